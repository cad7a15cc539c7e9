"""Write dvr_D32768_fp64.json: the binary64 oracle's propagation of the
benchmark's sinc-DVR configuration at full size, for the GPU tests.

Configuration (paper Sec. VII centered Chebyshev propagation of the
harmonic-oscillator sinc-DVR operator; Sec. III analytic generation):
D = 32768 on [-20, 20], m = omega = 1, the binary32 entries with the
sum-rule compensated diagonal, initial state the displaced Gaussian at
x0 = 3, sigma = 1 rounded to complex64, dt = 0.05, order K from the
coefficient rule at tol 1e-10 with the analytic bounds.  Every product is the
oracle's binary64 FFT-Toeplitz product (``oracle.DVR.apply_fft``), pinned
against the row-by-row product in the oracle tests.

Recorded per step: the rel-L2 distance of the binary64 state to the exact
coherent state, its norm, and the state at 64 grid points x in [-5, 5].
Only the oracle is called.  Runtime: several minutes per step on 8 cores.

    python tests/golden/make_dvr_full_size.py [nsteps]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import chebyshev as ch  # noqa: E402
from paper_2606_31598_amd import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dvr_D32768_fp64.json")


def main(nsteps: int = 2) -> None:
    D, dt, x0 = 32768, 0.05, 3.0
    d = oracle.DVR(D)
    e0, e1 = d.spectral_bounds()
    c, R = 0.5 * (e0 + e1), 0.5 * (e1 - e0)
    K = ch.cheb_order(R * dt, 1e-10)
    psi = workloads.wavepacket(D).astype(np.complex64).astype(np.complex128)
    idx = np.searchsorted(d.x, np.linspace(-5.0, 5.0, 64))
    rec = {"_source": __doc__.strip().splitlines()[0], "D": D, "dt": dt, "x0": x0,
           "c": c, "R": R, "K": K, "tol": 1e-10, "sample_index": idx.tolist(), "steps": []}
    for step in range(1, nsteps + 1):
        t0 = time.time()
        psi = ch.propagate(lambda v: d.apply_fft(v), psi, c, R, dt, K, nsteps=1)
        exact = ch.coherent_state(d.x, step * dt, x0, d.dx)[None, :]
        err = float(np.linalg.norm(psi - exact) / np.linalg.norm(exact))
        rec["steps"].append({"step": step, "fp64_vs_exact": err,
                             "norm": float(np.linalg.norm(psi)),
                             "sample": [[float(z.real), float(z.imag)]
                                        for z in psi[0, idx]]})
        print(f"step {step}: fp64 vs exact {err:.3e} ({time.time() - t0:.0f} s)", flush=True)
        with open(OUT, "w") as f:
            json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2)
