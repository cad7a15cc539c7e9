"""GPU parity: Chebyshev propagation against the binary64 oracle.

The oracle runs the same centered Chebyshev expansion in binary64 on the same
binary32 generated entries; the harmonic-oscillator runs are also checked
against the exact coherent state.
"""
import numpy as np
import pytest

from oracle import chebyshev as ch
from paper_2606_31598_amd import workloads
from tests.gpu_util import rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_31598_amd import procmv
    procmv.load()
    return procmv


def test_gue_propagation_matches_oracle(pm, orc):
    D, nv, dt, steps = 700, 3, 0.05, 20
    op = pm.Operator.gue(D, seed=5).plan(256)
    psi0 = workloads.gaussian_vectors(D, nv, seed=6)
    P = to_dev(psi0)
    norms = op.propagate(P, dt, nsteps=steps, c=0.0, R=2.5, norms=True)
    got = to_host(P)
    H = orc.gue_dense(5, D)
    K = ch.cheb_order(2.5 * dt)
    ref = ch.propagate(lambda v: v @ H.T, psi0.astype(np.complex64), 0.0, 2.5, dt, K,
                       nsteps=steps)
    assert rel_l2(got, ref) < 1e-5
    assert np.max(np.abs(norms - 1.0)) < 1e-5


def test_gue_propagation_cached_identical(pm):
    D = 900
    psi0 = to_dev(workloads.gaussian_vectors(D, 2, seed=1))
    outs = []
    for strat, f in [(pm.PROCEDURAL, 0), (pm.PARTIAL, 0.5), (pm.FULL, 1)]:
        op = pm.Operator.gue(D, seed=2).plan(128, strat, f).set_tile_shape(1)
        P = psi0.clone()
        op.propagate(P, 0.05, nsteps=5)
        outs.append(to_host(P))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("D,steps", [(1024, 20), (4096, 4)])
def test_dvr_propagation_matches_oracle_and_closed_form(pm, orc, D, steps):
    dt = 0.05
    op = pm.Operator.dvr(D).plan(256)
    d = orc.DVR(D)
    e0, e1 = d.spectral_bounds()
    c, R = 0.5 * (e0 + e1), 0.5 * (e1 - e0)
    psi0 = workloads.wavepacket(D)
    P = to_dev(psi0)
    norms = op.propagate(P, dt, nsteps=steps, c=c, R=R, norms=True)
    got = to_host(P)
    Ht = np.ascontiguousarray(d.dense().T)
    K = ch.cheb_order(R * dt)
    ref = ch.propagate(lambda v: v.real @ Ht + 1j * (v.imag @ Ht),
                       psi0.astype(np.complex64), c, R, dt, K, nsteps=steps)
    exact = ch.coherent_state(d.x, steps * dt, 3.0, d.dx)[None, :]
    err_oracle = rel_l2(got, ref)
    err_exact = rel_l2(got, exact)
    print(f"D={D} steps={steps} K={K} err_vs_fp64={err_oracle:.3e} "
          f"err_vs_exact={err_exact:.3e} norm-1={norms[-1, 0] - 1:.2e}")
    assert err_oracle < 1e-4
    assert err_exact < 1e-4
    assert np.max(np.abs(norms - 1.0)) < 1e-4


def test_dvr_benchmark_configuration_one_step(pm, orc):
    """The benchmark's own configuration at full size (sinc-DVR D = 32768,
    dt = 0.05, K = 83,108 products, procedural b = 256, library bounds):
    checked through properties that hold at any size, since the binary64
    oracle cannot run 83,108 products of this size: the state stays
    normalised, and it matches the exact coherent state within the binary32
    error budget of one step (the growth with D and steps is documented with
    the accuracy sweep)."""
    D, dt = 32768, 0.05
    op = pm.Operator.dvr(D).plan(256, pm.PROCEDURAL)
    c, R = op.spectral_bounds()
    K = pm.cheb_order(R * dt, 1e-10)
    assert K == ch.cheb_order(R * dt, 1e-10)
    d = orc.DVR(D)
    P = to_dev(workloads.wavepacket(D))
    norms = op.propagate(P, dt, nsteps=1, K=K, c=c, R=R, norms=True)
    got = to_host(P)
    exact = ch.coherent_state(d.x, dt, 3.0, d.dx)[None, :]
    err = rel_l2(got, exact)
    print(f"D={D} K={K} err_vs_exact={err:.3e} norm-1={norms[-1, 0] - 1:.2e}")
    assert err < 1e-3                          # measured 5.0e-4
    assert abs(norms[-1, 0] - 1.0) < 2e-4      # measured -8.1e-5
