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


def step_budget(n):
    """1e-4 after 200 steps, rounding errors of independent steps adding in
    quadrature: 1e-4 sqrt(n / 200) after n steps."""
    return 1e-4 * np.sqrt(n / 200.0)


def _dvr_case(pm, orc, D, steps, precision):
    dt = 0.05
    op = pm.Operator.dvr(D).plan(256, precision=precision)
    d = orc.DVR(D)
    e0, e1 = d.spectral_bounds()
    c, R = 0.5 * (e0 + e1), 0.5 * (e1 - e0)
    psi0 = workloads.wavepacket(D)
    P = to_dev(psi0)
    norms = op.propagate(P, dt, nsteps=steps, c=c, R=R, norms=True)
    got = to_host(P)
    K = ch.cheb_order(R * dt)
    ref = ch.propagate(lambda v: d.apply_fft(v), psi0.astype(np.complex64), c, R, dt, K,
                       nsteps=steps)
    exact = ch.coherent_state(d.x, steps * dt, 3.0, d.dx)[None, :]
    return rel_l2(got, ref), rel_l2(got, exact), norms, K


def test_dvr_propagation_matches_oracle_and_closed_form(pm, orc):
    """Plain binary32 arithmetic at D = 1024 (121 products per step) stays
    within the scaled budget after 20 steps, against the binary64 oracle and
    the exact coherent state."""
    D, steps = 1024, 20
    err_oracle, err_exact, norms, K = _dvr_case(pm, orc, D, steps, pm.FP32)
    print(f"D={D} steps={steps} K={K} err_vs_fp64={err_oracle:.3e} "
          f"err_vs_exact={err_exact:.3e} norm-1={norms[-1, 0] - 1:.2e}")
    assert err_oracle < step_budget(steps)
    assert err_exact < step_budget(steps)
    assert np.max(np.abs(norms - 1.0)) < step_budget(steps)


def test_dvr_plain_binary32_error_grows_with_products(pm, orc):
    """At D = 4096 (1381 products per step) plain binary32 vectors and sums
    leave the scaled budget (the rounding of every product accumulates over
    the terms of a step), while the compensated arithmetic of the same
    operator stays far inside it."""
    D, steps = 4096, 4
    e_plain, _, _, _ = _dvr_case(pm, orc, D, steps, pm.FP32)
    e_comp, _, _, _ = _dvr_case(pm, orc, D, steps, pm.FP32_COMPENSATED)
    print(f"D={D} steps={steps} plain {e_plain:.2e} compensated {e_comp:.2e} "
          f"budget {step_budget(steps):.2e}")
    assert e_comp < step_budget(steps) < e_plain
    assert e_comp < e_plain / 10
