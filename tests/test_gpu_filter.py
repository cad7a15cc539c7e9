"""GPU parity: imaginary-time Chebyshev filter e^{-tau H} (paper Sec. I and
Sec. VII: TPQ states are random vectors filtered by e^{-beta H/2}) against the
binary64 oracle on the same binary32 entries and the same order K.

Tolerances: a CPU model of the library's arithmetic (complex64 Chebyshev
vectors, binary64 coefficient sum) differs from the binary64 filter by
4e-7 (GUE, tau = 1.5) and 6.9e-6 (sinc-DVR, tau = 0.5: the result is 5x
smaller than the input, so the vectors' rounding weighs 5x more); the tests
allow 5e-6 and 5e-5.  The long filter (tau = 6) is checked through what it
must produce, the oscillator ground level 1/2.
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


@pytest.mark.parametrize("b,strategy,frac", [(256, 0, 0.0), (128, 1, 0.5), (256, 2, 1.0)])
def test_gue_filter_matches_oracle(pm, orc, b, strategy, frac):
    D, nv, tau, c, R = 700, 3, 1.5, 0.0, 2.5
    op = pm.Operator.gue(D, seed=5).plan(b, strategy, frac)
    psi0 = workloads.gaussian_vectors(D, nv, seed=6).astype(np.complex64)
    K = ch.filter_order(R * tau, 1e-10)
    P = to_dev(psi0)
    norms = op.filter(P, tau, K=K, c=c, R=R, norms=True)
    got = to_host(P)
    H = orc.gue_dense(5, D)
    ref = ch.imag_time_filter(lambda v: v @ H.T, psi0.astype(np.complex128), c, R, tau, K)
    assert rel_l2(got, ref) < 5e-6
    assert np.allclose(norms, np.linalg.norm(ref, axis=1), rtol=5e-6)


def test_dvr_filter_matches_oracle(pm, orc):
    D, tau = 1024, 0.5
    op = pm.Operator.dvr(D).plan(256)
    d = orc.DVR(D)
    e0, e1 = d.spectral_bounds()
    c, R = 0.5 * (e0 + e1), 0.5 * (e1 - e0)
    K = ch.filter_order(R * tau, 1e-10)
    psi0 = workloads.wavepacket(D).astype(np.complex64)
    P = to_dev(psi0)
    op.filter(P, tau, K=K, c=c, R=R)
    ref = ch.imag_time_filter(lambda v: d.apply_rows(v), psi0.astype(np.complex128), c, R,
                              tau, K)
    assert rel_l2(to_host(P), ref) < 5e-5


def test_dvr_long_filter_reaches_the_ground_state(pm, orc):
    D, tau = 1024, 6.0
    op = pm.Operator.dvr(D).plan(256)
    P = to_dev(workloads.wavepacket(D))
    op.filter(P, tau)                        # analytic bounds, automatic order
    phi = to_host(P).astype(np.complex128)
    phi /= np.linalg.norm(phi)
    d = orc.DVR(D)
    energy = float(np.real(np.vdot(phi, d.apply_rows(phi))))
    # excited-state weight left after tau = 6 is ~e^{-12}; binary32 vectors
    assert abs(energy - 0.5) < 1e-4


def test_zero_tau_is_identity(pm):
    D = 300
    op = pm.Operator.gue(D, seed=2).plan(128)
    psi0 = workloads.gaussian_vectors(D, 2, seed=1).astype(np.complex64)
    P = to_dev(psi0)
    op.filter(P, 0.0, c=0.0, R=2.5)
    assert np.array_equal(to_host(P), psi0)


def test_filter_rejects_bad_arguments(pm):
    op = pm.Operator.gue(64, seed=1)
    P = to_dev(workloads.gaussian_vectors(64, 1, seed=1))
    with pytest.raises(pm.ProcmvError):
        op.filter(P, 1.0)                    # no plan yet
    op.plan(64)
    with pytest.raises(pm.ProcmvError):
        op.filter(P, -1.0)
    with pytest.raises(pm.ProcmvError):
        op.filter(P, 1e6, c=-1e3, R=1.0)     # e^{-tau E_min} overflows binary64
