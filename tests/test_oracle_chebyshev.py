"""Pins of the oracle's Chebyshev propagation (paper Sec. VII).

Bessel values against scipy's AMOS-based jv, the independent sum rule
J_0^2 + 2 sum J_k^2 = 1, the propagator against exact diagonalisation,
norm conservation, the t = 0 identity, the group property, and the
harmonic-oscillator coherent state.
"""
import numpy as np
import pytest
from scipy.special import jv

from oracle import chebyshev as ch
from paper_2606_31598_amd import workloads


@pytest.mark.parametrize("x", [0.125, 1.0, 7.5, 141.37, 5000.0])
def test_bessel_against_scipy(x):
    K = ch.cheb_order(x, 1e-12)
    j = ch.bessel_j_seq(x, K)
    ks = np.unique(np.linspace(0, K, 40).astype(int))
    assert np.max(np.abs(j[ks] - jv(ks, x))) < 1e-13
    # independent sum rule (the normalisation uses the even-index rule)
    assert abs(j[0] ** 2 + 2 * np.sum(j[1:] ** 2) - 1) < 1e-12


def test_order_rule():
    for x in [0.125, 3.0, 141.37, 2000.0]:
        K = ch.cheb_order(x, 1e-10)
        assert K >= x
        assert 2 * abs(jv(K, x)) < 1e-10 and 2 * abs(jv(K + 1, x)) < 1e-10
        assert not (2 * abs(jv(K - 1, x)) < 1e-10 and 2 * abs(jv(K, x)) < 1e-10) or K - 1 < x


def test_coefficients_reproduce_exponential():
    """sum_k a_k T_k(y) = exp(-i x y) on [-1, 1] (Jacobi-Anger)."""
    x = 40.0
    K = ch.cheb_order(x, 1e-14)
    a = ch.cheb_coeffs(x, K)
    y = np.linspace(-1, 1, 101)
    T = np.cos(np.outer(np.arange(K + 1), np.arccos(y)))
    assert np.max(np.abs(a @ T - np.exp(-1j * x * y))) < 1e-12


def _gue(orc, D, seed=1):
    return orc.gue_dense(seed, D)


def test_propagate_matches_eigh_gue(orc):
    D = 256
    H = _gue(orc, D)
    psi = workloads.gaussian_vectors(D, 2, seed=2)
    dt, c, R = 0.05, 0.0, 2.5
    K = ch.cheb_order(R * dt)
    out = ch.propagate(lambda v: v @ H.T, psi, c, R, dt, K, nsteps=20)
    U = ch.exact_propagator(H, 20 * dt)
    assert np.max(np.abs(out - psi @ U.T)) < 1e-9
    assert np.max(np.abs(np.linalg.norm(out, axis=1) - 1)) < 1e-10


def test_propagate_matches_eigh_dvr(orc):
    D = 256
    d = orc.DVR(D)
    H = d.dense()
    e0, e1 = d.spectral_bounds()
    c, R = (e0 + e1) / 2, (e1 - e0) / 2
    dt = 0.05
    K = ch.cheb_order(R * dt)
    psi = workloads.wavepacket(D)
    out = ch.propagate(lambda v: v @ H.T, psi, c, R, dt, K, nsteps=10)
    U = ch.exact_propagator(H, 10 * dt)
    assert np.max(np.abs(out - psi @ U.T)) < 1e-9


def test_propagate_identity_and_group(orc):
    D = 128
    H = _gue(orc, D, seed=4)
    psi = workloads.gaussian_vectors(D, 1, seed=8)
    ap = lambda v: v @ H.T
    same = ch.propagate(ap, psi, 0.0, 2.5, 0.0, 0)
    assert np.array_equal(same, psi)
    one = ch.propagate(ap, psi, 0.0, 2.5, 0.2, ch.cheb_order(0.5, 1e-14))
    two = ch.propagate(ap, psi, 0.0, 2.5, 0.1, ch.cheb_order(0.25, 1e-14), nsteps=2)
    assert np.max(np.abs(one - two)) < 1e-12


def test_coherent_state_closed_form(orc):
    D = 512
    d = orc.DVR(D)
    H = d.dense(rounded=False)
    psi0 = ch.coherent_state(d.x, 0.0, 3.0, d.dx)
    assert np.allclose(psi0, workloads.wavepacket(D)[0], atol=1e-12)
    for t in [0.7, 10.0]:
        U = ch.exact_propagator(H, t)
        assert np.linalg.norm(U @ psi0 - ch.coherent_state(d.x, t, 3.0, d.dx)) < 1e-10


def test_dvr_propagation_close_to_closed_form(orc):
    """FP32-rounded entries with the compensated diagonal, binary64 Chebyshev:
    within 1e-6 of the exact coherent state after 20 steps at D = 1024."""
    D = 1024
    d = orc.DVR(D)
    H = d.dense()
    e0, e1 = d.spectral_bounds()
    c, R = (e0 + e1) / 2, (e1 - e0) / 2
    dt = 0.05
    K = ch.cheb_order(R * dt)
    out = ch.propagate(lambda v: v @ H.T, workloads.wavepacket(D), c, R, dt, K,
                       nsteps=20)
    ref = ch.coherent_state(d.x, 20 * dt, 3.0, d.dx)
    assert np.linalg.norm(out[0] - ref) < 1e-6
