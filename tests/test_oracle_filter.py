"""Pins of the binary64 imaginary-time Chebyshev filter oracle (paper Sec. I
and Sec. VII: thermal pure quantum states are random vectors filtered by a
Chebyshev expansion of e^{-beta H/2}).

The filter is checked against what fixes it independently of its code: the
library's exponentially scaled modified Bessel functions (scipy ``ive``), the
matrix exponential by exact diagonalisation, the semigroup property, tau = 0,
and the harmonic-oscillator ground level 1/2 that a long filter projects onto.
"""
import numpy as np
import pytest
from scipy import special

import oracle
from oracle import chebyshev as ch
from paper_2606_31598_amd import workloads


@pytest.mark.parametrize("z", [0.3, 2.0, 17.5, 160.0, 900.0])
def test_scaled_bessel_i_matches_scipy(z):
    K = 60 + int(3 * np.sqrt(z))
    got = ch.bessel_i_scaled_seq(z, K)
    ref = special.ive(np.arange(K + 1), z)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-300)


def test_order_rule():
    for z in (0.5, 10.0, 200.0):
        K = ch.filter_order(z, 1e-10)
        v = special.ive(np.arange(K + 3), z)
        assert 2 * v[K] < 1e-10 and 2 * v[K + 1] < 1e-10
        assert K == 1 or not (2 * v[K - 1] < 1e-10 and 2 * v[K] < 1e-10)


def _eigh_filter(H, psi, tau):
    lam, U = np.linalg.eigh(H)
    return (U * np.exp(-tau * lam)) @ (U.conj().T @ psi.T)


@pytest.mark.parametrize("tau", [0.0, 0.4, 3.0])
def test_gue_filter_equals_matrix_exponential(tau):
    D = 96
    H = oracle.gue_dense(4, D)
    psi = workloads.gaussian_vectors(D, 2, seed=8)
    c, R = 0.0, 2.5
    K = ch.filter_order(R * tau, 1e-13)
    got = ch.imag_time_filter(lambda v: v @ H.T, psi, c, R, tau, K)
    ref = _eigh_filter(H, psi, tau).T
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-11


def test_semigroup():
    D = 80
    H = oracle.gue_dense(6, D)
    psi = workloads.gaussian_vectors(D, 1, seed=2)
    f = lambda v, t: ch.imag_time_filter(lambda x: x @ H.T, v, 0.0, 2.5, t,
                                         ch.filter_order(2.5 * t, 1e-13))
    a = f(f(psi, 0.7), 1.1)
    b = f(psi, 1.8)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-11


def test_dvr_filter_projects_on_the_ground_state():
    D = 256
    d = oracle.DVR(D, x_min=-10.0, x_max=10.0)
    H = d.dense(rounded=False)
    e0, e1 = d.spectral_bounds()
    c, R = 0.5 * (e0 + e1), 0.5 * (e1 - e0)
    psi = workloads.gaussian_vectors(D, 1, seed=3)
    tau = 12.0                     # e^{-tau (E_1 - E_0)} = e^{-12}
    # the result has norm ~1.6e-4: a 1e-15 coefficient cut keeps it to ~1e-11 relative
    K = ch.filter_order(R * tau, 1e-15)
    phi = ch.imag_time_filter(lambda v: v @ H.T, psi, c, R, tau, K)[0]
    phi /= np.linalg.norm(phi)
    energy = float(np.real(np.vdot(phi, H @ phi)))
    assert abs(energy - 0.5) < 1e-8
    ref = _eigh_filter(H, psi, tau).T[0]
    assert np.linalg.norm(phi - ref / np.linalg.norm(ref)) < 1e-10
