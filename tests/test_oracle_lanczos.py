"""Pins of the binary64 Lanczos spectral-bounds oracle (paper Sec. VII: Lanczos
estimates E_min, E_max before the centered Chebyshev propagation).

Each check rests on a fact fixed by linear algebra, not on the oracle's own
formulas: a full Krylov space reproduces the whole spectrum; the basis is
orthonormal and reduces H to the tridiagonal (the defining property of the
recurrence: a dropped term or a wrong sign breaks it); Ritz values lie inside
the spectrum (Cauchy interlacing); each Ritz value has an eigenvalue within
its residual estimate; the sinc-DVR oscillator's lowest level is 1/2.
"""
import numpy as np

import oracle
from oracle import lanczos as ol
from paper_2606_31598_amd import workloads


def _gue(D, seed=1):
    H = oracle.gue_dense(seed, D)
    return H, (lambda v: H @ v)


def test_full_krylov_space_gives_the_spectrum():
    D = 12
    H, ap = _gue(D)
    v0 = workloads.gaussian_vectors(D, 1, 5)[0]
    alpha, beta = ol.lanczos(ap, v0, D)
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    assert np.allclose(np.linalg.eigvalsh(T), np.linalg.eigvalsh(H), atol=1e-9)
    assert beta[-1] < 1e-9            # the Krylov space is invariant


def test_basis_is_orthonormal_and_tridiagonalises():
    D, m = 200, 30
    H, ap = _gue(D, seed=7)
    v0 = workloads.gaussian_vectors(D, 1, 6)[0]
    alpha, beta, V = ol.lanczos(ap, v0, m, return_basis=True)
    assert np.allclose(V.conj() @ V.T, np.eye(m), atol=1e-9)
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    assert np.allclose(V.conj() @ H @ V.T, T, atol=1e-9)


def test_ritz_values_interlace_and_residuals_bound_the_distance():
    D = 256
    H, ap = _gue(D, seed=3)
    lam = np.linalg.eigvalsh(H)
    b = ol.spectral_bounds(ap, workloads.gaussian_vectors(D, 1, 2)[0], m=40)
    assert b["theta_min"] >= lam[0] - 1e-10 and b["theta_max"] <= lam[-1] + 1e-10
    assert np.min(np.abs(lam - b["theta_min"])) <= b["r_min"] + 1e-10
    assert np.min(np.abs(lam - b["theta_max"])) <= b["r_max"] + 1e-10
    # semicircle of radius 2 for the normalised GUE-like operator
    assert 1.6 < b["theta_max"] <= lam[-1] and lam[0] <= b["theta_min"] < -1.6


def test_dvr_oscillator_bounds():
    D = 512
    dvr = oracle.DVR(D)
    H = dvr.dense(rounded=False)
    lam = np.linalg.eigvalsh(H)
    assert abs(lam[0] - 0.5) < 1e-6   # harmonic-oscillator ground level (n + 1/2)
    b = ol.spectral_bounds(lambda v: H @ v, workloads.gaussian_vectors(D, 1, 4)[0], m=40)
    assert lam[0] - 1e-9 <= b["theta_min"] and b["theta_max"] <= lam[-1] + 1e-9
    # the top of the spectrum converges fast: within 1e-3 relative
    assert abs(b["theta_max"] - lam[-1]) < 1e-3 * lam[-1]
    assert b["e_max"] >= lam[-1] - 1e-9
    # the analytic bound [0, pi^2/(2 dx^2) + max V] contains the spectrum
    lo, hi = dvr.spectral_bounds()
    assert lo <= lam[0] and lam[-1] <= hi
