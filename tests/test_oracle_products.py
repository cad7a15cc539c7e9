"""Pins of the oracle's binary64 products (paper Sec. II, Eq. blockmatvecindex).

The row-by-row C product is checked against an independent dense
materialisation (numpy matmul), against the Hermitian identity
<x, H y> = <H x, y>, against linearity, and for the sinc-DVR operator against
an FFT-based Toeplitz product and the harmonic-oscillator spectrum n + 1/2.
"""
import numpy as np
import pytest

from oracle import chebyshev as ch
from paper_2606_31598_amd import workloads


def test_gue_rows_match_dense(orc):
    D = 700
    X = workloads.gaussian_vectors(D, 3, seed=2)
    H = orc.gue_dense(1, D)
    Y = orc.gue_apply_rows(1, D, X)
    ref = X @ H.T
    assert np.max(np.abs(Y - ref)) < 1e-13
    rows = np.array([0, 5, 699, 350])
    Ys = orc.gue_apply_rows(1, D, X, rows)
    assert np.max(np.abs(Ys - ref[:, rows])) < 1e-13


def test_gue_hermitian_identity(orc):
    D = 513
    x = workloads.gaussian_vectors(D, 1, seed=3)
    y = workloads.gaussian_vectors(D, 1, seed=4)
    Hx = orc.gue_apply_rows(9, D, x)
    Hy = orc.gue_apply_rows(9, D, y)
    lhs = np.vdot(x[0], Hy[0])
    rhs = np.vdot(Hx[0], y[0])
    assert abs(lhs - rhs) < 1e-13


def test_gue_linearity(orc):
    D = 257
    x = workloads.gaussian_vectors(D, 2, seed=5)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    comb = (a * x[0] + b * x[1])[None]
    Y = orc.gue_apply_rows(3, D, np.vstack([x, comb]))
    assert np.max(np.abs(Y[2] - (a * Y[0] + b * Y[1]))) < 1e-13


def test_gue_norm_expectation(orc):
    """E ||H psi||^2 = 1 for a unit psi (row variances sum to 1)."""
    D = 2048
    x = workloads.gaussian_vectors(D, 8, seed=2)
    Y = orc.gue_apply_rows(1, D, x)
    n2 = np.sum(np.abs(Y) ** 2, axis=1)
    assert abs(n2.mean() - 1) < 0.05


def test_dvr_rows_match_dense_and_fft(orc):
    D = 1000
    d = orc.DVR(D)
    X = workloads.gaussian_vectors(D, 2, seed=6)
    Y = d.apply_rows(X)
    H = d.dense()
    ref = X @ H.T
    assert np.max(np.abs(Y - ref)) / np.max(np.abs(ref)) < 1e-14
    # FFT Toeplitz product: first column c = tk32 with the constant diagonal
    col = d.tk32.astype(np.float64).copy()
    col[0] = d.d32
    n = 2 * D
    circ = np.concatenate([col, [0.0], col[1:][::-1]])
    fc = np.fft.fft(circ, n)
    conv = np.fft.ifft(fc[None, :] * np.fft.fft(X, n, axis=1), axis=1)[:, :D]
    fftY = conv + X * d.v32.astype(np.float64)[None, :]
    assert np.max(np.abs(fftY - ref)) / np.max(np.abs(ref)) < 1e-10


@pytest.mark.parametrize("D", [256, 512])
def test_dvr_harmonic_spectrum(orc, D):
    d = orc.DVR(D)
    w = np.linalg.eigvalsh(d.dense(rounded=False))
    assert np.max(np.abs(w[:6] - (np.arange(6) + 0.5))) < 1e-8
    e_min, e_max = d.spectral_bounds()
    assert e_min <= w[0] and w[-1] <= e_max


def test_dvr_compensation_restores_low_spectrum(orc):
    D = 1024
    plain = orc.DVR(D, compensate=False)
    comp = orc.DVR(D, compensate=True)
    w_plain = np.linalg.eigvalsh(plain.dense())[:5]
    w_comp = np.linalg.eigvalsh(comp.dense())[:5]
    exact = np.arange(5) + 0.5
    assert np.max(np.abs(w_comp - exact)) < np.max(np.abs(w_plain - exact))
    assert np.max(np.abs(w_comp - exact)) < 1e-5
    # the exact tables are untouched by the choice
    assert np.array_equal(plain.tk32, comp.tk32) and plain.d0 == comp.d0


def test_dvr_entries_closed_form(orc):
    D = 101
    d = orc.DVR(D, x_min=-5.0, x_max=5.0)
    dx = 10.0 / 100
    assert d.dx == dx
    k = np.arange(1, D)
    assert np.allclose(d.tk64[1:], (-1.0) ** k / (dx * dx * k * k), rtol=1e-15)
    assert np.allclose(d.v64, 0.5 * d.x ** 2, rtol=1e-15)
    assert np.isclose(d.d0, np.pi ** 2 / (6 * dx * dx), rtol=1e-15)
    assert np.array_equal(d.tk32, d.tk64.astype(np.float32))


@pytest.mark.parametrize("D", [2, 3, 64, 777, 4096])
def test_dvr_fft_product_matches_rows(orc, D):
    """The oracle's FFT-Toeplitz product (used for long propagations) equals
    the row-by-row binary64 product of the same entries, rounded and exact
    tables, and is Hermitian: <x, H y> = <H x, y>."""
    d = orc.DVR(D)
    X = workloads.gaussian_vectors(D, 2, seed=D)
    for rounded in (True, False):
        a = d.apply_fft(X, rounded=rounded)
        b = d.apply_rows(X, rounded=rounded)
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-13
    Hx = d.apply_fft(X[:1])
    Hy = d.apply_fft(X[1:])
    lhs = np.vdot(X[0], Hy[0])
    rhs = np.vdot(Hx[0], X[1])
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(Hx) * np.linalg.norm(X[1])


def test_dvr_fft_propagation_matches_dense(orc):
    """Chebyshev propagation through the FFT product equals the one through
    the dense binary64 matrix (same entries) to rounding."""
    D, dt, steps = 512, 0.05, 5
    d = orc.DVR(D)
    H = d.dense()
    e0, e1 = d.spectral_bounds()
    c, R = (e0 + e1) / 2, (e1 - e0) / 2
    K = ch.cheb_order(R * dt)
    psi = workloads.wavepacket(D)
    a = ch.propagate(lambda v: d.apply_fft(v), psi, c, R, dt, K, nsteps=steps)
    b = ch.propagate(lambda v: v @ H.T, psi, c, R, dt, K, nsteps=steps)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-12
