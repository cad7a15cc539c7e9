"""Plain CPU oracle for the block-procedural matrix-free product phi = H psi.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package.  It shares no code with
the GPU library (``paper_2606_31598_amd``) and never imports it; the two meet
only through the seeded input recipes in ``paper_2606_31598_amd.workloads``,
which hold none of the method's arithmetic.

Contents
--------
* generators and the row-by-row binary64 product (C, ``oracle.c``; paper
  Sec. II Eqs. blockmatvec/blockmatvecindex, Sec. III seeded and analytic
  generation);
* dense materialisation at small D (the definition of the product, for
  cross-checks);
* Chebyshev propagation (``oracle.chebyshev``; paper Sec. VII, centered
  Chebyshev recurrence);
* the imaginary-time Chebyshev filter e^{-tau H} (``oracle.chebyshev``;
  paper Sec. I and VII, TPQ filtering);
* matrix-free Lanczos spectral bounds (``oracle.lanczos``; paper Sec. VII);
* the system-bath Kronecker operator (``oracle.kron``; paper Sec. VII example);
* planner formulas and the MLP surrogate in binary64 (``oracle.planner``;
  paper Sec. IV).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def lib():
    """Load liboracle.so, compiling it first if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.path.join(_HERE, "liboracle.so")
    if not os.path.exists(path):
        _build.build()
    L = ctypes.CDLL(path)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    f32p = ctypes.POINTER(ctypes.c_float)
    f64p = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    c = ctypes
    L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.orc_u01.argtypes = [c.c_uint32]
    L.orc_u01.restype = c.c_float
    L.orc_logf32.argtypes = [c.c_float]
    L.orc_logf32.restype = c.c_float
    L.orc_logf32_vec.argtypes = [f32p, c.c_int64, f32p]
    L.orc_sincos2pi_vec.argtypes = [f32p, c.c_int64, f32p, f32p]
    L.orc_box_muller_vec.argtypes = [u32p, u32p, c.c_int64, f32p, f32p]
    L.orc_philox_vec.argtypes = [u32p, c.c_int64, c.c_uint32, c.c_uint32, u32p]
    L.orc_gue_entries_f32.argtypes = [c.c_uint64, c.c_int64, c.c_int64,
                                      c.c_int32, c.c_int32, c.c_float,
                                      c.c_float, f32p]
    L.orc_gue_apply_rows_f64.argtypes = [c.c_uint64, c.c_int64, c.c_float,
                                         c.c_float, f64p, c.c_int64,
                                         c.c_int32, i64p, c.c_int64, f64p]
    L.orc_dvr_tables.argtypes = [c.c_int64, c.c_double, c.c_double,
                                 c.c_double, c.c_double, c.c_int32, f64p,
                                 f64p, f32p, f32p, f64p, f64p]
    L.orc_dvr_apply_rows_f64.argtypes = [f64p, f64p, c.c_double, c.c_int64,
                                         f64p, c.c_int64, c.c_int32, i64p,
                                         c.c_int64, f64p]
    L.orc_num_threads.restype = c.c_int32
    _lib = L
    return L


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# Philox4x32-10 and the FP32 Gaussian transform
# --------------------------------------------------------------------------
def philox(ctr, key):
    """Raw Philox4x32-10 block for one counter (4 words) and key (2 words)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32),
                            _p(out, ctypes.c_uint32))
    return out


def philox_many(ctrs, key):
    c = np.ascontiguousarray(ctrs, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    lib().orc_philox_vec(_p(c, ctypes.c_uint32), c.shape[0], int(key[0]),
                         int(key[1]), _p(out, ctypes.c_uint32))
    return out


def u01(x) -> np.float32:
    return np.float32(lib().orc_u01(int(x)))


def logf32(u):
    u = np.ascontiguousarray(u, dtype=np.float32)
    out = np.empty_like(u)
    lib().orc_logf32_vec(_p(u, ctypes.c_float), u.size, _p(out, ctypes.c_float))
    return out


def sincos2pi_f32(u):
    u = np.ascontiguousarray(u, dtype=np.float32)
    s = np.empty_like(u)
    c = np.empty_like(u)
    lib().orc_sincos2pi_vec(_p(u, ctypes.c_float), u.size,
                            _p(s, ctypes.c_float), _p(c, ctypes.c_float))
    return s, c


def box_muller_f32(x0, x1):
    x0 = np.ascontiguousarray(x0, dtype=np.uint32)
    x1 = np.ascontiguousarray(x1, dtype=np.uint32)
    z0 = np.empty(x0.shape, np.float32)
    z1 = np.empty(x0.shape, np.float32)
    lib().orc_box_muller_vec(_p(x0, ctypes.c_uint32), _p(x1, ctypes.c_uint32),
                             x0.size, _p(z0, ctypes.c_float),
                             _p(z1, ctypes.c_float))
    return z0, z1


# --------------------------------------------------------------------------
# Philox-GUE operator
# --------------------------------------------------------------------------
def gue_scales(D: int, R: float = 1.0):
    """Entry scales: re, im ~ N(0, 1/(2D)) off the diagonal, N(0, 1/D) on it.

    Computed in binary64 and rounded once to binary32; ``R`` divides both
    (the Chebyshev half-width when the generator emits the scaled operator).
    """
    s_off = np.float32(np.sqrt(1.0 / (2.0 * D)) / R)
    s_diag = np.float32(np.sqrt(1.0 / D) / R)
    return s_off, s_diag


def gue_entries(seed: int, r0: int, c0: int, nr: int, nc: int,
                s_off=None, s_diag=None, D=None):
    """Window H[r0:r0+nr, c0:c0+nc] of generated binary32 entries (complex64)."""
    if s_off is None:
        s_off, s_diag = gue_scales(D)
    out = np.empty((nr, nc, 2), np.float32)
    lib().orc_gue_entries_f32(int(seed), int(r0), int(c0), int(nr), int(nc),
                              float(s_off), float(s_diag),
                              _p(out, ctypes.c_float))
    return out[..., 0] + 1j * out[..., 1].astype(np.complex64)


def gue_dense(seed: int, D: int) -> np.ndarray:
    """Dense complex128 materialisation of the generated operator (small D)."""
    return gue_entries(seed, 0, 0, D, D, D=D).astype(np.complex128)


def gue_apply_rows(seed: int, D: int, X: np.ndarray, rows=None,
                   s_off=None, s_diag=None) -> np.ndarray:
    """Y[:, r] = sum_j H[rows[r], j] X[:, j] in binary64, X of shape (R, D)."""
    if s_off is None:
        s_off, s_diag = gue_scales(D)
    X = np.ascontiguousarray(np.atleast_2d(X), dtype=np.complex128)
    R = X.shape[0]
    assert X.shape[1] == D
    rows = np.arange(D, dtype=np.int64) if rows is None else \
        np.ascontiguousarray(rows, dtype=np.int64)
    Y = np.empty((R, rows.size), np.complex128)
    lib().orc_gue_apply_rows_f64(int(seed), int(D), float(s_off), float(s_diag),
                                 _p(X.view(np.float64), ctypes.c_double), D, R,
                                 _p(rows, ctypes.c_int64), rows.size,
                                 _p(Y.view(np.float64), ctypes.c_double))
    return Y


# --------------------------------------------------------------------------
# Sinc-DVR harmonic oscillator
# --------------------------------------------------------------------------
class DVR:
    """Tables of the sinc-DVR operator H = T_off + diag(V) + d I.

    ``tk64``/``v64``/``d0`` are the binary64 values of the definition;
    ``tk32``/``v32`` their binary32 roundings and ``d32`` the binary64
    diagonal constant that goes with them (sum-rule compensated when
    ``compensate``).
    """

    def __init__(self, D, x_min=-20.0, x_max=20.0, mass=1.0, omega=1.0,
                 compensate=True):
        self.D = int(D)
        self.x_min, self.x_max, self.mass, self.omega = x_min, x_max, mass, omega
        self.tk64 = np.empty(D, np.float64)
        self.v64 = np.empty(D, np.float64)
        self.tk32 = np.empty(D, np.float32)
        self.v32 = np.empty(D, np.float32)
        d = np.empty(2, np.float64)
        dx = np.empty(1, np.float64)
        lib().orc_dvr_tables(self.D, x_min, x_max, mass, omega,
                             1 if compensate else 0,
                             _p(self.tk64, ctypes.c_double),
                             _p(self.v64, ctypes.c_double),
                             _p(self.tk32, ctypes.c_float),
                             _p(self.v32, ctypes.c_float),
                             _p(d, ctypes.c_double), _p(dx, ctypes.c_double))
        self.d0, self.d32 = float(d[0]), float(d[1])
        self.dx = float(dx[0])
        self.x = x_min + np.arange(D) * self.dx

    def spectral_bounds(self):
        """E_min = 0 (T and V are positive semidefinite); E_max = largest
        symbol value pi^2/(2 m dx^2) plus max V (Gershgorin-type bound)."""
        e_min = 0.0
        e_max = np.pi ** 2 / (2.0 * self.mass * self.dx ** 2) + float(self.v64.max())
        return e_min, e_max

    def dense(self, rounded=True) -> np.ndarray:
        """Dense real binary64 matrix (small D)."""
        tk = self.tk32.astype(np.float64) if rounded else self.tk64
        v = self.v32.astype(np.float64) if rounded else self.v64
        d = self.d32 if rounded else self.d0
        idx = np.arange(self.D)
        H = tk[np.abs(idx[:, None] - idx[None, :])]
        H[idx, idx] = v + d
        return H

    def apply_fft(self, X, rounded=True) -> np.ndarray:
        """Binary64 product H X of the same entries as ``apply_rows``, for
        any D: the Toeplitz part sum_j t(i - j) x_j is a linear convolution,
        evaluated by embedding the symbol t(-(D-1)) .. t(D-1) in a circulant
        of length N >= 2D - 1 and multiplying in Fourier space (numpy FFT);
        the diagonal (v_i + d) x_i is added directly.  X: (nvec, D)."""
        D = self.D
        tk = self.tk32.astype(np.float64) if rounded else self.tk64
        v = self.v32.astype(np.float64) if rounded else self.v64
        d = self.d32 if rounded else self.d0
        X = np.atleast_2d(np.asarray(X, dtype=np.complex128))
        N = 1 << int(np.ceil(np.log2(2 * D - 1))) if D > 1 else 1
        sym = self._fft_symbol(N, tk)
        Xp = np.zeros((X.shape[0], N), np.complex128)
        Xp[:, :D] = X
        Y = np.fft.ifft(np.fft.fft(Xp, axis=1) * sym[None, :], axis=1)[:, :D]
        return Y + (v + d)[None, :] * X

    def _fft_symbol(self, N, tk):
        """FFT of the circulant column c[k] = t(k) for 0 <= k < D,
        c[N - k] = t(-k) = t(k) for 0 < k < D, zero elsewhere (t(0) = 0)."""
        key = (N, tk.ctypes.data if tk is self.tk64 else "r")
        cache = getattr(self, "_sym_cache", None)
        if cache is not None and cache[0] == key:
            return cache[1]
        c = np.zeros(N, np.float64)
        c[1:self.D] = tk[1:self.D]
        c[N - self.D + 1:] = tk[1:self.D][::-1]
        sym = np.fft.fft(c)
        self._sym_cache = (key, sym)
        return sym

    def apply_rows(self, X, rows=None, rounded=True) -> np.ndarray:
        """Row-by-row binary64 product with the generated (or exact) entries."""
        D = self.D
        tk = self.tk32.astype(np.float64) if rounded else self.tk64
        v = self.v32.astype(np.float64) if rounded else self.v64
        d = self.d32 if rounded else self.d0
        X = np.ascontiguousarray(np.atleast_2d(X), dtype=np.complex128)
        R = X.shape[0]
        rows = np.arange(D, dtype=np.int64) if rows is None else \
            np.ascontiguousarray(rows, dtype=np.int64)
        Y = np.empty((R, rows.size), np.complex128)
        tk = np.ascontiguousarray(tk)
        v = np.ascontiguousarray(v)
        lib().orc_dvr_apply_rows_f64(_p(tk, ctypes.c_double),
                                     _p(v, ctypes.c_double), float(d), D,
                                     _p(X.view(np.float64), ctypes.c_double),
                                     D, R, _p(rows, ctypes.c_int64), rows.size,
                                     _p(Y.view(np.float64), ctypes.c_double))
        return Y
