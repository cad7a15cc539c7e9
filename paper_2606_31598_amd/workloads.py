"""Seeded synthetic inputs for the products and propagations.

This module only draws input data: right-hand-side vectors, the initial
wavepacket, instance sizes of a batch, sampled row indices and planner
workloads.  It holds none of the operator's arithmetic (no matrix entries,
no products, no propagation), so the GPU library's callers and the CPU
reference checks can both take their inputs from here.
"""
import numpy as np


def gaussian_vectors(D: int, nvec: int, seed: int) -> np.ndarray:
    """nvec complex Gaussian vectors of length D, each normalised to 1.

    Shape (nvec, D), complex128: vector v is row v (the vector-contiguous
    layout of the library).
    """
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nvec, D)) + 1j * rng.standard_normal((nvec, D))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


def grid(D: int, x_min: float = -20.0, x_max: float = 20.0) -> np.ndarray:
    """Equispaced grid with both end points, spacing (x_max - x_min)/(D - 1)."""
    return x_min + np.arange(D) * ((x_max - x_min) / (D - 1))


def wavepacket(D: int, x0: float = 3.0, sigma: float = 1.0,
               x_min: float = -20.0, x_max: float = 20.0) -> np.ndarray:
    """Displaced Gaussian exp(-(x - x0)^2 / (2 sigma^2)) at rest, normalised
    on the grid (complex128, shape (1, D))."""
    x = grid(D, x_min, x_max)
    psi = np.exp(-0.5 * ((x - x0) / sigma) ** 2).astype(np.complex128)
    psi /= np.linalg.norm(psi)
    return psi[None, :]


def batch_sizes(n: int = 256, lo: int = 512, hi: int = 8192,
                seed: int = 0xC2) -> np.ndarray:
    """Instance dimensions drawn uniformly from [lo, hi] (inclusive)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=n).astype(np.int64)


def sampled_rows(D: int = 262144, n: int = 4096, seed: int = 3) -> np.ndarray:
    """n distinct row indices in [0, D), sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(D, size=n, replace=False)).astype(np.int64)


def planner_workloads(n: int, seed: int, log2_d=(12, 18), nvec_max: int = 64,
                      budget_gb=(16.0, 256.0), reuse=(1, 500)) -> list:
    """Planner problems: D = 2^k, nvec, memory budget, reuse count, family.

    D is a power of two in the given range, nvec log-uniform in [1, nvec_max]
    (integer), the budget log-uniform in GB, the reuse count log-uniform
    (integer), the family 0 (Philox-GUE) or 1 (sinc-DVR).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        k = int(rng.integers(log2_d[0], log2_d[1] + 1))
        nv = int(round(np.exp(rng.uniform(0.0, np.log(nvec_max)))))
        bud = float(np.exp(rng.uniform(np.log(budget_gb[0]), np.log(budget_gb[1]))))
        ru = int(round(np.exp(rng.uniform(np.log(reuse[0]), np.log(reuse[1])))))
        fam = int(rng.integers(0, 2))
        out.append({"D": 1 << k, "nvec": max(nv, 1), "budget_gb": bud,
                    "reuse": max(ru, 1), "family": fam})
    return out


def system_matrices(d_s: int, n_int: int, seed: int) -> tuple:
    """Synthetic system-side matrices of a system-bath operator: a Hermitian
    H_S and n_int Hermitian couplings A_a, each (G + G^H)/2 of a complex
    Gaussian G, rounded to complex64 values (returned as complex128)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(1 + n_int):
        G = rng.standard_normal((d_s, d_s)) + 1j * rng.standard_normal((d_s, d_s))
        out.append((0.5 * (G + G.conj().T)).astype(np.complex64).astype(np.complex128))
    return out[0], out[1:]
