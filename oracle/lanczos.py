"""Matrix-free Lanczos estimate of the spectral bounds, in binary64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper Sec. VII: before the centered Chebyshev propagation, a short run of
matrix-free Lanczos iterations (m = 40 in the paper's run) estimates E_min and
E_max, which give the shift c = (E_max + E_min)/2 and half-width
R = (E_max - E_min)/2.  The paper does not spell out the iteration, the start
vector or any safety margin; the readings taken here:

* plain Hermitian Lanczos (three-term recurrence, no reorthogonalisation):
  v_1 = v0/||v0||; for j = 1..m: w = H v_j, alpha_j = Re <v_j, w>,
  w <- w - alpha_j v_j - beta_{j-1} v_{j-1}, beta_j = ||w||,
  v_{j+1} = w / beta_j; stop early only when beta_j is exactly zero;
* the start vector is an input (a seeded complex Gaussian in the tests);
* the extreme Ritz values theta of the tridiagonal T_m (diagonal alpha,
  off-diagonal beta_1..beta_{m-1}) are widened by their residual estimates
  |beta_m s_m| (s = the unit eigenvector of T_m, s_m its last entry), which
  bound the distance from each Ritz value to the spectrum:
  E_min = theta_min - r_min, E_max = theta_max + r_max.

A numpy eigen-solver serves as the tridiagonal step.
"""
import numpy as np


def lanczos(apply_h, v0: np.ndarray, m: int, return_basis: bool = False):
    """alpha[0..n), beta[0..n) of n <= m Lanczos steps (beta[j] = ||w|| after
    step j, so beta[n-1] is the residual coupling beta_m)."""
    v = np.asarray(v0, np.complex128).ravel()
    v = v / np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    alpha, beta, basis = [], [], []
    for _ in range(m):
        basis.append(v)
        w = np.asarray(apply_h(v), np.complex128).ravel()
        a = float(np.real(np.vdot(v, w)))
        w = w - a * v - b_prev * v_prev
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        if b == 0.0:
            break
        v_prev, v, b_prev = v, w / b, b
    alpha, beta = np.array(alpha), np.array(beta)
    if return_basis:
        return alpha, beta, np.array(basis)
    return alpha, beta


def ritz_bounds(alpha: np.ndarray, beta: np.ndarray) -> dict:
    """Extreme Ritz values of T_m, their residual estimates and the widened
    bounds with the Chebyshev shift and half-width."""
    n = alpha.size
    T = np.diag(alpha) + np.diag(beta[:n - 1], 1) + np.diag(beta[:n - 1], -1)
    theta, S = np.linalg.eigh(T)
    r_min = abs(beta[n - 1] * S[n - 1, 0])
    r_max = abs(beta[n - 1] * S[n - 1, n - 1])
    e_min = theta[0] - r_min
    e_max = theta[-1] + r_max
    return {"theta_min": float(theta[0]), "theta_max": float(theta[-1]),
            "r_min": float(r_min), "r_max": float(r_max),
            "e_min": float(e_min), "e_max": float(e_max),
            "c": 0.5 * (e_max + e_min), "R": 0.5 * (e_max - e_min), "steps": n}


def spectral_bounds(apply_h, v0: np.ndarray, m: int = 40) -> dict:
    alpha, beta = lanczos(apply_h, v0, m)
    out = ritz_bounds(alpha, beta)
    out["alpha"], out["beta"] = alpha, beta
    return out
