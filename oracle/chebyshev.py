"""Chebyshev real-time propagation in binary64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper Sec. VII (centered Chebyshev propagation, citing Tal-Ezer & Kosloff
1984): with spectral bounds E_min, E_max the operator is rescaled to
Ht = (H - c I)/R, c = (E_max + E_min)/2, R = (E_max - E_min)/2, and the
Chebyshev vectors obey q_0 = psi, q_1 = Ht q_0, q_{l+1} = 2 Ht q_l - q_{l-1}.
The paper does not print the expansion coefficients; they follow from the
Jacobi-Anger expansion e^{-i z cos(theta)} = sum_k (2 - delta_k0) (-i)^k
J_k(z) cos(k theta), so that

    psi(t + dt) = e^{-i c dt} sum_{k=0}^{K} a_k q_k,
    a_k = (2 - delta_k0) (-i)^k J_k(R dt).

The order K follows the coefficient-tolerance rule (paper: "--cheb-tol" and
the Chebyshev-order discussion in Sec. VII): the first k >= R dt at which two
consecutive coefficients fall below the tolerance.
"""
import math

import numpy as np


def bessel_j_seq(x: float, kmax: int) -> np.ndarray:
    """J_0(x) .. J_kmax(x) for x >= 0 by Miller's backward recurrence.

    J_{k-1} = (2k/x) J_k - J_{k+1}, started far above max(kmax, x) from
    (0, tiny), rescaled to avoid overflow, and normalised with the sum rule
    J_0 + 2 sum_{k>=1} J_{2k} = 1.
    """
    if x == 0.0:
        out = np.zeros(kmax + 1)
        out[0] = 1.0
        return out
    top = int(max(kmax, x)) + 30 + int(20.0 * max(x, 1.0) ** (1.0 / 3.0))
    j = np.zeros(top + 2)
    j[top + 1] = 0.0
    j[top] = 1e-300
    for k in range(top, 0, -1):
        j[k - 1] = (2.0 * k / x) * j[k] - j[k + 1]
        if abs(j[k - 1]) > 1e250:
            j[k - 1:] *= 1e-250
    norm = j[0] + 2.0 * j[2::2].sum()
    return j[: kmax + 1] / norm


def cheb_order(x: float, tol: float = 1e-10) -> int:
    """Smallest k >= x with 2|J_k(x)| < tol and 2|J_{k+1}(x)| < tol."""
    kmax = int(x) + 60 + int(30.0 * max(x, 1.0) ** (1.0 / 3.0))
    j = bessel_j_seq(x, kmax + 1)
    k = int(math.ceil(x))
    while k + 1 <= kmax:
        if 2.0 * abs(j[k]) < tol and 2.0 * abs(j[k + 1]) < tol:
            return k
        k += 1
    raise RuntimeError("order search ran past the table")


def cheb_coeffs(x: float, K: int) -> np.ndarray:
    """a_k = (2 - delta_k0) (-i)^k J_k(x), k = 0..K (complex128)."""
    j = bessel_j_seq(x, K)
    k = np.arange(K + 1)
    a = ((-1j) ** (k % 4)) * j * 2.0
    a[0] = j[0]
    return a.astype(np.complex128)


def propagate(apply_h, psi, c: float, R: float, dt: float, K: int,
              nsteps: int = 1, record=False):
    """nsteps Chebyshev steps of exp(-i H dt) applied to psi (shape (nvec, D)).

    ``apply_h(v)`` returns H v in binary64 for v of shape (nvec, D).
    Returns the final state, or the list of states after every step when
    ``record``.
    """
    a = cheb_coeffs(R * dt, K)
    phase = np.exp(-1j * c * dt)
    psi = np.array(psi, dtype=np.complex128, copy=True)
    states = []

    def ht(v):
        return (apply_h(v) - c * v) / R

    for _ in range(nsteps):
        q0 = psi
        acc = a[0] * q0
        if K >= 1:
            q1 = ht(q0)
            acc = acc + a[1] * q1
            for k in range(2, K + 1):
                q2 = 2.0 * ht(q1) - q0
                acc = acc + a[k] * q2
                q0, q1 = q1, q2
        psi = phase * acc
        if record:
            states.append(psi.copy())
    return states if record else psi


def coherent_state(x: np.ndarray, t: float, x0: float, dx: float) -> np.ndarray:
    """Harmonic-oscillator coherent state (m = omega = hbar = 1) on a grid.

    Initial state pi^{-1/4} exp(-(x - x0)^2 / 2) (a Gaussian of width 1 at
    x0, momentum 0).  Its exact evolution keeps the shape, moves the centre
    to x0 cos t with momentum -x0 sin t, and picks up the phase
    -t/2 + (x0^2/2) sin t cos t.  Grid amplitudes carry sqrt(dx) so that the
    discrete norm is 1.
    """
    xc = x0 * np.cos(t)
    p = -x0 * np.sin(t)
    phase = -0.5 * t + 0.5 * x0 * x0 * np.sin(t) * np.cos(t)
    return (np.pi ** -0.25) * np.sqrt(dx) * np.exp(
        -0.5 * (x - xc) ** 2 + 1j * (p * x + phase))


def exact_propagator(H: np.ndarray, t: float) -> np.ndarray:
    """exp(-i H t) from the eigendecomposition of a Hermitian matrix."""
    w, V = np.linalg.eigh(H)
    return (V * np.exp(-1j * w * t)) @ V.conj().T


# --------------------------------------------------------------------------
# Imaginary-time filter (paper Sec. I and Sec. VII: TPQ states are random
# vectors filtered by a Chebyshev expansion of e^{-beta H/2}).  The paper does
# not print its coefficients; they follow from the generating function
# e^{z cos(theta)} = I_0(z) + 2 sum_k I_k(z) cos(k theta) with theta -> theta + pi:
#   e^{-tau (c + R x)} = e^{-tau c} [I_0(z) + 2 sum_k (-1)^k I_k(z) T_k(x)],
# z = R tau, written with the scaled e^{-z} I_k(z) and the factor e^{-tau (c - R)}.
# --------------------------------------------------------------------------
def bessel_i_scaled_seq(z: float, kmax: int) -> np.ndarray:
    """e^{-z} I_k(z), k = 0..kmax, z >= 0, by Miller's backward recurrence
    I_{k-1} = (2k/z) I_k + I_{k+1}, normalised by e^{-z} (I_0 + 2 sum I_k) = 1."""
    if z == 0.0:
        out = np.zeros(kmax + 1)
        out[0] = 1.0
        return out
    top = max(kmax, int(math.sqrt(80.0 * max(z, 1.0))) + 40) + 30
    v = np.zeros(top + 2)
    v[top] = 1e-300
    for k in range(top, 0, -1):
        v[k - 1] = (2.0 * k / z) * v[k] + v[k + 1]
        if v[k - 1] > 1e250:
            v[k - 1:] *= 1e-250
    norm = v[0] + 2.0 * v[1:].sum()
    return v[: kmax + 1] / norm


def filter_order(z: float, tol: float = 1e-10) -> int:
    """First k (>= 1) with 2 e^{-z} I_k(z) < tol and 2 e^{-z} I_{k+1}(z) < tol."""
    kmax = int(math.sqrt(80.0 * max(z, 1.0))) + 60
    v = bessel_i_scaled_seq(z, kmax + 1)
    for k in range(kmax + 1):
        if 2.0 * v[k] < tol and 2.0 * v[k + 1] < tol:
            return max(k, 1)
    raise RuntimeError("order search ran past the table")


def imag_time_filter(apply_h, psi, c: float, R: float, tau: float, K: int):
    """e^{-tau H} psi (not normalised) by the Chebyshev expansion above;
    ``apply_h(v)`` returns H v in binary64 for v of shape (nvec, D)."""
    z = R * tau
    iv = bessel_i_scaled_seq(z, K)
    a = 2.0 * iv * np.where(np.arange(K + 1) % 2 == 1, -1.0, 1.0)
    a[0] = iv[0]
    psi = np.array(psi, dtype=np.complex128, copy=True)

    def ht(v):
        return (apply_h(v) - c * v) / R

    q0 = psi
    acc = a[0] * q0
    if K >= 1:
        q1 = ht(q0)
        acc = acc + a[1] * q1
        for k in range(2, K + 1):
            q2 = 2.0 * ht(q1) - q0
            acc = acc + a[k] * q2
            q0, q1 = q1, q2
    return math.exp(-tau * (c - R)) * acc
