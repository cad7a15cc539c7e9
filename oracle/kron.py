"""System-bath Kronecker operator, binary64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper Sec. VII (18-qubit example): the code's Hamiltonian is
H = H_S (x) I_B + I_S (x) H_B + g sum_a A_a (x) B_a, applied matrix-free to
psi in C^{d_S} (x) C^{d_B}.  With psi stored as the d_S x d_B matrix Psi
(psi[s d_B + j] = Psi[s, j]) the definition of the Kronecker product gives
(H psi)[s, j] = sum_t H_S[s,t] Psi[t,j] + (H_B Psi[s,:])_j
               + g sum_a sum_t A_a[s,t] (B_a Psi[t,:])_j,
so every bath operator acts on the d_S rows of Psi together (R = d_S vectors,
paper Sec. IV-A).  The paper does not give the distribution of its bath
operators; the tests use Philox-GUE operators of distinct seeds.
"""
import numpy as np


def kron_dense(HS, HB, A_list, B_list, g):
    """The dense D x D matrix, D = d_S d_B (small sizes only)."""
    dS, dB = HS.shape[0], HB.shape[0]
    H = np.kron(HS, np.eye(dB)) + np.kron(np.eye(dS), HB)
    for A, B in zip(A_list, B_list):
        H = H + g * np.kron(A, B)
    return H


def kron_apply(HS, apply_hb, A_list, apply_b_list, g, psi):
    """H psi for psi of length d_S d_B; ``apply_hb(P)`` and each
    ``apply_b_list[a](P)`` return the bath operator applied to every row of the
    (d_S, d_B) matrix P, in binary64."""
    dS = HS.shape[0]
    P = np.asarray(psi, np.complex128).reshape(dS, -1)
    Y = HS @ P + apply_hb(P)
    for A, ap in zip(A_list, apply_b_list):
        Y = Y + g * (A @ ap(P))
    return Y.reshape(-1)
