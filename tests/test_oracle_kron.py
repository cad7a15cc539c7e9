"""Pins of the system-bath Kronecker oracle (paper Sec. VII example:
H = H_S (x) I + I (x) H_B + g sum_a A_a (x) B_a): the matrix-free form agrees
with numpy's Kronecker product, the operator is Hermitian, and with H_S = 0,
g = 0 it is block diagonal with H_B on every system index."""
import numpy as np

import oracle
from oracle import kron as ok
from paper_2606_31598_amd import workloads


def _ops(dB, n_int):
    HB = oracle.gue_dense(21, dB)
    Bs = [oracle.gue_dense(22 + a, dB) for a in range(n_int)]
    return HB, Bs


def test_matrix_free_equals_numpy_kron():
    dS, dB, g = 3, 40, 0.37
    HS, As = workloads.system_matrices(dS, 2, seed=5)
    HB, Bs = _ops(dB, 2)
    psi = workloads.gaussian_vectors(dS * dB, 1, seed=9)[0]
    dense = ok.kron_dense(HS, HB, As, Bs, g)
    got = ok.kron_apply(HS, lambda P: P @ HB.T, As, [lambda P, B=B: P @ B.T for B in Bs], g, psi)
    assert np.allclose(got, dense @ psi, atol=1e-12)
    # the library's bath products: Philox-GUE rows through the row-by-row oracle
    rows = lambda seed: (lambda P: oracle.gue_apply_rows(seed, dB, P))
    got2 = ok.kron_apply(HS, rows(21), As, [rows(22), rows(23)], g, psi)
    assert np.allclose(got2, dense @ psi, atol=1e-12)


def test_hermitian_and_block_diagonal_case():
    dS, dB = 4, 32
    HS, As = workloads.system_matrices(dS, 1, seed=2)
    HB, Bs = _ops(dB, 1)
    H = ok.kron_dense(HS, HB, As, Bs, 0.8)
    assert np.allclose(H, H.conj().T, atol=1e-14)
    H0 = ok.kron_dense(np.zeros((dS, dS)), HB, As, Bs, 0.0)
    for s in range(dS):
        assert np.allclose(H0[s * dB:(s + 1) * dB, s * dB:(s + 1) * dB], HB)
    assert np.count_nonzero(np.abs(H0) > 0) == dS * np.count_nonzero(np.abs(HB) > 0)
