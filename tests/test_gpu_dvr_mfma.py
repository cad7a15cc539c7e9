"""GPU parity of the matrix-core sinc-DVR Toeplitz kernels (one vector)
against the binary64 oracle and against the VALU Toeplitz kernel.

Both kernels cut the operator into 32 x 32 Toeplitz blocks T_d (one per block
offset d) and apply each to all output blocks at once on the matrix cores:
kind 2 in binary32 MFMA, kind 3 on the bfloat16 matrix cores with an exact
three-piece split of every binary32 operand (six piece products, binary32
accumulation).  Ragged D, operators smaller than one block and both
arithmetics (plain and compensated, whose tables drop the band |i - j| < 32)
are covered, with the tolerances of binary32 products.
"""
import numpy as np
import pytest

from oracle import chebyshev as ch
from paper_2606_31598_amd import workloads
from tests.gpu_util import rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_31598_amd import procmv
    procmv.load()
    return procmv


@pytest.mark.parametrize("kind", [2, 3])
@pytest.mark.parametrize("D", [2, 33, 100, 1000, 2047, 5000, 16384, 20000])
def test_mfma_toeplitz_matches_oracle(pm, orc, D, kind):
    d = orc.DVR(D)
    # inputs rounded to complex64 first: the oracle applies the operator to
    # exactly the vector the GPU reads (for the smooth vector the rounding
    # alone, times the stencil's cancellation, would exceed the tolerance)
    X = workloads.gaussian_vectors(D, 1, seed=D).astype(np.complex64)
    S = workloads.wavepacket(D).astype(np.complex64)
    for prec in (pm.FP32, pm.FP32_COMPENSATED):
        op = pm.Operator.dvr(D).plan(256, precision=prec).set_dvr_kernel(kind)
        err = rel_l2(to_host(op.apply(to_dev(X))), d.apply_rows(X))
        print(f"D={D} kind={kind} precision={prec} random {err:.2e}")
        assert err < 1e-5
        if prec == pm.FP32_COMPENSATED:
            # smooth vector: error of the rescaled operator (H - c)/R, the
            # quantity the propagation accumulates (see test_gpu_compensated)
            ref_s = d.apply_rows(S)
            R = 0.5 * d.spectral_bounds()[1]
            got_s = to_host(op.apply(to_dev(S)))
            sc = float(np.linalg.norm(got_s - ref_s) / (R * np.linalg.norm(S)))
            err_s = rel_l2(got_s, ref_s)
            print(f"D={D} kind={kind} compensated smooth rel {err_s:.2e} scaled {sc:.1e}")
            assert err_s < 1e-5 or sc < 1e-9
        op.close()


@pytest.mark.parametrize("D", [40000, 65536, 100003])
def test_split_kernel_large_operators(pm, orc, D):
    """Above the benchmark's size the chunks are as long as the LDS window
    allows (70-72 offsets) and, for D = 100003, the last row group is
    ragged; 256 sampled rows of each product against the binary64 row
    oracle, both arithmetics."""
    d = orc.DVR(D)
    rows = workloads.sampled_rows(D, 256, seed=21)
    X = workloads.gaussian_vectors(D, 1, seed=D % 1000).astype(np.complex64)
    S = workloads.wavepacket(D).astype(np.complex64)
    R = 0.5 * d.spectral_bounds()[1]
    for prec in (pm.FP32, pm.FP32_COMPENSATED):
        op = pm.Operator.dvr(D).plan(256, precision=prec).set_dvr_kernel(3)
        err = rel_l2(to_host(op.apply(to_dev(X)))[:, rows], d.apply_rows(X, rows))
        got_s = to_host(op.apply(to_dev(S)))[:, rows]
        ref_s = d.apply_rows(S, rows)
        err_s = rel_l2(got_s, ref_s)
        sc = float(np.linalg.norm(got_s - ref_s) / (R * np.linalg.norm(S[:, rows])))
        print(f"D={D} precision={prec} random {err:.2e} smooth {err_s:.2e} (scaled {sc:.1e})")
        assert err < 1e-5
        if prec == pm.FP32_COMPENSATED:
            assert err_s < 1e-5 or sc < 1e-9
        op.close()


@pytest.mark.parametrize("kind", [2, 3])
def test_mfma_and_valu_toeplitz_agree(pm, kind):
    """Same entries, different summation order (and, for kind 3, the
    split's dropped products): the products agree to binary32 rounding."""
    D = 20000
    X = to_dev(workloads.gaussian_vectors(D, 1, seed=3))
    op = pm.Operator.dvr(D).plan(256)
    a = to_host(op.set_dvr_kernel(1).apply(X))
    b = to_host(op.set_dvr_kernel(kind).apply(X))
    assert rel_l2(b, a) < 2e-6


def test_split_kernel_is_deterministic_and_row_exact_on_integers(pm, orc):
    """Small integers are exact in every piece and product: with a vector of
    integers in [-8, 8] the split products reproduce the binary64 row sums of
    the binary32 entries to a few binary32 roundings of the partial sums, and
    two launches give the same bits."""
    D = 3000
    d = orc.DVR(D)
    rng = np.random.default_rng(11)
    X = (rng.integers(-8, 9, D) + 1j * rng.integers(-8, 9, D)).astype(np.complex64)[None, :]
    op = pm.Operator.dvr(D).plan(256).set_dvr_kernel(3)
    a = to_host(op.apply(to_dev(X)))
    b = to_host(op.apply(to_dev(X)))
    assert np.array_equal(a, b)
    assert rel_l2(a, d.apply_rows(X)) < 1e-6


@pytest.mark.parametrize("kind", [2, 3])
def test_mfma_propagation_matches_oracle(pm, orc, kind):
    """Compensated propagation with a matrix-core product at D = 4096,
    20 steps, against the binary64 oracle and the scaled budget."""
    D, dt, steps = 4096, 0.05, 20
    d = orc.DVR(D)
    e0, e1 = d.spectral_bounds()
    c, R = 0.5 * (e0 + e1), 0.5 * (e1 - e0)
    op = pm.Operator.dvr(D).plan(256, precision=pm.FP32_COMPENSATED).set_dvr_kernel(kind)
    psi0 = workloads.wavepacket(D).astype(np.complex64)
    P = to_dev(psi0)
    op.propagate(P, dt, nsteps=steps, c=c, R=R)
    ref = ch.propagate(lambda v: d.apply_fft(v), psi0, c, R, dt, ch.cheb_order(R * dt),
                       nsteps=steps)
    err = rel_l2(to_host(P), ref)
    print(f"D={D} kind={kind} steps={steps} vs fp64 {err:.2e}")
    assert err < 1e-4 * np.sqrt(steps / 200.0)


@pytest.mark.parametrize("D", [16384, 32768, 49152])
def test_xcd_placed_reduction_covers_every_row(pm, orc, D):
    """At D = 2048 G with G a multiple of 8 the reduction after the split
    kernel takes its 64-row blocks in XCD order (a permutation of the
    blocks).  Both arithmetics, output pre-filled with NaN: every row is
    written once and matches the binary64 FFT product of the same entries."""
    import torch
    d = orc.DVR(D)
    X = workloads.gaussian_vectors(D, 1, seed=7).astype(np.complex64)
    ref = d.apply_fft(X)
    for prec in (pm.FP32, pm.FP32_COMPENSATED):
        op = pm.Operator.dvr(D).plan(256, precision=prec).set_dvr_kernel(3)
        Y = torch.full((1, D), float("nan"), dtype=torch.complex64, device="cuda")
        got = to_host(op.apply(to_dev(X), Y))
        assert np.isfinite(got).all(), (D, prec)
        worst = float(np.abs(got - ref).max() / np.abs(ref).max())
        print(f"D={D} precision={prec}: max row error {worst:.2e} of max |Hx|")
        assert worst < 1e-5
        op.close()
