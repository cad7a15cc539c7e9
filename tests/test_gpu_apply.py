"""GPU parity: generated entries and products against the binary64 oracle.

Entries must match the oracle's generator bit for bit; products must be
within rel-L2 1e-5 of the binary64 product (FP32 arithmetic), and every
storage mode must give bit-identical products for the same input.
"""
import numpy as np
import pytest

from paper_2606_31598_amd import workloads
from tests.gpu_util import rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_31598_amd import procmv
    procmv.load()
    return procmv


@pytest.mark.parametrize("D,win", [
    (2048, (0, 0, 256, 256)), (2048, (1700, 100, 348, 333)),
    (1000, (0, 0, 1000, 1000)), (262144, (262000, 100, 144, 200)),
    (262144, (5, 131072, 64, 300))])
def test_gue_entries_bit_exact(pm, orc, D, win):
    r0, c0, nr, nc = win
    op = pm.Operator.gue(D, seed=1)
    got = to_host(op.entries(r0, c0, nr, nc))
    want = orc.gue_entries(1, r0, c0, nr, nc, D=D)
    assert got.dtype == np.complex64
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_generator_short_arithmetic_matches_ieee(pm):
    """The kernels' short division and square root give the IEEE results on
    every one of the 2^23 uniforms the generator can draw (exhaustive)."""
    assert pm.selftest_generator() == (0, 0)


def test_dvr_entries_bit_exact(pm, orc):
    D = 4096
    op = pm.Operator.dvr(D)
    d = orc.DVR(D)
    got = to_host(op.entries(0, 0, 300, 4096))
    idx_i = np.arange(300)[:, None]
    idx_j = np.arange(4096)[None, :]
    want = d.tk32[np.abs(idx_i - idx_j)]
    want[np.arange(300), np.arange(300)] = d.v32[:300]
    assert np.array_equal(got.real, want) and np.all(got.imag == 0)


def test_c0_ten_repeated_matvecs(pm, orc):
    """D = 2048 GUE, b = 256, procedural, psi = normalised Gaussian seed 2."""
    D = 2048
    op = pm.Operator.gue(D, seed=1).plan(256, pm.PROCEDURAL)
    psi = workloads.gaussian_vectors(D, 1, seed=2)
    ref = orc.gue_apply_rows(1, D, psi)
    X = to_dev(psi)
    outs = [to_host(op.apply(X)) for _ in range(10)]
    for o in outs:
        assert rel_l2(o, ref) <= TOL_FP32
        assert np.array_equal(o, outs[0])
    # chained H^3 psi against the oracle chain
    Y = X
    R = psi
    for _ in range(3):
        Y = op.apply(Y)
        R = orc.gue_apply_rows(1, D, R)
    assert rel_l2(to_host(Y), R) <= 3 * TOL_FP32


@pytest.mark.parametrize("D,nvec,b", [(1, 1, 64), (65, 3, 64), (777, 5, 128),
                                      (1000, 11, 256), (4096, 4, 512),
                                      (3001, 16, 1024)])
def test_gue_ragged_and_multivector(pm, orc, D, nvec, b):
    op = pm.Operator.gue(D, seed=7).plan(b, pm.PROCEDURAL)
    X = workloads.gaussian_vectors(D, nvec, seed=D + nvec)
    got = to_host(op.apply(to_dev(X)))
    ref = orc.gue_apply_rows(7, D, X)
    assert rel_l2(got, ref) <= TOL_FP32


@pytest.mark.parametrize("gen", ["gue", "dvr"])
@pytest.mark.parametrize("nvec,shape", [(4, 1), (1, 0)])
def test_storage_modes_agree(pm, orc, gen, nvec, shape):
    """Every storage mode gives the same product.  Cached modes read the very
    entries the generator emits, with the same arithmetic in the same order,
    so with one tile shape they are bit-identical to each other for every
    block size, and for GUE also to the procedural mode.  One vector at shape
    0 covers the pipelined kernel of fully cached super-tiles (full cache, and
    the cached super-tiles of a partial cache at b = 512) against the mixed
    super-tiles of b = 128.  The procedural sinc-DVR mode runs the Toeplitz
    kernel (different summation order): equal within binary32 rounding."""
    D = 1500
    Xh = workloads.gaussian_vectors(D, nvec, seed=3)
    X = to_dev(Xh)
    outs = {}
    for strat, f in [(pm.PROCEDURAL, 0.0), (pm.PARTIAL, 0.5), (pm.PARTIAL, 0.25),
                     (pm.FULL, 1.0)]:
        for b in (128, 512):
            op = pm.Operator.gue(D, seed=4) if gen == "gue" else pm.Operator.dvr(D)
            op.plan(b, strat, f).set_tile_shape(shape)
            info = op.plan_info()
            if strat == pm.FULL:
                assert info["p_cache"] == info["n_pair"]
            if strat == pm.PARTIAL:
                assert info["p_cache"] == int(np.floor(f * info["n_pair"]))
            outs[(strat, f, b)] = to_host(op.apply(X))
            op.close()
    ref = orc.gue_apply_rows(4, D, Xh) if gen == "gue" else orc.DVR(D).apply_rows(Xh)
    # four or more vectors of a full cache stream on the matrix cores: a
    # different kernel, equal within binary32 rounding only
    full_mfma = nvec >= 4
    cached = [v for k, v in outs.items()
              if k[0] != pm.PROCEDURAL and not (full_mfma and k[0] == pm.FULL)]
    for o in cached[1:]:
        assert np.array_equal(o, cached[0])
    for k, v in outs.items():
        if full_mfma and k[0] == pm.FULL:
            assert rel_l2(v, ref) <= TOL_FP32
    procs = [v for k, v in outs.items() if k[0] == pm.PROCEDURAL]
    assert np.array_equal(procs[0], procs[1])
    if gen == "gue":
        assert np.array_equal(procs[0], cached[0])
    for o in (procs[0], cached[0]):
        assert rel_l2(o, ref) <= TOL_FP32


@pytest.mark.parametrize("gen", ["gue", "dvr"])
def test_default_shapes_partial_cache(pm, orc, gen):
    """Default tile shapes (one launch per super-tile class: cached, generated,
    mixed) on partial caches at both sides of the super-tile edge, against the
    binary64 oracle, at a size with several super-tiles and a ragged tail."""
    D = 2000
    Xh = workloads.gaussian_vectors(D, 2, seed=5)
    ref = orc.gue_apply_rows(6, D, Xh) if gen == "gue" else orc.DVR(D).apply_rows(Xh)
    for b, f in [(128, 0.5), (256, 0.25), (512, 0.75), (1024, 0.5)]:
        for nv in (1, 2):
            op = pm.Operator.gue(D, seed=6) if gen == "gue" else pm.Operator.dvr(D)
            op.plan(b, pm.PARTIAL, f)
            got = to_host(op.apply(to_dev(Xh[:nv])))
            assert rel_l2(got, ref[:nv]) <= TOL_FP32, (b, f, nv)
            op.close()


@pytest.mark.parametrize("D,nvec", [(2, 1), (63, 2), (3001, 3), (8192, 2),
                                     (16383, 1), (32768, 1), (32768, 5)])
def test_dvr_apply_random_vectors(pm, orc, D, nvec):
    """Procedural sinc-DVR (Toeplitz kernel, both tile shapes), ragged D;
    at D >= 16384 checked on sampled rows."""
    op = pm.Operator.dvr(D).plan(256, pm.PROCEDURAL)
    X = workloads.gaussian_vectors(D, nvec, seed=9)
    got = to_host(op.apply(to_dev(X)))
    rows = np.arange(D) if D <= 8192 else workloads.sampled_rows(D, 256, seed=5)
    ref = orc.DVR(D).apply_rows(X, rows)
    assert rel_l2(got[:, rows], ref) <= TOL_FP32


def test_hermitian_identity_on_gpu(pm):
    D = 3000
    op = pm.Operator.gue(D, seed=11).plan(256)
    x = workloads.gaussian_vectors(D, 1, seed=1)
    y = workloads.gaussian_vectors(D, 1, seed=2)
    Hx = to_host(op.apply(to_dev(x)))[0].astype(np.complex128)
    Hy = to_host(op.apply(to_dev(y)))[0].astype(np.complex128)
    xs = x[0].astype(np.complex64).astype(np.complex128)
    ys = y[0].astype(np.complex64).astype(np.complex128)
    assert abs(np.vdot(xs, Hy) - np.vdot(Hx, ys)) < 1e-5


def test_errors_reported(pm):
    import torch
    op = pm.Operator.gue(512, seed=1)
    X = torch.zeros((1, 512), dtype=torch.complex64, device="cuda")
    with pytest.raises(pm.ProcmvError) as e:
        op.apply(X)
    assert e.value.status == 4
    op.plan(64)
    with pytest.raises(pm.ProcmvError) as e:
        op.apply(X, X)
    assert e.value.status == 1
    with pytest.raises(pm.ProcmvError) as e:
        op.plan(64, pm.FULL, precision=7)
    assert e.value.status == 1
    # empty vector sets and empty batches are argument errors, caught on the host
    import ctypes
    L = pm.load()
    Y = torch.zeros_like(X)
    p = ctypes.c_void_p
    assert L.procmv_apply(op._h, p(X.data_ptr()), 512, p(Y.data_ptr()), 512, 0, None) == 1
    h = ctypes.c_void_p()
    assert L.procmv_batch_create((ctypes.c_void_p * 1)(), 0, 1, ctypes.byref(h)) == 1


@pytest.mark.parametrize("nvec", [1, 2, 4, 8])
def test_every_tile_shape_matches_oracle(pm, orc, nvec):
    """Each VALU tile shape, explicitly, procedural and cached, single and
    batched, against the binary64 oracle (the autotuners may pick any)."""
    import torch
    D = 1500
    Xh = workloads.gaussian_vectors(D, nvec, seed=21)
    ref = orc.gue_apply_rows(9, D, Xh)
    for strat, f in ((pm.PROCEDURAL, 0.0), (pm.PARTIAL, 0.5)):
        for shape in (0, 1, 2):
            op = pm.Operator.gue(D, seed=9).plan(256, strat, f).set_tile_shape(shape)
            got = to_host(op.apply(to_dev(Xh)))
            assert rel_l2(got, ref) <= TOL_FP32, (strat, shape)
            if nvec in (1, 2, 4, 8):
                B = pm.Batch([op], nvec)
                X = torch.from_numpy(Xh.astype(np.complex64).ravel()).cuda()
                Y = torch.empty_like(X)
                B.configure(shape, 256, 0)
                B.apply(X, Y)
                gb = Y.cpu().numpy().reshape(nvec, D)
                assert rel_l2(gb, ref) <= TOL_FP32, ("batch", strat, shape)
                B.close()
            op.close()


@pytest.mark.parametrize("b", [192, 256])
def test_tall_tiles_stay_inside_cache_slots(pm, orc, b):
    """One vector at tile shape 2 has 128-row tiles; D = 12000 (256-row
    super-tiles) lets them run, and a partial cache of block size b reads
    whole tiles from one slot only when 128 divides b: the library launches
    shape 1 for b = 192 (procmv_tile_shape_fit) and shape 2 for b = 256.
    Both against the binary64 oracle on sampled rows; the batched launch
    with a cached b = 64 instance goes through the batch autotuner, which
    tries every shape."""
    import torch
    D = 12000
    assert pm.tile_shape_fit(1, 2, D, b) == (1 if b % 128 else 2)
    X = workloads.gaussian_vectors(D, 1, seed=31)
    rows = workloads.sampled_rows(D, 512, seed=32)
    ref = orc.gue_apply_rows(13, D, X, rows=rows)
    op = pm.Operator.gue(D, seed=13).plan(b, pm.PARTIAL, 0.5).set_tile_shape(2)
    got = to_host(op.apply(to_dev(X)))[:, rows]
    assert rel_l2(got, ref) <= TOL_FP32
    ops = [op, pm.Operator.gue(700, seed=14).plan(64, pm.FULL, 1.0)]
    B = pm.Batch(ops, 1)
    Xb = np.concatenate([X[0], workloads.gaussian_vectors(700, 1, seed=33)[0]])
    Xd = torch.from_numpy(Xb.astype(np.complex64)).cuda()
    Yd = torch.empty_like(Xd)
    B.autotune(Xd, Yd, reps=1)
    B.apply(Xd, Yd)
    Yb = to_host(Yd)
    assert rel_l2(Yb[:D][rows], ref[0]) <= TOL_FP32
    ref2 = orc.gue_apply_rows(14, 700, Xb[None, D:])
    assert rel_l2(Yb[D:], ref2[0]) <= TOL_FP32
    B.close()
