"""The allocation-free product procmv_apply_noalloc, called through the C
ABI, against procmv_apply: the same kernels in the same order, with the
partial slots in the library's static device workspace instead of the
operator's own buffer, so the outputs agree bit for bit.  Two calls in a
row, the second on a smaller input, show that the workspace's leftover
contents from the first call do not leak into the second."""
import numpy as np
import pytest

from paper_2606_31598_amd import workloads
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_31598_amd import procmv
    procmv.load()
    return procmv


def _apply_noalloc(pm, op, X, Y):
    px, ldx, nv = pm._vec_arg(X, op.D)
    py, ldy, _ = pm._vec_arg(Y, op.D)
    return pm.load().procmv_apply_noalloc(op._h, px, ldx, py, ldy, nv, pm._stream())


def test_noalloc_matches_apply_on_two_calls(pm):
    import torch
    cases = [
        # one vector of the compensated sinc-DVR operator at D = 20000: the
        # split-bf16 matrix-core product (26 partial slots)
        (pm.Operator.dvr(20000).plan(256, precision=pm.FP32_COMPENSATED), 1, 13),
        # smaller: GUE, 4 vectors, half-cached: 64-wide-edge super-tiles of a ragged D
        (pm.Operator.gue(3000, seed=7).plan(256, pm.PARTIAL, 0.5), 4, 11),
        # smaller still: one vector of the compensated sinc-DVR operator (VALU)
        (pm.Operator.dvr(1500).plan(128, precision=pm.FP32_COMPENSATED), 1, 12),
    ]
    for op, nv, seed in cases:
        X = to_dev(workloads.gaussian_vectors(op.D, nv, seed=seed))
        ref = to_host(op.apply(X))
        Y = torch.full_like(X, complex(np.nan, np.nan))
        st = _apply_noalloc(pm, op, X, Y)
        assert st == 0, pm.load().procmv_last_error()
        got = to_host(Y)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (op.D, nv)


def test_noalloc_rejects_products_beyond_the_workspace(pm):
    import torch
    # 257 partial slots of 65536 complex64 = 134 MB, above the 64 MiB workspace
    op = pm.Operator.gue(65536, seed=1).plan(256)
    X = torch.zeros((1, 65536), dtype=torch.complex64, device="cuda")
    Y = torch.zeros_like(X)
    assert _apply_noalloc(pm, op, X, Y) == 1
    assert b"static workspace" in pm.load().procmv_last_error()
