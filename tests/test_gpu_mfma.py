"""GPU parity of the multi-vector matrix-core path.

Binary32 MFMA products must be within rel-L2 1e-5 of the binary64 oracle,
split-bfloat16 products within 2e-5; at D = 262144 (16 vectors, 25% canonical
cache) the check runs on 4096 sampled rows.
"""
import numpy as np
import pytest

from paper_2606_31598_amd import workloads
from tests.gpu_util import rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 2e-5}


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_31598_amd import procmv
    procmv.load()
    return procmv


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("D,nvec,strat,f,b", [
    (1000, 16, 0, 0.0, 256), (2048, 9, 1, 0.5, 256), (777, 20, 2, 1.0, 128),
    (3001, 1, 0, 0.0, 512), (513, 4, 1, 0.25, 64), (4500, 5, 2, 1.0, 256),
    (6000, 8, 0, 0.0, 1024)])
def test_gue_mfma_parity(pm, orc, prec, D, nvec, strat, f, b):
    if prec == 0 and nvec < 4:
        pytest.skip("binary32 with fewer than 4 vectors runs on the VALU kernel")
    op = pm.Operator.gue(D, seed=3).plan(b, strat, f, precision=prec)
    X = workloads.gaussian_vectors(D, nvec, seed=nvec + 1)
    got = to_host(op.apply(to_dev(X)))
    ref = orc.gue_apply_rows(3, D, X)
    err = rel_l2(got, ref)
    print(f"GUE D={D} nvec={nvec} strat={strat} prec={prec}: rel-L2 {err:.2e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_mfma_storage_modes_identical(pm, prec):
    D = 1200
    X = to_dev(workloads.gaussian_vectors(D, 16, seed=5))
    outs = []
    for strat, f in [(0, 0.0), (1, 0.5), (2, 1.0)]:
        op = pm.Operator.gue(D, seed=8).plan(256, strat, f, precision=prec)
        outs.append(to_host(op.apply(X)))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_dvr_split_bf16(pm, orc):
    D = 4096
    op = pm.Operator.dvr(D).plan(256, pm.PROCEDURAL, precision=pm.SPLIT_BF16)
    X = workloads.gaussian_vectors(D, 16, seed=4)
    got = to_host(op.apply(to_dev(X)))
    ref = orc.DVR(D).apply_rows(X)
    assert rel_l2(got, ref) <= TOL[1]


@pytest.fixture(scope="module")
def c3_reference(orc):
    D = 262144
    X = workloads.gaussian_vectors(D, 16, seed=2)
    rows = workloads.sampled_rows(D, 4096, seed=3)
    ref = orc.gue_apply_rows(1, D, X, rows)
    return D, X, rows, ref


@pytest.mark.parametrize("prec", [0, 1])
def test_c3_beyond_hbm_sampled_rows(pm, c3_reference, prec):
    """GUE seed 1, D = 262144 (dense complex64 would need 512 GiB), 16 vectors,
    25% canonical block cache at b = 512."""
    import torch
    D, X, rows, ref = c3_reference
    op = pm.Operator.gue(D, seed=1).plan(512, pm.PARTIAL, 0.25, precision=prec)
    info = op.plan_info()
    assert info["p_cache"] == int(0.25 * info["n_pair"])
    Y = op.apply(to_dev(X))
    got = to_host(Y)[:, rows]
    err = rel_l2(got, ref)
    print(f"C3 prec={prec}: rel-L2 {err:.2e} over {rows.size} rows x 16 vectors")
    assert err <= TOL[prec]
    del Y
    op.close()
    torch.cuda.empty_cache()
