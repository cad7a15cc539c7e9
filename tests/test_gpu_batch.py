"""GPU parity of batched products and batched Chebyshev propagation.

A batch of independent operators goes through one persistent launch over
super-tiles of edge 256 for every instance.  Its products must not depend on
the persistent grid or the item order (same kernels, fixed reduction order:
bit-identical), must equal the per-instance product bit for bit where the
instance's own product runs the same kernel on the same super-tiles (edge
256: D > 11264) and within binary32 rounding elsewhere, the captured HIP graph must reproduce the eager
step on every replay, and every instance must match the binary64 oracle.
"""
import numpy as np
import pytest

from oracle import chebyshev as ch
from paper_2606_31598_amd import workloads
from tests.gpu_util import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_31598_amd import procmv
    procmv.load()
    return procmv


def _packed(sizes, nvec, seed):
    parts = [workloads.gaussian_vectors(int(D), nvec, seed=seed + k).ravel()
             for k, D in enumerate(sizes)]
    return np.concatenate(parts)


def _unpack(buf, sizes, nvec):
    out, o = [], 0
    for D in sizes:
        out.append(buf[o:o + nvec * D].reshape(nvec, D))
        o += nvec * D
    return out


# nvec = 8 takes the matrix cores: the batch runs the four-wave kernel form and
# single products the eight-wave form, which must agree bit for bit
@pytest.mark.parametrize("nvec", [1, 4, 8])
def test_batched_apply_equals_per_instance(pm, orc, nvec):
    import torch
    sizes = [700, 64, 1500, 257, 1024, 3, 999, 11520]
    ops = [pm.Operator.gue(D, seed=10 + k).plan(256) for k, D in enumerate(sizes)]
    B = pm.Batch(ops, nvec)
    Xh = _packed(sizes, nvec, seed=1)
    X = torch.from_numpy(Xh.astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    Xs = _unpack(Xh, sizes, nvec)
    refs = [orc.gue_apply_rows(10 + k, D, Xs[k]) for k, D in enumerate(sizes)]
    singles = []
    for k, (op, D) in enumerate(zip(ops, sizes)):
        Xk = X[int(B.offsets[k]):int(B.offsets[k]) + nvec * D].view(nvec, D)
        singles.append(op.apply(Xk).cpu().numpy())
    outs = {}
    for cfg in [(2, 1024, 0), (2, 256, 1), (0, 256, 1), (0, 2048, 0), (1, 2048, 0)]:
        B.configure(*cfg)
        B.apply(X, Y)
        got = _unpack(Y.cpu().numpy(), sizes, nvec)
        outs[cfg] = got
        for k, D in enumerate(sizes):
            assert rel_l2(got[k], refs[k]) <= 1e-5, (cfg, D)
            assert rel_l2(got[k], singles[k]) <= 1e-5, (cfg, D)
        if cfg[0] == 0:
            # single products default to tile shape 0; the D = 11520 operator
            # plans the batch's super-tile edge too
            assert np.array_equal(got[-1], singles[-1])
    for a, b in zip(outs[(2, 1024, 0)], outs[(2, 256, 1)]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[(0, 256, 1)], outs[(0, 2048, 0)]):
        assert np.array_equal(a, b)


def test_batched_propagation_graph_replays(pm, orc):
    import torch
    sizes = [300, 1000, 77, 640]
    nvec = 2
    ops = [pm.Operator.gue(D, seed=20 + k).plan(128) for k, D in enumerate(sizes)]
    B = pm.Batch(ops, nvec)
    p0 = _packed(sizes, nvec, seed=5).astype(np.complex64)
    eager = torch.from_numpy(p0).cuda()
    graph = eager.clone()
    dt, c, R = 0.05, 0.0, 2.5
    for rep in range(3):
        B.propagate(eager, dt, 1, c, R, graph=False)
        torch.cuda.synchronize()
        nrm = B.propagate(graph, dt, 1, c, R, graph=True, norms=True)
        torch.cuda.synchronize()
        assert torch.equal(eager, graph), f"replay {rep} differs from the eager step"
        assert np.max(np.abs(nrm - 1.0)) < 1e-5
    # per-instance propagation agrees within binary32 rounding (its plan uses
    # a smaller super-tile edge at these sizes)
    for k, (op, D) in enumerate(zip(ops, sizes)):
        single = torch.from_numpy(_unpack(p0, sizes, nvec)[k].copy()).cuda()
        op.propagate(single, dt, nsteps=3, c=c, R=R)
        got = graph[int(B.offsets[k]):int(B.offsets[k]) + nvec * D].view(nvec, D)
        assert rel_l2(got.cpu().numpy(), single.cpu().numpy()) <= 1e-5
    # oracle on two instances
    for k in (0, 2):
        H = orc.gue_dense(20 + k, sizes[k])
        ref = ch.propagate(lambda v: v @ H.T, _unpack(p0, sizes, nvec)[k], c, R, dt,
                           ch.cheb_order(R * dt), nsteps=3)
        got = graph[int(B.offsets[k]):int(B.offsets[k]) + nvec * sizes[k]].view(
            nvec, sizes[k]).cpu().numpy()
        assert rel_l2(got, ref) < 1e-5


def test_c2_batch_shape_autotuned(pm, orc):
    """256 GUE instances, seeds 1..256, D uniform in [512, 8192], 4 vectors:
    one autotuned persistent launch per product; sampled instances checked."""
    import torch
    sizes = workloads.batch_sizes(256)
    ops = [pm.Operator.gue(int(D), seed=k + 1).plan(256) for k, D in enumerate(sizes)]
    B = pm.Batch(ops, 4)
    Xh = _packed(sizes, 4, seed=100)
    X = torch.from_numpy(Xh.astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    ms = B.autotune(X, Y, reps=2)
    info = B.info()
    print(f"C2 autotuned: {ms:.2f} ms per batched product, config {info}")
    B.apply(X, Y)
    got = _unpack(Y.cpu().numpy(), sizes, 4)
    Xs = _unpack(Xh, sizes, 4)
    # every instance against the binary64 oracle on 64 sampled rows (all four
    # vectors), ragged sizes and several super-tile bands included
    worst = 0.0
    for k, D in enumerate(sizes):
        rows = workloads.sampled_rows(int(D), 64, seed=1000 + k)
        ref = orc.gue_apply_rows(k + 1, int(D), Xs[k], rows=rows)
        err = rel_l2(got[k][:, rows], ref)
        worst = max(worst, err)
        assert err <= 1e-5, (k, int(D), err)
    print(f"C2: worst sampled rel-L2 over 256 instances {worst:.2e}")


def test_c2_graph_propagation_100_steps(pm, orc):
    """The C2 batch (256 instances, 4 vectors) propagated 100 steps of
    dt = 0.05 through the captured HIP graph; eight instances (the six
    smallest and two near the median size) against the oracle's binary64
    propagation of the same entries, every instance's norms conserved."""
    import torch
    sizes = workloads.batch_sizes(256)
    ops = [pm.Operator.gue(int(D), seed=k + 1).plan(256) for k, D in enumerate(sizes)]
    B = pm.Batch(ops, 4)
    p0 = _packed(sizes, 4, seed=300).astype(np.complex64)
    P = torch.from_numpy(p0).cuda()
    dt, c, R, steps = 0.05, 0.0, 2.5, 100
    nrm = B.propagate(P, dt, steps, c, R, graph=True, norms=True)
    torch.cuda.synchronize()
    assert np.max(np.abs(nrm - 1.0)) < 1e-4
    got = _unpack(P.cpu().numpy(), sizes, 4)
    start = _unpack(p0, sizes, 4)
    order = np.argsort(sizes)
    pick = list(order[:6]) + list(order[127:129])
    K = ch.cheb_order(R * dt)
    for k in pick:
        H = orc.gue_dense(int(k) + 1, int(sizes[k]))
        ref = ch.propagate(lambda v: v @ H.T, start[k], c, R, dt, K, nsteps=steps)
        err = rel_l2(got[k], ref)
        print(f"instance {int(k)} D={int(sizes[k])}: rel-L2 vs binary64 {err:.2e}")
        assert err < 1e-4


@pytest.mark.parametrize("strat,f", [(0, 0.0), (1, 0.5), (2, 1.0)])
def test_batched_dvr_instances(pm, orc, strat, f):
    """Sinc-DVR batches: procedural (VALU batched kernel with the closed-form
    entries) and cached (matrix-core batched kernel, 4 vectors) against the
    binary64 oracle, instance by instance."""
    import torch
    sizes = [300, 1000, 777, 2048]
    nvec = 4
    ops = [pm.Operator.dvr(D).plan(256, strat, f) for D in sizes]
    B = pm.Batch(ops, nvec)
    Xh = _packed(sizes, nvec, seed=9)
    X = torch.from_numpy(Xh.astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    B.apply(X, Y)
    got = _unpack(Y.cpu().numpy(), sizes, nvec)
    Xs = _unpack(Xh, sizes, nvec)
    for k, D in enumerate(sizes):
        ref = orc.DVR(D).apply_rows(Xs[k])
        assert rel_l2(got[k], ref) <= 1e-5, (D, strat)
