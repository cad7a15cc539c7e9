"""Pins of the planner formulas (paper Sec. IV) and the surrogate network.

The formulas reproduce the worked numbers the paper prints for its 18-qubit
run (Sec. VII); the network's analytic gradients match central finite
differences.
"""
import json
import os

import numpy as np

from oracle import planner as pl

HERE = os.path.dirname(os.path.abspath(__file__))


def test_paper_worked_numbers():
    g = json.load(open(os.path.join(HERE, "golden", "paper_worked_numbers.json")))
    dS, dB = g["d_S"], g["d_B"]
    assert pl.mem_full(2 ** 18, 2 ** 18) == g["dense_complex64_D2p18_bytes"]["value"]
    assert pl.mem_full(dB, dB) == g["bath_operator_dB65536_bytes"]["value"]
    b = dB // g["n_blk"]
    assert b == 4096
    assert pl.mem_partial(1, b) == g["block_b4096_bytes"]["value"]
    assert pl.mem_full(dB, dB, n_op=1, p_row=g["p_row"]) == g["row_slice_bytes"]["value"]
    assert pl.mem_full(dB, dB, n_op=g["n_op"], p_row=g["p_row"]) == g["per_gpu_two_ops_bytes"]["value"]
    F = pl.flops_mv(dB, dB, dS, n_op=g["n_op"])
    want = g["work_per_hpsi_flops"]
    assert abs(F / want["value"] - 1) < want["rel_tol"]
    assert pl.waves(g["n_task"], g["gpu_groups"]) == 5
    s = pl.bench_score(g["n_task"], g["gpu_groups"], g["t_mv_s"]["value"])
    assert abs(s - g["score_s"]["value"]) < g["score_s"]["abs_tol"]


def test_cache_pairs_and_feasibility():
    assert pl.n_pair(16) == 136
    assert pl.n_pair(512) == 131328
    b = 512
    # a quarter of the canonical pairs of D = 2^18 at b = 512
    m = 0.25 * pl.n_pair(512) * 8 * b * b
    assert pl.p_cache(512, b, m) == 32832
    assert pl.p_cache(8, 256, 1e15) == 36
    assert pl.feasible(10, [20, 12], alpha=0.9)
    assert not pl.feasible(11, [20, 12], alpha=0.9)
    assert abs(pl.b_target(128 * 2 ** 20) - 4096) < 1e-9


def test_mlp_gradients_finite_difference():
    rng = np.random.default_rng(0)
    p = pl.mlp_init(seed=1)
    z = rng.standard_normal((32, 8))
    t = rng.standard_normal(32)
    loss, g = pl.mlp_loss_grad(p, z, t)
    h = 1e-6
    for k in p:
        flat = p[k].ravel()
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = pl.mlp_loss_grad(p, z, t)
            flat[i] = old - h
            lm, _ = pl.mlp_loss_grad(p, z, t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].ravel()[i]) < 1e-6 * max(1.0, abs(fd))


def test_mlp_adam_fits_smooth_target():
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (512, 8))
    y = np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2]
    p = pl.mlp_init(seed=2)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(val) for k, val in p.items()}
    l0, _ = pl.mlp_loss_grad(p, x, y)
    for t in range(1, 1501):
        loss, g = pl.mlp_loss_grad(p, x, y)
        pl.adam_step(p, g, m, v, t, lr=3e-3)
    assert loss < 0.02 * l0
