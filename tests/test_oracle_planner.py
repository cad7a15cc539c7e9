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


MM = {"gen_rate": (2.7e11, 5e11), "dvr_rate": 1.4e13, "cache_bw": 4e12,
      "flop_rate": 1e14, "launch_s": 2e-5}


def test_adam_step_by_hand():
    """Kingma & Ba's update, worked by hand for one scalar: lr = 0.1,
    beta = (0.9, 0.999), eps = 1e-8, p0 = 1.
    Step 1, g = 0.5: m = 0.05, v = 2.5e-4, m^ = 0.5, v^ = 0.25,
      p = 1 - 0.1 * 0.5 / (0.5 + 1e-8) = 0.900000002.
    Step 2, g = -0.2: m = 0.045 - 0.02 = 0.025, v = 2.4975e-4 + 4e-5 = 2.8975e-4,
      m^ = 0.025 / 0.19 = 0.1315789474, v^ = 2.8975e-4 / 0.001999 = 0.1449474737,
      p = 0.900000002 - 0.1 * 0.1315789474 / 0.3807196...= 0.8654394181."""
    from oracle import planner as opl
    p = {"w": np.array([1.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    opl.adam_step(p, {"w": np.array([0.5])}, m, v, 1, lr=0.1)
    assert abs(m["w"][0] - 0.05) < 1e-15 and abs(v["w"][0] - 2.5e-4) < 1e-18
    assert abs(p["w"][0] - 0.900000002) < 1e-12
    opl.adam_step(p, {"w": np.array([-0.2])}, m, v, 2, lr=0.1)
    assert abs(m["w"][0] - 0.025) < 1e-15 and abs(v["w"][0] - 2.8975e-4) < 1e-17
    assert abs(p["w"][0] - 0.8654394181) < 1e-9


def test_analytic_time_by_hand():
    """The analytic model at three points, worked by hand with
    R_gen = 2.7e11 (GUE), R_dvr = 1.4e13, cache 4e12 B/s, F = 1e14 flop/s,
    launch 2e-5 s.
    A: GUE D = 4096, 1 vector, b = 256, procedural: 4096 * 4097 / 2 =
       8,390,656 generated entries / 2.7e11 = 3.10765e-5 s against
       8 * 4096^2 / 1e14 = 1.342e-6 s of flops: t_apply = 5.10765e-5, no fill.
    B: the same, full cache: 16 blocks, 136 pairs of 256^2 complex64 =
       71,303,168 B read once per product, 3.78258e-5 s; fill generates the
       8,912,896 cached entries (whole diagonal blocks) and writes them:
       3.30107e-5 + 1.78258e-5 = 5.08365e-5 s.
    C: sinc-DVR D = 32768, 1 vector, procedural: Toeplitz source
       32768^2 / 1.4e13 = 7.67e-5 s is below the 8.58993e-5 s of flops:
       t_apply = 1.058993e-4 s."""
    from oracle import planner as opl
    tf, ta = opl.analytic_time(MM, 4096, 1, 0, 256, opl.PROCEDURAL, 0.0, 1)
    assert tf == 0.0 and abs(ta - 5.10765037e-5) < 1e-13
    tf, ta = opl.analytic_time(MM, 4096, 1, 0, 256, opl.FULL, 1.0, 7)
    assert abs(ta - 3.7825792e-5) < 1e-13 and abs(tf - 5.0836518e-5) < 1e-12
    tf, ta = opl.analytic_time(MM, 32768, 1, 1, 256, opl.PROCEDURAL, 0.0, 1)
    assert abs(ta - 1.0589934592e-4) < 1e-13


def test_analytic_choice_limits():
    """One product never pays for a cache fill; hundreds of products pick
    the full cache when it fits; a budget too small for any plan gives None."""
    from oracle import planner as opl
    c = opl.candidates()
    q1, _ = opl.analytic_choice(MM, 32768, 1, 256e9, 1, 0)
    q500, _ = opl.analytic_choice(MM, 32768, 1, 256e9, 500, 0)
    assert c[q1][1] == opl.PROCEDURAL and c[q500][1] == opl.FULL
    assert opl.analytic_choice(MM, 262144, 64, 1e6, 1, 0)[0] is None


def test_library_analytic_planner_matches_oracle():
    """procmv_plan_model_time on every candidate and procmv_plan_choose
    (planner 0) against the oracle's Algorithm 1, over dimensions, vector
    counts, families, reuse counts and budgets (host-only entry points)."""
    from oracle import planner as opl
    from paper_2606_31598_amd import procmv as pm
    mm = pm.MachineModel()
    mm.gen_rate[0], mm.gen_rate[1] = MM["gen_rate"]
    mm.dvr_rate, mm.cache_bw = MM["dvr_rate"], MM["cache_bw"]
    mm.flop_rate, mm.launch_s = MM["flop_rate"], MM["launch_s"]
    assert pm.plan_candidates() == opl.candidates()
    n_choices = 0
    for D in (700, 4096, 3 * 2 ** 13, 32768, 5 * 2 ** 14, 262144):
        for nvec in (1, 2, 3, 4, 7, 8, 16, 64):
            for fam in (0, 1):
                for reuse in (1, 7, 500):
                    for q, (b, st, f) in enumerate(opl.candidates()):
                        lt = pm.plan_model_time(mm, D, nvec, fam, b, st, f, reuse)
                        ot = opl.analytic_time(MM, D, nvec, fam, b, st, f, reuse)
                        for a, o in zip(lt, ot):
                            assert abs(a - o) <= 1e-12 * max(abs(o), 1e-300), (D, nvec, q)
                    for budget in (16e9, 256e9):
                        oq, osc = opl.analytic_choice(MM, D, nvec, budget, reuse, fam)
                        try:
                            lq, lsc = pm.plan_choose(0, D, nvec, budget, reuse, fam, mm=mm)
                        except pm.ProcmvError as e:
                            assert e.status == 3 and oq is None
                            continue
                        assert lq == oq and abs(lsc - osc) <= 1e-12 * osc, (D, nvec, fam)
                        n_choices += 1
    assert n_choices > 500
