"""The committed planner data: the plan-trial log measured on MI355X and the
surrogate network trained on it (paper Sec. IV-D: the surrogate is fitted to
logged plan trials of the library and then ranks the feasible candidates).

Host-only checks: the log covers the candidate grid of both operator families
with at least 2000 measured trials, and the trained parameters, run through
the oracle's binary64 forward pass, reproduce the training error recorded
with them and rank plans better than the fixed procedural plan on held-out
(budget, reuse) draws.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import planner as opl

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2606_31598_amd", "data")
TRIALS = os.path.join(DATA, "mi355x_plan_trials.jsonl")
MODEL = os.path.join(DATA, "mi355x_planner_mlp.json")

pytestmark = pytest.mark.skipif(not (os.path.exists(TRIALS) and os.path.exists(MODEL)),
                                reason="no committed plan trials / trained model")


def _unflatten(flat):
    """Library layout W1 (8x64, row-major), b1, W2 (64x64), b2, W3 (64), b3."""
    flat = np.asarray(flat, np.float64)
    o, p = 0, {}
    for name, shape in (("W1", (8, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
                        ("W3", (64, 1)), ("b3", (1,))):
        n = int(np.prod(shape))
        p[name] = flat[o:o + n].reshape(shape)
        o += n
    assert o == flat.size
    return p


def test_trial_log_covers_the_grid():
    rows = [json.loads(line) for line in open(TRIALS)]
    assert rows[0]["kind"] == "machine_model"
    trials = [r for r in rows if r["kind"] != "machine_model"]
    ok = [r for r in trials if r.get("status") == "ok"]
    assert len(ok) >= 2000
    assert {r["family"] for r in ok} == {0, 1}
    assert {r["D"] for r in ok} == {1 << k for k in range(12, 19)}
    assert {r["nvec"] for r in ok} == {1, 2, 4, 8, 16, 32, 64}
    for r in ok:
        assert r["t_apply_ms"] > 0 and r["t_fill_ms"] >= 0
        assert 0 <= r["cand"] < 30
    # every infeasible trial is a plan that does not fit the device
    assert all(r.get("status") in ("ok", "infeasible") for r in trials)


def test_trained_network_matches_oracle_forward():
    from paper_2606_31598_amd import planner
    model = json.load(open(MODEL))
    p = _unflatten(model["params"])
    norm = np.asarray(model["norm"], np.float64)
    mu, sd = norm[:8], norm[8:]
    _, table = planner.load_trials(TRIALS)
    X, y = planner.training_set(table, draws=model.get("draws", 2))
    assert X.shape[0] == model["n_train"]
    pred = opl.mlp_forward(p, (X.astype(np.float64) - mu) / sd)[0]
    mse = float(np.mean((pred - y) ** 2))
    # the recorded error was computed by the binary32 GPU forward pass
    assert abs(mse - model["train_log_mse"]) <= 1e-3 * max(1.0, model["train_log_mse"])
    # a useful fit: the spread of log time over the set is far larger
    assert mse < 0.1 * float(np.var(y))


def test_learned_ranking_beats_fixed_plan_on_held_out_draws():
    """Regret against exhaustive measured search, with the network evaluated
    by the oracle's binary64 forward pass (no library compute)."""
    from paper_2606_31598_amd import planner, procmv as pm, workloads
    model = json.load(open(MODEL))
    p = _unflatten(model["params"])
    norm = np.asarray(model["norm"], np.float64)
    mu, sd = norm[:8], norm[8:]
    _, table = planner.load_trials(TRIALS)
    cands = pm.plan_candidates()
    q_proc = [q for q, c in enumerate(cands) if c[0] == 256 and c[1] == pm.PROCEDURAL][0]
    learned, fixed = [], []
    for w in workloads.planner_workloads(600, seed=777, nvec_max=64):
        D, fam, bud, reuse = w["D"], w["family"], w["budget_gb"] * 1e9, w["reuse"]
        nv = min(planner.NVECS, key=lambda v: abs(math.log(v) - math.log(w["nvec"])))
        feas, feats = {}, {}
        for q, (b, st, f) in enumerate(cands):
            if b > D and b != cands[0][0]:
                continue
            x, _, fe = pm.plan_features(D, nv, bud, reuse, fam, b, st, f)
            if fe and (D, nv, fam, q) in table:
                tf, ta = table[(D, nv, fam, q)]
                feas[q], feats[q] = tf + reuse * ta, x
        if not feas:
            continue
        qs = list(feas)
        z = (np.array([feats[q] for q in qs], np.float64) - mu) / sd
        ql = qs[int(np.argmin(opl.mlp_forward(p, z)[0]))]
        best = min(feas.values())
        learned.append(feas[ql] / best - 1.0)
        fixed.append(feas[q_proc] / best - 1.0 if q_proc in feas else float("inf"))
        if len(learned) >= 200:
            break
    learned, fixed = np.array(learned), np.minimum(np.array(fixed), 1e3)
    assert learned.size >= 150
    assert np.mean(learned) < np.mean(fixed)
    assert np.median(learned) <= np.median(fixed)
