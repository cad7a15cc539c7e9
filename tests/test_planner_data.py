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


HELDOUT = os.path.join(DATA, "mi355x_plan_heldout.jsonl")


@pytest.mark.skipif(not os.path.exists(HELDOUT), reason="no committed held-out trials")
def test_held_out_log_covers_its_grid():
    """The held-out trials are a fresh exhaustive measurement on (D, nvec)
    points outside the training grid (3 * 2^k and 5 * 2^k sizes, vector
    counts that are not powers of two), both families."""
    from paper_2606_31598_amd import planner
    rows = [json.loads(line) for line in open(HELDOUT)]
    trials = [r for r in rows if r["kind"] != "machine_model"]
    ok = [r for r in trials if r.get("status") == "ok"]
    assert {r["D"] for r in ok} == set(planner.HELDOUT_D)
    assert {r["nvec"] for r in ok} == set(planner.HELDOUT_NVEC)
    assert {r["family"] for r in ok} == {0, 1}
    train_d = {1 << k for k in range(12, 19)}
    assert not (set(planner.HELDOUT_D) & train_d)
    assert not (set(planner.HELDOUT_NVEC) & set(planner.NVECS))
    # every (D, nvec, family) point has every candidate that fits measured
    pts = {(r["D"], r["nvec"], r["family"]) for r in ok}
    assert len(pts) == len(planner.HELDOUT_D) * len(planner.HELDOUT_NVEC) * 2
    for r in ok:
        assert r["t_apply_ms"] > 0 and r["t_fill_ms"] >= 0


@pytest.mark.skipif(not os.path.exists(HELDOUT), reason="no committed held-out trials")
def test_learned_ranking_on_held_out_sizes():
    """200 held-out workloads (seed 4242) on sizes the network never saw:
    the learned choice, from the oracle's binary64 forward pass of the
    trained parameters, against the exhaustive measured search.  It is
    within 10 % of the best measured plan on at least 90 % of them and beats
    the fixed procedural plan b = 256 in mean and median regret."""
    from paper_2606_31598_amd import planner, procmv as pm
    model = json.load(open(MODEL))
    p = _unflatten(model["params"])
    norm = np.asarray(model["norm"], np.float64)
    mu, sd = norm[:8], norm[8:]
    _, table = planner.load_trials(HELDOUT)
    cands = pm.plan_candidates()
    q_proc = [q for q, c in enumerate(cands) if c[0] == 256 and c[1] == pm.PROCEDURAL][0]
    learned, fixed = [], []
    for w in planner.heldout_workloads(200, seed=4242):
        D, nv, fam, bud, reuse = (w["D"], w["nvec"], w["family"], w["budget_gb"] * 1e9,
                                  w["reuse"])
        feas, feats = {}, {}
        for q, (b, st, f) in enumerate(cands):
            if b > D and b != cands[0][0]:
                continue
            x, _, fe = pm.plan_features(D, nv, bud, reuse, fam, b, st, f)
            if fe and (D, nv, fam, q) in table:
                tf, ta = table[(D, nv, fam, q)]
                feas[q], feats[q] = tf + reuse * ta, x
        assert feas
        qs = list(feas)
        z = (np.array([feats[q] for q in qs], np.float64) - mu) / sd
        ql = qs[int(np.argmin(opl.mlp_forward(p, z)[0]))]
        best = min(feas.values())
        learned.append(feas[ql] / best - 1.0)
        fixed.append(feas[q_proc] / best - 1.0 if q_proc in feas else float("inf"))
    learned, fixed = np.array(learned), np.minimum(np.array(fixed), 1e3)
    print(f"held-out learned mean {learned.mean():.3f} median {np.median(learned):.4f} "
          f"within 10% {np.mean(learned <= 0.1):.3f}; procedural mean {fixed.mean():.3f}")
    assert learned.size == 200
    assert np.mean(learned <= 0.10) >= 0.90
    assert np.mean(learned) < 0.10
    assert np.mean(learned) < np.mean(fixed)
    assert np.median(learned) <= np.median(fixed)
