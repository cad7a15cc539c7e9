"""Execution planner driver: measured plan trials, surrogate training, and
evaluation against exhaustive measured search (paper Sec. IV, Algorithms 1-3).

The candidate grid, memory model, features, analytic cost model, surrogate
kernels and the final choice live in the C library; this module runs the
measurement campaign (each trial a library-measured fill and product time,
logged as one JSON line like the paper's plan-trial log), builds the training
set, trains the network on the GPU through the library, and scores planners.

    python -m paper_2606_31598_amd.planner collect --out trials.jsonl
    python -m paper_2606_31598_amd.planner train --trials trials.jsonl --out model.json
    python -m paper_2606_31598_amd.planner evaluate --trials trials.jsonl --model model.json
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import procmv as pm
from . import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TRIALS = os.path.join(HERE, "data", "mi355x_plan_trials.jsonl")
DEFAULT_MODEL = os.path.join(HERE, "data", "mi355x_planner_mlp.json")

LOG2_D = range(12, 19)
NVECS = (1, 2, 4, 8, 16, 32, 64)
BUDGET_MAX = 256e9
DEFAULT_HELDOUT = os.path.join(HERE, "data", "mi355x_plan_heldout.jsonl")
# Problems the network never saw: dimensions 3 2^k and 5 2^k and vector
# counts that are not powers of two (the training grid is D = 2^12..2^18,
# nvec = 1, 2, 4, ..., 64).
HELDOUT_D = (5120, 6144, 10240, 12288, 20480, 24576, 40960, 49152, 81920, 98304)
HELDOUT_NVEC = (3, 5, 6, 12, 24, 48)


def log(msg):
    print(f"[planner] {msg}", file=sys.stderr, flush=True)


def calibrate(stream=None):
    """Machine constants of the analytic model from library microbenchmarks."""
    D = 16384
    tf, ta = pm.measure(pm.GEN_PHILOX_GUE, D, 1, 256, pm.PROCEDURAL, reps=3)
    gen_gue = 0.5 * D * (D + 1) / (ta * 1e-3)
    tf, ta = pm.measure(pm.GEN_SINC_DVR, D, 1, 256, pm.FULL, 1.0, reps=3)
    gen_dvr = 0.5 * D * (D + 1) / (tf * 1e-3)            # fill rate of the closed form
    tf, tdv = pm.measure(pm.GEN_SINC_DVR, D, 1, 256, pm.PROCEDURAL, reps=3)
    dvr_rate = D * D / (tdv * 1e-3)
    tf, tc = pm.measure(pm.GEN_PHILOX_GUE, D, 1, 256, pm.FULL, 1.0, reps=3)
    cache_bw = 0.5 * D * (D + 1) * 8.0 / (tc * 1e-3)
    tf, tm = pm.measure(pm.GEN_PHILOX_GUE, 4096, 16, 256, pm.FULL, 1.0, reps=3)
    flop = 8.0 * 4096 * 4096 * 16 / (tm * 1e-3)
    tf, tl = pm.measure(pm.GEN_PHILOX_GUE, 256, 1, 128, pm.PROCEDURAL, reps=10)
    mm = pm.MachineModel()
    mm.gen_rate[0], mm.gen_rate[1] = gen_gue, gen_dvr
    mm.dvr_rate, mm.cache_bw, mm.flop_rate, mm.launch_s = dvr_rate, cache_bw, flop, tl * 1e-3
    return mm


def model_dict(mm):
    return {"gen_rate": [mm.gen_rate[0], mm.gen_rate[1]], "dvr_rate": mm.dvr_rate,
            "cache_bw": mm.cache_bw, "flop_rate": mm.flop_rate, "launch_s": mm.launch_s}


def model_from(d):
    mm = pm.MachineModel()
    mm.gen_rate[0], mm.gen_rate[1] = d["gen_rate"]
    mm.dvr_rate, mm.cache_bw, mm.flop_rate, mm.launch_s = (
        d["dvr_rate"], d["cache_bw"], d["flop_rate"], d["launch_s"])
    return mm


def load_planners(trials=DEFAULT_TRIALS, model=DEFAULT_MODEL):
    """The calibrated analytic model and the trained network (parameters and
    feature normalisation) for procmv_plan_choose / procmv_plan_auto."""
    m = json.load(open(model))
    mm = model_from(m["machine_model"]) if "machine_model" in m else load_trials(trials)[0]
    return mm, np.array(m["params"], np.float32), np.array(m["norm"], np.float32)


def collect(out_path, log2_d=LOG2_D, nvecs=NVECS, families=(0, 1), reps=2, dims=None,
            calibrate_model=True):
    """Measure fill and product time of every memory-feasible candidate on the
    (D, nvec, family) grid; one JSON line per trial."""
    import torch
    torch.zeros(1, device="cuda")       # initialise the device before timing
    cands = pm.plan_candidates()
    n = 0
    dims = list(dims) if dims is not None else [1 << k for k in log2_d]
    with open(out_path, "w") as fh:
        if calibrate_model:
            mm = calibrate()
            fh.write(json.dumps({"kind": "machine_model", **model_dict(mm)}) + "\n")
        for D in dims:
            for fam in families:
                for nv in nvecs:
                    for q, (b, st, f) in enumerate(cands):
                        if b > D and b != cands[0][0]:
                            continue
                        _, mt, fe = pm.plan_features(D, nv, BUDGET_MAX, 2, fam, b, st, f)
                        rec = {"kind": "trial", "D": D, "nvec": nv, "family": fam,
                               "cand": q, "block_size": b, "strategy": st, "fraction": f,
                               "m_tot": mt}
                        if not fe:
                            rec["status"] = "infeasible"
                        else:
                            t0 = time.perf_counter()
                            r = pm.measure(fam, D, nv, b, st, f, seed=1, warmup=1, reps=reps)
                            if r is None:
                                rec["status"] = "oom"
                            else:
                                rec["status"] = "ok"
                                rec["t_fill_ms"], rec["t_apply_ms"] = r
                            rec["wall_s"] = time.perf_counter() - t0
                        fh.write(json.dumps(rec) + "\n")
                        fh.flush()
                        n += 1
                    log(f"D={D} family={fam} nvec={nv}: {n} trials so far")
    return n


def load_trials(path=DEFAULT_TRIALS):
    mm, table = None, {}
    for line in open(path):
        r = json.loads(line)
        if r["kind"] == "machine_model":
            mm = model_from(r)
        elif r.get("status") == "ok":
            table[(r["D"], r["nvec"], r["family"], r["cand"])] = (r["t_fill_ms"], r["t_apply_ms"])
    return mm, table


def t_total(tf, ta, reuse):
    return tf + reuse * ta


def training_set(table, draws=4, seed=1234):
    """One record per (measured trial, draw of budget and reuse): features of
    the pair and the measured total time t_fill + reuse t_apply (ms)."""
    rng = np.random.default_rng(seed)
    cands = pm.plan_candidates()
    X, y = [], []
    for (D, nv, fam, q), (tf, ta) in sorted(table.items()):
        b, st, f = cands[q]
        for _ in range(draws):
            bud = float(np.exp(rng.uniform(np.log(16.0), np.log(256.0)))) * 1e9
            reuse = int(round(np.exp(rng.uniform(0.0, np.log(500.0)))))
            x, mt, fe = pm.plan_features(D, nv, bud, max(reuse, 1), fam, b, st, f)
            if not fe:
                continue
            X.append(x)
            y.append(math.log(t_total(tf, ta, max(reuse, 1))))
    return np.array(X, np.float32), np.array(y, np.float32)


def train(table, epochs=4000, lr=3e-3, seed=0, draws=4):
    X, y = training_set(table, draws=draws)
    mu = X.mean(0)
    sd = X.std(0)
    sd[sd == 0] = 1.0
    Z = (X - mu) / sd
    rng = np.random.default_rng(seed)
    p = np.zeros(pm.mlp_param_count(), np.float32)
    # He-normal initial weights, zero biases (layout W1, b1, W2, b2, W3, b3)
    o = 0
    for (fan_in, fan_out) in ((8, 64), (64, 64), (64, 1)):
        p[o:o + fan_in * fan_out] = rng.standard_normal(fan_in * fan_out) * math.sqrt(2.0 / fan_in)
        o += fan_in * fan_out + fan_out
    params, hist = pm.mlp_train(Z, y, p, epochs, lr)
    pred = pm.mlp_predict(params, Z)
    return {"params": params.tolist(), "norm": np.concatenate([mu, sd]).tolist(),
            "n_train": int(y.size), "draws": draws, "epochs": epochs, "lr": lr,
            "train_log_mse": float(np.mean((pred - y) ** 2)),
            "loss_first": float(hist[0]), "loss_last": float(hist[-1])}


def evaluate(table, mm, model, n=200, seed=777):
    """Held-out workloads: regret of each planner against the best measured
    feasible plan (exhaustive measured search over the candidate grid)."""
    cands = pm.plan_candidates()
    params = np.array(model["params"], np.float32)
    norm = np.array(model["norm"], np.float32)
    wls = workloads.planner_workloads(n * 3, seed=seed, nvec_max=64)
    res = {"learned": [], "analytic": [], "procedural": []}
    used = 0
    for w in wls:
        if used >= n:
            break
        D, fam, bud, reuse = w["D"], w["family"], w["budget_gb"] * 1e9, w["reuse"]
        nv = min(NVECS, key=lambda v: abs(math.log(v) - math.log(w["nvec"])))
        feas = {}
        for q, (b, st, f) in enumerate(cands):
            if b > D and b != cands[0][0]:
                continue
            _, _, fe = pm.plan_features(D, nv, bud, reuse, fam, b, st, f)
            if fe and (D, nv, fam, q) in table:
                tf, ta = table[(D, nv, fam, q)]
                feas[q] = t_total(tf, ta, reuse)
        if not feas:
            continue
        best = min(feas.values())
        ql, _ = pm.plan_choose(1, D, nv, bud, reuse, fam, params=params, norm=norm)
        qa, _ = pm.plan_choose(0, D, nv, bud, reuse, fam, mm=mm)
        qp = [q for q, c in enumerate(cands) if c[0] == 256 and c[1] == pm.PROCEDURAL][0]
        for name, q in (("learned", ql), ("analytic", qa), ("procedural", qp)):
            t = feas.get(q)
            res[name].append(float("inf") if t is None else t / best - 1.0)
        used += 1
    out = {"n_workloads": used}
    for name, r in res.items():
        r = np.array(r)
        out[name] = {"mean_regret": float(np.mean(np.minimum(r, 1e3))),
                     "median_regret": float(np.median(r)),
                     "within_10pct": float(np.mean(r <= 0.10))}
    return out


def heldout_workloads(n=200, seed=4242):
    """Held-out problems: (D, nvec) from the held-out sets, family, budget
    log-uniform in [16, 256] GB and reuse log-uniform in [1, 500]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        out.append({"D": int(rng.choice(HELDOUT_D)), "nvec": int(rng.choice(HELDOUT_NVEC)),
                    "family": int(rng.integers(0, 2)),
                    "budget_gb": float(np.exp(rng.uniform(np.log(16.0), np.log(256.0)))),
                    "reuse": max(1, int(round(np.exp(rng.uniform(0.0, np.log(500.0))))))})
    return out


def evaluate_heldout(table, mm, model, n=200, seed=4242, k_bench=4):
    """Regret t_chosen / t_best - 1 against the exhaustive measured search on
    problems outside the training grid, for the learned (Algorithm 3,
    direct), analytic (Algorithm 1), measured (Algorithm 2: analytic top
    k_bench, best measured) and hybrid (learned top k_bench, best measured)
    planners and the fixed procedural plan b = 256.  The measured planners
    take their times from the same exhaustive table."""
    cands = pm.plan_candidates()
    params = np.array(model["params"], np.float32)
    norm = np.array(model["norm"], np.float32)
    names = ("learned", "analytic", "measured", "hybrid", "procedural")
    res = {k: [] for k in names}
    qp = [q for q, c in enumerate(cands) if c[0] == 256 and c[1] == pm.PROCEDURAL][0]
    used = 0
    for w in heldout_workloads(n, seed):
        D, nv, fam, bud, reuse = w["D"], w["nvec"], w["family"], w["budget_gb"] * 1e9, w["reuse"]
        feas = {}
        for q, (b, st, f) in enumerate(cands):
            if b > D and b != cands[0][0]:
                continue
            _, _, fe = pm.plan_features(D, nv, bud, reuse, fam, b, st, f)
            if fe and (D, nv, fam, q) in table:
                tf, ta = table[(D, nv, fam, q)]
                feas[q] = t_total(tf, ta, reuse)
        if not feas:
            continue
        best = min(feas.values())
        ol, _ = pm.plan_rank(1, D, nv, bud, reuse, fam, params=params, norm=norm)
        oa, _ = pm.plan_rank(0, D, nv, bud, reuse, fam, mm=mm)
        meas = lambda order: min(order[:k_bench], key=lambda q: feas.get(q, float("inf")))
        for name, q in (("learned", ol[0]), ("analytic", oa[0]), ("measured", meas(oa)),
                        ("hybrid", meas(ol)), ("procedural", qp)):
            t = feas.get(q)
            res[name].append(float("inf") if t is None else t / best - 1.0)
        used += 1
    out = {"n_workloads": used, "k_bench": k_bench}
    for name, r in res.items():
        r = np.array(r)
        out[name] = {"mean_regret": float(np.mean(np.minimum(r, 1e3))),
                     "median_regret": float(np.median(r)),
                     "within_10pct": float(np.mean(r <= 0.10))}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["collect", "train", "evaluate", "all", "collect-heldout",
                                    "evaluate-heldout"])
    ap.add_argument("--heldout", default=DEFAULT_HELDOUT)
    ap.add_argument("--trials", default=DEFAULT_TRIALS)
    ap.add_argument("--out", default=None)
    ap.add_argument("--model", default=DEFAULT_MODEL)
    ap.add_argument("--min-log2d", type=int, default=12)
    ap.add_argument("--families", default="0,1")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--max-log2d", type=int, default=18)
    ap.add_argument("--nvecs", default=",".join(str(v) for v in NVECS))
    args = ap.parse_args(argv)
    if args.cmd == "collect-heldout":
        fams = tuple(int(f) for f in args.families.split(","))
        n = collect(args.out or args.heldout, nvecs=HELDOUT_NVEC, families=fams,
                    reps=args.reps, dims=HELDOUT_D, calibrate_model=False)
        log(f"{n} held-out trials written")
        return
    if args.cmd == "evaluate-heldout":
        mm, _ = load_trials(args.trials)
        _, table = load_trials(args.heldout)
        model = json.load(open(args.model))
        print(json.dumps(evaluate_heldout(table, mm, model)), flush=True)
        return
    if args.cmd in ("collect", "all"):
        out = args.out or args.trials
        fams = tuple(int(f) for f in args.families.split(","))
        n = collect(out, log2_d=range(args.min_log2d, args.max_log2d + 1), families=fams,
                    nvecs=tuple(int(v) for v in args.nvecs.split(",")), reps=args.reps)
        log(f"{n} trials written to {out}")
        args.trials = out
    if args.cmd in ("train", "all"):
        mm, table = load_trials(args.trials)
        model = train(table)
        model["machine_model"] = model_dict(mm)
        out = args.out if args.cmd == "train" and args.out else args.model
        json.dump(model, open(out, "w"))
        log(f"trained on {model['n_train']} records: log-MSE {model['train_log_mse']:.4f}")
        args.model = out
    if args.cmd in ("evaluate", "all"):
        mm, table = load_trials(args.trials)
        model = json.load(open(args.model))
        print(json.dumps(evaluate(table, mm, model)), flush=True)


if __name__ == "__main__":
    main()
