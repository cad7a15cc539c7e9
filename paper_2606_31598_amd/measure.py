"""Timings of the product on the paper's configurations (one MI355X).

    python -m paper_2606_31598_amd.measure c0|c2|c3|modes [--reps N]

Each sub-command prints JSON lines with the measured quantities of one
configuration; accuracy against the binary64 reference lives in the tests.

* c0 -- Philox-GUE D = 2048, b = 256, procedural, one vector: ten repeated
  products (paper Sec. V, small dense case).
* c2 -- 256 uneven Philox-GUE instances (D uniform in [512, 8192], seeds
  1..256), four vectors: one persistent batched launch (autotuned) against
  one product per instance, and batched Chebyshev steps replayed from a HIP
  graph against per-instance steps.
* c3 -- Philox-GUE D = 262144, 16 vectors, b = 512: procedural and 25%
  canonical cache, binary32 and split-bfloat16 matrix-core products; cache
  fill time and the bandwidth of the cached part.
* probe -- a few products of each configuration above (C0: 20; C2: 3 batched;
  C3: 2 per arithmetic and storage mode), for hardware-counter and
  kernel-trace runs.
* modes -- single-vector products of one operator (Philox-GUE or sinc-DVR,
  D = 32768 by default, b = 256) in each storage mode: procedural, 50%
  canonical cache, full cache; cache bytes and the rate they are read at.
"""
import argparse
import json
import time

import numpy as np


def _cuda():
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    return torch


def _emit(rec):
    print(json.dumps(rec), flush=True)


def _time(fn, reps, torch):
    """Mean seconds per call over `reps` calls (HIP events, after one warm call)."""
    fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def c0(reps):
    torch = _cuda()
    from . import procmv as pm, workloads
    D = 2048
    op = pm.Operator.gue(D, seed=1).plan(256, pm.PROCEDURAL)
    X = torch.from_numpy(workloads.gaussian_vectors(D, 1, seed=2).astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    t = _time(lambda: op.apply(X, Y), max(reps, 10), torch)
    shape, tuned = op.autotune(1, reps=max(reps, 10))
    t_tuned = _time(lambda: op.apply(X, Y), max(reps, 10), torch)
    _emit({"config": "c0", "workload": "Philox-GUE D=2048 b=256 procedural, 1 vector",
           "us_per_product": t * 1e6, "gelem_s": D * D / t / 1e9,
           "autotuned_shape": shape, "us_per_product_autotuned": t_tuned * 1e6,
           "gelem_s_autotuned": D * D / t_tuned / 1e9})


def c2(reps):
    torch = _cuda()
    from . import procmv as pm, workloads
    sizes = workloads.batch_sizes(256)
    nvec = 4
    ops = [pm.Operator.gue(int(D), seed=k + 1).plan(256) for k, D in enumerate(sizes)]
    B = pm.Batch(ops, nvec)
    parts = [workloads.gaussian_vectors(int(D), nvec, seed=100 + k).ravel()
             for k, D in enumerate(sizes)]
    X = torch.from_numpy(np.concatenate(parts).astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    elems = float(np.sum(sizes.astype(np.float64) ** 2))
    tuned_ms = B.autotune(X, Y, reps=2)
    t_batch = _time(lambda: B.apply(X, Y), reps, torch)
    views = [(X[int(o):int(o) + nvec * int(D)].view(nvec, int(D)),
              Y[int(o):int(o) + nvec * int(D)].view(nvec, int(D)))
             for o, D in zip(B.offsets, sizes)]

    def per_instance():
        for op, (xv, yv) in zip(ops, views):
            op.apply(xv, yv)
    t_each = _time(per_instance, max(1, reps // 4), torch)
    _emit({"config": "c2", "workload": "256 Philox-GUE instances, D in [512, 8192], 4 vectors",
           "sum_D2": elems, "batched_ms_per_product": t_batch * 1e3,
           "batched_gelem_s": elems / t_batch / 1e9,
           "batched_gelem_s_x4": nvec * elems / t_batch / 1e9,
           "per_instance_ms_per_product": t_each * 1e3,
           "per_instance_gelem_s": elems / t_each / 1e9,
           "speedup": t_each / t_batch, "autotune_ms": tuned_ms, "batch_config": B.info()})
    # Chebyshev steps (dt = 0.05, spectral interval c = 0, R = 2.5)
    dt, c, R = 0.05, 0.0, 2.5
    K = pm.cheb_order(R * dt, 1e-10)
    psi = X.clone()
    nsteps = 20
    B.propagate(psi, dt, 1, c, R, graph=True)      # capture + first replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.propagate(psi, dt, nsteps, c, R, graph=True)
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / nsteps
    t0 = time.perf_counter()
    B.propagate(psi, dt, 2, c, R, graph=False)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / 2
    psis = [p.clone() for p, _ in views]
    t0 = time.perf_counter()
    for op, p in zip(ops, psis):
        op.propagate(p, dt, nsteps=1, K=K, c=c, R=R)
    torch.cuda.synchronize()
    t_inst = time.perf_counter() - t0
    _emit({"config": "c2", "chebyshev_K": K,
           "batched_graph_steps_per_s": 1.0 / t_graph,
           "batched_eager_steps_per_s": 1.0 / t_eager,
           "per_instance_steps_per_s": 1.0 / t_inst,
           "graph_gelem_s": (K + 1) * elems / t_graph / 1e9})


def c3(reps):
    torch = _cuda()
    from . import procmv as pm, workloads
    D, nvec, b = 262144, 16, 512
    X = torch.from_numpy(workloads.gaussian_vectors(D, nvec, seed=2).astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    for strat, f in ((pm.PROCEDURAL, 0.0), (pm.PARTIAL, 0.25)):
        for prec, pname in ((pm.FP32, "fp32"), (pm.SPLIT_BF16, "split_bf16")):
            op = pm.Operator.gue(D, seed=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            op.plan(b, strat, f, precision=prec)
            torch.cuda.synchronize()
            t_plan = time.perf_counter() - t0
            info = op.plan_info()
            t = _time(lambda: op.apply(X, Y), reps, torch)
            rec = {"config": "c3", "workload": f"Philox-GUE D={D}, {nvec} vectors, b={b}",
                   "strategy": "procedural" if f == 0 else f"partial {f}", "precision": pname,
                   "plan_s": t_plan, "cache_gb": info["cache_bytes"] / 1e9,
                   "ms_per_product": t * 1e3, "gelem_s": D * D / t / 1e9,
                   "gelem_s_x16": nvec * D * D / t / 1e9}
            _emit(rec)
            op.close()
            torch.cuda.synchronize()


def probe():
    torch = _cuda()
    from . import procmv as pm, workloads
    # C0
    D = 2048
    op = pm.Operator.gue(D, seed=1).plan(256, pm.PROCEDURAL)
    X = torch.from_numpy(workloads.gaussian_vectors(D, 1, seed=2).astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    for _ in range(20):
        op.apply(X, Y)
    torch.cuda.synchronize()
    op.close()
    _emit({"probe": "c0", "products": 20})
    # C2: the default batch configuration (no autotuning)
    sizes = workloads.batch_sizes(256)
    nvec = 4
    ops = [pm.Operator.gue(int(Dk), seed=k + 1).plan(256) for k, Dk in enumerate(sizes)]
    B = pm.Batch(ops, nvec)
    parts = [workloads.gaussian_vectors(int(Dk), nvec, seed=100 + k).ravel()
             for k, Dk in enumerate(sizes)]
    X = torch.from_numpy(np.concatenate(parts).astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    for _ in range(3):
        B.apply(X, Y)
    torch.cuda.synchronize()
    _emit({"probe": "c2", "products": 3, "batch_config": B.info()})
    del B, ops
    # C3
    D, nvec, b = 262144, 16, 512
    X = torch.from_numpy(workloads.gaussian_vectors(D, nvec, seed=2).astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    for strat, f in ((pm.PROCEDURAL, 0.0), (pm.PARTIAL, 0.25)):
        for prec, pname in ((pm.FP32, "fp32"), (pm.SPLIT_BF16, "split_bf16")):
            op = pm.Operator.gue(D, seed=1).plan(b, strat, f, precision=prec)
            for _ in range(2):
                op.apply(X, Y)
            torch.cuda.synchronize()
            op.close()
            torch.cuda.synchronize()
            _emit({"probe": "c3", "strategy": "procedural" if f == 0 else f"partial {f}",
                   "precision": pname, "products": 2})


def modes(reps, family="gue", D=32768):
    torch = _cuda()
    from . import procmv as pm, workloads
    X = torch.from_numpy(workloads.gaussian_vectors(D, 1, seed=2).astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    for name, strat, f in (("procedural", pm.PROCEDURAL, 0.0), ("partial 0.5", pm.PARTIAL, 0.5),
                           ("full", pm.FULL, 1.0)):
        op = pm.Operator.gue(D, seed=1) if family == "gue" else pm.Operator.dvr(D)
        op.plan(256, strat, f)
        info = op.plan_info()
        t = _time(lambda: op.apply(X, Y), reps, torch)
        _emit({"config": "modes", "workload": f"{family} D={D} b=256, 1 vector", "strategy": name,
               "us_per_product": t * 1e6, "gelem_s": D * D / t / 1e9,
               "cache_gb": info["cache_bytes"] / 1e9,
               "cache_read_gb_s": info["cache_bytes"] / t / 1e9})
        op.close()
        torch.cuda.synchronize()


def lanczos(reps, m=40):
    """Lanczos spectral bounds (m steps) against m plain products, on the
    benchmark's operator and the small GUE one."""
    torch = _cuda()
    from . import procmv as pm, workloads
    for name, D in (("dvr", 32768), ("gue", 2048), ("gue", 32768)):
        op = pm.Operator.gue(D, seed=1) if name == "gue" else pm.Operator.dvr(D)
        op.plan(256)
        X = torch.from_numpy(workloads.gaussian_vectors(D, 1, seed=2).astype(np.complex64)).cuda()
        Y = torch.empty_like(X)
        t_l = _time(lambda: op.lanczos_bounds(X, m), reps, torch)
        t_p = _time(lambda: op.apply(X, Y), reps * m, torch)
        b = op.lanczos_bounds(X, m)
        _emit({"config": "lanczos", "workload": f"{name} D={D} b=256 procedural, m={m}",
               "ms_per_call": t_l * 1e3, "ms_m_products": t_p * m * 1e3,
               "overhead": t_l / (t_p * m) - 1.0, "e_min": b["e_min"], "e_max": b["e_max"]})
        op.close()
        torch.cuda.synchronize()


def filt(reps):
    """Imaginary-time filter e^{-tau H} on one vector: time per call and per
    Chebyshev term, automatic order (coefficient cut 1e-10)."""
    torch = _cuda()
    from . import procmv as pm, workloads
    for name, D, tau in (("gue", 32768, 2.0), ("dvr", 32768, 0.01)):
        op = pm.Operator.gue(D, seed=1) if name == "gue" else pm.Operator.dvr(D)
        op.plan(256)
        c, R = op.spectral_bounds()
        K = pm.filter_order(R * tau, 1e-10)
        X0 = torch.from_numpy(workloads.gaussian_vectors(D, 1, seed=2).astype(np.complex64)).cuda()
        X = X0.clone()
        t = _time(lambda: (X.copy_(X0), op.filter(X, tau, K=K)), reps, torch)
        _emit({"config": "filter", "workload": f"{name} D={D} b=256 procedural, tau={tau}",
               "K": K, "ms_per_filter": t * 1e3, "us_per_term": t / (K + 1) * 1e6})
        op.close()
        torch.cuda.synchronize()


def kron(reps):
    """System-bath Kronecker product at the paper's run shape: d_S = 4,
    d_B = 65536, one interaction term (two Philox-GUE bath operators):
    procedural at block sizes 4096 (the paper's autotuned choice) and 256, and
    fully cached (34 GB of canonical blocks), with one 181-term Chebyshev
    step on the cached operators."""
    torch = _cuda()
    from . import procmv as pm, workloads
    dS, dB = 4, 65536
    HS, As = workloads.system_matrices(dS, 1, seed=3)
    X = torch.from_numpy(workloads.gaussian_vectors(dS * dB, 1, seed=4)[0]
                         .astype(np.complex64).reshape(dS, dB)).cuda()
    Y = torch.empty_like(X)
    flops = 2 * 8 * dS * dB * dB          # two bath operators, 8 flop per complex MAC
    for b, strat, f in ((4096, pm.PROCEDURAL, 0.0), (256, pm.PROCEDURAL, 0.0),
                        (256, pm.FULL, 1.0)):
        HB = pm.Operator.gue(dB, seed=41).plan(b, strat, f)
        B = pm.Operator.gue(dB, seed=42).plan(b, strat, f)
        t = _time(lambda: pm.kron_apply(HB, [B], HS, As, 0.5, X, Y), reps, torch)
        name = "procedural" if f == 0 else "full cache"
        rec = {"config": "kron", "workload": f"system-bath d_S={dS} d_B={dB} n_int=1, b={b} {name}",
               "cache_gb": (HB.plan_info()["cache_bytes"] + B.plan_info()["cache_bytes"]) / 1e9,
               "ms_per_apply": t * 1e3, "flop_per_apply": flops, "tflop_s": flops / t / 1e12}
        if f == 1.0:
            # one real-time Chebyshev step at the paper's order (181 terms per step)
            P = X.clone()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            pm.kron_propagate(HB, [B], HS, As, 0.5, P, 0.01, 1, 0.0, 10.0, K=181)
            e1.record()
            torch.cuda.synchronize()
            rec["cheb_step_K181_s"] = e0.elapsed_time(e1) / 1e3
        _emit(rec)
        HB.close()
        B.close()
        torch.cuda.synchronize()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["c0", "c2", "c3", "probe", "modes", "lanczos", "filter", "kron"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--family", choices=["gue", "dvr"], default="gue")
    ap.add_argument("--D", type=int, default=32768)
    args = ap.parse_args(argv)
    if args.cmd == "modes":
        modes(args.reps, args.family, args.D)
    elif args.cmd == "lanczos":
        lanczos(args.reps)
    elif args.cmd == "filter":
        filt(args.reps)
    elif args.cmd == "kron":
        kron(args.reps)
    elif args.cmd == "probe":
        probe()
    else:
        {"c0": c0, "c2": c2, "c3": c3}[args.cmd](args.reps)


if __name__ == "__main__":
    main()
