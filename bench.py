"""Benchmark: Gelem/s of H applied and Chebyshev steps/s on one MI355X.

Default workload: sinc-DVR harmonic oscillator, D = 32768 on x in [-20, 20],
wavepacket at x0 = 3 (sigma = 1), Chebyshev propagation with dt = 0.05 and
the order from the Bessel-coefficient rule.  One benchmark step is one
Chebyshev time step: K + 1 coefficient terms, K products H q (each one
generated-block product over all D^2 entries, by default the split-bf16
matrix-core Toeplitz kernel, plus its fixed-order reduction with the
recurrence and the binary64 accumulation fused), and the final rounding and
binary64 norm.  The
default arithmetic is the compensated binary32 one (band in difference form,
hi + lo recurrence vectors), which keeps the state within 1e-4 sqrt(n/200)
of the exact one; --precision fp32 gives the plain binary32 arithmetic.

The JSON line reports the whole-step throughput in matrix elements applied
per second, the throughput of each storage mode (procedural, 50% partial
cache, full cache) for single products, the roofline position of the
dominant kernel (from HIP events recorded around sampled launches in the
timed region), the error of the propagated state against the exact coherent
state with its budget, and the binary64 oracle timed on a bounded sample on
the host.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("Gelem/s of H applied (procedural vs cached) & Chebyshev steps/s "
          "at stated err")
PEAK_FP32_TFLOPS = 157.3   # MI355X fp32: vector and dense matrix cores (published)
PEAK_BF16_TFLOPS = 2500.0  # MI355X bf16 dense matrix cores (published)
PEAK_HBM_GBS = 8000.0
# the split-bf16 product applies six bfloat16 piece products per entry and
# vector component (hh, hm, mh, hl, lh, mm) where a binary32 product applies one
SPLIT_PRODUCTS = 6
KINDS = {"auto": 0, "valu": 1, "mfma": 2, "split": 3}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


CSRC = os.path.join(ROOT, "paper_2606_31598_amd", "csrc")
# dominant kernel per --dvr-kernel: (counter summary, kernel source)
PMC = {"split": (os.path.join(ROOT, "profiles", "dvr_toeplitz_bf16x6_D32768_pmc.txt"),
                 os.path.join(CSRC, "dvr_bf16.hip")),
       "mfma": (os.path.join(ROOT, "profiles", "dvr_toeplitz_mfma_D32768_pmc.txt"),
                os.path.join(CSRC, "dvr_mfma.hip")),
       "valu": (os.path.join(ROOT, "profiles", "dvr_toeplitz_D32768_pmc.txt"),
                os.path.join(CSRC, "dvr.hip"))}
KERNEL_NAMES = {"split": "dvr_toeplitz_bf16x6_kernel", "mfma": "dvr_toeplitz_mfma_kernel",
                "valu": "dvr_toeplitz_kernel"}


def resolve_kernel(choice, D):
    """Kernel the library runs for one vector of the procedural operator."""
    if choice == "auto":
        return "split" if D >= 16384 else "valu"
    return choice


def counted_traffic(kernel):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel source has
    changed since the counters were taken."""
    import hashlib
    summary, source = PMC[kernel]
    if not os.path.exists(summary):
        return None
    vals = {}
    for line in open(summary):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    digest = hashlib.sha256(open(source, "rb").read()).hexdigest()
    if vals.get("source_sha256") != digest:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measure_apply(pm, op, X, reps, warm=2):
    """Mean seconds per product over `reps` products (HIP events)."""
    import torch
    for _ in range(warm):
        op.apply(X, Y=None)
    Y = torch.empty_like(X)
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    op.profile(1)
    e0.record(s)
    for _ in range(reps):
        op.apply(X, Y)
    e1.record(s)
    torch.cuda.synchronize()
    prof = op.profile_read()
    op.profile(0)
    return e0.elapsed_time(e1) / 1e3 / reps, prof


def cpu_baseline_dvr(D, budget_s=10.0):
    """Binary64 oracle (row-by-row product) on a bounded sample: the rows of
    one product, doubled until a quarter of the budget is reached, then whole
    products repeated until the budget is spent (the Chebyshev step itself,
    K products, would take the oracle hours)."""
    import numpy as np
    import oracle
    from paper_2606_31598_amd import workloads
    d = oracle.DVR(D)
    X = workloads.wavepacket(D)
    rows, elapsed = 64, 0.0
    while True:
        idx = np.arange(rows, dtype=np.int64) * (D // rows)
        t0 = time.perf_counter()
        d.apply_rows(X, idx)
        elapsed = time.perf_counter() - t0
        if elapsed > budget_s / 4 or rows >= D:
            break
        rows = min(D, rows * 4)
    n_prod = 0
    if rows >= D:
        idx = np.arange(D, dtype=np.int64)
        elapsed = 0.0
        t0 = time.perf_counter()
        while elapsed < budget_s:
            d.apply_rows(X, idx)
            n_prod += 1
            elapsed = time.perf_counter() - t0
        elems = float(n_prod) * D * D
        what = f"{n_prod} whole products ({D} x {D})"
    else:
        elems = float(rows) * D
        what = f"{rows} of {D} rows x {D} columns"
    return {"value": elems / elapsed / 1e9, "unit": "Gelem/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"binary64 row-by-row sinc-DVR product, {what}, 1 vector "
                      f"({elapsed:.2f} s)"}


def stated_error_dvr(psi_host, D, t):
    """rel-L2 of the propagated state against the exact coherent state."""
    import numpy as np
    import oracle
    from oracle import chebyshev as ch
    d = oracle.DVR(D)
    ref = ch.coherent_state(d.x, t, 3.0, d.dx)
    return float(np.linalg.norm(psi_host[0] - ref) / np.linalg.norm(ref))


def run_dvr(args):
    import numpy as np
    import torch
    from paper_2606_31598_amd import procmv as pm
    from paper_2606_31598_amd import workloads

    D, dt, b = args.D, 0.05, args.block
    strat = {"procedural": pm.PROCEDURAL, "partial": pm.PARTIAL,
             "full": pm.FULL}[args.strategy]
    frac = {"procedural": 0.0, "partial": 0.5, "full": 1.0}[args.strategy]
    prec = {"fp32": pm.FP32, "compensated": pm.FP32_COMPENSATED}[args.precision]
    log(f"DVR D={D} b={b} strategy={args.strategy} precision={args.precision}")
    kind = KINDS[args.dvr_kernel]
    op = pm.Operator.dvr(D).plan(b, strat, frac, precision=prec).set_dvr_kernel(kind)
    c, R = op.spectral_bounds()
    K = pm.cheb_order(R * dt, 1e-10)
    log(f"c={c:.6g} R={R:.6g} K={K} (H products per step)")
    psi = torch.from_numpy(workloads.wavepacket(D).astype(np.complex64)).cuda()
    s = torch.cuda.current_stream()
    for w in range(args.warmup):
        op.propagate(psi, dt, nsteps=1, K=K, c=c, R=R)
        torch.cuda.synchronize()
        log(f"warmup step {w + 1}/{args.warmup} done")
    op.profile(args.profile_every)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    for k in range(args.steps):
        op.propagate(psi, dt, nsteps=1, K=K, c=c, R=R)
        if args.steps > 1:
            log(f"timed step {k + 1}/{args.steps} enqueued")
    e1.record(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = op.profile_read()
    op.profile(0)
    wall = t1 - t0
    ev = e0.elapsed_time(e1) / 1e3
    log(f"timed {args.steps} steps: wall {wall:.3f} s, events {ev:.3f} s")
    elems = float(args.steps) * K * D * D
    value = elems / wall / 1e9
    psi_host = psi.cpu().numpy()
    t_total = (args.warmup + args.steps) * dt

    tile_avg = prof["tile_ms"] / max(prof["tile_n"], 1) / 1e3
    red_avg = prof["reduce_ms"] / max(prof["reduce_n"], 1) / 1e3
    flops = 4.0 * D * D      # real entry x complex vector: 2 FMA per element
    kern = resolve_kernel(args.dvr_kernel, D)
    if kern == "split":
        # algorithmic work of the split-bf16 product: six piece products
        roof = {"bound": "mfma", "achieved": SPLIT_PRODUCTS * flops / tile_avg / 1e12,
                "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "mfma" if kern == "mfma" else "alu",
                "achieved": flops / tile_avg / 1e12, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = counted_traffic(kern)
    out = {
        "metric": METRIC, "value": value, "unit": "Gelem/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3 split of f32 (f32 accumulate)" if kern == "split" else "f32",
        "data": "synthetic",
        "config": {"workload": f"sinc-DVR harmonic oscillator D={D}, x in [-20,20], "
                               f"wavepacket x0=3 sigma=1, Chebyshev dt={dt}, "
                               f"K={K} products per step, {args.strategy}, "
                               f"{args.precision} arithmetic",
                   "D": D, "nvec": 1, "K": K, "dt": dt, "strategy": args.strategy,
                   "arithmetic": args.precision},
        "cheb_steps_per_s": args.steps / wall,
        "h_products_per_s": args.steps * K / wall,
        "tile_kernel_avg_us": tile_avg * 1e6,
        "reduce_kernel_avg_us": red_avg * 1e6,
        "timed_launches": {"tile": prof["tile_n"], "reduce": prof["reduce_n"],
                           "sampled_every": args.profile_every},
        "dominant_kernel": KERNEL_NAMES[kern],
        "roofline": roof,
        # binary32-equivalent rate of the product (4 D^2 flop) against the
        # binary32 peak, for comparison with the binary32 kernels
        "fp32_equivalent": {"achieved": flops / tile_avg / 1e12, "peak": PEAK_FP32_TFLOPS,
                            "unit": "TFLOP/s", "frac": flops / tile_avg / 1e12 / PEAK_FP32_TFLOPS},
    }

    if args.modes:
        X = torch.from_numpy(workloads.gaussian_vectors(D, 1, seed=2)
                             .astype(np.complex64)).cuda()
        modes = {}
        for name, st, f in [("procedural", pm.PROCEDURAL, 0.0),
                            ("partial50", pm.PARTIAL, 0.5),
                            ("full", pm.FULL, 1.0)]:
            o2 = pm.Operator.dvr(D).plan(b, st, f, precision=prec).set_dvr_kernel(kind)
            t, pr = measure_apply(pm, o2, X, args.mode_reps)
            info = o2.plan_info()
            ta = pr["tile_ms"] / max(pr["tile_n"], 1) / 1e3
            modes[name] = {"gelem_s": D * D / t / 1e9, "us_per_product": t * 1e6,
                           "tile_us": ta * 1e6,
                           "cache_gb": info["cache_bytes"] / 1e9,
                           "cache_read_gb_s": info["cache_bytes"] / ta / 1e9}
            log(f"mode {name}: {modes[name]['gelem_s']:.1f} Gelem/s")
            o2.close()
            torch.cuda.synchronize()
        out["modes"] = modes

    if args.cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_dvr(D)
        n_steps = args.warmup + args.steps
        out["err_vs_exact"] = stated_error_dvr(psi_host, D, t_total)
        out["err_steps"] = n_steps
        out["err_time"] = t_total
        # target: 1e-4 after 200 steps, rounding errors of independent steps
        # adding in quadrature
        out["err_budget"] = 1e-4 * math.sqrt(n_steps / 200.0)
    return out


def pmc_probe(args):
    """Short fixed workload for hardware-counter runs: 20 products of the
    benchmark operator (the dominant kernel) and 20 device copies of 256 MiB
    (a plain copy kernel of known traffic, for scaling the counters)."""
    import numpy as np
    import torch
    from paper_2606_31598_amd import procmv as pm
    from paper_2606_31598_amd import workloads
    D = args.D
    prec = {"fp32": pm.FP32, "compensated": pm.FP32_COMPENSATED}[args.precision]
    kind = KINDS[args.dvr_kernel]
    op = pm.Operator.dvr(D).plan(args.block, precision=prec).set_dvr_kernel(kind)
    X = torch.from_numpy(workloads.gaussian_vectors(D, 1, seed=2).astype(np.complex64)).cuda()
    Y = torch.empty_like(X)
    for _ in range(20):
        op.apply(X, Y)
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(20):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": "done", "D": D, "copy_bytes": src.numel() * 4}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--D", type=int, default=32768)
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--strategy", default="procedural",
                    choices=["procedural", "partial", "full"])
    ap.add_argument("--precision", default="compensated", choices=["fp32", "compensated"],
                    help="binary32 arithmetic of the products and the recurrence")
    ap.add_argument("--dvr-kernel", default="auto", choices=list(KINDS),
                    help="procedural sinc-DVR product: split = bf16 matrix cores with an "
                         "exact three-piece split, mfma = binary32 matrix cores, valu = "
                         "binary32 FMA; auto = the library's choice (split from D = 16384)")
    ap.add_argument("--profile-every", type=int, default=256,
                    help="dispatch-stamp every n-th product and reduction launch (HIP "
                         "events; stamping every 16th costs about 2%% of the step)")
    ap.add_argument("--mode-reps", type=int, default=50)
    ap.add_argument("--no-modes", dest="modes", action="store_false")
    ap.add_argument("--no-cpu", dest="cpu", action="store_false")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short fixed run for hardware-counter collection")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    if args.pmc_probe:
        pmc_probe(args)
        return
    out = run_dvr(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
