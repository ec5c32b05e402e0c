"""Benchmark of the sampled block matrix product on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (paper-scale block sampling): M 4096 x 65536 and N 65536 x 4096
float32, column j of M and row j of N scaled by independent lognormal(0, 1.5)
factors, 1024 uneven blocks of 16..112 columns / rows, c in {64, 128, 256}
draws with the block probabilities (1.4) "norm", uniform, and (1.2) "exact".

One step is one pass of the whole path over that input, resident in HBM:
the norm pass, the exact product MN with the per-block norms ||M^k N_k||_F
that (1.2) needs and ||MN||_F, then for each of the 9 (rule, c) pairs the
design and draws, the gather of C and D, and the sketched product CD with
||MN - CD||_F in its epilogue.

Printed: one JSON line. ``value`` is the whole step's matrix-core throughput
(algorithmic flops of the 9 sketched products and the exact product, divided
by the step time); the line also carries the norm-pass bandwidth, the
per-kernel rates measured with HIP events on the launch stream, the relative
errors per (rule, c), the roofline of the dominant kernel and the float64 CPU
reference timed on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("sketched-GEMM TFLOP/s + norm-pass GB/s at fixed rel ||MN−CD||_F error, "
          "1 MI355X")
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
RULES = ("norm", "uniform", "exact")
CS = (64, 128, 256)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-linear-layer", action="store_true",
                    help="skip the bf16 linear-layer forward/backward leg")
    ap.add_argument("--no-section4", action="store_true",
                    help="skip the paper's Section 4 stratified-sampling leg")
    ap.add_argument("--section4-sweeps", action="store_true",
                    help="run the paper's Table 1 experiments (Cases I/II, c, K and c0 sweeps) and print their JSON")
    ap.add_argument("--bound-checks", action="store_true",
                    help="the probability error bounds of Thms 3.3, 4.2, 4.4 at the Section 4 sizes")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 512-problem batched leg")
    ap.add_argument("--no-section4-sweeps", action="store_true",
                    help="skip the compact Table 1 sweep record of the default run")
    ap.add_argument("--no-bound-checks", action="store_true",
                    help="skip the compact bound-check record of the default run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for "
                         "the HBM byte counters of a profiler run)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarize two rocprofv3 counter_collection.csv files (FETCH_SIZE, "
                         "WRITE_SIZE) of a --calibration-copy run into profiles/hbm_traffic.json "
                         "and exit (no GPU use)")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_CSV", "COMMAND"),
                    help="print a markdown kernel-time table from a rocprofv3 kernel_trace.csv "
                         "(float32 products split into exact and sketched) and exit (no GPU use)")
    return ap.parse_args()


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2105_04940_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_key, src_hash, launches_flops):
    """HBM bytes per launch of the kernel from the committed counter summary,
    if it was taken from the current source (else None)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_key)
    if not ent or ent.get("source_hash") != src_hash:
        return None
    return ent.get("bytes_per_launch")


CAL_BYTES = 256 << 20   # the --calibration-copy size


def pmc_summary(fetch_csv, write_csv, command):
    """HBM bytes per launch of the float32 products from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the counter reads for
    the plain 256 MiB copy. A float32 product launched right after the
    block-Gram kernel is the exact MN; the others are sketched products."""
    import csv

    def rows(path, counter):
        out = []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]),
                                float(r["Counter_Value"]) * 1024.0))
        out.sort()
        return out

    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rs = rows(path, counter)
        copies = [v for _, name, grid, v in rs if "copyBuffer" in name and v > CAL_BYTES / 8]
        if not copies:
            raise SystemExit(f"{path}: no calibration copy found")
        factor = CAL_BYTES / copies[0]
        groups = {"sketch_gemm": [], "exact_gemm": []}
        prev = ""
        for _, name, grid, v in rs:
            if _is_f32_product(name):
                groups["exact_gemm" if "block_gram" in prev else "sketch_gemm"].append(v * factor)
            if "copyBuffer" not in name:
                prev = name
        res[counter] = (factor, {k: (float(np.mean(v)) if v else None, len(v))
                                 for k, v in groups.items()})
    gh = source_hash("gemm.hip", "gemm_common.h")
    out = {"command": command, "calibration": {
        "copy_bytes": CAL_BYTES, "fetch_factor": res["FETCH_SIZE"][0],
        "write_factor": res["WRITE_SIZE"][0]}}
    for key in ("sketch_gemm", "exact_gemm"):
        f, nf = res["FETCH_SIZE"][1][key]
        w, nw = res["WRITE_SIZE"][1][key]
        if f is None or w is None:
            continue
        out[key] = {"source_hash": gh, "fetch_bytes": f, "write_bytes": w,
                    "bytes_per_launch": f + w, "launches": [nf, nw]}
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def _is_f32_product(name):
    """The single-problem float32 product kernels (128 x 128 and 256 x 256
    tiles), not the grouped ones of the batched path."""
    return "sgemm_kernel" in name or "sgemm_lds_kernel" in name


def _short(name):
    name = name.replace("(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in name:             # drop the argument list
        if ch == "(" and depth == 0 and out:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).replace("void ", "")


def trace_summary(trace_csv, command):
    """Kernel-time table from a rocprofv3 kernel trace; a float32 product
    launched right after the block-Gram kernel is the exact MN, the others
    are sketched products."""
    import csv
    with open(trace_csv) as fh:
        recs = sorted(csv.DictReader(fh), key=lambda r: int(r["Dispatch_Id"]))
    stats = {}
    prev = ""
    for r in recs:
        name = _short(r["Kernel_Name"])
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        key = name
        if _is_f32_product(name):
            key = name + (" — exact MN" if "block_gram" in prev else " — sketched CD")
        stats.setdefault(key, []).append(us)
        if "copyBuffer" not in name:
            prev = name
    total = sum(sum(v) for v in stats.values())
    print(f"Command (repository root, one MI355X):\n\n```\n{command}\n```\n")
    print("| kernel | calls | avg (us) | min (us) | max (us) | total (ms) | % |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for k, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        print(f"| `{k}` | {len(v)} | {np.mean(v):.1f} | {min(v):.1f} | {max(v):.1f} | "
              f"{sum(v) / 1e3:.2f} | {100 * sum(v) / total:.1f} |")


def cpu_baseline(M, N, off, target_s):
    """The float64 oracle, as it stands, on the same step: norms, exact MN,
    per-block ||M^k N_k||_F^2, then for each (rule, c) the design, draws,
    sketch, CD and its error. If the whole step would take much longer than
    ``target_s`` seconds, a slab of M's first r rows and N's first r columns
    (full inner dimension) stands in, r sized from a timed probe. The value is
    the step's algorithmic flops (as on the GPU) per second."""
    from oracle import method as om
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    n = M.shape[1]
    r = M.shape[0]
    # probe: one exact product on a 512-row slab predicts the step time
    t0 = time.perf_counter()
    om.exact_product(M[:512, :], N[:, :512])
    probe = time.perf_counter() - t0
    # the step costs about 8 such products (MN, the per-block products, the
    # sketches); it scales with r^2
    r = int(min(r, max(256, 128 * math.floor(512 * math.sqrt(target_s / (8 * probe)) / 128))))
    Ms, Ns = M[:r, :], N[:, :r]
    t0 = time.perf_counter()
    col, row = om.column_row_sq(Ms, Ns)
    MN = om.exact_product(Ms, Ns)
    bp = om.block_product_sq(Ms, Ns, off)
    flops = 2.0 * r * n * r
    Ls = []
    for rule in RULES:
        for c in CS:
            design, *_ = om.plan(Ms, Ns, off, c, prob=rule, col_row=(col, row),
                                 blkprod_sq=bp if rule == "exact" else None)
            draws = om.sample(design, 0, 0)
            C, D = om.sketch(Ms, Ns, draws)
            CD = om.sketch_product(C, D)
            om.judge(MN, CD)
            flops += 2.0 * r * r * draws.L
            Ls.append(draws.L)
    dt = time.perf_counter() - t0
    return {
        "value": flops / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": int(threads),
        "cpu_model": cpu_model_string(),
        "host_cpus": os.cpu_count(),
        "tiny_workload": tiny_oracle_seconds(),
        "kind": "oracle",
        "sample": (f"one whole step of the oracle in float64 (norms, exact MN, per-block "
                   f"norms, 9 x (design, draws, sketch, CD, error), L = {Ls}) on M[:{r}, :] "
                   f"(x{n}) and N[:, :{r}]; {dt:.1f} s"),
        "seconds": dt,
    }


def cpu_model_string():
    """The host CPU as /proc/cpuinfo names it, with its family / model /
    stepping numbers and clock (a virtualized host may report only a short
    model name)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ":" in ln:
                    k, v = ln.split(":", 1)
                    info.setdefault(k.strip(), v.strip())
    except OSError:
        return ""
    parts = [info.get("model name", "")]
    ids = [f"{k} {info[k]}" for k in ("vendor_id", "cpu family", "model", "stepping") if k in info]
    if ids:
        parts.append("(" + ", ".join(ids) + ")")
    if "cpu MHz" in info:
        parts.append(f"{float(info['cpu MHz']):.0f} MHz")
    if "cache size" in info:
        parts.append(f"cache {info['cache size']}")
    return " ".join(x for x in parts if x)


def tiny_oracle_seconds(reps=5):
    """The oracle on the tiny workload (M 256x1024, N 1024x256 float64, 64
    blocks of 16, c = 16, rule (1.4)), whole run (norms, design, draws,
    sketch, CD, exact MN, error): median seconds with every BLAS thread and
    with one."""
    import workloads as wl
    from oracle import method as om
    M, N, off = wl.tiny(0)

    def timeit():
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            om.run(M, N, off, 16, seed=0, prob="norm")
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    out = {"all_threads_s": timeit()}
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            out["single_thread_s"] = timeit()
    except Exception as e:   # threadpoolctl missing: report that, not a number
        out["single_thread_s"] = None
        out["single_thread_note"] = f"threadpoolctl unavailable: {e}"
    return out


def section4_sweeps_compact(r):
    """The Table 1 sweep reduced to the mean relative error per (case,
    experiment, point, method), 4 significant digits, and the paper's
    findings on Case II."""
    out = {"replications": r["replications"], "ssm_budget": r["ssm_budget"],
           "experiments": "vary_c: Exps 1/3 (K=10, c0=5000); vary_K: Exps 2/4 (c=5e4, c0=5000); "
                          "vary_c0: Exp 5 (c=5e4, K=10)"}
    for case in ("caseI", "caseII"):
        out[case] = {exp: {pt: {meth: float(f"{v['rel_mean']:.4g}") for meth, v in pts.items()}
                           for pt, pts in pts_all.items()}
                     for exp, pts_all in r[case].items()}
    out["paper_findings_case_II"] = r["paper_findings_case_II"]
    return out


def bound_checks_compact(r):
    """Per case and method: theta's, beta, the variance bound against the
    design's expected squared error, and per delta the exceedance fraction;
    the checks and whether all hold."""
    out = {"replications": r["replications"], "deltas": r["deltas"]}
    for case in ("caseI", "caseII"):
        out[case] = {}
        for name, v in r[case].items():
            out[case][name] = {"theta1": v["theta1"], "theta2": v["theta2"], "beta": v["beta"],
                               "expected_over_var_bound": v["expected_over_var_bound"],
                               "sq_err_mean_over_expected": v["sq_err_mean_over_expected"],
                               "exceed_frac": {d: x["exceed_frac"] for d, x in v["per_delta"].items()}}
    out["checks_failed"] = [k for k, ok in r["checks"].items() if not ok]
    out["checks_total"] = len(r["checks"])
    out["all_hold"] = r["all_hold"]
    return out


def stream_copy_GBps(torch, nbytes=1 << 30, reps=10):
    """A plain device-to-device copy of nbytes (torch's copy kernel): bytes
    read plus written per second, the box's own streaming reference."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / ms / 1e6


def fused_vs_materialized(h, pk, torch, Md, Nd, off, c, reps=3):
    """The paper-scale problem as a batch of one (rule (1.4), c draws): the
    sketched product with the gather fused into its loads against gathering C,
    D first, per tile shape, as the batch tuner times them (HIP events)."""
    b = pk.Batch(h, [dict(M=Md, N=Nd, off=off, c=c, prob="norm", seed=0, trial=0)])
    t = b.tune(reps=reps)
    b.run()
    torch.cuda.synchronize()
    L = int(b.L[0].item())
    flops = 2.0 * Md.shape[0] * Nd.shape[1] * L
    ms = t["ms"][1]
    n = len(pk.BATCH_TILES)
    best_f = min(v for v in ms[:2 * n] if v > 0)
    best_m = min(v for v in ms[2 * n:4 * n] if v > 0) if any(v > 0 for v in ms[2 * n:4 * n]) else None
    out = {"c": c, "L": L,
           "fused_ms": best_f, "fused_TFLOPs": flops / best_f / 1e9,
           "materialized_ms": best_m,
           "materialized_TFLOPs": flops / best_m / 1e9 if best_m else None,
           "note": "materialized includes its gather; tiles of the batched grouped product"}
    b.close()
    torch.cuda.empty_cache()
    return out


def linear_layer_leg(h, pk, wl, torch, steps, warmup):
    """The differentiable linear layer Y ~ X W (bf16, 512 blocks of 32,
    c = 128): forward (norms, plan, gather, sketched product) and backward
    (draws merged per block; dX[:, drawn] = w G W_U^T and dW[drawn, :] =
    w X_U^T G over the L_U distinct drawn columns, written by the products'
    epilogues, the undrawn columns / rows zeroed), beside the dense backward
    G W^T, X^T G with torch's bf16 matmul for context."""
    dev = "cuda:0"
    X, W, G = wl.linear_layer()
    off = wl.equal_blocks(X.shape[1], 512)
    Xd = torch.from_numpy(X).to(dev).to(torch.bfloat16)
    Wd = torch.from_numpy(W).to(dev).to(torch.bfloat16)
    Gd = torch.from_numpy(G).to(dev)
    del X, W, G
    b, d_in = Xd.shape
    d_out = Wd.shape[1]
    c = 128
    prob = pk.Problem(Xd, Wd, off, c, seed=11)

    def fwd():
        col, row, blk = h.norms(prob)
        pl = h.plan(prob, col, row, blk, sync=False)
        C, D = h.sketch(prob, pl, out_dtype=torch.bfloat16)
        Y, _ = h.sketch_gemm(C, D, pl)
        return pl, C, D, Y

    def ev():
        return torch.cuda.Event(enable_timing=True)

    fw, bw = [], []
    for it in range(warmup + steps):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record()
        pl, C, D, Y = fwd()
        e1.record()
        dX, dW = h.backward(prob, pl, None, None, Gd, compute=torch.bfloat16)
        e2.record()
        if it >= warmup:
            fw.append((e0, e1))
            bw.append((e1, e2))
    L = int(pl.col_off[-1].item())
    L_u = 32 * int(torch.unique(pl.idx).numel())   # distinct drawn columns
    # dense backward in bf16 for context (transposed operands made contiguous)
    G16 = Gd.to(torch.bfloat16)
    Wt = Wd.t().contiguous()
    Xt = Xd.t().contiguous()
    dense = []
    for it in range(warmup + steps):
        e0, e1 = ev(), ev()
        e0.record()
        torch.mm(G16, Wt)
        torch.mm(Xt, G16)
        e1.record()
        if it >= warmup:
            dense.append((e0, e1))
    torch.cuda.synchronize()
    ms = lambda ev_list: float(np.mean([s.elapsed_time(e) for s, e in ev_list]))
    t_f, t_b, t_d = ms(fw), ms(bw), ms(dense)
    bwd_flops = 2 * (2.0 * b * d_out * L_u)
    return {
        "workload": (f"linear layer X {b}x{d_in}, W {d_in}x{d_out} bf16, 512 blocks of 32, "
                     f"c={c}, G {b}x{d_out} float32"),
        "L": L,
        "L_distinct": L_u,
        "backward_flops": bwd_flops,
        "forward_ms": t_f,
        "backward_ms": t_b,
        "backward_TFLOPs": bwd_flops / t_b / 1e9,
        "backward_frac_bf16_peak": bwd_flops / t_b / 1e9 / 2500.0,
        "dense_backward_ms_torch_bf16": t_d,
        "backward_speedup_vs_dense": t_d / t_b,
    }


def batched_leg(h, pk, wl, torch, steps, warmup):
    """512 independent problems (m, p in [256, 2048], n in [4096, 32768],
    blocks of 8..128, c in [16, 256], inputs written on the device) as one
    batched pass: grouped norm pass, per-problem plans, grouped exact and
    sketched products. Tuned once, then timed eagerly and as a graph."""
    items, mats = wl.batched_device_inputs(512)
    probs = [dict(M=M, N=N, off=it["off"], c=it["c"], prob="norm", seed=0, trial=t)
             for t, (it, (M, N)) in enumerate(zip(items, mats))]
    b = pk.Batch(h, probs)
    tuning = b.tune(reps=2)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(warmup):
            fn()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    eager_ms = timed(b.run)
    b.capture()
    graph_ms = timed(b.replay)
    L = b.L.cpu().numpy()
    e2 = b.err2_mn2.cpu().numpy()
    rel = np.sqrt(e2[0::2] / e2[1::2])
    m = np.array([it["m"] for it in items], np.float64)
    n = np.array([it["n"] for it in items], np.float64)
    p = np.array([it["p"] for it in items], np.float64)
    exact_flops = float(np.sum(2 * m * n * p))
    sketch_flops = float(np.sum(2 * m * p * L))
    norm_bytes = float(np.sum((m * n + n * p) * 4))
    best = [tuning["ms"][g][2 * tuning["cfg"][g] + tuning["lpt"][g]] for g in range(2)]
    out = {
        "workload": ("512 independent block-sampling problems: m, p uniform in [256, 2048], n uniform in "
                     "[4096, 32768], uneven blocks of 8..128, c uniform in [16, 256], rule (1.4), float32 "
                     "inputs from the counter-based stream written on the device; one pass = grouped norm "
                     "pass + per-problem plans + grouped exact MN + grouped sketched CD (gather fused, or "
                     "sketches materialized group by group, as tuned) + per-problem errors"),
        "pass_ms_eager": eager_ms,
        "pass_ms_graph": graph_ms,
        "TFLOPs_graph": (exact_flops + sketch_flops) / graph_ms / 1e9,
        "exact_TFLOPs": exact_flops / best[0] / 1e9,
        "sketch_TFLOPs": sketch_flops / best[1] / 1e9,
        "frac_fp32_peak_sketch": sketch_flops / best[1] / 1e9 / FP32_PEAK_TFLOPS,
        "exact_flops": exact_flops, "sketch_flops": sketch_flops, "norm_bytes": norm_bytes,
        "tuning": tuning,
        "rel_err": {"mean": float(rel.mean()), "min": float(rel.min()), "max": float(rel.max())},
        "L_total": int(L.sum()),
    }
    b.close()
    del mats, probs
    torch.cuda.empty_cache()
    return out


def section4_leg(h, pk, wl, torch, reps=100, warmup=3):
    """The paper's Section 4 setting in float64: m = 26, p = 28, n = 5e5 in
    K = 10 blocks of 5e4, c = 5e4, Cases I (Gaussian) and II (t_1, location
    1). Per method, one step is everything the method computes before its
    estimate is judged: norm pass, then ||M^k N_k||_F per block (OPL) or the
    pilot with c0 = 5000 (ONU, ONMCNR), plan, gather and sketched product
    with its error against the exact MN (computed once, outside the timing).
    Mean relative error over `reps` replications (trials), as the paper
    averages 100."""
    dev = "cuda:0"
    methods = {"UU": dict(prob="uniform", alloc="uniform"),
               "ONC": dict(prob="norm", alloc="norm"),
               "OPL": dict(prob="norm", alloc="opt"),
               "ONU": dict(prob="norm", alloc="two_step", pilot="uniform"),
               "ONMCNR": dict(prob="norm", alloc="two_step", pilot="norm")}
    K, c, c0 = 10, 50000, 5000

    def ev():
        return torch.cuda.Event(enable_timing=True)

    out = {"workload": ("paper Section 4: M 26x500000, N 500000x28 float64, K=10 blocks of 50000, c=50000, "
                        "c0=5000 (two-step pilots), Case I Gaussian rows/columns with Toeplitz covariances, "
                        "Case II multivariate t_1 with location 1; stratified sampling (Alg. 2 / Alg. 3)"),
           "replications": reps}
    for case in (1, 2):
        M, N = wl.case_data(case)
        off = wl.equal_blocks(M.shape[1], K)
        Md = torch.from_numpy(M).to(dev)
        Nd = torch.from_numpy(N).to(dev)
        del M, N
        base = pk.Problem(Md, Nd, off, c, mode="stratified")
        MN, _, mn_sq = h.exact(base, store=True)
        # norm pass bandwidth on this shape
        col, row, blk = h.norms(base)
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(10):
            h.norms(base)
        e1.record()
        torch.cuda.synchronize()
        norm_ms = e0.elapsed_time(e1) / 10
        res = {"norm_pass_ms": norm_ms,
               "norm_pass_GBps": (Md.numel() + Nd.numel()) * 8 / norm_ms / 1e6}
        for name, kw in methods.items():
            ms, errs = [], []
            for t in range(warmup + reps):
                prob = pk.Problem(Md, Nd, off, c, mode="stratified", c0=c0, seed=0, trial=t, **kw)
                a, b = ev(), ev()
                a.record()
                col, row, blk = h.norms(prob)
                if kw["alloc"] == "opt":
                    _, prob.blkprod_sq, _ = h.exact(prob, store=False, blocknorm=True)
                if kw["alloc"] == "two_step":
                    prob.pilot_sq = h.pilot(prob, col, row, blk)
                pl = h.plan(prob, col, row, blk, sync=False)
                C, D = h.sketch(prob, pl)
                _, err = h.sketch_gemm(C, D, pl, MN=MN, store=False)
                b.record()
                if t >= warmup:
                    ms.append((a, b))
                    errs.append(err)
            torch.cuda.synchronize()
            times = [x.elapsed_time(y) for x, y in ms]
            rel = np.sqrt(torch.cat(errs).cpu().numpy() / mn_sq.item())
            res[name] = {"ms_per_step_median": float(np.median(times)),
                         "rel_err_mean": float(rel.mean()), "rel_err_std": float(rel.std())}
        out[f"case{'I' * case}"] = res
        del Md, Nd, MN
        torch.cuda.empty_cache()
    return out


def section4_sweeps(h, pk, wl, torch, reps=100):
    """The paper's Table 1 experiments at its sizes (m = 26, p = 28,
    n = 5e5, float64, Cases I and II, `reps` replications per point):
    1/3 vary c at K = 10, c0 = 5000; 2/4 vary K at c = 5e4, c0 = 5000; 5
    varies c0 at c = 5e4, K = 10. Methods: UU, ONC, OPL (Alg. 2), ONU,
    ONMCNR (Alg. 3) and SSM (block sampling with (1.4); the paper gives no
    budget for it, so it draws round(c / n_k) blocks: a sketch as wide as
    Alg. 2's). Per point and method: mean / std of the relative error and
    the median step time (as in the Section 4 leg). The paper's qualitative
    findings are evaluated on the Case II means."""
    dev = "cuda:0"
    methods = {"UU": dict(mode="stratified", prob="uniform", alloc="uniform"),
               "ONC": dict(mode="stratified", prob="norm", alloc="norm"),
               "OPL": dict(mode="stratified", prob="norm", alloc="opt"),
               "ONU": dict(mode="stratified", prob="norm", alloc="two_step", pilot="uniform"),
               "ONMCNR": dict(mode="stratified", prob="norm", alloc="two_step", pilot="norm"),
               "SSM": dict(mode="block", prob="norm")}

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def point(Md, Nd, MN, mn2, K, c, c0, names):
        off = wl.equal_blocks(Md.shape[1], K)
        out = {}
        for name in names:
            kw = methods[name]
            cc = max(1, round(c / (Md.shape[1] / K))) if name == "SSM" else c
            ms, errs = [], []
            for t in range(2 + reps):
                prob = pk.Problem(Md, Nd, off, cc, c0=c0, seed=0, trial=t, **kw)
                a, b = ev(), ev()
                a.record()
                col, row, blk = h.norms(prob)
                if kw.get("alloc") == "opt":
                    _, prob.blkprod_sq, _ = h.exact(prob, store=False, blocknorm=True)
                if kw.get("alloc") == "two_step":
                    prob.pilot_sq = h.pilot(prob, col, row, blk)
                pl = h.plan(prob, col, row, blk, sync=False)
                C, D = h.sketch(prob, pl)
                _, err = h.sketch_gemm(C, D, pl, MN=MN, store=False)
                b.record()
                if t >= 2:
                    ms.append((a, b))
                    errs.append(err)
            torch.cuda.synchronize()
            rel = np.sqrt(torch.cat(errs).cpu().numpy() / mn2)
            out[name] = {"rel_mean": float(rel.mean()), "rel_std": float(rel.std()),
                         "ms": float(np.median([x.elapsed_time(y) for x, y in ms]))}
        return out

    a2 = ["UU", "ONC", "OPL", "SSM"]
    a23 = ["UU", "ONC", "OPL", "ONU", "ONMCNR"]
    res = {"replications": reps, "ssm_budget": "round(c / n_k) block draws"}
    for case in (1, 2):
        M, N = wl.case_data(case)
        Md = torch.from_numpy(M).to(dev)
        Nd = torch.from_numpy(N).to(dev)
        del M, N
        MN, _, mn_sq = h.exact(pk.Problem(Md, Nd, [0, Md.shape[1]], 1), store=True)
        mn2 = mn_sq.item()
        print(f"section 4 sweeps: case {case}", file=sys.stderr, flush=True)
        cs = [50000, 100000, 200000, 350000, 500000]
        Ks = [10, 50, 100, 250, 500]
        c0s = [500, 1000, 5000, 20000, 50000]
        r = {"vary_c": {str(c): point(Md, Nd, MN, mn2, 10, c, 5000, sorted(set(a2 + a23))) for c in cs},
             "vary_K": {str(K): point(Md, Nd, MN, mn2, K, 50000, 5000, sorted(set(a2 + a23))) for K in Ks},
             "vary_c0": {str(c0): point(Md, Nd, MN, mn2, 10, 50000, c0, ["ONC", "OPL", "ONU", "ONMCNR"])
                         for c0 in c0s}}
        res[f"case{'I' * case}"] = r
        del Md, Nd, MN
        torch.cuda.empty_cache()

    # the paper's qualitative findings, on the Case II means
    r2 = res["caseII"]
    m = lambda grp, key, name: r2[grp][key][name]["rel_mean"]
    claims = {
        "OPL and ONC more accurate than SSM (every c, every K)":
            all(m(g, k, x) < m(g, k, "SSM") for g in ("vary_c", "vary_K") for k in r2[g] for x in ("OPL", "ONC")),
        "UU more accurate than SSM somewhere (the paper says it may be)":
            any(m(g, k, "UU") < m(g, k, "SSM") for g in ("vary_c", "vary_K") for k in r2[g]),
        "OPL the most accurate of Alg. 2 / Alg. 3 (within 2 %) at every c and K":
            all(m(g, k, "OPL") <= 1.02 * min(m(g, k, x) for x in a23) for g in ("vary_c", "vary_K") for k in r2[g]),
        "ONMCNR within 10 % of OPL at every c (K = 10)":
            all(m("vary_c", k, "ONMCNR") <= 1.10 * m("vary_c", k, "OPL") for k in r2["vary_c"]),
        "ONMCNR the least accurate of ONC, OPL, ONU, ONMCNR at the largest K (smallest c0 / K)":
            m("vary_K", "500", "ONMCNR") >= max(m("vary_K", "500", x) for x in ("ONC", "OPL", "ONU")),
        "ONMCNR within 2 % of OPL at the largest c0":
            m("vary_c0", "50000", "ONMCNR") <= 1.02 * m("vary_c0", "50000", "OPL"),
        "ONC within 10 % of OPL at every point":
            all(m(g, k, "ONC") <= 1.10 * m(g, k, "OPL") for g in ("vary_c", "vary_K", "vary_c0") for k in r2[g]),
    }
    res["paper_findings_case_II"] = claims
    return res


def bound_checks(h, pk, wl, torch, reps=100, deltas=(0.5, 0.1, 0.01)):
    """The probability error bounds at the paper's Section 4 sizes (m = 26,
    p = 28, n = 5e5 float64 in K = 10 blocks of 5e4, c = 5e4, c0 = 5000,
    Cases I and II), for the methods they cover: OPL (Thm 3.3, (3.12)), ONC
    (Thm 4.2, (4.4)), ONU and ONMCNR (Thm 4.4, (4.9); the bound changes with
    every pilot). Per method over `reps` trials: theta_1, theta_2 (and the
    range of the pilot's theta^_1, theta^_2), the sampled beta, phi, the
    variance bound against E ||MN - CD||_F^2 of the design and the mean
    squared error; per delta the bound, the fraction of trials whose squared
    error exceeds it (the theorems claim at most delta) and the empirical
    (1 - delta) quantile of the squared error over the bound."""
    dev = "cuda:0"
    methods = {"OPL": dict(prob="norm", alloc="opt"),
               "ONC": dict(prob="norm", alloc="norm"),
               "ONU": dict(prob="norm", alloc="two_step", pilot="uniform"),
               "ONMCNR": dict(prob="norm", alloc="two_step", pilot="norm")}
    K, c, c0 = 10, 50000, 5000
    out = {"workload": "paper Section 4 sizes, float64, K=10 blocks of 50000, c=50000, c0=5000",
           "replications": reps, "deltas": list(deltas)}
    checks = {}
    for case in (1, 2):
        print(f"bound checks: case {case}", file=sys.stderr, flush=True)
        M, N = wl.case_data(case)
        off = wl.equal_blocks(M.shape[1], K)
        Md = torch.from_numpy(M).to(dev)
        Nd = torch.from_numpy(N).to(dev)
        del M, N
        base = pk.Problem(Md, Nd, off, c, mode="stratified")
        MN, bp, _ = h.exact(base, store=True, blocknorm=True)
        col, row, blk = h.norms(base)
        res = {}
        for name, kw in methods.items():
            err2, g = [], []
            for t in range(reps):
                prob = pk.Problem(Md, Nd, off, c, mode="stratified", c0=c0, seed=0, trial=t, **kw)
                if kw["alloc"] == "opt":
                    prob.blkprod_sq = bp
                if kw["alloc"] == "two_step":
                    prob.pilot_sq = h.pilot(prob, col, row, blk)
                pl = h.plan(prob, col, row, blk, sync=False)
                C, D = h.sketch(prob, pl)
                _, e = h.sketch_gemm(C, D, pl, MN=MN, store=False)
                err2.append(e)
                g.append(h.bound(prob, col, row, blk, bp, pl, deltas=deltas))
            e2 = torch.cat(err2).cpu().numpy()
            exp = np.array([x["expected"] for x in g])
            r = {"beta": min(x["beta"] for x in g), "theta1": g[0]["theta1"], "theta2": g[0]["theta2"],
                 "phi_range": [min(x["phi"] for x in g), max(x["phi"] for x in g)],
                 "var_bound_median": float(np.median([x["var_bound"] for x in g])),
                 "expected_sq_err_mean": float(exp.mean()),
                 "sq_err_mean": float(e2.mean()),
                 "sq_err_mean_over_expected": float(e2.mean() / exp.mean()),
                 "std_errors_from_expected": float((e2.mean() - exp.mean()) / (e2.std(ddof=1) / np.sqrt(reps))),
                 "expected_over_var_bound": float(np.max(exp / np.array([x["var_bound"] for x in g])))}
            if kw["alloc"] == "two_step":
                r["theta1_hat_range"] = [min(x["theta1_hat"] for x in g), max(x["theta1_hat"] for x in g)]
                r["theta2_hat_range"] = [min(x["theta2_hat"] for x in g), max(x["theta2_hat"] for x in g)]
            per = {}
            for j, d in enumerate(deltas):
                b = np.array([x["bound"][j] for x in g])
                per[str(d)] = {"bound_median": float(np.median(b)),
                               "exceed_frac": float(np.mean(e2 > b)),
                               "quantile_over_bound": float(np.quantile(e2, 1 - d) / np.median(b))}
                checks[f"case{'I' * case} {name} delta={d}: exceedance <= delta"] = bool(np.mean(e2 > b) <= d)
            r["per_delta"] = per
            checks[f"case{'I' * case} {name}: E||MN-CD||^2 <= variance bound"] = bool(r["expected_over_var_bound"] <= 1)
            checks[f"case{'I' * case} {name}: mean squared error within 5 s.e. of its expectation"] = \
                bool(abs(r["std_errors_from_expected"]) <= 5)
            res[name] = r
        out[f"case{'I' * case}"] = res
        del Md, Nd, MN
        torch.cuda.empty_cache()
    out["checks"] = checks
    out["all_hold"] = all(checks.values())
    return out


def main():
    args = parse()
    if args.trace_summary:
        trace_summary(*args.trace_summary)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1],
                    "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -d <dir> -o run -- "
                    "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-linear-layer --no-batched "
                    "--no-section4 --no-section4-sweeps --no-bound-checks --calibration-copy")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the path "
              "runs on one MI355X; multi-GPU sharding is a design note, not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2105_04940_amd as pk
    import workloads as wl

    if args.section4_sweeps:
        print(json.dumps(section4_sweeps(pk.Handle(0), pk, wl, torch)))
        return
    if args.bound_checks:
        print(json.dumps(bound_checks(pk.Handle(0), pk, wl, torch)))
        return
    dev = "cuda:0"
    M, N, off = wl.paper_scale()
    m, n = M.shape
    p = N.shape[1]
    Md = torch.from_numpy(M).to(dev)
    Nd = torch.from_numpy(N).to(dev)
    h = pk.Handle(0)
    if args.calibration_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    torch.cuda.synchronize()

    timers = {}   # name -> list of (start, end) events

    def timed(name, fn):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        out = fn()
        e.record()
        timers.setdefault(name, []).append((s, e))
        return out

    def sketch_leg(record, col, row, blk, MN, bp, compute, tag):
        res = {}
        for rule in RULES:
            for c in CS:
                prob = pk.Problem(Md, Nd, off, c, prob=rule, seed=0, trial=0,
                                  blkprod_sq=bp if rule == "exact" else None)
                pl = h.plan(prob, col, row, blk, sync=False)
                C, D = h.sketch(prob, pl, out_dtype=compute)
                CD, err = (timed(f"{tag}_c{c}", lambda: h.sketch_gemm(C, D, pl, MN=MN))
                           if record else h.sketch_gemm(C, D, pl, MN=MN))
                res[(rule, c)] = (err, pl, CD)
        return res

    def mx_leg(record, col, row, blk, MN, bp):
        res = {}
        for rule in RULES:
            for c in CS:
                prob = pk.Problem(Md, Nd, off, c, prob=rule, seed=0, trial=0,
                                  blkprod_sq=bp if rule == "exact" else None)
                pl = h.plan(prob, col, row, blk, sync=False)
                C8, Cs, Dt8, Ds = h.sketch_mx(prob, pl)
                CD, err = (timed(f"mx_c{c}", lambda: h.sketch_gemm_mx(C8, Cs, Dt8, Ds, pl, MN=MN))
                           if record else h.sketch_gemm_mx(C8, Cs, Dt8, Ds, pl, MN=MN))
                res[(rule, c)] = (err, pl, CD)
        return res

    def step(record):
        res = {}
        base = pk.Problem(Md, Nd, off, CS[-1])
        col, row, blk = (timed("norm_pass", lambda: h.norms(base)) if record
                         else h.norms(base))
        MN, bp, mn2 = (timed("exact_gemm", lambda: h.exact(base, store=True, blocknorm=True))
                       if record else h.exact(base, store=True, blocknorm=True))
        for rule in RULES:
            for c in CS:
                prob = pk.Problem(Md, Nd, off, c, prob=rule, seed=0, trial=0,
                                  blkprod_sq=bp if rule == "exact" else None)
                pl = (timed("plan", lambda: h.plan(prob, col, row, blk, sync=False)) if record
                      else h.plan(prob, col, row, blk, sync=False))
                C, D = (timed("gather", lambda: h.sketch(prob, pl)) if record
                        else h.sketch(prob, pl))
                CD, err = (timed(f"sketch_gemm_c{c}", lambda: h.sketch_gemm(C, D, pl, MN=MN))
                           if record else h.sketch_gemm(C, D, pl, MN=MN))
                res[(rule, c)] = (err, pl)
        return res, mn2

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    timers.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, mn2 = step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    def avg_ms(name):
        return float(np.mean([s.elapsed_time(e) for s, e in timers[name]]))

    # bf16 sketches of the same draws (beside the float32 step, not in it)
    base = pk.Problem(Md, Nd, off, CS[-1])
    col, row, blk = h.norms(base)
    # the norm pass on its own: 20 back-to-back calls between two events (the
    # events around each call inside the step leave the GPU idle for about
    # 10 us each, which the per-call figure includes)
    torch.cuda.synchronize()
    n0, n1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n0.record()
    for _ in range(20):
        h.norms(base)
    n1.record()
    torch.cuda.synchronize()
    t_norm_b2b = n0.elapsed_time(n1) / 20
    MN, bp, _ = h.exact(base, store=True, blocknorm=True)
    f32 = sketch_leg(False, col, row, blk, MN, bp, torch.float32, "f32")
    for _ in range(args.warmup):
        sketch_leg(False, col, row, blk, MN, bp, torch.bfloat16, "bf16")
    for _ in range(args.steps):
        b16 = sketch_leg(True, col, row, blk, MN, bp, torch.bfloat16, "bf16")
    torch.cuda.synchronize()
    # MX E4M3 sketches of the same draws
    for _ in range(args.warmup):
        mx_leg(False, col, row, blk, MN, bp)
    for _ in range(args.steps):
        mx8 = mx_leg(True, col, row, blk, MN, bp)
    torch.cuda.synchronize()

    mn2v = mn2.item()
    rel_err = {}
    Ls = {}
    for (rule, c), (err, pl) in res.items():
        rel_err[f"{rule}/c{c}"] = math.sqrt(err.item() / mn2v)
        Ls[f"{rule}/c{c}"] = int(pl.col_off[-1].item())

    # algorithmic work
    norm_bytes = (m * n + n * p) * 4
    exact_flops = 2.0 * m * n * p
    sketch_flops = {c: float(np.mean([2.0 * m * p * Ls[f"{r}/c{c}"] for r in RULES])) for c in CS}
    step_flops = exact_flops + sum(2.0 * m * p * L for L in Ls.values())

    t_norm_step = avg_ms("norm_pass")
    t_norm = t_norm_b2b
    t_exact = avg_ms("exact_gemm")
    t_sk = {c: avg_ms(f"sketch_gemm_c{c}") for c in CS}
    kernels = {
        "norm_pass": {"ms": t_norm, "GB/s": norm_bytes / t_norm / 1e6, "timing": "20 back-to-back passes",
                      "in_step_ms": t_norm_step, "in_step_GB/s": norm_bytes / t_norm_step / 1e6},
        "exact_gemm": {"ms": t_exact, "TFLOP/s": exact_flops / t_exact / 1e9},
        "plan": {"ms": avg_ms("plan")},
        "gather": {"ms": avg_ms("gather"),
                   "GB/s": float(np.mean([2 * (m + p) * Ls[k] * 4 for k in Ls])) / avg_ms("gather") / 1e6},
    }
    for c in CS:
        kernels[f"sketch_gemm_c{c}"] = {"ms": t_sk[c], "TFLOP/s": sketch_flops[c] / t_sk[c] / 1e9,
                                        "mean_L": sketch_flops[c] / (2.0 * m * p)}
    sk_total_ms = sum(t_sk[c] for c in CS) * len(RULES)
    sk_total_flops = sum(sketch_flops[c] for c in CS) * len(RULES)
    sketch_tflops = sk_total_flops / sk_total_ms / 1e9

    # dominant kernel of the step by time: the sketched products (one kernel,
    # 9 launches) or the exact product with block norms (one launch)
    gh = source_hash("gemm.hip", "gemm_common.h")
    if sk_total_ms >= t_exact:
        dom = "sketch_gemm"
        achieved = sketch_tflops
        per_launch = sk_total_flops / (3 * len(CS))
    else:
        dom = "exact_gemm"
        achieved = exact_flops / t_exact / 1e9
        per_launch = exact_flops
    traffic = traffic_from_profile(dom, gh, per_launch)
    # the box's own matrix-core rates (register operands, outside the timed
    # region): the spec peaks assume a clock the power limit holds lower
    mpk = {d: h.peak_probe(d) for d in ("f32", "bf16", "f8e4m3")}
    roofline = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
                "flops_per_launch": per_launch, "measured_peak": mpk["f32"],
                "frac_of_measured_peak": achieved / mpk["f32"]}
    copy_gbs = stream_copy_GBps(torch)
    norm_roof = {"kernel": "norm_pass", "bound": "hbm", "achieved": kernels["norm_pass"]["GB/s"],
                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": kernels["norm_pass"]["GB/s"] / HBM_PEAK_GBS, "bytes_per_launch": norm_bytes,
                 "measured_copy_GBps": copy_gbs,
                 "frac_of_measured_copy": kernels["norm_pass"]["GB/s"] / copy_gbs}
    fvm = fused_vs_materialized(h, pk, torch, Md, Nd, off, CS[-1])

    t_b16 = {c: avg_ms(f"bf16_c{c}") for c in CS}
    b16_flops = sum(sketch_flops[c] for c in CS) * len(RULES)
    b16_ms = sum(t_b16[c] for c in CS) * len(RULES)
    bf16 = {
        "sketch_gemm_TFLOPs": b16_flops / b16_ms / 1e9,
        "peak": 2500.0, "unit": "TFLOP/s",
        "frac": b16_flops / b16_ms / 1e9 / 2500.0,
        "measured_peak": mpk["bf16"], "frac_of_measured_peak": b16_flops / b16_ms / 1e9 / mpk["bf16"],
        "speedup_vs_f32": sk_total_ms / b16_ms,
        "per_c": {f"c{c}": {"ms": t_b16[c], "TFLOP/s": sketch_flops[c] / t_b16[c] / 1e9} for c in CS},
        "rel_err": {f"{r}/c{c}": math.sqrt(b16[(r, c)][0].item() / mn2v) for r in RULES for c in CS},
        "cd_rel_diff_vs_f32": {f"{r}/c{c}": float(((b16[(r, c)][2] - f32[(r, c)][2]).norm()
                                                   / f32[(r, c)][2].norm()).item())
                               for r in RULES for c in CS},
    }
    t_mx = {c: avg_ms(f"mx_c{c}") for c in CS}
    mx_ms = sum(t_mx[c] for c in CS) * len(RULES)
    mx = {
        "format": "OCP MX E4M3 (E8M0 scale per 32 sketch columns), float32 accumulator across instructions",
        "sketch_gemm_TFLOPs": b16_flops / mx_ms / 1e9,
        "peak": 5000.0, "unit": "TFLOP/s",
        "frac": b16_flops / mx_ms / 1e9 / 5000.0,
        "measured_peak": mpk["f8e4m3"], "frac_of_measured_peak": b16_flops / mx_ms / 1e9 / mpk["f8e4m3"],
        "speedup_vs_f32": sk_total_ms / mx_ms,
        "speedup_vs_bf16": b16_ms / mx_ms,
        "per_c": {f"c{c}": {"ms": t_mx[c], "TFLOP/s": sketch_flops[c] / t_mx[c] / 1e9} for c in CS},
        "rel_err": {f"{r}/c{c}": math.sqrt(mx8[(r, c)][0].item() / mn2v) for r in RULES for c in CS},
        "cd_rel_diff_vs_f32": {f"{r}/c{c}": float(((mx8[(r, c)][2] - f32[(r, c)][2]).norm()
                                                   / f32[(r, c)][2].norm()).item())
                               for r in RULES for c in CS},
    }

    out = {
        "metric": METRIC,
        "value": step_flops / (ms_per_step * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("paper-scale block sampling: M 4096x65536, N 65536x4096 float32 with "
                         "lognormal(0,1.5) column/row factors, K=1024 uneven blocks 16..112, "
                         "c in {64,128,256}, rules norm (1.4) / uniform / exact (1.2); step = norm "
                         "pass + exact MN with block norms + 9 x (plan, gather, sketched CD + error)"),
            "m": m, "n": n, "p": p, "K": len(off) - 1, "c": list(CS), "rules": list(RULES),
            "parallelism": "single GPU",
        },
        "sketch_gemm_TFLOPs": sketch_tflops,
        "norm_pass_GBps": kernels["norm_pass"]["GB/s"],
        "rel_err": rel_err,
        "L": Ls,
        "kernels": kernels,
        "roofline": roofline,
        "roofline_norm_pass": norm_roof,
        "sketch_fused_vs_materialized": fvm,
        "bf16": bf16,
        "mx_e4m3": mx,
    }
    if not args.no_linear_layer:
        del Md, Nd, MN, res, f32, b16, mx8
        torch.cuda.empty_cache()
        out["linear_layer"] = linear_layer_leg(h, pk, wl, torch, args.steps, args.warmup)
    if not args.no_section4:
        print("section 4 leg", file=sys.stderr, flush=True)
        out["section4"] = section4_leg(h, pk, wl, torch)
    if not args.no_section4_sweeps:
        print("section 4 sweeps", file=sys.stderr, flush=True)
        out["section4_sweeps"] = section4_sweeps_compact(section4_sweeps(h, pk, wl, torch))
    if not args.no_bound_checks:
        print("bound checks", file=sys.stderr, flush=True)
        out["bound_checks"] = bound_checks_compact(bound_checks(h, pk, wl, torch))
    if not args.no_batched:
        torch.cuda.empty_cache()
        out["batched"] = batched_leg(h, pk, wl, torch, max(2, args.steps // 2), 1)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(M, N, off, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    h.close()


if __name__ == "__main__":
    main()
