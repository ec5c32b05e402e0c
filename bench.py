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
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for "
                         "the HBM byte counters of a profiler run)")
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


def cpu_baseline(M, N, off, target_s):
    """The float64 oracle, as it stands, on a bounded slab of the same
    workload: the first r rows of M and columns of N with the full inner
    dimension, rule norm, c = 256. r grows until the run takes about
    ``target_s`` seconds."""
    from oracle import method as om
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    r = 256
    while True:
        Ms = M[:r, :]
        Ns = N[:, :r]
        t0 = time.perf_counter()
        res = om.run(Ms, Ns, off, 256, seed=0, prob="norm")
        dt = time.perf_counter() - t0
        if dt >= target_s / 2 or r >= M.shape[0]:
            break
        r = min(M.shape[0], r * 2)
    n = M.shape[1]
    flops = 2.0 * r * n * r + 2.0 * r * r * res.draws.L
    return {
        "value": flops / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"oracle norm pass, design, draws, sketch, CD and exact MN in float64 on "
                   f"M[:{r}, :] (x{n}) and N[:, :{r}], rule norm, c=256, L={res.draws.L}; "
                   f"{dt:.1f} s"),
        "seconds": dt,
    }


def linear_layer_leg(h, pk, wl, torch, steps, warmup):
    """The differentiable linear layer Y ~ X W (bf16, 512 blocks of 32,
    c = 128): forward (norms, plan, gather, sketched product) and backward
    (dC = G D^T, dD = C^T G and the scatter into dX, dW), beside the dense
    backward G W^T, X^T G with torch's bf16 matmul for context."""
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
        dX, dW = h.backward(prob, pl, C, D, Gd)
        e2.record()
        if it >= warmup:
            fw.append((e0, e1))
            bw.append((e1, e2))
    L = int(pl.col_off[-1].item())
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
    bwd_flops = 2 * (2.0 * b * d_out * L)
    return {
        "workload": (f"linear layer X {b}x{d_in}, W {d_in}x{d_out} bf16, 512 blocks of 32, "
                     f"c={c}, G {b}x{d_out} float32"),
        "L": L,
        "forward_ms": t_f,
        "backward_ms": t_b,
        "backward_TFLOPs": bwd_flops / t_b / 1e9,
        "backward_frac_bf16_peak": bwd_flops / t_b / 1e9 / 2500.0,
        "dense_backward_ms_torch_bf16": t_d,
        "backward_speedup_vs_dense": t_d / t_b,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the path "
              "runs on one MI355X; multi-GPU sharding is a design note, not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2105_04940_amd as pk
    import workloads as wl

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
    MN, bp, _ = h.exact(base, store=True, blocknorm=True)
    f32 = sketch_leg(False, col, row, blk, MN, bp, torch.float32, "f32")
    for _ in range(args.warmup):
        sketch_leg(False, col, row, blk, MN, bp, torch.bfloat16, "bf16")
    for _ in range(args.steps):
        b16 = sketch_leg(True, col, row, blk, MN, bp, torch.bfloat16, "bf16")
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

    t_norm = avg_ms("norm_pass")
    t_exact = avg_ms("exact_gemm")
    t_sk = {c: avg_ms(f"sketch_gemm_c{c}") for c in CS}
    kernels = {
        "norm_pass": {"ms": t_norm, "GB/s": norm_bytes / t_norm / 1e6},
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
    gh = source_hash("gemm.hip", "common.h")
    if sk_total_ms >= t_exact:
        dom = "sketch_gemm"
        achieved = sketch_tflops
        per_launch = sk_total_flops / (3 * len(CS))
    else:
        dom = "exact_gemm"
        achieved = exact_flops / t_exact / 1e9
        per_launch = exact_flops
    traffic = traffic_from_profile(dom, gh, per_launch)
    roofline = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
                "flops_per_launch": per_launch}
    norm_roof = {"kernel": "norm_pass", "bound": "hbm", "achieved": kernels["norm_pass"]["GB/s"],
                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": kernels["norm_pass"]["GB/s"] / HBM_PEAK_GBS, "bytes_per_launch": norm_bytes}

    t_b16 = {c: avg_ms(f"bf16_c{c}") for c in CS}
    b16_flops = sum(sketch_flops[c] for c in CS) * len(RULES)
    b16_ms = sum(t_b16[c] for c in CS) * len(RULES)
    bf16 = {
        "sketch_gemm_TFLOPs": b16_flops / b16_ms / 1e9,
        "peak": 2500.0, "unit": "TFLOP/s",
        "frac": b16_flops / b16_ms / 1e9 / 2500.0,
        "speedup_vs_f32": sk_total_ms / b16_ms,
        "per_c": {f"c{c}": {"ms": t_b16[c], "TFLOP/s": sketch_flops[c] / t_b16[c] / 1e9} for c in CS},
        "rel_err": {f"{r}/c{c}": math.sqrt(b16[(r, c)][0].item() / mn2v) for r in RULES for c in CS},
        "cd_rel_diff_vs_f32": {f"{r}/c{c}": float(((b16[(r, c)][2] - f32[(r, c)][2]).norm()
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
        "bf16": bf16,
    }
    if not args.no_linear_layer:
        del Md, Nd, MN, res, f32, b16
        torch.cuda.empty_cache()
        out["linear_layer"] = linear_layer_leg(h, pk, wl, torch, args.steps, args.warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(M, N, off, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    h.close()


if __name__ == "__main__":
    main()
