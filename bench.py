#!/usr/bin/env python3
"""Benchmark of the MI355X dimension-lifted FFT.

Default workload: one complex64 transform of n = 2^24 points through the lift
<4096 4096> (two HBM passes: column FFTs with the inter-level twiddle and the
reshape-transpose folded into the store, then row FFTs with the final
transpose folded into the store).  A step is one full transform; inputs are
resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-extras]

Throughput is 5 n log2(n) / t (GFLOP/s).  The roofline block reports the
dominant kernel (the slower of the two level launches) against the 8 TB/s
HBM peak with its algorithmic bytes (read + write of every element once per
launch), timed with HIP events on the stream the kernels run on.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FFT GFLOP/s (5n·log2n/t) & HBM GB/s vs peak, batched/MFMA vs plain, at stated error"
HBM_PEAK_GBS = 8000.0


def gflops(n, batch, seconds):
    return 5.0 * n * math.log2(max(n, 2)) * batch / seconds / 1e9


def time_events(fn, reps, torch):
    """Average duration (ms) of fn() over reps, by HIP events on the current stream."""
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def kernel_name(p):
    """Device symbol (demangled) of the kernel a pass descriptor launches."""
    lg = int(math.log2(p["N"]))
    tin, tout = str(p["in_tile_fast"]).lower(), str(p["out_tile_fast"]).lower()
    if p["mfma"] != "none":
        return "k_pass_mfma<%d, %d>" % (lg, 1 if p["mfma"] == "split_bf16" else 2)
    if p["kernel_mode"] == 3:
        return "k_pass_pair<%d, %s, %s>" % (lg, tin, tout)
    return "k_pass<float, %d, %d, %s, %s>" % (lg, p["kernel_mode"], tin, tout)


def level_times_in_chain(plan, x, out, reps, torch):
    """Average duration (ms) of each level launch run in sequence, level l
    reading what level l - 1 wrote, with events between the launches."""
    levels = plan.num_levels
    bufs = [x] + [torch.empty_like(x) for _ in range(min(levels - 1, 2))]
    chain = []
    for lvl in range(levels):
        src = bufs[0] if lvl == 0 else bufs[1 + (lvl - 1) % 2]
        dst = out if lvl + 1 == levels else bufs[1 + lvl % 2]
        chain.append((lvl, src, dst))
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(levels + 1)] for _ in range(reps)]
    for lvl, src, dst in chain:
        plan.run_level(lvl, src, dst)
    for r in range(reps):
        ev[r][0].record()
        for lvl, src, dst in chain:
            plan.run_level(lvl, src, dst)
            ev[r][lvl + 1].record()
    torch.cuda.synchronize()
    return [sum(ev[r][lvl].elapsed_time(ev[r][lvl + 1]) for r in range(reps)) / reps for lvl in range(levels)]


def rel_err(got, want, np):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run a plain device copy of the same buffer (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(a sharded transform would need an all-to-all exchange between GPUs).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0803_2386_amd import fft as mfft
    from paper_0803_2386_amd import inputs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n, batch, lift = 1 << 24, 1, [4096, 4096]
    x_np = inputs.uniform_complex(n, seed=args.seed, dtype=np.complex64)
    x = torch.from_numpy(x_np).to(dev)
    out = torch.empty_like(x)
    plan = mfft.Plan(n, batch, lift, dtype=torch.complex64)
    print(f"[bench] workload c64 n=2^24 lift {lift}; warmup {args.warmup}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        plan.forward(x, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.forward(x, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = gflops(n, batch, ms_per_step / 1e3)
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step, {value:.1f} GFLOP/s",
          file=sys.stderr, flush=True)

    if args.copy_ref:
        ref = torch.empty_like(x)
        copy_ms = time_events(lambda: ref.copy_(x), args.steps, torch)
        print(f"[bench] reference copy of {8 * n} B: {copy_ms:.4f} ms", file=sys.stderr, flush=True)

    # Per-level kernel durations, each level in its place in the chain
    # x -> workspace -> ... -> out (so the cache state matches the full
    # transform), timed by HIP events on the launch stream.
    levels = plan.num_levels
    level_ms = level_times_in_chain(plan, x, out, args.steps, torch)
    step_event_ms = time_events(lambda: plan.forward(x, out=out), args.steps, torch)
    dom = int(np.argmax(level_ms))
    bytes_per_launch = 2 * 8 * n * batch  # read + write every element once
    achieved = bytes_per_launch / (level_ms[dom] * 1e-3) / 1e9
    desc = plan.describe()
    kernel_names = [kernel_name(p) for p in desc["passes"]]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": kernel_names[dom], "level": dom,
                "level_ms": [round(v, 5) for v in level_ms],
                "algorithmic_bytes_per_launch": bytes_per_launch}

    result = {"metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
              "data": "synthetic", "config": {"workload": "c64 1-D FFT n=2^24, lift <4096 4096>",
                                              "n": n, "batch": batch, "lift": lift},
              "roofline": roofline,
              "hbm_gbs_step": round(2 * bytes_per_launch / (ms_per_step * 1e-3) / 1e9, 1),
              "event_ms_per_step": round(step_event_ms, 5)}

    if not args.no_parity or not args.no_cpu_baseline:
        import oracle
        y = out.cpu().numpy().astype(np.complex128)
        xin = x_np.astype(np.complex128)
        t2 = time.perf_counter()
        want = oracle.fft(xin)
        t3 = time.perf_counter()
        err = rel_err(y, want, np)
        result["error_vs_fp64_oracle"] = {"rel_l2": err, "tolerance": 2e-6 * 24, "pass": err <= 2e-6 * 24}
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = {"value": round(gflops(n, 1, t3 - t2), 3), "unit": "GFLOP/s", "cores": 1,
                                      "kind": "oracle",
                                      "sample": "one full n=2^24 transform of the same input (FP64 Van Loan "
                                                "radix-2, single thread), %.2f s" % (t3 - t2)}

    if not args.no_extras:
        result["extras"] = extras(args, torch, np, mfft, inputs)

    print(json.dumps(result), flush=True)


def extras(args, torch, np, mfft, inputs):
    """Other workloads, timed the same way (context for the headline line)."""
    ex = {}
    dev = torch.device("cuda", 0)
    reps = max(5, args.steps // 2)
    # Uneven batch: one persistent launch vs one plain launch per size.
    sizes = [int(s) for s in inputs.uneven_sizes(8192, 6, 14, seed=args.seed)]
    total = sum(sizes)
    flops = sum(5.0 * s * math.log2(s) for s in sizes)
    xb = inputs.device_uniform_complex(total, args.seed, torch.complex64, dev)
    ob = torch.empty_like(xb)
    rec = {"transforms": len(sizes), "elements": total}
    for name, kw in (("persistent", {}), ("per_size", {"per_size": True}),
                     ("persistent_graph", {"graph": True})):
        p = mfft.BatchedPlan(sizes, **kw)
        for _ in range(3):
            p.forward(xb, out=ob)
        ms = time_events(lambda: p.forward(xb, out=ob), reps, torch)
        rec[name] = {"ms": round(ms, 5), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
                     "hbm_gbs": round(16 * total / (ms * 1e-3) / 1e9, 1)}
        p.close()
    ex["uneven_batch_8192_2^6..2^14"] = rec
    # Differentiable workload: forward + adjoint, 256 x 2^16, lift <256 256>.
    n, B = 1 << 16, 256
    p = mfft.Plan(n, B, [256, 256])
    xa = inputs.device_uniform_complex(n * B, args.seed + 1, torch.complex64, dev)
    ya = torch.empty_like(xa)
    za = torch.empty_like(xa)

    def fwd_adj():
        p.forward(xa, out=ya)
        p.adjoint(ya, out=za)
    fwd_adj()
    ms = time_events(fwd_adj, reps, torch)
    ex["fwd_adj_b256_2^16"] = {"ms": round(ms, 5), "gflops": round(2 * gflops(n, B, ms * 1e-3), 1),
                               "hbm_gbs": round(4 * 16 * n * B / (ms * 1e-3) / 1e9, 1)}
    p.close()
    # Latency of the complex128 n = 2^10 transform (single workgroup).
    p = mfft.Plan(1 << 10, 1, None, dtype=torch.complex128)
    xc = inputs.device_uniform_complex(1 << 10, args.seed + 2, torch.complex128, dev)
    yc = torch.empty_like(xc)
    for _ in range(10):
        p.forward(xc, out=yc)
    ex["c128_n1024_us_per_call"] = round(1e3 * time_events(lambda: p.forward(xc, out=yc), 200, torch), 3)
    p.close()
    return ex


if __name__ == "__main__":
    main()
