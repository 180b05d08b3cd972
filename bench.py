#!/usr/bin/env python3
"""Benchmark of the MI355X dimension-lifted FFT.

Headline workload: one complex64 transform of n = 2^24 points through the lift
<4096 4096> (two HBM passes: column FFTs with the inter-level twiddle and the
reshape-transpose folded into the store, then row FFTs with the final
transpose folded into the store).  A step is one full transform; inputs are
resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-extras]
                    [--extras uneven,fwd_adj,split_mfma,tuned,hypercube,defaults,c128]

Throughput is 5 n log2(n) / t (GFLOP/s).  The roofline block reports the
dominant kernel (the slower of the two level launches, each timed in its place
in the x -> workspace -> out chain with HIP events on the launch stream)
against the 8 TB/s HBM peak with its algorithmic bytes (read + write of every
element once per launch); `traffic` is the HBM bytes per launch that the
rocprofv3 FETCH_SIZE / WRITE_SIZE counters measured for the same kernel
source (profiles/traffic.json), or null when the kernel source has changed
since.  The extras time the other workloads (uneven batch, forward+adjoint,
split-precision matrix-core levels, the tuned lift, the default lifts against
the former near-equal ones, complex128 latency); the
CPU leg times the FP64 oracle and states the error of every result against it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FFT GFLOP/s (5n·log2n/t) & HBM GB/s vs peak, batched/MFMA vs plain, at stated error"
HBM_PEAK_GBS = 8000.0
MFMA_DENSE_PEAK_TFLOPS = 2500.0  # bf16 / fp16 dense matrix-core peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


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


def step_percentiles(fn, reps, torch, np):
    """p10 / p50 / p90 of single-step durations (ms), one event pair a step."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return [round(float(np.percentile(t, q)), 5) for q in (10, 50, 90)]


_sweep = {}


def cold_step_ms(fn, reps, torch, np):
    """Median single-step duration (ms) with the L2 and the 256 MB Infinity
    Cache evicted before every step by a read-only sweep of 1 GiB (a read
    leaves no dirty lines to be written back inside the timed step)."""
    if "buf" not in _sweep:
        _sweep["buf"] = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    buf = _sweep["buf"]
    t = []
    for _ in range(reps):
        _ = buf.sum()  # the read-only sweep
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        t.append(a.elapsed_time(b))
    return float(np.median(t))


def chained_copy_gbs(x, reps, torch):
    """Read+write bandwidth (GB/s) of plain device copies of x's size chained
    through three buffers (each copy reads what the previous one wrote, a
    working set larger than the Infinity Cache, like the transform's chain).
    The best of torch's device-to-device copy and an elementwise pass over a
    float32 view (multiply by one, which streams 16 bytes a lane and runs
    about 40% faster than the copy on MI355X)."""
    bufs = [x.clone(), torch.empty_like(x), torch.empty_like(x)]
    flt = [b.view(torch.float32) for b in bufs]
    ops = (lambda i: bufs[(i + 1) % 3].copy_(bufs[i % 3]),
           lambda i: torch.mul(flt[i % 3], 1.0, out=flt[(i + 1) % 3]))
    best = 0.0
    for op in ops:
        for i in range(3):
            op(i)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for i in range(reps):
            op(i)
        e.record()
        e.synchronize()
        ms = s.elapsed_time(e) / reps
        best = max(best, 2 * x.numel() * x.element_size() / (ms * 1e-3) / 1e9)
    return best


def kernel_name(p):
    """Device symbol (demangled, without the direction argument) of the
    kernel a pass descriptor launches."""
    lg = int(math.log2(p["N"]))
    tin, tout = str(p["in_tile_fast"]).lower(), str(p["out_tile_fast"]).lower()
    if p["mfma"] != "none":
        prec = 1 if p["mfma"] == "split_bf16" else 2
        if p["kernel_mode"] == 3:
            return "k_pass_mfma_pair<%d, %d, %s, %s>" % (lg, prec, tin, tout)
        return "k_pass_mfma<%d, %d>" % (lg, prec)
    if p["kernel_mode"] == 3:
        return "k_pass_pair<%d, %s, %s>" % (lg, tin, tout)
    if p["kernel_mode"] == 4:
        return "k_small<%d>" % lg
    return "k_pass<float, %d, %d, %s, %s, %d>" % (lg, p["kernel_mode"], tin, tout, p["lg_radix"])


def sources_digest(paths):
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter runs of `kernel`, if
    its sources are unchanged since they were taken, else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            entry = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not entry:
        return None
    try:
        if sources_digest(entry["sources"]) != entry["sources_sha256"]:
            return None
    except OSError:
        return None
    return int(entry["hbm_bytes_per_launch"])


def rel_err_rows(got, want, np):
    got = np.atleast_2d(got)
    want = np.atleast_2d(want)
    return float((np.linalg.norm(got - want, axis=-1) / np.linalg.norm(want, axis=-1)).max())


def headline(args, torch, np, mfft, inputs):
    dev = torch.device("cuda", 0)
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

    level_ms = level_times_in_chain(plan, x, out, args.steps, torch)
    step_event_ms = time_events(lambda: plan.forward(x, out=out), args.steps, torch)
    per_step = step_percentiles(lambda: plan.forward(x, out=out), args.steps, torch, np)
    cold = cold_step_ms(lambda: plan.forward(x, out=out), max(5, args.steps // 5), torch, np)
    copy_gbs = chained_copy_gbs(x, args.steps, torch)
    dom = int(np.argmax(level_ms))
    bytes_per_launch = 2 * 8 * n * batch  # read + write every element once
    achieved = bytes_per_launch / (level_ms[dom] * 1e-3) / 1e9
    desc = plan.describe()
    names = [kernel_name(p) for p in desc["passes"]]
    traffic = measured_traffic(names[dom])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": names[dom], "level": dom, "level_kernels": names,
                "level_ms": [round(v, 5) for v in level_ms],
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "measured_copy_gbs": round(copy_gbs, 1),
                "frac_of_measured_copy": round(achieved / copy_gbs, 4)}
    result = {"metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
              "data": "synthetic", "config": {"workload": "c64 1-D FFT n=2^24, lift <4096 4096>",
                                              "n": n, "batch": batch, "lift": lift},
              "roofline": roofline,
              "hbm_gbs_step": round(2 * bytes_per_launch / (ms_per_step * 1e-3) / 1e9, 1),
              "event_ms_per_step": round(step_event_ms, 5),
              "event_ms_per_step_p10_p50_p90": per_step,
              "cold_ms_per_step_median": round(cold, 5)}
    sample = {"x": x_np, "y": out.cpu().numpy()}
    plan.close()
    return result, sample


def extras(args, torch, np, mfft, inputs):
    """Other workloads, timed the same way (context for the headline line).
    Returns the records and, per record, host copies of a few transforms for
    the error statement of the CPU leg."""
    from paper_0803_2386_amd import tune
    ex, samples = {}, {}
    dev = torch.device("cuda", 0)
    reps = max(5, args.steps // 2)
    chosen = set(args.extras.split(","))

    def want(name):
        return "all" in chosen or name in chosen

    if want("uneven"):
        # Uneven batch: one fused launch (default grid: one workgroup per task;
        # resident grid: persistent, two workgroups per CU; the autotuner's
        # grid, also replayed from a HIP graph) vs one plain launch per size.
        sizes = [int(s) for s in inputs.uneven_sizes(8192, 6, 14, seed=args.seed)]
        total = sum(sizes)
        offs = np.concatenate([[0], np.cumsum(sizes)])
        flops = sum(5.0 * s * math.log2(s) for s in sizes)
        xb = inputs.device_uniform_complex(total, args.seed, torch.complex64, dev)
        ob = torch.empty_like(xb)
        rec = {"transforms": len(sizes), "elements": total}
        pick = [0, int(np.argmax(sizes)), len(sizes) - 1]
        probe = mfft.BatchedPlan(sizes, host_only=True)
        d = probe.describe()
        probe.close()
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        resident = cus * max(1, (160 * 1024) // d["lds_bytes"])
        rec["tasks"] = d["tasks"]

        def entry(ms, p):
            return {"ms": round(ms, 5), "grid": p.describe()["persistent_blocks"], "task_lg": p.describe()["task_lg"],
                    "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
                    "hbm_gbs": round(16 * total / (ms * 1e-3) / 1e9, 1),
                    "frac_hbm_peak": round(16 * total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        best = tune.tune_batched(sizes, grids=(0, resident // 2, resident, 2 * resident, 3 * resident,
                                               4 * resident))
        tuned = best["tuning"] or {}
        for name, kw in (("one_launch", {}), ("resident_grid", {"tuning": {"persistent_blocks": resident}}),
                         ("per_size", {"per_size": True}), ("tuned", {"tuning": tuned}),
                         ("tuned_graph", {"tuning": tuned, "graph": True})):
            p = mfft.BatchedPlan(sizes, **kw)
            for _ in range(3):
                p.forward(xb, out=ob)
            ms = time_events(lambda: p.forward(xb, out=ob), reps, torch)
            rec[name] = entry(ms, p)
            if name in ("tuned", "tuned_graph", "per_size"):
                rec[name]["cold_ms_median"] = round(cold_step_ms(lambda: p.forward(xb, out=ob), 7, torch, np), 5)
            if name == "tuned_graph":
                xs, ys = xb.cpu().numpy(), ob.cpu().numpy()
                samples["uneven_batch"] = [(xs[offs[i]:offs[i + 1]], ys[offs[i]:offs[i + 1]], 2e-6 * math.log2(sizes[i]))
                                           for i in pick]
                # The whole batch, for the oracle on all host cores and the
                # error of every transform.
                samples["uneven_batch_all"] = {"x": xs, "y": ys, "sizes": sizes, "offsets": offs}
            p.close()
        rec["tuned"]["tuner_ms"] = round(best["ms"], 5)
        # The tuned launch recorded into a caller's HIP graph (torch capture
        # on a side stream, 10 launches a graph, each graph replayed): a
        # serving loop's form, free of the per-launch cost of a one-node graph.
        p = mfft.BatchedPlan(sizes, tuning=tuned)
        cg = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            p.forward(xb, out=ob)
            with torch.cuda.graph(cg, stream=side):
                for _ in range(10):
                    p.forward(xb, out=ob)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        cg.replay()
        ms = time_events(cg.replay, 20, torch) / 10
        rec["tuned_caller_graph"] = entry(ms, p)
        rec["tuned_caller_graph"]["launches_per_graph"] = 10
        p.close()
        del cg
        # one plain launch per transform (8192 launches, timed once)
        plans = {n: mfft.Plan(n, 1, None) for n in set(sizes)}
        views = [xb[offs[i]:offs[i + 1]] for i in range(len(sizes))]
        outs = [ob[offs[i]:offs[i + 1]] for i in range(len(sizes))]

        def singles():
            for i, s_ in enumerate(sizes):
                plans[s_].forward(views[i], out=outs[i])
        singles()
        ms = time_events(singles, 1, torch)
        rec["single_launches"] = {"ms": round(ms, 4), "launches": len(sizes),
                                  "hbm_gbs": round(16 * total / (ms * 1e-3) / 1e9, 1)}
        for q in plans.values():
            q.close()
        rec["one_launch_vs_per_size"] = round(rec["per_size"]["ms"] / rec["one_launch"]["ms"], 3)
        rec["tuned_graph_vs_per_size"] = round(rec["per_size"]["ms"] / rec["tuned_graph"]["ms"], 3)
        rec["tuned_caller_graph_vs_per_size"] = round(rec["per_size"]["ms"] / rec["tuned_caller_graph"]["ms"], 3)
        rec["one_launch_vs_single_launches"] = round(rec["single_launches"]["ms"] / rec["one_launch"]["ms"], 1)
        ex["uneven_batch_8192_2^6..2^14"] = rec
        del xb, ob

    if want("fwd_adj"):
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
        lv = level_times_in_chain(p, xa, ya, reps, torch)
        d = p.describe()
        gbs = 4 * 16 * n * B / (ms * 1e-3) / 1e9
        ex["fwd_adj_b256_2^16"] = {"ms": round(ms, 5), "gflops": round(2 * gflops(n, B, ms * 1e-3), 1),
                                   "hbm_gbs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                                   "cold_ms_median": round(cold_step_ms(fwd_adj, 7, torch, np), 5),
                                   "forward_level_ms": [round(v, 5) for v in lv],
                                   "forward_level_frac_hbm_peak": [
                                       round(16 * n * B / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) for v in lv],
                                   "kernels": [kernel_name(q) for q in d["passes"]]}
        p.close()
        del xa, ya, za

    if want("split_mfma"):
        # Split-precision matrix-core levels vs FP32, 256 x 2^20, under both
        # two-level lifts: <256 4096> (4096-point columns first, 64-byte runs)
        # and <4096 256> (256-point columns first, 1 KB runs on both sides of
        # each level).  Each figure is the median of three timed trials.
        n, B = 1 << 20, 256
        xm = inputs.device_uniform_complex(n * B, args.seed + 3, torch.complex64, dev)
        ym = torch.empty_like(xm)
        rows = [0, B - 1]
        xs = xm.view(B, n)[rows].cpu().numpy()
        rec = {}
        best = {}
        for lift in ([256, 4096], [4096, 256]):
            lk = "lift_%dx%d" % tuple(lift)
            rec[lk] = {}
            for prec in ("native", "split_bf16", "split_fp16"):
                p = mfft.Plan(n, B, lift, prec=prec)
                d = p.describe()
                p.forward(xm, out=ym)
                mreps = max(3, reps // 2)
                ms = sorted(time_events(lambda: p.forward(xm, out=ym), mreps, torch) for _ in range(3))[1]
                lv = level_times_in_chain(p, xm, ym, mreps, torch)
                levels = len(d["passes"])
                r = {"ms": round(ms, 4), "gflops": round(gflops(n, B, ms * 1e-3), 1),
                     "hbm_gbs": round(2 * levels * 8 * n * B / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm_peak": round(2 * levels * 8 * n * B / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "level_ms": [round(v, 4) for v in lv],
                     "level_frac_hbm_peak": [round(16 * n * B / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) for v in lv],
                     "kernels": [kernel_name(q) for q in d["passes"]]}
                stages = sum(int(math.log2(q["N"])) // 4 for q in d["passes"] if q["mfma"] != "none")
                if stages:
                    # 6 MFMA 16x16x32 per 16 butterflies of a stage: 384 flops a point.
                    tf = 384.0 * stages * n * B / (ms * 1e-3) / 1e12
                    r["mfma_stages"] = stages
                    r["mfma_tflops"] = round(tf, 1)
                    r["mfma_frac_dense_peak"] = round(tf / MFMA_DENSE_PEAK_TFLOPS, 4)
                bound = 2e-6 * math.log2(n) if prec != "split_bf16" else 2.0 * stages * 2.0 ** -16
                samples["mfma_%s_%s" % (prec, lk)] = [(xs[i], ym.view(B, n)[rows[i]].cpu().numpy(), bound)
                                                      for i in range(len(rows))]
                rec[lk][prec] = r
                if prec not in best or ms < best[prec][0]:
                    best[prec] = (ms, lk)
                p.close()
        rec["best"] = {k: {"ms": round(v[0], 4), "lift": v[1]} for k, v in best.items()}
        rec["split_over_native_at_best_lifts"] = {k: round(best[k][0] / best["native"][0], 4)
                                                  for k in ("split_bf16", "split_fp16")}
        ex["split_mfma_b256_2^20"] = rec
        del xm, ym

    if want("tuned"):
        # The autotuner's lift and tile widths for n = 2^24 (up to three levels).
        with tempfile.TemporaryDirectory() as td:
            os.environ["MOA_FFT_TUNE_CACHE"] = os.path.join(td, "tune.json")
            best = tune.tune(1 << 24, 1, max_levels=3, reps=5, use_cache=False)
        # The pick, timed like the headline (warm-up, then --steps calls).
        n = 1 << 24
        p = mfft.Plan(n, 1, best["lift"], tuning=best["tuning"])
        xt = inputs.device_uniform_complex(n, args.seed, torch.complex64, dev)
        yt = torch.empty_like(xt)
        for _ in range(args.warmup):
            p.forward(xt, out=yt)
        ms = time_events(lambda: p.forward(xt, out=yt), args.steps, torch)
        p.close()
        ex["tuned_2^24"] = {"lift": best["lift"], "tuning": best["tuning"], "ms": round(ms, 5),
                            "gflops": round(gflops(n, 1, ms * 1e-3), 1), "tuner_ms": round(best["ms"], 5),
                            "candidates": best["tried"]}
        del xt, yt
        # The register radix as a tuning dimension (Ch. 1, "Performance of the
        # General-Radix FFT"): 1024 transforms of 2^14 points, the tuner's
        # schedule against the fixed radix-16 one, timed the same way.
        n, B = 1 << 14, 1024
        with tempfile.TemporaryDirectory() as td:
            os.environ["MOA_FFT_TUNE_CACHE"] = os.path.join(td, "tune.json")
            best = tune.tune(n, B, max_levels=1, reps=10, use_cache=False)
        xr = inputs.device_uniform_complex(n * B, args.seed + 6, torch.complex64, dev)
        yr = torch.empty_like(xr)
        rec = {"n": n, "batch": B}
        for name, lift, tuning in (("radix16", None, None), ("tuned", best["lift"], best["tuning"])):
            p = mfft.Plan(n, B, lift, tuning=tuning)
            for _ in range(3):
                p.forward(xr, out=yr)
            ms = time_events(lambda: p.forward(xr, out=yr), reps, torch)
            rec[name] = {"ms": round(ms, 5), "gflops": round(gflops(n, B, ms * 1e-3), 1),
                         "frac_hbm_peak": round(16 * n * B / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "stage_lg_radices": [q["stage_lg_radices"] for q in p.describe()["passes"]],
                         "tuning": tuning}
            samples.setdefault("radix_" + name, []).append(
                (xr.view(B, n)[0].cpu().numpy(), yr.view(B, n)[0].cpu().numpy(), 2e-6 * 14))
            p.close()
        rec["tuned_vs_radix16"] = round(rec["radix16"]["ms"] / rec["tuned"]["ms"], 3)
        ex["radix_tuned_b1024_2^14"] = rec
        del xr, yr

    if want("nd"):
        # Multi-dimensional transforms of 2^24 complex64 points: 4096 x 4096
        # (two axis launches) and 256^3 (three), both through the level kernels.
        for dims in ((4096, 4096), (256, 256, 256)):
            p = mfft.NDPlan(dims, 1)
            N = 1 << 24
            xn = inputs.device_uniform_complex(N, args.seed + 5, torch.complex64, dev)
            yn = torch.empty_like(xn)
            for _ in range(3):
                p.forward(xn, out=yn)
            ms = time_events(lambda: p.forward(xn, out=yn), reps, torch)
            lv = level_times_in_chain(p, xn, yn, reps, torch)
            d = p.describe()
            dom = int(np.argmax(lv))
            ach = 16 * N / (lv[dom] * 1e-3) / 1e9
            ex["nd_" + "x".join(str(v) for v in dims)] = {
                "ms": round(ms, 5), "gflops": round(gflops(N, 1, ms * 1e-3), 1),
                "hbm_gbs": round(len(lv) * 16 * N / (ms * 1e-3) / 1e9, 1),
                "cold_ms_median": round(cold_step_ms(lambda: p.forward(xn, out=yn), 7, torch, np), 5),
                "level_ms": [round(v, 5) for v in lv], "kernels": [kernel_name(q) for q in d["passes"]],
                "roofline": {"kernel": kernel_name(d["passes"][dom]), "achieved_gbs": round(ach, 1),
                             "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": 16 * N}}
            xs = xn.cpu().numpy().reshape(dims)
            samples["nd_" + "x".join(str(v) for v in dims)] = {"x": xs, "y": yn.cpu().numpy().reshape(dims)}
            p.close()
            del xn, yn

    if want("hypercube"):
        # Ch. 6 workload: a 13-qubit complex64 density matrix (2^26 elements,
        # 512 MiB).  The hyper-cube transpose to its block-diagonal view for
        # two gated qubits (pure movement: read + write of every element), and
        # the in-place gates rho <- G rho G^H by direct indexing (the same
        # bytes), against a plain device copy of the same buffer.
        from paper_0803_2386_amd import hypercube as hcube
        nq = 13
        N = 1 << nq
        rho = inputs.device_uniform_complex(N * N, args.seed + 4, torch.complex64, dev).view(N, N)
        tgt = torch.empty_like(rho)
        nbytes = 2 * 8 * N * N
        rec = {"qubits": nq, "elements": N * N, "bytes_per_launch": nbytes}
        hreps = max(5, reps // 2)

        def rate(ms):
            gbs = nbytes / (ms * 1e-3) / 1e9
            return {"ms": round(ms, 5), "hbm_gbs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        tgt.copy_(rho)
        rec["device_copy"] = rate(time_events(lambda: tgt.copy_(rho), hreps, torch))
        for gated in ([0, 2], [11, 12]):
            t = hcube.block_diagonal_transpose_vector(nq, gated)
            hcube.hypercube_transpose(rho.view(-1), t, out=tgt.view(-1))
            r = rate(time_events(lambda: hcube.hypercube_transpose(rho.view(-1), t, out=tgt.view(-1)), hreps, torch))
            r["cold_ms_median"] = round(cold_step_ms(
                lambda: hcube.hypercube_transpose(rho.view(-1), t, out=tgt.view(-1)), 5, torch, np), 5)
            r["t"] = t
            rec["transpose_gated_%d_%d" % tuple(gated)] = r
        rng = np.random.default_rng(args.seed)
        for gated in ([0, 2], [11, 12], [0, 1, 2, 3]):
            k = 1 << len(gated)
            z = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
            U = torch.from_numpy(np.linalg.qr(z)[0].astype(np.complex64)).to(dev)
            hcube.density_gate(tgt, U, gated)
            r = rate(time_events(lambda: hcube.density_gate(tgt, U, gated), hreps, torch))
            r["cold_ms_median"] = round(cold_step_ms(lambda: hcube.density_gate(tgt, U, gated), 5, torch, np), 5)
            rec["gate_" + "_".join(str(b) for b in gated)] = r
        ex["hypercube_13_qubits_c64"] = rec
        del rho, tgt

    if want("defaults"):
        # The planner's default lifts where they depart from the fewest levels
        # of near-equal size, each against that former default, whole
        # transforms timed alike (median of three trials).
        rec = {}
        for n, B, dt, former in ((1 << 20, 256, torch.complex64, [1024, 1024]),
                                 (1 << 28, 1, torch.complex64, [16384, 16384]),
                                 (1 << 25, 1, torch.complex128, [8192, 4096])):
            xd = inputs.device_uniform_complex(n * B, args.seed + 9, dt, dev)
            yd = torch.empty_like(xd)
            r = {}
            for name, lift in (("default", None), ("near_equal", former)):
                p = mfft.Plan(n, B, lift, dtype=dt)
                p.forward(xd, out=yd)
                ms = sorted(time_events(lambda: p.forward(xd, out=yd), max(3, reps // 2), torch)
                            for _ in range(3))[1]
                r[name] = {"lift": p.describe()["lift"], "ms": round(ms, 4)}
                p.close()
            r["speedup"] = round(r["near_equal"]["ms"] / r["default"]["ms"], 3)
            rec["%s_2^%d_x%d" % ("c64" if dt == torch.complex64 else "c128", n.bit_length() - 1, B)] = r
            del xd, yd
        ex["default_lifts"] = rec

    if want("c128"):
        # Latency of the complex128 n = 2^10 transform (single workgroup).
        p = mfft.Plan(1 << 10, 1, None, dtype=torch.complex128)
        xc = inputs.device_uniform_complex(1 << 10, args.seed + 2, torch.complex128, dev)
        yc = torch.empty_like(xc)
        for _ in range(10):
            p.forward(xc, out=yc)
        ex["c128_n1024_us_per_call"] = round(1e3 * time_events(lambda: p.forward(xc, out=yc), 200, torch), 3)
        samples["c128_n1024"] = [(xc.cpu().numpy(), yc.cpu().numpy(), 1e-13)]
        ex["c128_n1024_replay"] = c128_replay_us(p, xc, torch, np)
        p.close()
    return ex, samples


def c128_replay_us(p, x, torch, np, calls=100, replays=20):
    """Per-call time of the single-workgroup transform without host launch
    cost: `calls` back-to-back transforms recorded into one HIP graph (torch
    capture of the library's launches on the capture stream), replayed
    `replays` times, each replay timed with HIP events.  Returns the median,
    p10 and p90 in microseconds per call, or the error text if the capture
    fails (the eager figure stands regardless)."""
    try:
        out = torch.empty_like(x)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(calls):
                p.forward(x, out=out)
        g.replay()
        torch.cuda.synchronize()
        ms = []
        for _ in range(replays):
            s = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            s.record()
            g.replay()
            e.record()
            e.synchronize()
            ms.append(s.elapsed_time(e))
        del g
        us = 1e3 * np.asarray(ms) / calls
        return {"calls_per_replay": calls, "replays": replays, "median_us": round(float(np.median(us)), 3),
                "p10_us": round(float(np.percentile(us, 10)), 3), "p90_us": round(float(np.percentile(us, 90)), 3)}
    except Exception as exc:  # noqa: BLE001 -- reported, not fatal
        return {"error": f"{type(exc).__name__}: {exc}"}


def host_info():
    """CPU model and core counts of the host the oracle ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def oracle_uneven_leg(full, ex, np):
    """The FP64 oracle over the whole uneven batch on OpenMP threads (the
    usable cores, at most 16), timed on a buffer already in host memory, and
    the error of every GPU transform of the batch against it."""
    import oracle
    sizes, offs = full["sizes"], full["offsets"]
    flops = sum(5.0 * s * math.log2(s) for s in sizes)
    threads = max(1, min(16, host_info()["usable_cores"] or 1))
    want = full["x"].astype(np.complex128)
    t0 = time.perf_counter()
    oracle.fft_packed_inplace(want, sizes, threads=threads)
    sec = time.perf_counter() - t0
    y = full["y"].astype(np.complex128)
    err2 = np.add.reduceat(np.abs(y - want) ** 2, offs[:-1])
    ref2 = np.add.reduceat(np.abs(want) ** 2, offs[:-1])
    rel = np.sqrt(err2 / np.maximum(ref2, 1e-300))
    tol = 2e-6 * np.log2(np.asarray(sizes, np.float64))
    if ex is not None:
        ex.setdefault("error_vs_fp64_oracle_all", {})["uneven_batch"] = {
            "rel_l2_max": float(rel.max()), "max_ratio_to_tolerance": float((rel / tol).max()),
            "transforms": len(sizes), "pass": bool((rel <= tol).all())}
    return {"value": round(flops / sec / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "seconds": round(sec, 3),
            "sample": "the whole uneven batch (%d transforms of 2^6..2^14, %d points), FP64 recursive radix-2 oracle, "
                      "OpenMP over the transforms, one run" % (len(sizes), int(offs[-1]))}


def cpu_baseline_leg(args, np, result, sample, samples):
    """Time the FP64 oracle on the host (full headline transforms repeated to
    about 10 s, one thread) and state the error of every GPU result against
    it."""
    import oracle
    xin = sample["x"].astype(np.complex128)
    # Repeat the full transform until about 10 s of CPU work (at most 12 runs).
    runs, spent = 0, 0.0
    while runs < 12 and (runs == 0 or spent < 10.0):
        t0 = time.perf_counter()
        want = oracle.fft(xin)
        spent += time.perf_counter() - t0
        runs += 1
    err = rel_err_rows(sample["y"].astype(np.complex128), want, np)
    n = xin.size
    per = spent / runs
    result["error_vs_fp64_oracle"] = {"rel_l2": err, "tolerance": 2e-6 * math.log2(n),
                                      "pass": err <= 2e-6 * math.log2(n)}
    result["cpu_baseline"] = {"value": round(gflops(n, 1, per), 3), "unit": "GFLOP/s", "cores": 1,
                              "kind": "oracle",
                              "sample": "%d full n=2^%d transforms of the headline input (FP64 recursive radix-2 oracle, "
                                        "single thread), %.2f s each, %.1f s in all"
                                        % (runs, int(math.log2(n)), per, spent)}
    result["cpu_baseline"]["host"] = host_info()
    full = samples.pop("uneven_batch_all", None)
    if full is not None:
        result["cpu_baseline"]["uneven_batch"] = oracle_uneven_leg(full, result.get("extras"), np)
    ex = result.get("extras")
    if not ex:
        return
    errs = {}
    for name in [k for k in samples if k.startswith("nd_")]:
        nd = samples.pop(name)
        xs = nd["x"].astype(np.complex128)
        want = oracle.fftn(xs, xs.ndim)
        e = float(np.linalg.norm(nd["y"].astype(np.complex128) - want) / np.linalg.norm(want))
        tol = 2e-6 * math.log2(xs.size)
        errs[name] = {"rel_l2_max": e, "transforms": 1, "tolerance": tol, "pass": e <= tol}
    for name, cases in samples.items():
        worst, ok = 0.0, True
        for xs, ys, tol in cases:
            e = rel_err_rows(ys.astype(np.complex128), oracle.fft(xs.astype(np.complex128)), np)
            worst = max(worst, e)
            ok = ok and e <= tol
        errs[name] = {"rel_l2_max": worst, "transforms": len(cases), "tolerance": cases[0][2], "pass": ok}
    ex["error_vs_fp64_oracle"] = errs


def profile_run(args, torch, np, mfft, inputs):
    """Launch one workload's kernels W + K times and nothing else (no tuner,
    no oracle), then one 128 MiB device copy, so a rocprofv3 kernel trace or
    counter run sees exactly those dispatches."""
    dev = torch.device("cuda", 0)
    w = args.profile
    free = []
    if w == "headline":
        n = 1 << 24
        x = inputs.device_uniform_complex(n, args.seed, torch.complex64, dev)
        y = torch.empty_like(x)
        p = mfft.Plan(n, 1, [4096, 4096])
        fn = lambda: p.forward(x, out=y)  # noqa: E731
    elif w == "uneven":
        sizes = [int(s) for s in inputs.uneven_sizes(8192, 6, 14, seed=args.seed)]
        x = inputs.device_uniform_complex(sum(sizes), args.seed, torch.complex64, dev)
        y = torch.empty_like(x)
        p = mfft.BatchedPlan(sizes, tuning={"persistent_blocks": args.grid})
        fn = lambda: p.forward(x, out=y)  # noqa: E731
    elif w == "fwd_adj":
        n, B = 1 << 16, 256
        x = inputs.device_uniform_complex(n * B, args.seed + 1, torch.complex64, dev)
        y, z = torch.empty_like(x), torch.empty_like(x)
        p = mfft.Plan(n, B, [256, 256])
        free.append(z)

        def fn():
            p.forward(x, out=y)
            p.adjoint(y, out=z)
    elif w.startswith("split_"):
        # split_<prec>[_4096x256]: 256 x 2^20 under lift <256 4096>, or <4096 256>
        n, B = 1 << 20, 256
        x = inputs.device_uniform_complex(n * B, args.seed + 3, torch.complex64, dev)
        y = torch.empty_like(x)
        prec = w[:-len("_4096x256")] if w.endswith("_4096x256") else w
        lift = [4096, 256] if w.endswith("_4096x256") else [256, 4096]
        p = mfft.Plan(n, B, lift, prec="native" if prec == "split_native" else prec)
        fn = lambda: p.forward(x, out=y)  # noqa: E731
    elif w == "default_2p28":
        # one complex64 transform of 2^28 points under its default lift
        n = 1 << 28
        x = inputs.device_uniform_complex(n, args.seed + 9, torch.complex64, dev)
        y = torch.empty_like(x)
        p = mfft.Plan(n, 1, None)
        fn = lambda: p.forward(x, out=y)  # noqa: E731
    elif w in ("nd2", "nd3"):
        dims = (4096, 4096) if w == "nd2" else (256, 256, 256)
        x = inputs.device_uniform_complex(1 << 24, args.seed + 5, torch.complex64, dev)
        y = torch.empty_like(x)
        p = mfft.NDPlan(dims, 1)
        fn = lambda: p.forward(x, out=y)  # noqa: E731
    elif w in ("hc_transpose", "hc_gate", "hc_gate4"):
        from paper_0803_2386_amd import hypercube as hcube
        N = 1 << 13
        x = inputs.device_uniform_complex(N * N, args.seed + 4, torch.complex64, dev).view(N, N)
        y = torch.empty_like(x)
        p = None
        if w == "hc_transpose":
            t = hcube.block_diagonal_transpose_vector(13, [0, 2])
            fn = lambda: hcube.hypercube_transpose(x.view(-1), t, out=y.view(-1))  # noqa: E731
        elif w == "hc_gate":
            U = torch.eye(4, dtype=torch.complex64, device=dev)
            fn = lambda: hcube.density_gate(y, U, [0, 2])  # noqa: E731
        else:
            U = torch.eye(16, dtype=torch.complex64, device=dev)
            fn = lambda: hcube.density_gate(y, U, [0, 1, 2, 3])  # noqa: E731
    else:
        raise SystemExit(f"bench.py: unknown --profile workload {w!r}")
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    for _ in range(args.steps):
        fn()
    torch.cuda.synchronize()
    ref = torch.empty(1 << 24, dtype=torch.complex64, device=dev)
    src = torch.ones_like(ref)
    ref.copy_(src)
    torch.cuda.synchronize()
    if p is not None:
        p.close()
    print(f"[bench] profile {w}: {args.warmup} + {args.steps} launches, then a 128 MiB copy", file=sys.stderr,
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (and the error statement)")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="all",
                    help="comma list of extra workloads: uneven, fwd_adj, split_mfma, tuned, nd, hypercube, "
                         "defaults, c128 "
                         "(default all)")
    ap.add_argument("--profile", default=None,
                    help="kernel-only run for rocprofv3: warm-up, then --steps launches of one workload's kernels "
                         "(headline, uneven, fwd_adj, split_native, split_bf16, split_fp16 -- each of the split "
                         "ones also with the suffix _4096x256 for that lift --, nd2, nd3, hc_transpose, hc_gate, hc_gate4), "
                         "then a device copy of 128 MiB (the counters' reference); prints nothing else")
    ap.add_argument("--grid", type=int, default=1536,
                    help="--profile uneven: workgroups of the fused launch (the tuner's usual pick)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run a plain device copy of the same buffer (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the transform runs on one GPU; --gpus {args.gpus} is not supported "
              "(a sharded transform would need an all-to-all exchange between GPUs).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0803_2386_amd import fft as mfft
    from paper_0803_2386_amd import inputs

    torch.cuda.set_device(torch.device("cuda", 0))
    if args.profile:
        profile_run(args, torch, np, mfft, inputs)
        return
    result, sample = headline(args, torch, np, mfft, inputs)
    samples = {}
    if not args.no_extras:
        result["extras"], samples = extras(args, torch, np, mfft, inputs)
    if not args.no_cpu_baseline:
        cpu_baseline_leg(args, np, result, sample, samples)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
