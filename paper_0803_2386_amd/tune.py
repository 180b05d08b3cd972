"""Autotuner: picks the lift, the per-level tile widths and the per-level
register radix of a plan by timing candidates on the device, and the grid
and streaming mode of an uneven batch's fused launch.

The paper leaves the blocking size c as a run-time parameter to be chosen per
machine (Ch. 1 and Ch. 3, "Results and Discussion": the best c was found by
experiment, not from the cache size), and so is the radix of the butterflies
(Ch. 1, "Performance of the General-Radix FFT", Table 4: the best radix was
measured, not derived).  Here the candidates are lifts whose
levels each fit one workgroup, in the paper's uniform form
<2^p_max c ... c> and in balanced mixed forms, each with a few tile widths;
every candidate is planned through the C ABI, timed with HIP events, and the
fastest is cached in a JSON file keyed by device, dtype, precision, n, batch,
the search limits and a digest of the built library
(``$MOA_FFT_TUNE_CACHE``, default ``~/.cache/moa_fft_tune.json``).  Timing is
the only thing done here; all arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import itertools
import json
import os
import threading
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from . import capi

_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("MOA_FFT_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                             "moa_fft_tune.json"))


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


_lib_digest = None


def library_digest() -> str:
    """Short sha256 of the built library: a rebuilt kernel set invalidates
    the cached picks of the old one."""
    global _lib_digest
    if _lib_digest is None:
        import hashlib
        h = hashlib.sha256()
        with open(capi.LIB_PATH, "rb") as f:
            for chunk in iter(lambda: f.read(1 << 20), b""):
                h.update(chunk)
        _lib_digest = h.hexdigest()[:16]
    return _lib_digest


def _key(device_name: str, dtype_code: int, n: int, batch: int, prec: int, max_levels: int = 3,
         limit: Optional[int] = None, refine: int = 5, radix: bool = True) -> str:
    """Cache key: the problem, the search that answered it (a search cut
    short by a candidate limit is not the answer of a full one) and the
    library it timed."""
    return (f"{device_name}|{'c64' if dtype_code == capi.MOA_C64 else 'c128'}|p{prec}|n{n}|b{batch}"
            f"|L{max_levels}|lim{limit or 0}|r{refine}|rad{int(radix)}|lib{library_digest()}")


RADIX_CHOICES = (2, 3, 5)   # log2 of radix 4, 8, 32 (0 = the default radix 16)


def radix_candidates(n: int, batch: int, lift: Sequence[int], tuning: Optional[dict], dtype_code: int,
                     prec: int) -> List[dict]:
    """Tunings that change one level's register radix of (lift, tuning),
    keeping everything else; only those that plan."""
    base = dict(tuning or {})
    L = len(lift)
    cur = list(base.get("lg_radix", [0] * L))
    out = []
    for lvl in range(L):
        for g in RADIX_CHOICES:
            if cur[lvl] == g:
                continue
            t = dict(base)
            lr = list(cur)
            lr[lvl] = g
            t["lg_radix"] = lr
            if _plan_ok(n, batch, lift, dtype_code, prec, t) is not None:
                out.append(t)
    return out


def lift_candidates(n: int, dtype_code: int = capi.MOA_C64, max_levels: int = 3) -> List[List[int]]:
    """Lifts (outermost factor first) whose levels fit one workgroup: the
    paper's uniform blocking <2^p_max c ... c> for every c, plus all
    factorizations into at most `max_levels` powers of two."""
    d = n.bit_length() - 1
    maxlg = capi.moa_fft_max_block(dtype_code).bit_length() - 1
    out = set()
    if d <= maxlg:
        out.add((n,))
    for lam in range(1, maxlg + 1):        # paper's uniform block c = 2^lam
        if lam >= d:
            continue
        l_max = -(-d // lam) - 1
        p_max = d - l_max * lam
        if l_max + 1 <= max_levels:
            out.add(tuple([1 << p_max] + [1 << lam] * l_max))
    for L in range(2, max_levels + 1):       # mixed factorizations
        for parts in itertools.product(range(1, maxlg + 1), repeat=L):
            if sum(parts) == d:
                out.add(tuple(1 << p for p in parts))
    return sorted((list(c) for c in out), key=lambda c: (len(c), c))


def _plan_ok(n, batch, lift, dtype_code, prec, tuning) -> Optional[dict]:
    try:
        h = capi.moa_fft_plan(n, batch, lift, dtype_code, prec, capi.MOA_FFT_FLAG_HOST_ONLY, tuning)
    except capi.MoaError:
        return None
    try:
        return json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)


def candidates(n: int, batch: int, dtype_code: int = capi.MOA_C64, prec: int = capi.MOA_FFT_PREC_NATIVE,
               max_levels: int = 3, widths: Sequence[int] = (0, 1, 2, 4, 8, 16, 32, 64)) -> List[Tuple[List[int], dict]]:
    """(lift, tuning) pairs that plan successfully (host-only validation)."""
    out = []
    for lift in lift_candidates(n, dtype_code, max_levels):
        L = len(lift)
        for w in widths:
            tuning = {"cols_per_block": [w] * L} if w else None
            if _plan_ok(n, batch, lift, dtype_code, prec, tuning) is not None:
                out.append((lift, tuning))
    return out


def _timing_input(torch, numel: int, dtype, dev):
    """Seeded U[-1, 1) re/im on the device: candidates are timed on data like
    the workload's (an all-zero buffer runs measurably faster on MI355X)."""
    real = torch.float32 if dtype == torch.complex64 else torch.float64
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    x = torch.rand(2 * numel, dtype=real, device=dev, generator=g)
    return x.mul_(2).sub_(1).view(dtype)


def _time_plan(torch, plan, x, out, reps: int) -> float:
    for _ in range(2):
        plan.forward(x, out=out)
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        plan.forward(x, out=out)
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def first_round_lifts(n: int, batch: int, dtype_code: int = capi.MOA_C64, prec: int = capi.MOA_FFT_PREC_NATIVE,
                      max_levels: int = 3) -> List[List[int]]:
    """The lifts the tuner times first, with the planner's defaults: every
    lift of `lift_candidates` that plans.  With a split precision only those
    with a level on the matrix cores, where any has one: a lift of FP32
    levels only would answer a split-precision request with FP32."""
    ok = []
    for lift in lift_candidates(n, dtype_code, max_levels):
        d = _plan_ok(n, batch, lift, dtype_code, prec, None)
        if d is not None:
            ok.append((lift, any(p["mfma"] != "none" for p in d["passes"])))
    if prec != capi.MOA_FFT_PREC_NATIVE and any(m for _, m in ok):
        return [lift for lift, m in ok if m]
    return [lift for lift, _ in ok]


def tune(n: int, batch: int = 1, dtype=None, prec: str = "native", max_levels: int = 3, reps: int = 10,
         candidates_limit: Optional[int] = None, use_cache: bool = True, verbose: bool = False,
         refine: int = 5, radix: bool = True) -> dict:
    """Time the candidate lifts/tile widths/radices for (n, batch) on the
    current device; returns {"lift", "tuning", "ms", "tried"} and caches it.

    Rounds: every lift of `first_round_lifts` with the planner's defaults
    (with a split precision, those with a matrix-core level); every tile width for the
    `refine` fastest lifts; then (radix=True) for the three fastest so far,
    each level's register radix changed one level at a time, and the best
    change of every level combined."""
    import torch

    from . import fft as mfft
    dtype = dtype or torch.complex64
    dcode = mfft._dtype_code(dtype)
    pcode = mfft._PREC[prec]
    dev = torch.device("cuda", torch.cuda.current_device())
    name = torch.cuda.get_device_name(dev)
    key = _key(name, dcode, n, batch, pcode, max_levels, candidates_limit, refine, radix)
    if use_cache:
        with _lock:
            hit = _load_cache().get(key)
        if hit:
            return hit
    x = _timing_input(torch, n * batch, dtype, dev)
    out = torch.empty_like(x)
    timed = []

    def run(cands):
        for lift, tuning in cands:
            if candidates_limit and len(timed) >= candidates_limit:
                return
            plan = mfft.Plan(n, batch, lift, dtype=dtype, prec=prec, tuning=tuning)
            ms = _time_plan(torch, plan, x, out, reps)
            plan.close()
            timed.append({"lift": list(lift), "tuning": tuning, "ms": ms})
            if verbose:
                print(f"tune n={n} batch={batch} lift={lift} tuning={tuning}: {ms:.4f} ms", flush=True)

    run([(lift, None) for lift in first_round_lifts(n, batch, dcode, pcode, max_levels)])
    top = sorted(timed, key=lambda r: r["ms"])[:max(1, refine)]
    for r in top:
        run([c for c in candidates(n, batch, dcode, pcode, max_levels=len(r["lift"]))
             if c[0] == r["lift"] and c[1] is not None])
    if radix:
        for r in sorted(timed, key=lambda r: r["ms"])[:3]:
            lift, tuning = r["lift"], r["tuning"]
            before = len(timed)
            run([(lift, t) for t in radix_candidates(n, batch, lift, tuning, dcode, pcode)])
            trial = [q for q in timed[before:]]
            # combine the best radix of each level when several levels gained
            per_level = {}
            for q in trial:
                lr = q["tuning"]["lg_radix"]
                base_lr = (tuning or {}).get("lg_radix", [0] * len(lift))
                lvl = next(i for i in range(len(lift)) if lr[i] != base_lr[i])
                if q["ms"] < r["ms"] and (lvl not in per_level or q["ms"] < per_level[lvl]["ms"]):
                    per_level[lvl] = q
            if len(per_level) > 1:
                t = dict(tuning or {})
                lr = list(t.get("lg_radix", [0] * len(lift)))
                for lvl, q in per_level.items():
                    lr[lvl] = q["tuning"]["lg_radix"][lvl]
                t["lg_radix"] = lr
                if _plan_ok(n, batch, lift, dcode, pcode, t) is not None:
                    run([(lift, t)])
    best = dict(min(timed, key=lambda r: r["ms"]))
    best["tried"] = len(timed)
    if use_cache:
        with _lock:
            c = _load_cache()
            c[key] = best
            _save_cache(c)
    return best


def tune_batched(sizes: Sequence[int], dtype=None, grids: Iterable[int] = (0, 256, 512, 768, 1024, 1536, 2048),
                 reps: int = 10, verbose: bool = False, streams: Iterable[int] = (0, 1, -1),
                 task_lgs: Iterable[int] = (13, 12, 11)) -> dict:
    """Time the task packing (log2 of the most points a task packs: 13, the
    default, or fewer for more and shorter tasks) and the grid of an uneven
    batch's fused launch (0 = one workgroup per task, the default; smaller
    grids make it persistent), then the streaming modes of its loads and
    stores (0 = by size, 1 = always, -1 = never) at the best of those;
    returns the best tuning."""
    import torch

    from . import fft as mfft
    dtype = dtype or torch.complex64
    dev = torch.device("cuda", torch.cuda.current_device())
    total = int(sum(sizes))
    x = _timing_input(torch, total, dtype, dev)
    out = torch.empty_like(x)
    best = None
    seen = set()
    for tl in task_lgs:
        for g in grids:
            tuning = {}
            if g:
                tuning["persistent_blocks"] = int(g)
            if tl != 13:
                tuning["batch_task_lg"] = int(tl)
            plan = mfft.BatchedPlan(sizes, dtype=dtype, tuning=tuning or None)
            d = plan.describe()
            grid = d["persistent_blocks"]
            if (tl, grid) in seen:  # a grid at least the task count is one workgroup a task
                plan.close()
                continue
            seen.add((tl, grid))
            ms = _time_plan(torch, plan, x, out, reps)
            plan.close()
            if verbose:
                print(f"tune batched task_lg={tl} tasks={d['tasks']} grid={grid}: {ms:.4f} ms", flush=True)
            if best is None or ms < best["ms"]:
                best = {"tuning": tuning or None, "grid": grid, "task_lg": tl, "ms": ms}
    for sm in streams:
        if sm == 0:
            continue
        tuning = dict(best["tuning"] or {})
        tuning["stream"] = int(sm)
        plan = mfft.BatchedPlan(sizes, dtype=dtype, tuning=tuning)
        ms = _time_plan(torch, plan, x, out, reps)
        plan.close()
        if verbose:
            print(f"tune batched task_lg={best['task_lg']} grid={best['grid']} stream={sm}: {ms:.4f} ms", flush=True)
        if ms < best["ms"]:
            best = {"tuning": tuning, "grid": best["grid"], "task_lg": best["task_lg"], "ms": ms}
    return best


def tuned_plan(n: int, batch: int = 1, dtype=None, prec: str = "native", **kw):
    """A Plan with the tuned lift and tile widths (tuning on first use)."""
    from . import fft as mfft
    r = tune(n, batch, dtype, prec, **kw)
    import torch
    return mfft.Plan(n, batch, r["lift"], dtype=dtype or torch.complex64, prec=prec, tuning=r["tuning"])
