"""Host-side tests of the C-ABI library (no GPU needed): it loads, exports
every function include/moa_fft.h declares, validates arguments with the
documented status codes, and lowers lifts to pass descriptors that compute the
DFT.  The descriptors are checked by interpreting them on the CPU (gather by
the stated strides, DFT, inter-level twiddle, scatter) against the FP64
oracle, and their index maps against the MoA index oracle."""
import ctypes
import itertools
import json
import os
import re

import numpy as np
import pytest

import oracle
from oracle import moa
from paper_0803_2386_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = capi.MOA_FFT_FLAG_HOST_ONLY


@pytest.fixture(scope="module", autouse=True)
def built_library():
    if not os.path.exists(capi.LIB_PATH):
        import paper_0803_2386_amd.build as b
        b.build()
    capi.load()


def declared_functions():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    return sorted(set(re.findall(r"^\s*(?:const char\*|moa_status_t|int64_t)\s+(moa_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(capi.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(capi.EXPORTED) == names


def test_status_strings():
    for code, name in [(0, "MOA_OK"), (1, "MOA_ERR_NULL"), (2, "MOA_ERR_SIZE"), (3, "MOA_ERR_LIFT"),
                       (4, "MOA_ERR_BATCH"), (5, "MOA_ERR_DTYPE"), (6, "MOA_ERR_ALLOC"), (7, "MOA_ERR_HIP"),
                       (8, "MOA_ERR_STATE"), (9, "MOA_ERR_ARG"), (10, "MOA_ERR_TUNING"),
                       (11, "MOA_ERR_SCRATCH")]:
        assert capi.moa_fft_status_string(code) == name
    assert capi.moa_fft_status_string(99) == "MOA_ERR_UNKNOWN"
    assert capi.moa_fft_max_block(capi.MOA_C64) == 1 << 14
    assert capi.moa_fft_max_block(capi.MOA_C128) == 1 << 13


def status_of(fn, *a, **k):
    try:
        h = fn(*a, **k)
    except capi.MoaError as e:
        return e.status
    capi.moa_fft_destroy(h)
    return capi.MOA_OK


@pytest.mark.parametrize("args,want", [
    (dict(n=0), capi.MOA_ERR_SIZE), (dict(n=3), capi.MOA_ERR_SIZE), (dict(n=1 << 31), capi.MOA_ERR_SIZE),
    (dict(n=16, batch=0), capi.MOA_ERR_BATCH), (dict(n=16, batch=-4), capi.MOA_ERR_BATCH),
    (dict(n=16, lift_shape=[4, 8]), capi.MOA_ERR_LIFT), (dict(n=24 * 0 + 32, lift_shape=[4, 6]), capi.MOA_ERR_LIFT),
    (dict(n=1 << 15, lift_shape=[1 << 15]), capi.MOA_ERR_LIFT),
    (dict(n=1 << 14, lift_shape=[1 << 14], dtype=capi.MOA_C128), capi.MOA_ERR_LIFT),
    (dict(n=512, lift_shape=[2] * 9), capi.MOA_ERR_LIFT), (dict(n=16, lift_shape=[16, 1]), capi.MOA_ERR_LIFT),
    (dict(n=16, dtype=7), capi.MOA_ERR_DTYPE), (dict(n=16, prec=9), capi.MOA_ERR_DTYPE),
    (dict(n=16, dtype=capi.MOA_C128, prec=capi.MOA_FFT_PREC_SPLIT_BF16), capi.MOA_ERR_DTYPE),
    (dict(n=16, flags=HOST | 0x100), capi.MOA_ERR_ARG), (dict(n=16, flags=HOST | capi.MOA_FFT_FLAG_PER_SIZE),
                                                          capi.MOA_ERR_ARG),
    (dict(n=4096, lift_shape=[64, 64], tuning=dict(cols_per_block=[3])), capi.MOA_ERR_TUNING),
    (dict(n=4096, lift_shape=[64, 64], tuning=dict(cols_per_block=[128])), capi.MOA_ERR_TUNING),
    (dict(n=1 << 24, lift_shape=[4096, 4096], tuning=dict(cols_per_block=[16])), capi.MOA_ERR_TUNING),
    (dict(n=16), capi.MOA_OK), (dict(n=1), capi.MOA_OK), (dict(n=1 << 30), capi.MOA_OK),
])
def test_plan_validation(args, want):
    args = dict(args)
    args["flags"] = args.get("flags", 0) | HOST
    assert status_of(capi.moa_fft_plan, **args) == want


def test_null_pointers():
    lib = capi.load()
    assert lib.moa_fft_plan(None, 16, 1, None, 0, 0, 0, HOST) == capi.MOA_ERR_NULL
    h = ctypes.c_void_p()
    assert lib.moa_fft_plan(ctypes.byref(h), 16, 1, None, 2, 0, 0, HOST) == capi.MOA_ERR_NULL
    assert lib.moa_fft_plan_batched(ctypes.byref(h), None, 4, 0, HOST) == capi.MOA_ERR_NULL
    assert lib.moa_fft_exec(None, 0, None, None, None) == capi.MOA_ERR_NULL
    assert lib.moa_fft_destroy(None) == capi.MOA_OK
    size = ctypes.c_size_t()
    assert lib.moa_fft_workspace_size(None, ctypes.byref(size)) == capi.MOA_ERR_NULL


def test_host_only_plan_cannot_execute_and_describe_truncates():
    lib = capi.load()
    h = capi.moa_fft_plan(1024, 2, None, flags=HOST)
    try:
        buf = ctypes.create_string_buffer(16)
        assert lib.moa_fft_exec(h, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == capi.MOA_ERR_STATE
        assert lib.moa_fft_exec(h, 5, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == capi.MOA_ERR_ARG
        assert lib.moa_fft_describe(h, buf, 16) == capi.MOA_ERR_ARG
        assert len(buf.value) == 15
        assert json.loads(capi.moa_fft_describe(h))["n"] == 1024
    finally:
        capi.moa_fft_destroy(h)


def test_exec_noalloc_validation_on_the_host():
    """The allocation-free execution validates on the host before any HIP
    call: a plan needing more workspace than the static array is refused
    with MOA_ERR_SCRATCH, a host-only plan within it with MOA_ERR_STATE."""
    lib = capi.load()
    fn = lib.moa_fft_exec_noalloc
    buf = ctypes.c_void_p(256)
    assert fn(None, 0, buf, buf, None) == capi.MOA_ERR_NULL
    big = capi.moa_fft_plan(1 << 24, 1, [4096, 4096], flags=HOST | capi.MOA_FFT_FLAG_NO_WORKSPACE)
    fits = capi.moa_fft_plan(1 << 23, 1, [2048, 4096], flags=HOST | capi.MOA_FFT_FLAG_NO_WORKSPACE)
    fits128 = capi.moa_fft_plan(1 << 22, 1, [1024, 4096], dtype=capi.MOA_C128, flags=HOST)
    over128 = capi.moa_fft_plan(1 << 21, 3, [512, 4096], dtype=capi.MOA_C128, flags=HOST)
    try:
        assert capi.moa_fft_workspace_size(big) == 128 << 20
        assert fn(big, 0, buf, buf, None) == capi.MOA_ERR_SCRATCH
        assert fn(over128, 1, buf, buf, None) == capi.MOA_ERR_SCRATCH
        assert capi.moa_fft_workspace_size(fits) == capi.MOA_FFT_SCRATCH_BYTES
        assert fn(fits, 0, buf, buf, None) == capi.MOA_ERR_STATE
        assert fn(fits128, 1, buf, buf, None) == capi.MOA_ERR_STATE
        assert fn(fits, 2, buf, buf, None) == capi.MOA_ERR_ARG
        assert fn(fits, 0, None, buf, None) == capi.MOA_ERR_NULL
        d = json.loads(capi.moa_fft_describe(fits))
        assert d["workspace_bytes"] == 64 << 20 and d["workspace_owned"] is False
        assert json.loads(capi.moa_fft_describe(fits128))["workspace_owned"] is True
    finally:
        for h in (big, fits, fits128, over128):
            capi.moa_fft_destroy(h)
    # a destroyed plan is not a live plan
    assert fn(big, 0, buf, buf, None) == capi.MOA_ERR_STATE


@pytest.mark.parametrize("sizes,want", [([3], capi.MOA_ERR_SIZE), ([64, 1 << 15], capi.MOA_ERR_SIZE),
                                        ([], capi.MOA_ERR_BATCH), ([1 << 14], capi.MOA_OK)])
def test_batched_validation(sizes, want):
    if not sizes:
        lib = capi.load()
        h = ctypes.c_void_p()
        arr = (ctypes.c_int64 * 1)(64)
        assert lib.moa_fft_plan_batched(ctypes.byref(h), arr, 0, 0, HOST) == want
        return
    assert status_of(capi.moa_fft_plan_batched, sizes, flags=HOST) == want


def describe(n, batch=1, lift=None, dtype=capi.MOA_C64, tuning=None, prec=capi.MOA_FFT_PREC_NATIVE):
    h = capi.moa_fft_plan(n, batch, lift, dtype=dtype, prec=prec, flags=HOST, tuning=tuning)
    try:
        return json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)


def test_default_lifts():
    assert describe(1 << 24)["lift"] == [4096, 4096]
    assert describe(1 << 16)["lift"] == [256, 256]
    assert describe(1 << 14)["lift"] == [1 << 14]
    # complex64, 2^19 .. 2^23 points in batches of 2^24 points or more: a
    # 4096-point level, first up to 2^25 points a batch, last beyond (first
    # at 2^23 always); smaller batches keep the near-equal split
    assert describe(1 << 20)["lift"] == [1024, 1024]
    assert describe(1 << 20, batch=15)["lift"] == [1024, 1024]
    assert describe(1 << 20, batch=16)["lift"] == [256, 4096]
    assert describe(1 << 20, batch=32)["lift"] == [256, 4096]
    assert describe(1 << 20, batch=33)["lift"] == [4096, 256]
    assert describe(1 << 22, batch=64)["lift"] == [4096, 1024]
    assert describe(1 << 19, batch=128)["lift"] == [4096, 128]
    assert describe(1 << 23, batch=32)["lift"] == [2048, 4096]
    assert describe(1 << 23, batch=8)["lift"] == [2048, 4096]
    # 2^23 points in batches of up to 2^25 points: three levels
    assert describe(1 << 23)["lift"] == [256, 128, 256]
    assert describe(1 << 23, batch=4)["lift"] == [256, 128, 256]
    assert describe(1 << 18, batch=128)["lift"] == [512, 512]
    # 2^25 points and more: <256 4096 2^(d-20)>
    assert describe(1 << 25)["lift"] == [256, 4096, 32]
    assert describe(1 << 28)["lift"] == [256, 4096, 256]
    assert describe(1 << 30)["lift"] == [256, 4096, 1024]
    # complex128: the near-equal split of the fewest levels, but three
    # levels <256 256 2^(d-16)> at 2^23 .. 2^26 points
    assert describe(1 << 14, dtype=capi.MOA_C128)["lift"] == [128, 128]
    assert describe(1 << 20, dtype=capi.MOA_C128)["lift"] == [1024, 1024]
    assert describe(1 << 22, dtype=capi.MOA_C128)["lift"] == [2048, 2048]
    assert describe(1 << 23, dtype=capi.MOA_C128)["lift"] == [256, 256, 128]
    assert describe(1 << 26, dtype=capi.MOA_C128)["lift"] == [256, 256, 1024]
    assert describe(1 << 27, dtype=capi.MOA_C128)["lift"] == [512, 512, 512]
    assert describe(1 << 30, dtype=capi.MOA_C128)["lift"] == [1024, 1024, 1024]
    d = describe(1 << 24, lift=[4096, 4096])
    assert d["levels"] == [4096, 4096] and len(d["passes"]) == 2
    assert d["workspace_bytes"] == 8 << 24


@pytest.mark.parametrize("prec", [capi.MOA_FFT_PREC_SPLIT_FP16, capi.MOA_FFT_PREC_SPLIT_BF16])
def test_default_split_lifts_use_the_matrix_cores(prec):
    """With a split precision the default lift keeps the FP32 level count but
    cuts the levels into whole radix-16 digits, shorter levels first, so that
    they run on the matrix cores; bits left over from whole digits go to the
    first level, the only one that stays in FP32, and it takes as few as the
    12-bit levels after it allow.  From 2^25 points the FP32 default
    <256 4096 2^(d-20)> already has two matrix-core levels."""
    want = {12: [4096], 16: [256, 256], 20: [4096, 256], 24: [4096, 4096], 13: [8192], 14: [16384],
            15: [4096, 8], 17: [4096, 32], 19: [4096, 128], 22: [4096, 1024], 25: [256, 4096, 32],
            26: [256, 4096, 64], 27: [256, 4096, 128], 28: [256, 4096, 256], 29: [256, 4096, 512],
            30: [256, 4096, 1024]}
    for lg in range(1, 31):
        d = describe(1 << lg, batch=64, prec=prec)
        native = describe(1 << lg, batch=64)
        assert len(d["passes"]) == len(native["passes"]), lg
        assert lg == 4 or any(p["mfma"] != "none" for p in d["passes"]) or lg % 4 and lg < 15, lg
    for lg, lift in want.items():
        d = describe(1 << lg, batch=4, prec=prec)
        assert d["lift"] == lift, lg
        native = describe(1 << lg, batch=4)
        assert len(d["passes"]) == len(native["passes"]), lg
        # passes run innermost level first: the first takes the leftover bits
        for i, p in enumerate(d["passes"]):
            on_mfma = p["N"] in (16, 256, 4096)
            assert (p["mfma"] != "none") == on_mfma, (lg, i)
            assert on_mfma or i == 0, (lg, i)
    # a length of at most 2^12 points stays one level; only 16, 256, 4096 use MFMA
    assert describe(1 << 11, batch=64, prec=prec)["lift"] == [2048]
    assert describe(1 << 8, batch=64, prec=prec)["passes"][0]["mfma"] != "none"
    # a matrix-core tile gathers 2^11 points: with fewer transforms the level
    # runs in FP32 (an explicit tile width below that stays an error)
    assert describe(16, batch=128, prec=prec)["passes"][0]["mfma"] != "none"
    assert describe(16, batch=64, prec=prec)["passes"][0]["mfma"] == "none"
    assert describe(256, batch=4, lift=[256], prec=prec)["passes"][0]["mfma"] == "none"
    assert describe(256, batch=8, lift=[256], prec=prec)["passes"][0]["mfma"] != "none"
    with pytest.raises(capi.MoaError) as e:
        describe(256, batch=64, lift=[256], prec=prec, tuning=dict(cols_per_block=[4]))
    assert e.value.status == capi.MOA_ERR_TUNING


def _row(k, layout, stride):
    lg = layout["block_lg"]
    if lg >= 30:
        return k * stride
    return (k & ((1 << lg) - 1)) * stride + (k >> lg) * layout["stride_hi"]


def _axis0(i0, W, layout, stride0):
    """Offset of value i0 of batch axis 0 (the tile digit): tile i0 // W at
    the tile stride, column pairs at the pair stride, stride0 within a pair."""
    w = i0 % W
    return (i0 // W) * layout["tile_stride"] + (w >> 1) * layout["pair_stride"] + (w & 1) * stride0


def _batch_offsets(p, side):
    """Offsets of every combination of the batch axes (axis 0 slowest in the
    product) on one side ("in" or "out") of a pass."""
    axes = p["batch_axes"]
    lay = p[side + "_layout"]
    key = side + "_stride"
    offs = np.zeros(1, dtype=np.int64)
    for d, a in enumerate(axes):
        r = np.arange(a["size"], dtype=np.int64)
        o = _axis0(r, p["tile_width"], lay, a[key]) if d == 0 else r * a[key]
        offs = (offs[:, None] + o[None, :]).ravel()
    return offs


def interpret(desc, x, sign):
    """Run the plan's pass descriptors on the CPU: every pass gathers each
    transform by its strides and layouts, takes the DFT, applies the
    inter-level twiddle omega_root^(d0 k) (d0 = value of batch axis 0) and
    scatters it."""
    total = x.size
    ws = np.zeros(total, complex)
    out = np.zeros(total, complex)
    src = x
    for p in desc["passes"]:
        N = p["N"]
        ise, osk = p["dft_axis"]["in_stride"], p["dft_axis"]["out_stride"]
        axes = p["batch_axes"]
        dst_name = p["out"]
        snapshot = src.copy()
        dst = ws if dst_name == "workspace" else out
        k = np.arange(N)
        kin, kout = _row(k, p["in_layout"], ise), _row(k, p["out_layout"], osk)
        for idx in itertools.product(*[range(a["size"]) for a in axes]):
            ib = _axis0(idx[0], p["tile_width"], p["in_layout"], axes[0]["in_stride"]) + sum(
                i * a["in_stride"] for i, a in zip(idx[1:], axes[1:]))
            ob = _axis0(idx[0], p["tile_width"], p["out_layout"], axes[0]["out_stride"]) + sum(
                i * a["out_stride"] for i, a in zip(idx[1:], axes[1:]))
            X = oracle.dft_brute(snapshot[ib + kin], sign) if N <= 64 else oracle.fft(snapshot[ib + kin], sign)
            root = p["twiddle_root"]
            if root:
                e = (idx[0] * k) % root
                X = X * np.array([oracle.root(int(ee), root, sign) for ee in e])
            dst[ob + kout] = X
        src = dst
    return src


def interpret_fast(desc, x, sign):
    """Vectorized interpret(): the same gathers, transforms, twiddles and
    scatters with index arrays (FP64 transforms by the oracle's batch call,
    twiddles exp(sign 2 pi i e / root) with e reduced exactly)."""
    total = x.size
    bufs = {"workspace": np.zeros(total, complex), "y": np.zeros(total, complex)}
    src = x
    for p in desc["passes"]:
        N = p["N"]
        k = np.arange(N, dtype=np.int64)
        ib = _batch_offsets(p, "in")
        ob = _batch_offsets(p, "out")
        gi = ib[:, None] + _row(k, p["in_layout"], p["dft_axis"]["in_stride"])[None, :]
        go = ob[:, None] + _row(k, p["out_layout"], p["dft_axis"]["out_stride"])[None, :]
        X = oracle.fft_batch(np.ascontiguousarray(src[gi]), sign, threads=oracle.max_threads())
        root = p["twiddle_root"]
        if root:
            reps = gi.shape[0] // p["batch_axes"][0]["size"]
            d0 = np.repeat(np.arange(p["batch_axes"][0]["size"], dtype=np.int64), reps)
            e = (d0[:, None] * k[None, :]) % root
            X = X * np.exp(sign * 2j * np.pi * e / root)
        dst = bufs[p["out"]]
        dst[go] = X
        src = dst.copy()
    return src


@pytest.mark.parametrize("n,batch,lift", [
    (64, 1, [8, 8]), (256, 2, [16, 16]), (512, 1, [2, 16, 16]), (1024, 3, [4, 8, 32]),
    (4096, 1, [64, 64]), (2048, 1, [2, 4, 2, 8, 16]), (32, 2, [2, 4, 4]), (128, 1, [128]), (8, 4, None),
    (4096, 2, [16, 256]),
])
def test_lowering_computes_the_dft(n, batch, lift):
    desc = describe(n, batch, lift)
    rng = np.random.default_rng(n + batch)
    x = rng.uniform(-1, 1, n * batch) + 1j * rng.uniform(-1, 1, n * batch)
    for sign in (-1, 1):
        got = interpret(desc, x, sign).reshape(batch, n)
        want = oracle.fft(x.reshape(batch, n), sign)
        assert np.abs(got - want).max() < 1e-11 * n, (n, batch, lift, sign)
    for p in desc["passes"]:
        assert p["threads"] <= 1024 and p["lds_bytes"] <= 160 * 1024
        assert p["threads"] % 64 == 0 or p["threads"] < 64 or p["blocks"] >= 1


def test_two_level_store_is_the_reshape_transpose():
    # The first pass of a lift <r c> writes frequency k0 of column a'' at
    # position k0 * r + a'': the paper's reshape-transpose of the <c r> view,
    # i.e. the transpose of <c r> rho^ x read back as <c r>.
    r, c = 8, 4
    d = describe(r * c, 1, [r, c])
    p0, p1 = d["passes"]
    assert p0["N"] == c and p0["dft_axis"] == {"in_stride": r, "out_stride": r}
    assert p0["batch_axes"] == [{"size": r, "in_stride": 1, "out_stride": 1}]
    assert p0["twiddle_root"] == r * c
    # last pass: final transpose X[k0 + c k1] <- position k0 * r + a'
    assert p1["dft_axis"] == {"in_stride": 1, "out_stride": c}
    assert p1["batch_axes"] == [{"size": c, "in_stride": r, "out_stride": 1}]
    # index oracle: the final transpose as the reversal of the digit axes
    D = moa.MArray([c, r], list(range(r * c)))
    X = moa.transpose(D, [1, 0])
    for k0 in range(c):
        for k1 in range(r):
            # element k0 * r + k1 of D lands at gamma(<k1 k0>; <r c>) = k1 * c + k0
            assert moa.psi([k1, k0], X) == k0 * r + k1


def test_batched_plan_partitions_the_transforms():
    sizes = [64, 128, 64, 16384, 8, 8192, 8192, 1, 64] * 3
    h = capi.moa_fft_plan_batched(sizes, flags=HOST)
    try:
        d = json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)
    assert d["count"] == len(sizes) and d["elements"] == sum(sizes)
    groups = d["sizes_by_task_group"]
    assert [g["n"] for g in groups] == sorted(set(sizes), reverse=True)
    assert sum(g["tasks"] for g in groups) == d["tasks"]
    assert d["lds_bytes"] <= 160 * 1024 and d["threads"] == 512


def test_batched_grid_defaults_to_one_workgroup_per_task():
    """The fused launch has one workgroup per task unless a tuned grid caps it
    (then each workgroup walks the tasks with a grid stride); a negative grid
    is rejected."""
    sizes = [64, 128, 64, 16384, 8, 8192, 8192, 1, 64] * 40

    def grid(tuning):
        h = capi.moa_fft_plan_batched(sizes, flags=HOST, tuning=tuning)
        try:
            d = json.loads(capi.moa_fft_describe(h))
        finally:
            capi.moa_fft_destroy(h)
        return d["persistent_blocks"], d["tasks"]

    g, tasks = grid(None)
    assert g == tasks
    assert grid({"persistent_blocks": 7}) == (7, tasks)
    assert grid({"persistent_blocks": 10 * tasks}) == (tasks, tasks)
    assert status_of(capi.moa_fft_plan_batched, sizes, flags=HOST,
                     tuning={"persistent_blocks": -1}) == capi.MOA_ERR_TUNING


def test_batched_task_packing():
    """The task size of an uneven batch: at most 2^13 points a task by
    default; 2^12 or 2^11 pack fewer of the shorter transforms a task (each
    size group then has at least the tasks its points need at that size;
    a transform longer than the task size is one task); other sizes are
    refused."""
    sizes = [64, 128, 64, 16384, 8, 8192, 8192, 1, 64, 2048, 4] * 40

    def desc(tuning):
        h = capi.moa_fft_plan_batched(sizes, flags=HOST, tuning=tuning)
        try:
            return json.loads(capi.moa_fft_describe(h))
        finally:
            capi.moa_fft_destroy(h)

    base = desc(None)
    assert base["task_lg"] == 13 and desc({"batch_task_lg": 13})["tasks"] == base["tasks"]
    prev = base["tasks"]
    for tl in (12, 11):
        d = desc({"batch_task_lg": tl})
        assert d["task_lg"] == tl and d["tasks"] > prev
        prev = d["tasks"]
        for g in d["sizes_by_task_group"]:
            n, count = g["n"], sizes.count(g["n"])
            if n >= 1 << tl:
                assert g["tasks"] == count
            else:
                assert g["tasks"] >= -(-count * n // (1 << tl))
    for bad in (10, 14, -1):
        assert status_of(capi.moa_fft_plan_batched, sizes, flags=HOST,
                         tuning={"batch_task_lg": bad}) == capi.MOA_ERR_TUNING


def test_stream_choice():
    """Streaming loads of the caller's input: automatic while the input is at
    most 256 MiB, forced on or off by the tuning field, other values refused."""
    def stream(n, dtype=capi.MOA_C64, tuning=None):
        h = capi.moa_fft_plan(n, 1, None, dtype, capi.MOA_FFT_PREC_NATIVE, HOST, tuning)
        try:
            return json.loads(capi.moa_fft_describe(h))["stream"]
        finally:
            capi.moa_fft_destroy(h)

    assert stream(1 << 24) and stream(1 << 25)              # 128 and 256 MiB
    assert not stream(1 << 26)                              # 512 MiB
    assert not stream(1 << 25, capi.MOA_C128)               # 512 MiB
    assert stream(1 << 28, tuning={"stream": 1})
    assert not stream(1 << 10, tuning={"stream": -1})
    for bad in (2, -2):
        assert status_of(capi.moa_fft_plan, 1 << 10, 1, None, capi.MOA_C64, capi.MOA_FFT_PREC_NATIVE, HOST,
                         {"stream": bad}) == capi.MOA_ERR_TUNING
    h = capi.moa_fft_plan_batched([64, 16384] * 10, flags=HOST)
    try:
        assert json.loads(capi.moa_fft_describe(h))["stream"]
    finally:
        capi.moa_fft_destroy(h)


def test_batched_exec_level_validation():
    """exec_level on an uneven batch: host-only plans cannot run, levels are
    the size groups of a per-size plan (one level for the fused form)."""
    sizes = [64, 4096, 64, 16384, 1]
    for flags, groups in ((capi.MOA_FFT_FLAG_PER_SIZE, 4), (0, 1)):
        h = capi.moa_fft_plan_batched(sizes, flags=HOST | flags)
        try:
            assert capi.moa_fft_num_levels(h) == groups
            lib = capi.load()
            buf = ctypes.c_void_p(16)
            assert lib.moa_fft_exec_level(h, 0, groups, buf, buf, None) == capi.MOA_ERR_ARG
            assert lib.moa_fft_exec_level(h, 0, -1, buf, buf, None) == capi.MOA_ERR_ARG
            assert lib.moa_fft_exec_level(h, 0, 0, buf, buf, None) == capi.MOA_ERR_STATE
        finally:
            capi.moa_fft_destroy(h)


def test_pair_block_workspace_computes_the_dft():
    """The two-level <4096 4096> complex64 plan stores its workspace
    blockwise (column pairs of level 0, blocks of level 1's tile width):
    the level-0 stores are a permutation of the workspace, the level-1 loads
    read exactly that, and the two passes compose to the DFT."""
    n = 1 << 24
    desc = describe(n, 1, [4096, 4096])
    p0, p1 = desc["passes"]
    assert p0["out_layout"]["block_lg"] == 3 and p1["in_layout"]["block_lg"] == 1
    ob = _batch_offsets(p0, "out")
    go = (ob[:, None] + _row(np.arange(4096), p0["out_layout"], p0["dft_axis"]["out_stride"])[None, :]).ravel()
    assert np.array_equal(np.sort(go), np.arange(n))
    ib = _batch_offsets(p1, "in")
    gi = (ib[:, None] + _row(np.arange(4096), p1["in_layout"], p1["dft_axis"]["in_stride"])[None, :]).ravel()
    assert np.array_equal(np.sort(gi), np.arange(n))
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    got = interpret_fast(desc, x, -1)
    want = oracle.fft(x)
    assert np.abs(got - want).max() < 1e-9 * np.abs(want).max()



def describe_nd(dims, batch=1, dtype=capi.MOA_C64, prec=capi.MOA_FFT_PREC_NATIVE, tuning=None):
    h = capi.moa_fft_plan_nd(dims, batch, dtype=dtype, prec=prec, flags=HOST, tuning=tuning)
    try:
        return json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)


@pytest.mark.parametrize("dims,batch,kw,want", [
    ([3, 4], 1, {}, capi.MOA_ERR_SIZE), ([0, 4], 1, {}, capi.MOA_ERR_SIZE), ([1 << 15, 2], 1, {}, capi.MOA_ERR_SIZE),
    ([1 << 14, 2], 1, dict(dtype=capi.MOA_C128), capi.MOA_ERR_SIZE),
    ([1 << 14, 1 << 14, 8], 1, {}, capi.MOA_ERR_SIZE),        # 2^31 points
    ([], 1, {}, capi.MOA_ERR_ARG), ([2] * 9, 1, {}, capi.MOA_ERR_ARG),
    ([16, 16], 0, {}, capi.MOA_ERR_BATCH), ([16, 16], 1, dict(dtype=9), capi.MOA_ERR_DTYPE),
    ([16, 16], 1, dict(flags=capi.MOA_FFT_FLAG_PER_SIZE), capi.MOA_ERR_ARG),
    ([64, 64], 1, dict(tuning=dict(cols_per_block=[3])), capi.MOA_ERR_TUNING),
    ([4096, 4096], 1, {}, capi.MOA_OK), ([256, 256, 256], 1, {}, capi.MOA_OK), ([1, 1], 3, {}, capi.MOA_OK),
    ([1 << 14, 1 << 14, 4], 1, {}, capi.MOA_OK), ([2] * 8, 5, {}, capi.MOA_OK),
])
def test_nd_plan_validation(dims, batch, kw, want):
    kw = dict(kw)
    kw["flags"] = kw.get("flags", 0) | HOST
    if not dims:
        lib = capi.load()
        h = ctypes.c_void_p()
        arr = (ctypes.c_int64 * 1)(4)
        assert lib.moa_fft_plan_nd(ctypes.byref(h), 0, arr, 1, 0, 0, HOST) == want
        return
    assert status_of(capi.moa_fft_plan_nd, dims, batch, **kw) == want


def test_nd_null_pointers():
    lib = capi.load()
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * 2)(4, 4)
    assert lib.moa_fft_plan_nd(None, 2, arr, 1, 0, 0, HOST) == capi.MOA_ERR_NULL
    assert lib.moa_fft_plan_nd(ctypes.byref(h), 2, None, 1, 0, 0, HOST) == capi.MOA_ERR_NULL


@pytest.mark.parametrize("dims,batch", [
    ((8, 16), 1), ((16, 8), 3), ((4, 8, 2), 2), ((1, 64), 1), ((32, 1, 4), 1), ((2, 2, 2, 2), 2), ((1, 1), 2),
    ((64, 64), 1), ((4096, 2), 1), ((2, 4096), 1), ((16, 256), 2), ((16, 16, 16), 1),
])
def test_nd_lowering_computes_the_dft(dims, batch):
    desc = describe_nd(list(dims), batch)
    assert desc["kind"] == "nd" and desc["dims"] == list(dims) and desc["workspace_bytes"] == 0
    ext = [d for d in dims if d > 1]
    assert len(desc["passes"]) == max(1, len(ext))
    for p in desc["passes"]:
        assert p["twiddle_root"] == 0 and p["out"] == "y"
    rng = np.random.default_rng(sum(dims) + batch)
    N = int(np.prod(dims))
    x = rng.uniform(-1, 1, N * batch) + 1j * rng.uniform(-1, 1, N * batch)
    for sign in (-1, 1):
        got = interpret_fast(desc, x, sign).reshape((batch,) + tuple(dims))
        want = oracle.fftn(x.reshape((batch,) + tuple(dims)), len(dims), sign)
        assert np.abs(got - want).max() < 1e-11 * N, (dims, batch, sign)


def test_nd_headline_shapes_pick_the_wide_tile_kernels():
    d = describe_nd([4096, 4096])
    # contiguous rows first (one 4096-point row a tile), then the columns in
    # the paired-column kernel (unit-stride tile digit on both sides)
    assert [p["dft_axis"]["in_stride"] for p in d["passes"]] == [1, 4096]
    assert d["passes"][1]["kernel_mode"] == 3 and d["passes"][1]["in_tile_fast"] and d["passes"][1]["out_tile_fast"]
    d3 = describe_nd([256, 256, 256])
    assert [p["dft_axis"]["in_stride"] for p in d3["passes"]] == [1, 256, 65536]
    for p in d3["passes"][1:]:
        assert p["in_tile_fast"] and p["tile_width"] * 8 >= 128   # whole 128-byte lines per row


def test_stale_and_double_destroyed_handles_are_rejected():
    lib = capi.load()
    h = capi.moa_fft_plan(1024, 1, None, flags=HOST)
    assert lib.moa_fft_destroy(h) == capi.MOA_OK
    # the handle is gone: every call reports it without touching memory
    assert lib.moa_fft_destroy(h) == capi.MOA_ERR_STATE
    size = ctypes.c_size_t()
    lv = ctypes.c_int32()
    assert lib.moa_fft_workspace_size(h, ctypes.byref(size)) == capi.MOA_ERR_STATE
    assert lib.moa_fft_num_levels(h, ctypes.byref(lv)) == capi.MOA_ERR_STATE
    assert lib.moa_fft_exec(h, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == capi.MOA_ERR_STATE
    assert lib.moa_fft_describe_size(h, ctypes.byref(size)) == capi.MOA_ERR_STATE
    # a pointer that never was a plan
    junk = ctypes.create_string_buffer(256)
    assert lib.moa_fft_destroy(ctypes.cast(junk, ctypes.c_void_p)) == capi.MOA_ERR_STATE
    assert lib.moa_fft_num_levels(ctypes.cast(junk, ctypes.c_void_p), ctypes.byref(lv)) == capi.MOA_ERR_STATE


def test_hypercube_entry_points_validate_on_the_host():
    """Both hyper-cube calls refuse invalid arguments before any HIP call."""
    lib = capi.load()
    P = ctypes.c_void_p
    a, b = P(1 << 20), P(1 << 30)
    perm = (ctypes.c_int32 * 4)(2, 0, 3, 1)
    bad = (ctypes.c_int32 * 4)(2, 0, 2, 1)
    T = lib.moa_hypercube_transpose
    assert T(4, None, 8, a, b, None) == capi.MOA_ERR_NULL
    assert T(4, perm, 8, None, b, None) == capi.MOA_ERR_NULL
    assert T(0, perm, 8, a, b, None) == capi.MOA_ERR_SIZE
    assert T(35, perm, 8, a, b, None) == capi.MOA_ERR_SIZE
    assert T(4, bad, 8, a, b, None) == capi.MOA_ERR_ARG
    assert T(4, perm, 12, a, b, None) == capi.MOA_ERR_ARG
    assert T(4, perm, 8, P((1 << 20) + 8), b, None) == capi.MOA_ERR_ARG   # misaligned
    assert T(4, perm, 8, a, P((1 << 20) + 64), None) == capi.MOA_ERR_ARG  # overlapping
    g = (ctypes.c_int32 * 2)(0, 2)
    G = lib.moa_density_gate
    assert G(4, 2, None, a, capi.MOA_C64, b, None) == capi.MOA_ERR_NULL
    assert G(4, 2, g, None, capi.MOA_C64, b, None) == capi.MOA_ERR_NULL
    assert G(16, 2, g, a, capi.MOA_C64, b, None) == capi.MOA_ERR_SIZE
    assert G(4, 5, g, a, capi.MOA_C64, b, None) == capi.MOA_ERR_SIZE
    assert G(1, 2, g, a, capi.MOA_C64, b, None) == capi.MOA_ERR_SIZE
    assert G(4, 2, (ctypes.c_int32 * 2)(1, 1), a, capi.MOA_C64, b, None) == capi.MOA_ERR_ARG
    assert G(4, 2, (ctypes.c_int32 * 2)(0, 4), a, capi.MOA_C64, b, None) == capi.MOA_ERR_ARG
    assert G(4, 2, g, a, 7, b, None) == capi.MOA_ERR_DTYPE
    assert G(4, 2, g, a, capi.MOA_C64, P((1 << 30) + 8), None) == capi.MOA_ERR_ARG


def test_block_diagonal_transpose_vector_is_the_inverse_of_the_printed_one():
    from paper_0803_2386_amd import hypercube
    for n, gated in [(4, [0, 2]), (4, [1, 2]), (6, [5, 0, 3]), (3, [0])]:
        printed = moa.gate_transpose_vector(n, gated)
        assert hypercube.block_diagonal_transpose_vector(n, gated) == moa.inverse_permutation(printed)


@pytest.mark.parametrize("n,lift,dtype,prec,lg_radix,want", [
    (1 << 16, [256, 256], capi.MOA_C64, 0, [3, 2], capi.MOA_OK),
    (1 << 16, [256, 256], capi.MOA_C64, 0, [5, 0], capi.MOA_OK),
    (1 << 20, None, capi.MOA_C64, 0, [5, 5], capi.MOA_OK),
    (1 << 14, None, capi.MOA_C64, 0, [2], capi.MOA_OK),
    (1 << 16, [256, 256], capi.MOA_C128, 0, [3, 0], capi.MOA_ERR_TUNING),     # complex128: radix 16 only
    (1 << 16, [256, 256], capi.MOA_C64, 2, [3, 0], capi.MOA_ERR_TUNING),      # split precision
    (1 << 8, [16, 16], capi.MOA_C64, 0, [2, 0], capi.MOA_ERR_TUNING),         # a level below 2^5 points
    (1 << 16, [256, 256], capi.MOA_C64, 0, [1, 0], capi.MOA_ERR_TUNING),      # radix 2 is not offered
    (1 << 16, [256, 256], capi.MOA_C64, 0, [6, 0], capi.MOA_ERR_TUNING),
    (1 << 16, [256, 256], capi.MOA_C64, 0, [4, 4], capi.MOA_OK),              # 4 = the default
])
def test_radix_tuning_validation(n, lift, dtype, prec, lg_radix, want):
    st = status_of(capi.moa_fft_plan, n, 1, lift, dtype=dtype, prec=prec, flags=HOST,
                   tuning={"lg_radix": lg_radix})
    assert st == want


def test_radix_schedule_in_describe():
    h = capi.moa_fft_plan(1 << 16, 2, [256, 256], flags=HOST, tuning={"lg_radix": [3, 5]})
    try:
        d = json.loads(capi.moa_fft_describe(h))
        p0, p1 = d["passes"]
        assert p0["lg_radix"] == 3 and p0["stage_lg_radices"] == [3, 3, 2]
        assert p1["lg_radix"] == 5 and p1["stage_lg_radices"] == [5, 3] and p1["points_per_thread"] == 32
        assert p1["kernel_mode"] == 1
    finally:
        capi.moa_fft_destroy(h)
    h = capi.moa_fft_plan(1 << 24, 1, [4096, 4096], flags=HOST)
    try:
        assert [p["stage_lg_radices"] for p in json.loads(capi.moa_fft_describe(h))["passes"]] == [[4, 4, 4]] * 2
    finally:
        capi.moa_fft_destroy(h)
    h = capi.moa_fft_plan(1 << 10, 1, None, flags=HOST)   # the short-transform kernel: radix 4
    try:
        assert json.loads(capi.moa_fft_describe(h))["passes"][0]["stage_lg_radices"] == [2] * 5
    finally:
        capi.moa_fft_destroy(h)
