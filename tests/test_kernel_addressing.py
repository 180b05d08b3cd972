"""CPU check of the pass kernel's launch geometry before it runs on a GPU.

Mirrors, in numpy, the address arithmetic of k_pass (block decode with the
XCD remap, thread -> (column, row) map, register slots, LDS slots) for every
block and thread of a plan, and checks that every global load and store
stays inside the buffer, that every output element is written exactly once,
and that every LDS slot fits the dynamic LDS the plan requests."""
import json

import numpy as np
import pytest

from paper_0803_2386_amd import capi

HOST = capi.MOA_FFT_FLAG_HOST_ONLY


def lg_e(lgn):
    return min(lgn, 4)


def pad(i):
    return i + (i >> 4)


def mfma_pad(i):
    """LDS padding of the split-precision paired-column levels: one more spare
    slot every 256 elements."""
    return i + (i >> 4) + (i >> 8)


def row_off(r, layout, stride):
    """Offset of row r of a DFT axis: blockwise when the layout has a block."""
    lg = layout["block_lg"]
    if lg >= 30:
        return r * stride
    return (r & ((1 << lg) - 1)) * stride + (r >> lg) * layout["stride_hi"]


def col_off(w, layout, stride0):
    """Offset of column w inside a tile: pairs at pair_stride, stride0 within a pair."""
    return (w >> 1) * layout["pair_stride"] + (w & 1) * stride0


def check_small(p, total, elem_bytes):
    """The short-transform kernel: one workgroup of N / 4 threads; thread b
    loads rows b + r N / 4 and the last stage stores the same rows; every
    LDS slot of every stage fits the requested LDS."""
    N = p["N"]
    B = total // N
    ax = p["batch_axes"]
    assert len(ax) == 1 and ax[0]["size"] == B and ax[0]["in_stride"] == ax[0]["out_stride"] == N
    assert p["grid"] == p["blocks"] == B and p["tile_width"] == 1 and total == N * B
    assert p["threads"] == N // 4 and p["points_per_thread"] == 4
    assert p["dft_axis"]["in_stride"] == 1 and p["dft_axis"]["out_stride"] == 1
    # workgroup k, thread b: element k N + b + r N / 4 on load and store
    b = np.arange(N // 4)
    rows = (np.arange(B)[:, None, None] * N + b[None, :, None] + np.arange(4)[None, None, :] * (N // 4)).ravel()
    assert np.array_equal(np.sort(rows), np.arange(total))
    slots = [pad(i) for s_ in small_stage_slots(N) for i in s_]
    # the exchange tile (N padded), then omega_N^e for e < N (N <= 256) or
    # the 256-entry in-block table
    table0 = N + (N >> 4)
    entries = N if N <= 256 else 256
    assert max(slots) < table0 and (table0 + entries) * elem_bytes == p["lds_bytes"] <= 160 * 1024


def small_stage_slots(N):
    """LDS rows each radix-4 stage of the short-transform kernel writes."""
    lg = N.bit_length() - 1
    b = np.arange(N // 4)
    out = []
    for s in range(lg // 2):
        if s + 1 == lg // 2 and lg % 2 == 0:
            break
        NS = 1 << (2 * s)
        base = ((b >> (2 * s)) << (2 * s + 2)) + (b & (NS - 1))
        out.append((base[:, None] + np.arange(4)[None, :] * NS).ravel())
    return out


def small_model(x, sign=-1):
    """numpy model of the short-transform kernel's arithmetic order: radix-4
    Stockham stages (input r of butterfly b is row b + r N / 4, factor
    omega_{4 NS}^((b mod NS) r), output r to (b / NS) 4 NS + (b mod NS) + r NS),
    then a radix-2 stage (rows c, c + N / 2, factor omega_N^c) when log2 N is
    odd."""
    N = x.size
    lg = N.bit_length() - 1
    Q = N // 4
    b = np.arange(Q)
    cur = x.astype(np.complex128)
    for s in range(lg // 2):
        NS = 1 << (2 * s)
        v = np.stack([cur[b + r * Q] for r in range(4)])
        k = b & (NS - 1)
        for r in range(1, 4):
            e = (k * r) << (lg - 2 * s - 2)  # index into the kernel's table of omega_N
            assert e.max() < N
            v[r] *= np.exp(sign * 2j * np.pi * e / N)
        X = np.stack([sum(v[q] * np.exp(sign * 2j * np.pi * q * r / 4) for q in range(4)) for r in range(4)])
        base = ((b >> (2 * s)) << (2 * s + 2)) + k
        nxt = np.empty_like(cur)
        for r in range(4):
            nxt[base + r * NS] = X[r]
        cur = nxt
    if lg % 2:
        c = np.arange(N // 2)
        t = cur[c + N // 2] * np.exp(sign * 2j * np.pi * c / N)
        cur = np.concatenate([cur[c] + t, cur[c] - t])
    return cur


@pytest.mark.parametrize("lg", range(4, 13))
def test_short_transform_model_is_the_dft(lg):
    """The short kernel's stage order and indices compute the DFT (both
    directions), for every size it serves."""
    rng = np.random.default_rng(lg)
    x = rng.uniform(-1, 1, 1 << lg) + 1j * rng.uniform(-1, 1, 1 << lg)
    assert np.abs(small_model(x) - np.fft.fft(x)).max() <= 1e-12 * (1 << lg)
    assert np.abs(small_model(x, +1) - np.fft.ifft(x) * x.size).max() <= 1e-12 * (1 << lg)


@pytest.mark.parametrize("n,dtype", [(16, capi.MOA_C64), (32, capi.MOA_C128), (1024, capi.MOA_C128),
                                     (2048, capi.MOA_C64), (2048, capi.MOA_C128), (4096, capi.MOA_C64)])
def test_short_transform_kernel_selected(n, dtype):
    """A short transform (up to 2^12 points complex64, 2^11 complex128) takes
    the latency kernel alone or in a batch of at most 2048 transforms and
    2^19 points; a larger batch, a lifted plan or a tuned tile width does
    not."""
    def modes(batch, lift=None, tuning=None):
        h = capi.moa_fft_plan(n, batch, lift, dtype=dtype, flags=HOST, tuning=tuning)
        try:
            return [q["kernel_mode"] for q in json.loads(capi.moa_fft_describe(h))["passes"]]
        finally:
            capi.moa_fft_destroy(h)
    assert modes(1) == [4]
    assert modes(2) == [4]
    big = min(2048, (1 << 19) // n)
    assert modes(big) == [4]
    assert 4 not in modes(2 * big)
    if dtype == capi.MOA_C128:
        h = capi.moa_fft_plan(4096, 1, None, dtype=dtype, flags=HOST)
        try:
            assert json.loads(capi.moa_fft_describe(h))["passes"][0]["kernel_mode"] != 4
        finally:
            capi.moa_fft_destroy(h)
    assert 4 not in modes(1, [4, n // 4])
    assert 4 not in modes(1, tuning={"cols_per_block": [1]})


def check_pass(p, total, elem_bytes):
    N = p["N"]
    if p["kernel_mode"] == 4:
        return check_small(p, total, elem_bytes)
    mfma = p["mfma"] != "none"
    pair = p["kernel_mode"] == 3
    E = min(N, p["points_per_thread"]) if not mfma else 1
    if pair:
        # each thread owns two adjacent columns, 16 points of each, on 1024 threads
        E = 16
    TPC = N // E
    W = p["tile_width"]
    T = p["threads"]
    if pair:
        lgn = N.bit_length() - 1
        assert elem_bytes == 8 and W * N == 1 << 15
        assert T == (W // 2) * TPC == 1024
        if mfma:
            assert lgn in (8, 12)
        else:
            assert 12 <= lgn <= 14 and (p["in_tile_fast"] or p["out_tile_fast"])
    elif mfma:
        # 32 points a thread, copied in and out over i = t + m T
        assert T * 32 == W * N and T % 64 == 0 and T <= 512
        T = W * N  # check the full (column, row) set below
    else:
        assert T == W * TPC and T <= (1024 if p["kernel_mode"] == 2 else 512)
    axes = p["batch_axes"]
    nd = len(axes)
    blocks = p["blocks"]
    bid = np.arange(blocks, dtype=np.int64)
    if p["xcd_remap"] and p["grid"] == blocks:
        # one tile per workgroup: the remap must be a permutation of the tiles
        assert blocks % 8 == 0
        bid = (bid & 7) * (blocks >> 3) + (bid >> 3)
        assert np.array_equal(np.sort(bid), np.arange(blocks))
    elif p["xcd_remap"]:
        # persistent grid: XCD x walks tiles [x*chunk, (x+1)*chunk) with the
        # grid/8 workgroups it holds; together they must cover every tile once
        G = p["grid"]
        assert G % 8 == 0
        chunk = (blocks + 7) // 8
        seen = []
        for b in range(G):
            x, lw = b & 7, b >> 3
            seen.extend(range(x * chunk + lw, min(blocks, (x + 1) * chunk), G // 8))
        assert sorted(seen) == list(range(blocks))
    if nd == 1:
        tile, rest = bid, np.zeros_like(bid)
        assert blocks * W == axes[0]["size"]
    else:
        lg_tiles = (axes[0]["size"] // W).bit_length() - 1
        tile, rest = bid & ((1 << lg_tiles) - 1), bid >> lg_tiles
    ib = tile * p["in_layout"]["tile_stride"]
    ob = tile * p["out_layout"]["tile_stride"]
    assert p["in_layout"]["tile_stride"] == W * axes[0]["in_stride"] or pair
    assert p["out_layout"]["tile_stride"] == W * axes[0]["out_stride"] or pair
    for d in range(1, nd):
        if d == nd - 1:
            idx = rest
            assert idx.max() < axes[d]["size"]
        else:
            lg = axes[d]["size"].bit_length() - 1
            idx, rest = rest & ((1 << lg) - 1), rest >> lg
        ib = ib + idx * axes[d]["in_stride"]
        ob = ob + idx * axes[d]["out_stride"]
    t = np.arange(T)
    if pair:
        # pair index fastest on a unit-stride side (the FP32 kernel uses that
        # map on both sides), row fastest on the other side of a matrix-core
        # level; columns 2u and 2u + 1
        P = W // 2
        if mfma and not p["in_tile_fast"]:
            j, u = t % TPC, t // TPC
        else:
            u, j = t % P, t // P
        w = np.concatenate([2 * u, 2 * u + 1])
        j = np.concatenate([j, j])
    elif p["in_tile_fast"]:
        w, j = t % W, t // W
    else:
        j, w = t % TPC, t // TPC
    m = np.arange(E)
    # loads: block x thread x slot
    rows = j[:, None] + m[None, :] * TPC
    lane_in = (col_off(w, p["in_layout"], axes[0]["in_stride"])[:, None]
               + row_off(rows, p["in_layout"], p["dft_axis"]["in_stride"]))
    load = ib[:, None, None] + lane_in[None, :, :]
    assert load.min() >= 0 and load.max() < total
    if pair:
        # 32-bit lane byte offsets, and 16-byte alignment on a unit-stride side
        lane_out = (col_off(w, p["out_layout"], axes[0]["out_stride"])[:, None]
                    + row_off(rows, p["out_layout"], p["dft_axis"]["out_stride"]))
        assert lane_in.max() * 8 < 1 << 32 and lane_out.max() * 8 < 1 << 32
        even = slice(0, T)
        if p["in_tile_fast"]:
            assert np.all(load[:, even, :] % 2 == 0)
        if p["out_tile_fast"]:
            st = ob[:, None, None] + lane_out[None, :, :]
            assert np.all(st[:, even, :] % 2 == 0)
            assert st.min() >= 0 and st.max() < total
    # stores: every (column, k) of every block
    k = np.arange(N)
    ww = np.arange(W)
    store = (ob[:, None, None] + col_off(ww, p["out_layout"], axes[0]["out_stride"])[None, :, None]
             + row_off(k, p["out_layout"], p["dft_axis"]["out_stride"])[None, None, :])
    assert store.min() >= 0 and store.max() < total
    flat = np.sort(store.ravel())
    assert flat.size == total and np.array_equal(flat, np.arange(total)), "outputs not a permutation"
    # LDS slots
    cs = p["lds_col_stride"]
    top = ((W // 2 if pair else W) - 1) * cs + (mfma_pad(N - 1) if mfma and pair else pad(N - 1))
    assert (top + 1) * elem_bytes <= p["lds_bytes"] <= 160 * 1024


@pytest.mark.parametrize("n,batch,lift,dtype", [
    (1 << 24, 1, [4096, 4096], capi.MOA_C64),
    (1 << 16, 256, [256, 256], capi.MOA_C64),
    (1 << 20, 8, [256, 4096], capi.MOA_C64),
    (1 << 10, 1, None, capi.MOA_C128),
    (1 << 16, 3, [16, 16, 256], capi.MOA_C64),
    (2048, 2, [2, 4, 2, 8, 16], capi.MOA_C64),
    (1, 3, None, capi.MOA_C64), (2, 5, None, capi.MOA_C128), (64, 7, None, capi.MOA_C64),
    (1 << 14, 2, None, capi.MOA_C64), (1 << 13, 3, None, capi.MOA_C128), (1 << 15, 1, None, capi.MOA_C64),
    (1 << 18, 1, [64, 4096], capi.MOA_C64), (4096, 1, [256, 16], capi.MOA_C128),
    (1 << 20, 2, [4096, 256], capi.MOA_C64), (1 << 16, 4, [16, 4096], capi.MOA_C64),
    (1 << 21, 1, [8192, 256], capi.MOA_C64), (1 << 22, 1, [16384, 256], capi.MOA_C64),
    (1 << 21, 1, [256, 8192], capi.MOA_C64),
    (16, 1, None, capi.MOA_C64), (32, 1, None, capi.MOA_C128), (2048, 1, None, capi.MOA_C64),
    (4096, 1, None, capi.MOA_C128), (2048, 1, None, capi.MOA_C128), (256, 1, None, capi.MOA_C64),
    (512, 1, None, capi.MOA_C128), (16, 2048, None, capi.MOA_C64), (1024, 7, None, capi.MOA_C128),
    (4096, 128, None, capi.MOA_C64),
    # default lifts and wide far-writing tiles beyond the Infinity Cache
    (1 << 20, 1, None, capi.MOA_C64), (1 << 20, 17, None, capi.MOA_C64), (1 << 25, 1, None, capi.MOA_C64),
    (1 << 23, 2, None, capi.MOA_C64),
    (1 << 23, 1, None, capi.MOA_C128), (1 << 22, 8, [1024, 4096], capi.MOA_C64),
    (1 << 21, 16, [512, 4096], capi.MOA_C64), (1 << 23, 4, [2048, 4096], capi.MOA_C64),
    (1 << 22, 4, [1024, 4096], capi.MOA_C128),
])
def test_pass_kernel_geometry(n, batch, lift, dtype):
    h = capi.moa_fft_plan(n, batch, lift, dtype=dtype, flags=HOST)
    _check_plan(h, n, batch, dtype)


@pytest.mark.parametrize("n,lift", [(1 << 24, [4096, 4096]), (1 << 21, [8192, 256]), (1 << 22, [16384, 256]),
                                    (1 << 21, [256, 8192]), (1 << 18, [64, 4096])])
def test_paired_columns_selected(n, lift):
    """Complex64 levels of 2^12..2^14 points with a unit-stride tile side use
    the paired-column kernel with 2^15 / N columns a tile; others do not."""
    h = capi.moa_fft_plan(n, 1, lift, flags=HOST)
    try:
        d = json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)
    assert any(p["kernel_mode"] == 3 for p in d["passes"])
    for p in d["passes"]:
        big = 1 << 12 <= p["N"] <= 1 << 14
        tf = p["batch_axes"][0]["in_stride"] == 1 or p["batch_axes"][0]["out_stride"] == 1
        assert (p["kernel_mode"] == 3) == (big and tf)
        if p["kernel_mode"] == 3:
            assert p["tile_width"] * p["N"] == 1 << 15 and p["threads"] == 1024


@pytest.mark.parametrize("prec", [capi.MOA_FFT_PREC_SPLIT_BF16, capi.MOA_FFT_PREC_SPLIT_FP16])
@pytest.mark.parametrize("n,batch,lift", [(1 << 20, 4, [256, 4096]), (256, 64, None), (4096, 4, None),
                                          (1 << 16, 2, [16, 4096]), (1 << 16, 2, [256, 256]),
                                          (1 << 12, 3, [16, 256]), (1 << 20, 2, [256, 4096])])
def test_mfma_pass_geometry(n, batch, lift, prec):
    h = capi.moa_fft_plan(n, batch, lift, prec=prec, flags=HOST)
    d = _check_plan(h, n, batch, capi.MOA_C64)
    for p in d["passes"]:
        if p["mfma"] != "none":
            per_thread = 32
            assert p["threads"] % 64 == 0 and p["threads"] == p["tile_width"] * p["N"] // per_thread


def _check_plan(h, n, batch, dtype):
    try:
        d = json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)
    eb = 8 if dtype == capi.MOA_C64 else 16
    for p in d["passes"]:
        check_pass(p, n * batch, eb)
    return d


@pytest.mark.parametrize("cols", [1, 2, 4, 8, 16, 32, 64])
def test_tuned_geometry(cols):
    try:
        h = capi.moa_fft_plan(1 << 16, 4, [256, 256], flags=HOST, tuning=dict(cols_per_block=[cols, cols]))
    except capi.MoaError as e:
        assert e.status == capi.MOA_ERR_TUNING
        return
    try:
        d = json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)
    for p in d["passes"]:
        check_pass(p, 4 << 16, 8)


def test_batched_task_geometry():
    from paper_0803_2386_amd import inputs
    sizes = [int(s) for s in inputs.uneven_sizes(8192, 6, 14, seed=0)] + [1, 2, 4, 8, 16, 32]
    h = capi.moa_fft_plan_batched(sizes, flags=HOST)
    try:
        d = json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)
    # every task fits the workgroup and the LDS the launch requests: up to
    # 2^13 points at 16 a thread (one transform a thread below 16 points), a
    # 2^14-point transform as its two 2^13-point halves, on 512 threads; two
    # workgroups fit one CU
    assert d["threads"] == 512 and 2 * d["lds_bytes"] <= 160 * 1024
    for g in d["sizes_by_task_group"]:
        N = g["n"]
        lgn = N.bit_length() - 1
        Nt = min(N, 1 << 13)
        TPC = Nt >> min(Nt.bit_length() - 1, 4)
        base = Nt + (Nt >> 4)
        cs = base if TPC >= 16 else base + ((TPC - (base & 31) + 32) & 31)
        per = 1 if lgn == 14 else 512 // TPC
        assert per * min(Nt, 16) <= (1 << 13)
        if lgn > 4:  # more than one register stage: LDS exchange tile
            assert per * cs * 8 + 256 * 8 <= d["lds_bytes"]
        assert g["tasks"] == -(-sizes.count(N) // per)
    assert d["tasks"] == sum(g["tasks"] for g in d["sizes_by_task_group"])


@pytest.mark.parametrize("lgn", [4, 8, 12])
def test_mfma_pair_stage_indexing(lgn):
    """numpy mirror of the in-place radix-16 stages of the paired-column
    matrix-core kernel: the columns enter LDS in base-16 digit-reversed order;
    stage s, butterfly b (block b >> 4s, j = b mod 16^s) reads padded slots
    pad(base) + r * pstep, multiplies input r by omega_{16^(s+1)}^(j r) and
    writes output k to pad(base) + k * pstep; after the last stage slot k holds
    X[k].  Checks the slot sets (each slot read and written once a stage, the
    padded step equals pad(base + r 16^s) - pad(base)), the lane split of the
    16x16x32 operands (lane group g reads inputs 4g..4g+3 and writes outputs
    2g, 2g+1, 8+2g, 9+2g) and the result against numpy's FFT."""
    N = 1 << lgn
    nst, nb = lgn // 4, N // 16

    def rev16(p):
        r = 0
        for _ in range(nst):
            r, p = (r << 4) | (p & 15), p >> 4
        return r

    rng = np.random.default_rng(lgn)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    slots = np.zeros(pad(N - 1) + 1, complex)
    for p in range(N):
        slots[pad(rev16(p))] = x[p]
    F16 = np.exp(-2j * np.pi * np.outer(np.arange(16), np.arange(16)) / 16)
    for s in range(nst):
        ns = 1 << (4 * s)
        pstep = 1 if s == 0 else ns + (ns >> 4)
        read = np.zeros_like(slots, dtype=int)
        written = np.zeros_like(slots, dtype=int)
        new = slots.copy()
        for b in range(nb):
            j = b & (ns - 1)
            base = ((b >> (4 * s)) << (4 * s + 4)) + j
            pb = pad(base)
            for r in range(16):
                assert pad(base + r * ns) == pb + r * pstep
            idx = pb + np.arange(16) * pstep
            # lane group g holds inputs 4g..4g+3 and outputs {2g, 2g+1, 8+2g, 9+2g}
            ins = sorted(4 * g + i for g in range(4) for i in range(4))
            outs = sorted(q for g in range(4) for q in (2 * g, 2 * g + 1, 8 + 2 * g, 9 + 2 * g))
            assert ins == list(range(16)) and outs == list(range(16))
            read[idx] += 1
            written[idx] += 1
            xin = slots[idx] * np.exp(-2j * np.pi * j * np.arange(16) / (16 * ns))
            new[idx] = F16 @ xin
        used = np.array([pad(i) for i in range(N)])
        assert np.all(read[used] == 1) and np.all(written[used] == 1)
        slots = new
    got = np.array([slots[pad(k)] for k in range(N)])
    assert np.abs(got - np.fft.fft(x)).max() < 1e-9 * N


def _rev16(p, nst):
    r = 0
    for _ in range(nst):
        r = (r << 4) | (p & 15)
        p >>= 4
    return r


def _cycle_pairs_distinct(slots):
    """8-byte LDS accesses of one wave instruction: each run of 16 lanes (one
    LDS cycle) on 16 distinct bank pairs (slot mod 16)."""
    a = np.asarray(slots).reshape(4, 16) % 16
    return all(len(set(r.tolist())) == 16 for r in a)


@pytest.mark.parametrize("n,lift", [(1 << 20, [256, 4096]), (1 << 16, [16, 4096]), (1 << 16, [256, 256])])
def test_mfma_pair_lds_banks(n, lift):
    """Every LDS access of the split-precision paired-column levels (the tile
    scatter in digit-reversed order, the register-fused stages 0 and 1, the
    in-place stages from 2 on, the natural-order readback) puts the 16 lanes
    of each LDS cycle on distinct bank pairs, with the planned column stride.
    Lane (g, c) = (lane / 16, lane % 16) of the matrix-core operand layout."""
    h = capi.moa_fft_plan(n, 2, lift, prec=capi.MOA_FFT_PREC_SPLIT_FP16, flags=HOST)
    d = _check_plan(h, n, 2, capi.MOA_C64)
    seen = 0
    for p in d["passes"]:
        if p["mfma"] == "none" or p["kernel_mode"] != 3:
            continue
        seen += 1
        N = p["N"]
        lgn = N.bit_length() - 1
        NB, TPC, P, nst = N // 16, N // 16, (1 << 14) // N, lgn // 4
        cs = p["lds_col_stride"]
        assert cs >= mfma_pad(N - 1) + 1
        for wave in range(16):
            t = wave * 64 + np.arange(64)
            for tin in (False, True):
                u = (t & (P - 1)) if tin else (t >> (lgn - 4))
                j = (t >> (14 - lgn)) if tin else (t & (TPC - 1))
                for m in range(16):
                    assert _cycle_pairs_distinct([u[k] * cs + mfma_pad(_rev16(int(j[k]) + m * TPC, nst))
                                                  for k in range(64)])
                    assert _cycle_pairs_distinct(u * cs + mfma_pad(j + m * TPC))
            g, c = np.arange(64) // 16, np.arange(64) % 16
            for grp in range(4):
                gb = (wave * 4 + grp) * 16
                col = (gb >> (lgn - 4)) * cs
                b0 = gb & (NB - 1)
                for i in range(4):
                    assert _cycle_pairs_distinct(col + mfma_pad(16 * (b0 + c) + 4 * g + i))
                    assert _cycle_pairs_distinct(col + mfma_pad(16 * b0 + 4 * g + i + 16 * c))
                    for s in range(2, nst):
                        ns = 16 ** s

                        def slot(bf, r):
                            b = bf & (NB - 1)
                            return col + mfma_pad(((b // ns) * ns * 16) + (b % ns) + r * ns)
                        assert _cycle_pairs_distinct(slot(gb + c, 4 * g + i))
                        assert _cycle_pairs_distinct(slot(gb + 4 * g + i, c))
    assert seen >= 1


@pytest.mark.parametrize("n,batch,lift,widths", [
    # 256-point levels: 16 columns (128-byte runs); 64 columns where the rows
    # read lie 32 KB apart and 2^28 points leave 16384 tiles of 2^14
    (1 << 16, 256, [256, 256], [16, 16]),
    (1 << 20, 256, [4096, 256], [64, 8]),
    (1 << 16, 1024, [256, 256], [64, 16]),   # rows 2 KB apart, 2^26 points: 64 columns too
    (1 << 18, 256, [512, 512], [16, 16]),    # (512-point levels keep 16)
    (1 << 20, 16, [4096, 256], [16, 8]),     # 2^24 points: 1024 tiles of 2^14, too few
    (1 << 20, 256, [256, 4096], [8, 32]),    # rows written 32 KB apart, 2^28 points: 32 columns
    (1 << 20, 32, [256, 4096], [8, 16]),     # 256 points: 32 columns from 2^26 points only
    (1 << 24, 1, [256, 256, 256], [16, 16, 16]),
    (1 << 24, 4, [256, 256, 256], [64, 64, 32]),
    # 1024- and 2048-point levels: 128-byte runs up to 2^14 points a tile
    (1 << 20, 16, [1024, 1024], [16, 16]),
    (1 << 22, 4, [2048, 2048], [8, 8]),
    (1 << 18, 64, [512, 512], [16, 16]),
    (1 << 18, 64, [4096, 64], [64, 8]),      # 64-point levels: 2^12 points, 64 columns
    (1 << 21, 8, [512, 4096], [8, 8]),       # writing rows 32 KB apart only: 2^12 points
    (1 << 22, 4, [1024, 4096], [8, 4]),
    (1 << 21, 128, [512, 4096], [8, 16]),    # ... beyond the Infinity Cache: 128-byte runs, 2^13..2^14 points
    (1 << 22, 64, [1024, 4096], [8, 16]),
    (1 << 23, 32, [2048, 4096], [8, 8]),
    (1 << 21, 16, [512, 4096], [8, 16]),     # 2^25 points
    (1 << 22, 8, [1024, 4096], [8, 16]),
    (1 << 23, 4, [2048, 4096], [8, 8]),
    (1 << 30, 1, [1024, 1024, 1024], [16, 16, 16]),
    (1 << 24, 1, [4096, 4096], [8, 8]),      # paired columns
])
def test_default_tile_widths(n, batch, lift, widths):
    """The planner's default tile of a complex64 level with a unit-stride
    tile side: at least 128-byte runs (a level that only writes along the
    tile, rows 32 KB or more apart, keeps 2^12 points; from 2^25 points
    (2^26 at 256 points) 2^13 points and at least 128-byte runs up to 2^14
    points), 512-byte runs where
    the rows read lie 16 KB or more apart (or, at 256 points, once the level
    holds 2^26 points) and at least 2048 tiles of 2^14 points remain."""
    h = capi.moa_fft_plan(n, batch, lift, flags=HOST)
    try:
        d = json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)
    assert [p["tile_width"] for p in d["passes"]] == widths


@pytest.mark.parametrize("n,batch,lift,widths", [
    (1 << 20, 8, [1024, 1024], [8, 4]),      # read side: the largest tile, 2^13 points
    (1 << 18, 32, [512, 512], [16, 4]),
    (1 << 16, 128, [256, 256], [32, 8]),
    (1 << 22, 2, [2048, 2048], [4, 4]),
    (1 << 20, 8, [256, 4096], [2, 8]),       # write side only: 2^11 points
    (1 << 22, 2, [1024, 4096], [2, 4]),      # ... 64-byte runs, up to 128 MiB
    (1 << 22, 4, [1024, 4096], [2, 8]),      # from 256 MiB: 128-byte runs
    (1 << 21, 8, [512, 4096], [2, 8]),
    (1 << 23, 4, [2048, 4096], [2, 4]),      # (2^13 points at most)
    (1 << 20, 32, [256, 4096], [2, 8]),
    (1 << 18, 256, [512, 512], [16, 8]),     # rows 8 KB apart, 1 GiB: 128-byte runs too
    (1 << 20, 64, [1024, 1024], [8, 8]),
    (1 << 20, 8, [1024, 1024], [8, 4]),      # 128 MiB: 64-byte runs
])
def test_default_tile_widths_c128(n, batch, lift, widths):
    """Complex128 levels reading along a unit-stride tile side take the
    largest tile (2^13 points); write-side tiles keep 2^11 points and 64-byte
    runs, and 128-byte runs from 256 MiB at 512 .. 2048 points, whatever the
    spacing of the rows they write."""
    h = capi.moa_fft_plan(n, batch, lift, capi.MOA_C128, flags=HOST)
    try:
        d = json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)
    assert [p["tile_width"] for p in d["passes"]] == widths


@pytest.mark.parametrize("n,batch,lift", [(1 << 20, 16, [1024, 1024]), (1 << 16, 256, [256, 256]),
                                          (1 << 24, 1, [256, 256, 256]), (1 << 22, 64, [1024, 4096]),
                                          (1 << 21, 8, [512, 4096])])
def test_store_readback_across_columns_is_bank_conflict_free(n, batch, lift):
    """A level that reads along its columns and stores along its tile (up to
    16 columns, 16 or more threads a column) reads the LDS back across the
    columns before the store: lane t takes column t mod W, row t / W + m TPC.
    Each run of 16 lanes (one LDS cycle of 8-byte accesses) lands on 16
    distinct bank pairs with the planned column stride."""
    h = capi.moa_fft_plan(n, batch, lift, flags=HOST)
    try:
        d = json.loads(capi.moa_fft_describe(h))
    finally:
        capi.moa_fft_destroy(h)
    seen = 0
    for p in d["passes"]:
        W, N = p["tile_width"], p["N"]
        if p["in_tile_fast"] or not p["out_tile_fast"] or p["kernel_mode"] not in (0, 1, 2) or W > 16:
            continue
        TPC = N // p["points_per_thread"]
        if TPC < 16:
            continue
        seen += 1
        cs, lgw = p["lds_col_stride"], W.bit_length() - 1
        t = np.arange(p["threads"])
        wst, jst = t & (W - 1), t >> lgw
        for m in range(p["points_per_thread"]):
            slots = wst * cs + np.array([pad(int(r)) for r in jst + m * TPC])
            for c in range(0, len(t), 16):
                assert len(set((slots[c:c + 16] % 16).tolist())) == 16, (p["level"], m, c)
    assert seen >= 1


def test_nd_axis_tiles_widen_beyond_the_infinity_cache():
    """The 256-point axes of a 3-D transform of 2^26 points read 512-byte
    runs (64 columns) like the one-dimensional levels; below 2^26 points
    they keep 128-byte runs."""
    for batch, want in ((4, [16, 64, 64]), (1, [16, 16, 16])):
        h = capi.moa_fft_plan_nd([256, 256, 256], batch, flags=HOST)
        try:
            d = json.loads(capi.moa_fft_describe(h))
        finally:
            capi.moa_fft_destroy(h)
        assert [p["tile_width"] for p in d["passes"]] == want, batch
