// C ABI of the dimension-lifted FFT: validation, lowering of a lift to pass
// descriptors (the psi-calculus layer), twiddle tables, device resources and
// execution.  All host code; kernels live in the .hip files.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <unordered_set>
#include <vector>

#include "../../include/moa_fft.h"
#include "fft_internal.h"
#include "fft_mfma_layout.h"
#include "psi.hpp"

using moa::BatchTask;
using moa::PassDesc;
namespace psi = moa::psi;

namespace {

constexpr uint32_t kMagic = 0x4d4f4146u;  // "MOAF"
constexpr int kLgMaxN = 30;
constexpr uint32_t kKnownFlags =
    MOA_FFT_FLAG_HOST_ONLY | MOA_FFT_FLAG_PER_SIZE | MOA_FFT_FLAG_GRAPH | MOA_FFT_FLAG_NO_WORKSPACE;

bool is_pow2(int64_t x) { return x >= 1 && (x & (x - 1)) == 0; }
int lg2(int64_t x)
{
    int t = 0;
    while ((int64_t(1) << t) < x) ++t;
    return t;
}

// omega_L^e = exp(-2 pi i e / L) in float64 from the exact integer exponent:
// the quarter turn q = floor(4 e / L) is split off in integers, the rest is
// an angle in [0, pi/2) whose cosine and sine are then rotated by q.
void root_fp64(int64_t e, int64_t L, double* c, double* s)
{
    e %= L;
    if (e < 0) e += L;
    const int64_t q = (4 * e) / L;           // quadrant
    const int64_t r = 4 * e - q * L;          // remainder, in units of 1/(4L) turn
    const double a = (M_PI / 2.0) * double(r) / double(L);
    double cr = cos(a), sr = sin(a);
    double cc, ss;  // cos, sin of the full angle 2 pi e / L
    switch (q) {
        case 0: cc = cr; ss = sr; break;
        case 1: cc = -sr; ss = cr; break;
        case 2: cc = -cr; ss = -sr; break;
        default: cc = sr; ss = -cr; break;
    }
    *c = cc;
    *s = -ss;  // forward root: exp(-i theta)
}

struct GraphEntry {
    int dir;
    const void* in;
    void* out;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

struct moa_fft_plan_s {
    uint32_t magic = kMagic;
    bool batched = false;
    bool host_only = false;
    bool fp64 = false;
    int prec = MOA_FFT_PREC_NATIVE;
    uint32_t flags = 0;
    int64_t n = 0, batch = 0, total = 0;  // total = complex elements per buffer
    std::vector<int64_t> lift;            // as given: outermost first
    std::vector<int64_t> levels;          // f_0 (innermost, first pass) ...
    std::vector<int64_t> dims;            // multi-dimensional plan: the array shape (row-major); empty for 1-D
    std::vector<PassDesc> passes;
    // uneven batch
    std::vector<int64_t> sizes;
    std::vector<BatchTask> tasks;
    std::vector<int64_t> toff;
    std::vector<std::pair<int, int>> size_ranges;  // (first task, tasks) per distinct size
    int batch_threads = 0, batch_lds = 0, batch_grid = 0, batch_data_elems = 0;
    int batch_task_lg = 13;  // log2 of the most points a task packs
    // tables: element offsets in d_tables (units of one complex element)
    std::vector<double> tab_host;  // interleaved re/im, float64
    int64_t tw_blk_off = 0;
    // device resources
    void* d_tables = nullptr;
    void* d_ws = nullptr;
    size_t ws_bytes = 0;
    void* d_tasks = nullptr;
    void* d_toff = nullptr;
    int device = -1;
    int cus = 256;                 // compute units of the device (for persistent grids)
    bool stream = false;           // streaming access to data touched once (see moa_fft_tuning_t)
    std::vector<GraphEntry> graphs;
    std::mutex mu;
};

namespace {

size_t elem_bytes(bool fp64) { return fp64 ? 16 : 8; }
int max_lg_block(bool fp64) { return fp64 ? moa::kMaxLgBlockC128 : moa::kMaxLgBlockC64; }
int max_threads(bool) { return moa::kMaxThreads; }

// Append omega_L^e for e in [first, first + count) scaled by `step` to the
// host table; returns the element offset of the first entry.
int64_t add_table(moa_fft_plan_s* p, int64_t L, int64_t count, int64_t step)
{
    const int64_t off = int64_t(p->tab_host.size() / 2);
    p->tab_host.reserve(p->tab_host.size() + size_t(2 * count));
    for (int64_t e = 0; e < count; ++e) {
        double c, s;
        root_fp64(e * step, L, &c, &s);
        p->tab_host.push_back(c);
        p->tab_host.push_back(s);
    }
    return off;
}

int lgE(int lgn, int lge) { return lgn < lge ? lgn : lge; }

// Fill launch fields of a pass: tile width, mapping, LDS tile, grid.
// Matrix-core levels use one thread per 16 points like the VALU kernel, and
// need whole waves: at least 1024 points per workgroup.
moa_status_t finish_pass(PassDesc& d, bool fp64, int want_w, int cus)
{
    const int lgn = d.lgn;
    // A register radix other than 16 runs the level kernel's other-radix
    // instantiations: complex64, 2^5 .. 2^14 points, radix 4, 8 or 32.
    if (d.lgrad == moa::kLgRadixDefault) d.lgrad = 0;
    const bool other_radix = d.lgrad != 0;
    if (other_radix && (fp64 || d.mfma || lgn < 5 || lgn > moa::kMaxLgBlockC64 ||
                        (d.lgrad != 2 && d.lgrad != 3 && d.lgrad != 5)))
        return MOA_ERR_TUNING;
    const int maxT = max_threads(fp64);
    // Points per thread: 16, or 32 when 16 would need more than maxT threads
    // (complex64 only); the matrix-core kernel always holds 32.
    const bool in_tf = (d.in_s[0] == 1 && d.in_s_e != 1);
    const bool out_tf = (d.out_s[0] == 1 && d.out_s_k != 1);
    // Level-kernel variant for a tile of 2^(lgn+lgw) points: 16 points a
    // thread up to 512 threads (mode 0); beyond, 32 points a thread when the
    // level stores in its load pattern (mode 1), else 16 points a thread on
    // up to 1024 threads (mode 2).
    auto big = [&](int lgw) { return ((int64_t(1) << (lgn + lgw)) >> 4) > maxT; };
    auto kmode_for = [&](int lgw) {
        const bool tf = lgw > 0;
        // Radix 32 needs 32 points a thread: mode 1 (a level that stores in
        // its load pattern).
        if (d.lgrad == 5) return ((tf && in_tf) == (tf && out_tf)) ? 1 : -1;
        if (d.mfma || fp64 || !big(lgw)) return 0;
        return ((tf && in_tf) == (tf && out_tf)) ? 1 : 2;
    };
    auto lge_for = [&](int lgw) {
        if (d.mfma) return 5;
        return kmode_for(lgw) == 1 ? 5 : 4;
    };
    auto maxT_for = [&](int lgw) { return kmode_for(lgw) == 2 ? 1024 : (kmode_for(lgw) < 0 ? 0 : maxT); };
    auto tpc_for = [&](int lgw) { return 1 << (lgn - lgE(lgn, lge_for(lgw))); };
    const int min_lgw = d.mfma ? std::max(0, 11 - lgn) : 0;
    // A lone digit 0 may have any size: its tiles must divide it.
    int lg0 = d.lg[0];
    if (d.nd == 1) {
        lg0 = 0;
        while ((d.size[0] % (int64_t(2) << lg0)) == 0) ++lg0;
    }
    const int eb = int(elem_bytes(fp64));
    const int table_bytes = (moa::kTwBlkEntries + 256 * d.tw_parts + (d.mfma ? moa::kMfmaScaleElems : 0)) * eb;
    auto lds_for = [&](int lgw, bool tile_fast) {
        const int W = 1 << lgw;
        int lanes = tile_fast ? (W >= 16 ? 1 : 16 / W) : tpc_for(lgw);
        // A level that reads along its columns but stores along its tile
        // reads the LDS back across the columns before the store.  With 16
        // threads or more a column no LDS cycle of the stages spans two
        // columns, so up to 16 columns the stride serves that readback
        // instead (a stride of 16 slots put all 16 lanes of a cycle on one
        // bank pair): <1024 1024> x 16 0.129 against 0.134 ms, <1024 4096>
        // x 64 1.97 against 2.06 ms, <256 256 256> 0.141 against 0.144 ms.
        // (32 columns of 256 points ran 1 % slower so; complex128 levels,
        // 16-byte lanes, showed no difference and keep the former stride.)
        if (!fp64 && !tile_fast && out_tf && lgw > 0 && lgw <= 4 && tpc_for(lgw) >= 16)
            lanes = W >= 16 ? 1 : 16 / W;
        const int cs = moa::lds_col_stride(1 << lgn, lanes);
        return std::make_pair(cs, W * cs * eb + table_bytes);
    };
    // The matrix-core kernel always runs 32 points a thread (W N / 32 threads).
    auto threads_for = [&](int lgw) -> int64_t {
        if (d.mfma) return (int64_t(1) << (lgn + lgw)) >> 5;
        return (int64_t(1) << lgw) * tpc_for(lgw);
    };
    auto threads_ok = [&](int lgw) { return threads_for(lgw) <= maxT_for(lgw); };
    // Paired-column kernel (fft_pair.hip): a complex64 level of 2^12 .. 2^14
    // points with a unit-stride tile side keeps a tile of 2^(15-lgn) columns
    // in VGPRs (twice the LDS-bound width: 64-byte runs at N = 4096), moving
    // column pairs with 16-byte accesses.  It needs even strides on every
    // axis but digit 0 (so those accesses stay aligned), per-tile spans
    // below 2^32 bytes (32-bit lane offsets), at most 7 inter-level parts and
    // an inter-level root of at most 2^32 (32-bit exponents).
    // The split-precision matrix-core levels of 2^8 and 2^12 points use the
    // same tile in their own kernel (fft_mfma.hip), with any sides.
    auto pair_ok = [&](int lgw_) {
        if (fp64) return false;
        if (d.mfma ? (lgn != 8 && lgn != 12) : (lgn < 12 || lgn > 14 || !(in_tf || out_tf))) return false;
        if (lgw_ != 15 - lgn || lgw_ > lg0) return false;
        if (d.tw && (d.tw_parts > 7 || d.tw_lgroot > 32)) return false;
        const int64_t w1 = (int64_t(1) << lgw_) - 1, n1 = (int64_t(1) << lgn) - 1;
        if (w1 * d.in_s[0] + n1 * d.in_s_e >= (int64_t(1) << 29)) return false;
        if (w1 * d.out_s[0] + n1 * d.out_s_k >= (int64_t(1) << 29)) return false;
        if ((in_tf && d.in_s_e % 2) || (out_tf && d.out_s_k % 2)) return false;
        for (int i = 1; i < d.nd; ++i)
            if ((in_tf && d.in_s[i] % 2) || (out_tf && d.out_s[i] % 2)) return false;
        return true;
    };
    // One short transform (a single level, unit strides) is one workgroup
    // whatever the kernel, so its time is that workgroup's critical path:
    // the latency kernel (fft_small.hip) spreads it over N / 4 threads of 4
    // points, radix-4 stages.  A small batch of them runs one such workgroup
    // per transform.
    if (want_w <= 0 && !other_radix && !d.mfma && !d.tw && d.pre_lg == 0 && d.nd == 1 &&
        d.size[0] <= moa::kSmallMaxBatch &&
        (d.size[0] << lgn) <= (int64_t(1) << moa::kLgSmallMaxPoints) &&
        d.in_s_e == 1 && d.out_s_k == 1 && d.in_s[0] == (int64_t(1) << lgn) && d.out_s[0] == (int64_t(1) << lgn) &&
        lgn >= moa::kLgSmallMin && lgn <= (fp64 ? moa::kLgSmallMaxC128 : moa::kLgSmallMax)) {
        d.lgw = 0;
        d.lge = 2;
        d.kmode = 4;
        d.in_tile_fast = d.out_tile_fast = false;
        d.col_stride = moa::lds_padded_len(1 << lgn);
        d.data_elems = d.col_stride;
        d.lds_bytes = (d.data_elems + moa::small_table_entries(lgn)) * eb;  // exchange tile, then twiddles
        d.threads = 1 << (lgn - 2);
        d.blocks = d.size[0];  // one workgroup a transform
        d.grid = d.size[0];
        d.xcd_remap = 0;
        return MOA_OK;
    }
    const int eb0 = int(elem_bytes(fp64));
    auto finish_pair = [&](int lgw_) {
        const int P = 1 << (lgw_ - 1);
        d.lgw = lgw_;
        d.lge = 4;
        d.kmode = 3;
        d.in_tile_fast = in_tf;
        d.out_tile_fast = out_tf;
        const int lanes = std::max(1, 16 / P);
        d.col_stride = d.mfma ? moa::mfma_lds_col_stride(1 << lgn, lanes) : moa::lds_col_stride(1 << lgn, lanes);
        d.data_elems = P * d.col_stride;
        d.lds_bytes = (d.data_elems + moa::kTwBlkEntries + 256 * (d.tw ? d.tw_parts : 0) +
                       (d.mfma ? moa::kMfmaScaleElems + moa::kMfmaPairTwElems : 0)) * eb0;
        if (d.lds_bytes > moa::kLdsBytes) return want_w > 0 ? MOA_ERR_TUNING : MOA_ERR_LIFT;
        d.threads = 1024;
        int64_t blocks = d.size[0] >> lgw_;
        for (int i = 1; i < d.nd; ++i) blocks *= d.size[i];
        if (blocks >= (int64_t(1) << 31)) return MOA_ERR_BATCH;
        d.blocks = blocks;
        d.grid = blocks;  // one tile per workgroup
        d.xcd_remap = (blocks % 8 == 0 && blocks >= 16) ? 1 : 0;
        return MOA_OK;
    };
    if (!other_radix && (want_w > 0 ? (is_pow2(want_w) && pair_ok(lg2(want_w))) : pair_ok(15 - lgn)))
        return finish_pair(want_w > 0 ? lg2(want_w) : 15 - lgn);
    int lgw = 0;
    if (want_w > 0) {
        if (!is_pow2(want_w)) return MOA_ERR_TUNING;
        lgw = lg2(want_w);
        if (lgw > lg0 || lgw < min_lgw) return MOA_ERR_TUNING;
        if (!threads_ok(lgw)) return MOA_ERR_TUNING;
        if (lds_for(lgw, in_tf && lgw > 0).second > moa::kLdsBytes) return MOA_ERR_TUNING;
    } else {
        // Default tile: 2^12 points (2^11 for c128), so that several
        // workgroups share a CU and overlap each other's memory phases.  A
        // tile whose digit 0 is a unit-stride side takes at least 4 columns
        // (32-byte segments, the narrowest the L2 merges well); complex64
        // levels take at least 128-byte runs (16 columns), and 512-byte runs
        // (up to 2^14 points) where the rows they read lie 16 KB or more
        // apart and the level keeps at least 2048 such tiles.  Measured: a
        // 256-point level reading rows 32 KB apart, 16 columns 1.03 ms and
        // 64 columns 0.83 ms; 1024-point levels reading rows 8 and 32 KB
        // apart, 4 columns 120 / 118 us and 16 columns 70 / 83 us; whole
        // 2^24-point transforms <1024 1024> 0.182 -> 0.133 ms, <512 512>
        // 0.144 -> 0.109 ms, <2048 2048> 0.190 -> 0.165 ms.  Each up to the
        // thread limit, LDS and the digit itself.
        const int base_lg = fp64 ? 11 : 12;
        int target_lg = (in_tf || out_tf) ? std::max(base_lg, lgn + 2) : base_lg;
        // (A level that only writes along the tile, rows 32 KB or more apart,
        // keeps 2^12 points: 512- and 1024-point levels writing rows 32 KB
        // apart ran 9-10 % faster that way than with 16 columns; a 2048-point
        // level writing rows 16 KB apart was faster with 8 columns than 4.
        // Once a buffer of the level outgrows the Infinity Cache, such levels
        // of 256 .. 2048 points take 2^13 points and at least 128-byte runs
        // up to 2^14 points: 32 columns at 256 points, 16 at 512 and 1024, 8
        // at 2048; from 2^25 points (256 MiB), from 2^26 at 256 points.
        // Measured, 2^28 points: <256 4096> 1.83 against 1.91 ms (16
        // columns; 1.90 with 64), <512 4096> 1.94 against 2.18 ms (8; 2.24
        // with 32), <1024 4096> 2.05-2.08 against 2.88-2.90 ms (4), <2048
        // 4096> 2.20-2.22 against 3.16-3.20 ms (4), 2^30 <1024 1024 1024>
        // 15.3 against 19.0 ms; 2^25 points: <512 4096> 0.252 against 0.318
        // ms, <1024 4096> 0.275 against 0.452 ms, <2048 4096> 0.365 against
        // 0.447 ms, but <256 4096> 0.224 against 0.215 ms with 16 columns;
        // 2^24 points: the narrower tiles stay faster, <512 4096> 0.122
        // against 0.128 ms, <1024 4096> 0.131 against 0.142 ms.  Complex128
        // levels of 512 .. 2048 points take 128-byte runs (8 columns) up to
        // 2^13 points from 256 MiB, see below: 2^24 points <512 4096> 0.333
        // against 0.392 ms, <1024 4096> 0.353 against 0.383 ms, 2^25 points
        // 0.667 / 0.694 against 0.759 / 0.781 ms; at 2^23 points they tie.)
        const bool far_writes = !in_tf && out_tf && d.out_s_k * int64_t(eb) >= 32768;
        if (!fp64 && (in_tf || out_tf) && !far_writes) target_lg = std::max(target_lg, lgn + 4);
        int64_t level_bytes = (int64_t(1) << lgn) * eb;
        for (int i = 0; i < d.nd; ++i) level_bytes *= d.size[i];
        if (!fp64 && far_writes && lgn >= 8 && lgn <= 11 && level_bytes >= (int64_t(1) << (lgn == 8 ? 29 : 28)))
            target_lg = std::max(target_lg, std::min(14, std::max(13, lgn + 4)));
        // Complex128 write-side tiles of 512 .. 2048 points take 128-byte
        // runs from 256 MiB whatever the row spacing: 2^26 points <512 512>
        // 0.853 against 1.010 ms, <1024 1024> 0.915 against 1.056 ms (at
        // 2^23 points 4 columns stay faster, 0.135 against 0.137 ms).
        if (fp64 && !in_tf && out_tf && lgn >= 9 && lgn <= 11 && level_bytes >= (int64_t(1) << 28))
            target_lg = std::max(target_lg, std::min(13, lgn + 3));
        if (!fp64 && in_tf) {
            int64_t points = int64_t(1) << lgn;
            for (int i = 0; i < d.nd; ++i) points *= d.size[i];
            // (Also a 256-point level whose rows lie closer, over 2^26 points
            // or more: 1024 x 2^16 <256 256> 0.441 against 0.469 ms, 4096 x
            // 2^16 1.73 against 1.91 ms, 16 x 2^24 <256 256 256> 2.57 against
            // 2.79 ms, the 3-D 256^3 x 16 2.50 against 2.72 ms; 512-point
            // levels gained in 3-D and lost in 1-D, so they keep the rule.)
            const bool wide_rows = d.in_s_e * int64_t(eb) >= 16384 || (lgn == 8 && points >= (int64_t(1) << 26));
            if (wide_rows && (points >> 14) >= 2048)
                target_lg = std::max(target_lg, std::min(14, lgn + 6));
        }
        // Complex128 levels reading along a unit-stride tile side take the
        // largest tile, 2^13 points (measured, whole transforms: <1024 1024>
        // 0.156 -> 0.130 ms, <512 512> 0.138 -> 0.118 ms, <256 256> 0.109 ->
        // 0.104 ms, <4096 256> 1.34 -> 1.29 ms; write-side tiles keep 2^11).
        if (fp64 && in_tf) target_lg = std::max(target_lg, 13);
        lgw = std::min(min_lgw, lg0);
        while (lgw < lg0 && lgn + lgw + 1 <= std::max(target_lg, lgn + min_lgw) && threads_ok(lgw + 1) &&
               lds_for(lgw + 1, in_tf).second <= moa::kLdsBytes)
            ++lgw;
    }
    if (lgw < min_lgw) return MOA_ERR_LIFT;  // matrix-core level with too few transforms
    d.lgw = lgw;
    d.lge = lge_for(lgw);
    d.kmode = kmode_for(lgw);
    if (d.kmode < 0) return MOA_ERR_TUNING;  // radix 32 on a level whose store changes the thread map
    d.in_tile_fast = lgw > 0 && in_tf;
    d.out_tile_fast = lgw > 0 && out_tf;
    const auto cl = lds_for(lgw, d.in_tile_fast);
    d.col_stride = cl.first;
    d.data_elems = (1 << lgw) * cl.first;
    // LDS: data tile, then the in-block twiddle halves, then the inter-level
    // parts (then the scale slots of a matrix-core level).
    d.lds_bytes = (d.data_elems + moa::kTwBlkEntries + 256 * d.tw_parts + (d.mfma ? moa::kMfmaScaleElems : 0)) * eb;
    if (d.lds_bytes > moa::kLdsBytes) return want_w > 0 ? MOA_ERR_TUNING : MOA_ERR_LIFT;
    d.threads = int(threads_for(lgw));
    if (!threads_ok(lgw)) return want_w > 0 ? MOA_ERR_TUNING : MOA_ERR_LIFT;
    int64_t blocks = d.size[0] >> lgw;
    for (int i = 1; i < d.nd; ++i) blocks *= d.size[i];
    if (blocks >= (int64_t(1) << 31)) return MOA_ERR_BATCH;
    d.blocks = blocks;
    if (d.mfma || d.kmode == 2) {
        d.grid = blocks;  // one tile per workgroup
        d.xcd_remap = (blocks % 8 == 0 && blocks >= 16) ? 1 : 0;
    } else {
        // Persistent grid: the workgroups that fit at once (LDS and a
        // 1024-lane-per-CU register budget), a multiple of 8 so each XCD
        // walks its own contiguous run of tiles.
        const int per_cu = std::max(1, std::min(moa::kLdsBytes / d.lds_bytes, std::max(1, 1024 / d.threads)));
        int64_t g = std::min<int64_t>(blocks, int64_t(cus) * per_cu);
        if (g >= 8) g &= ~int64_t(7);
        d.grid = std::max<int64_t>(g, 1);
        d.xcd_remap = (d.grid % 8 == 0 && blocks >= 16) ? 1 : 0;
    }
    return MOA_OK;
}

// finish_pass for a level that may run on the matrix cores: a matrix-core
// tile holds at least 2^11 points, so a level with fewer transforms than that
// (say 64 transforms of 16 points) runs its butterflies in FP32 instead,
// unless the caller asked for a tile width.
moa_status_t finish_pass_prec(PassDesc& d, bool fp64, int want_w, int cus)
{
    moa_status_t st = finish_pass(d, fp64, want_w, cus);
    if (st == MOA_ERR_LIFT && d.mfma && want_w <= 0) {
        d.mfma = 0;
        st = finish_pass(d, fp64, want_w, cus);
    }
    return st;
}

void push_digit(PassDesc& d, int64_t size, int64_t in_s, int64_t out_s)
{
    d.size[d.nd] = size;
    d.lg[d.nd] = is_pow2(size) ? lg2(size) : -1;
    d.in_s[d.nd] = in_s;
    d.out_s[d.nd] = out_s;
    ++d.nd;
}

// Lower the lift to one pass descriptor per level.
//
// The vector of one transform is viewed as the digit array D of shape
// <f_0 f_1 ... f_{L-1}> (row-major, level-0 digit slowest): the psi view of
// the lift.  By the decimation-in-time split, level l takes the DFT over
// digit l for every value of the digits before it (already transformed,
// they index frequencies k_0..k_{l-1}) and every value a'' of the digits
// after it, then multiplies by omega_{f_l R_l}^(a'' k_l), R_l = pi(drop(l+1,
// f)).  Every level keeps the digit positions of D (read pattern = write
// pattern, so passes run in place in the workspace); the axis strides come
// from the PCT run lengths of D.  The last level writes the result through
// the final transpose: X = (reverse iota L) transpose D, i.e. frequency digit
// k_i lands at stride pi(take(i, f)).
// Workspace layout of a two-level lift <f0 f1> whose levels both run the
// paired-column kernel (column FFTs with 16-byte column-pair accesses, then
// row FFTs with the final transpose).  The plain layout keeps D's digit
// positions, so level 0 writes, and level 1 reads, 64-byte runs at a large
// stride.  Instead, element (k0, c) of the workspace goes to
//     (k0 >> b) B1 f1 + (c >> 1) 2 B1 + (k0 mod B1) 2 + (c mod 2),
// B1 = 2^b = level 1's tile width: the reshape-transpose of Ch. 3 taken
// blockwise, so that one level-0 tile writes, and one level-1 tile reads,
// runs of 2 B1 W0 elements (512 bytes at <4096 4096>) while level 0 still
// stores column pairs with 16-byte accesses.
void pair_block_workspace(moa_fft_plan_s* p)
{
    if (p->passes.size() != 2 || p->fp64 || p->prec != MOA_FFT_PREC_NATIVE || !p->dims.empty()) return;
    PassDesc& l0 = p->passes[0];
    PassDesc& l1 = p->passes[1];
    if (l0.kmode != 3 || l1.kmode != 3 || l0.mfma || l1.mfma) return;
    if (!l0.in_tile_fast || !l0.out_tile_fast || l1.in_tile_fast || !l1.out_tile_fast) return;
    const int64_t f1 = int64_t(1) << l1.lgn;
    const int b = l1.lgw;                       // log2 B1
    const int64_t B1 = int64_t(1) << b, W0 = int64_t(1) << l0.lgw;
    if (l0.lgn - 4 < b) return;                 // rows j + m TPC must step blockwise
    // Level 0 stores: column pair u of tile t at t W0 B1 + u 2 B1, row k0 blockwise.
    l0.out_pair_s = 2 * B1;
    l0.out_tile_s = W0 * B1;
    l0.out_s_k = 2;
    l0.out_lgb = b;
    l0.out_s_hi = B1 * f1;
    // Level 1 loads: column k0 = tile s, w at s B1 f1 + 2 w; row c as (c mod 2) + (c >> 1) 2 B1.
    l1.in_s[0] = 2;
    l1.in_pair_s = 4;
    l1.in_tile_s = B1 * f1;
    l1.in_s_e = 1;
    l1.in_lgb = 1;
    l1.in_s_hi = 2 * B1;
}

moa_status_t lower(moa_fft_plan_s* p, const moa_fft_tuning_t* tuning)
{
    const int L = int(p->levels.size());
    const psi::Vec D(p->levels.begin(), p->levels.end());
    const psi::Vec Rs = psi::axis_strides(D);                     // stride of digit i in x
    const psi::Vec rev_strides = psi::axis_strides(psi::reverse(D));
    psi::Vec perm(static_cast<size_t>(L));
    for (int i = 0; i < L; ++i) perm[size_t(i)] = L - 1 - i;
    const psi::Vec Xs = psi::transpose_view(rev_strides, perm);     // stride of k_i in X
    const int64_t n = p->n, B = p->batch;
    p->passes.clear();
    for (int l = 0; l < L; ++l) {
        PassDesc d;
        d.lgn = lg2(D[size_t(l)]);
        if (l < L - 1) {
            const int64_t Rl = Rs[size_t(l)];
            d.in_s_e = d.out_s_k = Rl;
            push_digit(d, Rl, 1, 1);                                   // a'': tile digit
            const int64_t outer = n / (D[size_t(l)] * Rl);
            if (outer > 1) push_digit(d, outer, D[size_t(l)] * Rl, D[size_t(l)] * Rl);
            if (B > 1) push_digit(d, B, n, n);
            d.tw = 1;
            d.tw_lgroot = lg2(D[size_t(l)] * Rl);
            d.tw_parts = (d.tw_lgroot + 7) / 8;
        } else {
            d.in_s_e = Rs[size_t(l)];
            d.out_s_k = Xs[size_t(l)];
            for (int i = 0; i < l; ++i) push_digit(d, D[size_t(i)], Rs[size_t(i)], Xs[size_t(i)]);
            if (B > 1 || d.nd == 0) push_digit(d, B, n, n);
        }
        d.pre_lg = 0;
        for (int i = 0; i < l; ++i) d.pre_lg += lg2(D[size_t(i)]);
        if (p->prec != MOA_FFT_PREC_NATIVE && d.lgn % 4 == 0 && d.lgn >= 4 && d.lgn <= 12) d.mfma = p->prec;
        const int want = tuning ? tuning->cols_per_block[l] : 0;
        if (tuning && (want < 0)) return MOA_ERR_TUNING;
        d.lgrad = tuning ? int((tuning->lg_radix >> (4 * l)) & 0xFu) : 0;
        moa_status_t st = finish_pass_prec(d, p->fp64, want, p->cus);
        if (st != MOA_OK) return st;
        // The level kernel applies the inter-level factor only when it stores
        // in its load pattern, which every non-final level of this lowering does.
        if (d.tw && !d.mfma && d.in_tile_fast != d.out_tile_fast) return MOA_ERR_STATE;
        p->passes.push_back(d);
    }
    pair_block_workspace(p);
    return MOA_OK;
}

// Lower a multi-dimensional transform (Ch. 1, "Conclusions for the General
// Radix Approach", and Ch. 3, "Conclusions": the lift extends to several
// dimensions).  The array of shape <n_0 ... n_{k-1}> (row-major) is already
// the lifted view of its ravel; its DFT is the 1-D DFT along every axis in
// turn, i.e. the levels of a lift with no inter-level factor between them
// and no digit reversal at the end.  Axis a (stride S_a = pi(drop(a+1, dims)),
// O_a = pi(take(a, dims)) outer values) becomes one pass: the DFT of length
// n_a at stride S_a for every value of the inner axes (digit 0, unit stride:
// the tile digit, so the tile reads and writes runs along the contiguous
// axes) and of the outer axes with the batch (one digit of stride n_a S_a).
// The contiguous last axis runs first, then the others outwards; every pass
// stores in its load pattern, so after the first pass (in -> out) the rest
// run in place in out and the plan needs no workspace.
moa_status_t lower_nd(moa_fft_plan_s* p, const moa_fft_tuning_t* tuning)
{
    const int k = int(p->dims.size());
    const psi::Vec D(p->dims.begin(), p->dims.end());
    const psi::Vec S = psi::axis_strides(D);  // stride of each axis
    const int64_t B = p->batch;
    p->passes.clear();
    p->levels.clear();
    int done_lg = 0;  // log2 of the points transformed by earlier passes
    for (int a = k - 1; a >= 0; --a) {
        const int64_t na = D[size_t(a)];
        if (na == 1) continue;
        const int64_t Sa = S[size_t(a)];
        const int64_t outer = psi::pi(psi::take(a, D)) * B;
        PassDesc d;
        d.lgn = lg2(na);
        d.in_s_e = d.out_s_k = Sa;
        if (Sa > 1) {
            push_digit(d, Sa, 1, 1);
            if (outer > 1) push_digit(d, outer, na * Sa, na * Sa);
        } else {
            push_digit(d, outer, na, na);
        }
        d.tw = 0;
        d.pre_lg = done_lg;
        if (p->prec != MOA_FFT_PREC_NATIVE && d.lgn % 4 == 0 && d.lgn >= 4 && d.lgn <= 12) d.mfma = p->prec;
        const int l = int(p->passes.size());
        const int want = tuning ? tuning->cols_per_block[l] : 0;
        if (want < 0) return MOA_ERR_TUNING;
        d.lgrad = tuning ? int((tuning->lg_radix >> (4 * l)) & 0xFu) : 0;
        moa_status_t st = finish_pass_prec(d, p->fp64, want, p->cus);
        if (st != MOA_OK) return st;
        p->passes.push_back(d);
        p->levels.push_back(na);
        done_lg += d.lgn;
    }
    if (p->passes.empty()) {
        // Every extent is 1: the transform is the identity, one pass of
        // length-1 transforms copies in to out.
        PassDesc d;
        d.lgn = 0;
        d.in_s_e = d.out_s_k = 1;
        push_digit(d, B, 1, 1);
        moa_status_t st = finish_pass(d, p->fp64, tuning ? tuning->cols_per_block[0] : 0, p->cus);
        if (st != MOA_OK) return st;
        p->passes.push_back(d);
        p->levels.push_back(1);
    }
    return MOA_OK;
}

// In-block table: omega_{2^14}^e for e < 128, then omega_{2^14}^(128 e) for
// e < 128.  Inter-level tables of a level with root 2^R: part p holds
// omega_{2^R}^(e 2^(8p)) for e < 256.
int64_t add_block_table(moa_fft_plan_s* p)
{
    const int64_t off = add_table(p, int64_t(1) << 14, 128, 1);
    add_table(p, int64_t(1) << 14, 128, 128);
    return off;
}

void build_tables(moa_fft_plan_s* p)
{
    p->tab_host.clear();
    p->tw_blk_off = add_block_table(p);
    for (PassDesc& d : p->passes) {
        if (!d.tw) continue;
        const int64_t root = int64_t(1) << d.tw_lgroot;
        d.tw_inter_off = add_table(p, root, 256, 1);
        for (int part = 1; part < d.tw_parts; ++part) add_table(p, root, 256, int64_t(1) << (8 * part));
    }
}

moa_status_t upload(moa_fft_plan_s* p)
{
    if (hipGetDevice(&p->device) != hipSuccess) return MOA_ERR_HIP;
    const size_t eb = elem_bytes(p->fp64);
    const size_t nel = p->tab_host.size() / 2;
    std::vector<unsigned char> buf(nel * eb);
    if (p->fp64) {
        memcpy(buf.data(), p->tab_host.data(), nel * eb);
    } else {
        float* f = reinterpret_cast<float*>(buf.data());
        for (size_t i = 0; i < 2 * nel; ++i) f[i] = float(p->tab_host[i]);
    }
    if (hipMalloc(&p->d_tables, buf.size()) != hipSuccess) return MOA_ERR_ALLOC;
    if (hipMemcpy(p->d_tables, buf.data(), buf.size(), hipMemcpyHostToDevice) != hipSuccess) return MOA_ERR_HIP;
    if (p->ws_bytes && !(p->flags & MOA_FFT_FLAG_NO_WORKSPACE)) {
        if (hipMalloc(&p->d_ws, p->ws_bytes) != hipSuccess) return MOA_ERR_ALLOC;
    }
    if (!p->tasks.empty()) {
        if (hipMalloc(&p->d_tasks, p->tasks.size() * sizeof(BatchTask)) != hipSuccess) return MOA_ERR_ALLOC;
        if (hipMalloc(&p->d_toff, p->toff.size() * sizeof(int64_t)) != hipSuccess) return MOA_ERR_ALLOC;
        if (hipMemcpy(p->d_tasks, p->tasks.data(), p->tasks.size() * sizeof(BatchTask), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(p->d_toff, p->toff.data(), p->toff.size() * sizeof(int64_t), hipMemcpyHostToDevice) !=
                hipSuccess)
            return MOA_ERR_HIP;
        if (moa::prepare_batched_kernel(p->fp64, p->batch_lds) != hipSuccess) return MOA_ERR_HIP;
    }
    for (const PassDesc& d : p->passes)
        if (moa::prepare_pass_kernel(p->fp64, d) != hipSuccess) return MOA_ERR_HIP;
    return MOA_OK;
}

void release(moa_fft_plan_s* p)
{
    for (GraphEntry& g : p->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    p->graphs.clear();
    if (p->d_tables) (void)hipFree(p->d_tables);
    if (p->d_ws) (void)hipFree(p->d_ws);
    if (p->d_tasks) (void)hipFree(p->d_tasks);
    if (p->d_toff) (void)hipFree(p->d_toff);
    p->d_tables = p->d_ws = p->d_tasks = p->d_toff = nullptr;
}

// Live plans.  A handle is valid from its constructor's success until its
// moa_fft_destroy; calls on any other pointer (a destroyed plan, a stray
// address) return an error instead of reading freed memory.
std::mutex& registry_mutex()
{
    static std::mutex m;
    return m;
}
std::unordered_set<const void*>& registry()
{
    static std::unordered_set<const void*> live;
    return live;
}

bool valid_plan(moa_fft_plan_t p)
{
    if (!p) return false;
    std::lock_guard<std::mutex> lock(registry_mutex());
    return registry().count(p) != 0;
}

// Status of a handle argument: MOA_ERR_NULL for NULL, MOA_ERR_STATE for a
// pointer that is not a live plan.
moa_status_t check_plan(moa_fft_plan_t p)
{
    if (!p) return MOA_ERR_NULL;
    return valid_plan(p) ? MOA_OK : MOA_ERR_STATE;
}

moa_status_t check_common(moa_fft_dtype_t dtype, moa_fft_prec_t prec, uint32_t flags)
{
    if (dtype != MOA_C64 && dtype != MOA_C128) return MOA_ERR_DTYPE;
    if (prec != MOA_FFT_PREC_NATIVE && prec != MOA_FFT_PREC_SPLIT_BF16 && prec != MOA_FFT_PREC_SPLIT_FP16)
        return MOA_ERR_DTYPE;
    if (prec != MOA_FFT_PREC_NATIVE && dtype != MOA_C64) return MOA_ERR_DTYPE;
    if (flags & ~kKnownFlags) return MOA_ERR_ARG;
    return MOA_OK;
}

moa_status_t finalize(moa_fft_plan_s* p, moa_fft_plan_t* out)
{
    if (!p->host_only) {
        moa_status_t st = upload(p);
        if (st != MOA_OK) {
            release(p);
            delete p;
            return st;
        }
    }
    try {
        std::lock_guard<std::mutex> lock(registry_mutex());
        registry().insert(p);
    } catch (...) {
        release(p);
        delete p;
        return MOA_ERR_ALLOC;
    }
    *out = p;
    return MOA_OK;
}

// ---------------------------------------------------------------------------
// JSON description
// ---------------------------------------------------------------------------

// log2 radices of a level's stages: the short-transform kernel runs radix-4
// stages (one radix-2 stage when log2 N is odd); the others stages of the
// level's largest radix, then one with the remaining radix.
std::string stage_radices(const PassDesc& d)
{
    std::string out = "[";
    auto add = [&](int r) {
        if (out.size() > 1) out += ",";
        out += std::to_string(r);
    };
    if (d.kmode == 4) {
        for (int left = d.lgn; left > 0; left -= std::min(2, left)) add(std::min(2, left));
    } else {
        const int g = d.lgrad ? d.lgrad : moa::kLgRadixDefault;
        if (d.lgn <= g) {
            if (d.lgn > 0) add(d.lgn);
        } else {
            for (int i = 0; i < d.lgn / g; ++i) add(g);
            if (d.lgn % g) add(d.lgn % g);
        }
    }
    return out + "]";
}

std::string describe_json(const moa_fft_plan_s* p)
{
    std::string s;
    char b[512];
    auto add = [&](const char* fmt, auto... args) {
        snprintf(b, sizeof(b), fmt, args...);
        s += b;
    };
    add("{\"kind\":\"%s\",\"dtype\":\"%s\",\"prec\":\"%s\",\"n\":%lld,\"batch\":%lld,\"elements\":%lld,",
        p->batched ? "uneven_batch" : (p->dims.empty() ? "lifted" : "nd"), p->fp64 ? "c128" : "c64",
        p->prec == MOA_FFT_PREC_NATIVE ? "native" : (p->prec == MOA_FFT_PREC_SPLIT_BF16 ? "split_bf16" : "split_fp16"),
        (long long)p->n, (long long)p->batch, (long long)p->total);
    add("\"host_only\":%s,\"workspace_bytes\":%zu,\"workspace_owned\":%s,\"stream\":%s,",
        p->host_only ? "true" : "false", p->ws_bytes,
        (p->ws_bytes && !(p->flags & MOA_FFT_FLAG_NO_WORKSPACE)) ? "true" : "false", p->stream ? "true" : "false");
    s += "\"lift\":[";
    for (size_t i = 0; i < p->lift.size(); ++i) add("%s%lld", i ? "," : "", (long long)p->lift[i]);
    if (!p->dims.empty()) {
        s += "],\"dims\":[";
        for (size_t i = 0; i < p->dims.size(); ++i) add("%s%lld", i ? "," : "", (long long)p->dims[i]);
    }
    s += "],\"levels\":[";
    for (size_t i = 0; i < p->levels.size(); ++i) add("%s%lld", i ? "," : "", (long long)p->levels[i]);
    s += "],\"passes\":[";
    for (size_t l = 0; l < p->passes.size(); ++l) {
        const PassDesc& d = p->passes[l];
        const bool last = l + 1 == p->passes.size();
        add("%s{\"level\":%zu,\"N\":%lld,\"in\":\"%s\",\"out\":\"%s\",\"dft_axis\":{\"in_stride\":%lld,"
            "\"out_stride\":%lld},\"batch_axes\":[",
            l ? "," : "", l, (long long)(int64_t(1) << d.lgn), l == 0 ? "x" : (p->dims.empty() ? "workspace" : "y"),
            (last || !p->dims.empty()) ? "y" : "workspace",
            (long long)d.in_s_e, (long long)d.out_s_k);
        for (int i = 0; i < d.nd; ++i)
            add("%s{\"size\":%lld,\"in_stride\":%lld,\"out_stride\":%lld}", i ? "," : "",
                (long long)d.size[i], (long long)d.in_s[i], (long long)d.out_s[i]);
        add("],\"in_layout\":{\"block_lg\":%d,\"stride_hi\":%lld,\"pair_stride\":%lld,\"tile_stride\":%lld},"
            "\"out_layout\":{\"block_lg\":%d,\"stride_hi\":%lld,\"pair_stride\":%lld,\"tile_stride\":%lld",
            d.in_lgb, (long long)d.in_s_hi, (long long)(d.in_pair_s ? d.in_pair_s : 2 * d.in_s[0]),
            (long long)(d.in_tile_s ? d.in_tile_s : (int64_t(1) << d.lgw) * d.in_s[0]), d.out_lgb, (long long)d.out_s_hi,
            (long long)(d.out_pair_s ? d.out_pair_s : 2 * d.out_s[0]),
            (long long)(d.out_tile_s ? d.out_tile_s : (int64_t(1) << d.lgw) * d.out_s[0]));
        add("},\"twiddle_root\":%lld,\"twiddle_parts\":%d,\"grid\":%lld,\"tile_width\":%d,\"threads\":%d,\"blocks\":%lld,\"lds_bytes\":%d,"
            "\"lds_col_stride\":%d,\"in_tile_fast\":%s,\"out_tile_fast\":%s,\"xcd_remap\":%d,\"mfma\":\"%s\","
            "\"points_per_thread\":%d,\"kernel_mode\":%d,\"lg_radix\":%d,\"stage_lg_radices\":%s}",
            d.tw ? (long long)(int64_t(1) << d.tw_lgroot) : 0LL, d.tw ? d.tw_parts : 0, (long long)d.grid, 1 << d.lgw,
            d.threads, (long long)d.blocks,
            d.lds_bytes, d.col_stride, d.in_tile_fast ? "true" : "false", d.out_tile_fast ? "true" : "false",
            d.xcd_remap, d.mfma == 0 ? "none" : (d.mfma == 1 ? "split_bf16" : "split_fp16"),
            (d.mfma || d.kmode == 3) ? 32 : (1 << lgE(d.lgn, d.lge)), d.kmode,
            d.kmode == 4 ? 2 : (d.lgrad ? d.lgrad : moa::kLgRadixDefault), stage_radices(d).c_str());
    }
    s += "]";
    if (p->batched) {
        add(",\"count\":%lld,\"tasks\":%zu,\"threads\":%d,\"lds_bytes\":%d,\"persistent_blocks\":%d,"
            "\"task_lg\":%d,\"per_size\":%s,\"sizes_by_task_group\":[",
            (long long)p->sizes.size(), p->tasks.size(), p->batch_threads, p->batch_lds, p->batch_grid, p->batch_task_lg,
            (p->flags & MOA_FFT_FLAG_PER_SIZE) ? "true" : "false");
        for (size_t i = 0; i < p->size_ranges.size(); ++i) {
            const auto& r = p->size_ranges[i];
            add("%s{\"n\":%lld,\"first_task\":%d,\"tasks\":%d}", i ? "," : "",
                (long long)(int64_t(1) << p->tasks[size_t(r.first)].lgn), r.first, r.second);
        }
        s += "]";
    }
    s += "}";
    return s;
}

moa_status_t make_graph(moa_fft_plan_s* p, int dir, const void* in, void* out, GraphEntry& g);
moa_status_t launch_all(moa_fft_plan_s* p, int dir, const void* in, void* out, void* ws, hipStream_t s);

// Fill the kernel argument blocks of every pass for one execution.
// Streaming (non-temporal) access to data a transform touches once: the
// first level's loads of the caller's input (while it fits the 256 MiB
// Infinity Cache they keep it from displacing the workspace the next level
// reads: the first level of the 2^24-point transform 108 -> 79 us; a 2 GiB
// input ran a few per cent slower with them, so the automatic choice is by
// size), and for an uneven batch its loads and its full-line output stores
// (8192 transforms: 99 -> 91 us).  Later levels read the workspace with
// plain loads, and the partial-line stores of a lifted level stay plain;
// streaming either was slower.
constexpr size_t kStreamAutoBytes = size_t(256) << 20;

moa_status_t stream_choice(const moa_fft_tuning_t* tuning, size_t in_bytes, bool& on)
{
    const int mode = tuning ? tuning->stream : 0;
    if (mode < -1 || mode > 1) return MOA_ERR_TUNING;
    on = mode == 1 || (mode == 0 && in_bytes <= kStreamAutoBytes);
    return MOA_OK;
}

// Buffers of the passes: a lifted 1-D plan reads `in` on level 0, runs its
// middle levels in place in the workspace `ws` and writes `out` on its last
// level; a multi-dimensional plan transforms one axis a pass, `in` -> `out`
// first, then in place in `out`.
// Fills args[0 .. passes) (a fixed array: an execution allocates nothing).
void pass_args(const moa_fft_plan_s* p, int dir, const void* in, void* out, void* ws, moa::PassArgs* args)
{
    const size_t eb = elem_bytes(p->fp64);
    const unsigned char* tb = static_cast<const unsigned char*>(p->d_tables);
    const size_t P = p->passes.size();
    const bool nd = !p->dims.empty();
    for (size_t l = 0; l < P; ++l) {
        const PassDesc& d = p->passes[l];
        moa::PassArgs a;
        memset(&a, 0, sizeof(a));
        if (nd) {
            a.in = l == 0 ? in : out;
            a.out = out;
        } else {
            a.in = l == 0 ? in : ws;
            a.out = (l + 1 == P) ? out : ws;
        }
        a.in_s_e = d.in_s_e;
        a.out_s_k = d.out_s_k;
        for (int i = 0; i < moa::kMaxDigits; ++i) {
            a.in_s[i] = d.in_s[i];
            a.out_s[i] = d.out_s[i];
            a.lg[i] = d.lg[i];
        }
        a.nd = d.nd;
        a.lgw = d.lgw;
        a.lg_tiles = d.nd == 1 ? 0 : d.lg[0] - d.lgw;
        a.col_stride = d.col_stride;
        a.tw_parts = d.tw ? d.tw_parts : 0;
        a.tw_lgroot = d.tw_lgroot;
        a.tw_inter = tb + size_t(d.tw_inter_off) * eb;
        a.tw_blk = tb + size_t(p->tw_blk_off) * eb;
        a.ntiles = d.blocks;
        a.data_elems = d.data_elems;
        a.xcd_remap = d.xcd_remap;
        a.pre_lg = d.pre_lg;
        a.sign = dir == MOA_FFT_FORWARD ? -1.0f : 1.0f;
        a.nt_in = (l == 0 && p->stream) ? 1 : 0;
        // The last level's output is written once; where its runs are whole
        // 128-byte lines (not the 64-byte runs of a paired level) the
        // persistent kernel stores it streaming too.
        a.nt_out = (l + 1 == P && p->stream && d.kmode != 3 && !d.mfma && !p->fp64 && d.out_tile_fast &&
                    (int64_t(1) << d.lgw) * int64_t(eb) >= 128)
                       ? 1
                       : 0;
        a.in_lgb = d.in_lgb;
        a.out_lgb = d.out_lgb;
        a.in_s_hi = d.in_s_hi;
        a.out_s_hi = d.out_s_hi;
        a.in_pair_s = d.in_pair_s ? d.in_pair_s : 2 * d.in_s[0];
        a.out_pair_s = d.out_pair_s ? d.out_pair_s : 2 * d.out_s[0];
        a.in_tile_s = d.in_tile_s ? d.in_tile_s : (int64_t(1) << d.lgw) * d.in_s[0];
        a.out_tile_s = d.out_tile_s ? d.out_tile_s : (int64_t(1) << d.lgw) * d.out_s[0];
        args[l] = a;
    }
}

moa::BatchArgs batch_args(const moa_fft_plan_s* p, int dir, const void* in, void* out, int task0, int ntasks)
{
    moa::BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.in = in;
    a.out = out;
    a.tasks = static_cast<const BatchTask*>(p->d_tasks);
    a.toff = static_cast<const int64_t*>(p->d_toff);
    a.tw_blk = static_cast<const unsigned char*>(p->d_tables) + size_t(p->tw_blk_off) * elem_bytes(p->fp64);
    a.task0 = task0;
    a.ntasks = ntasks;
    a.data_elems = p->batch_data_elems;
    a.sign = dir == MOA_FFT_FORWARD ? -1.0f : 1.0f;
    a.nt = p->stream ? 1 : 0;
    return a;
}

moa_status_t launch_all(moa_fft_plan_s* p, int dir, const void* in, void* out, void* ws, hipStream_t s)
{
    if (p->batched) {
        if (p->flags & MOA_FFT_FLAG_PER_SIZE) {
            for (const auto& r : p->size_ranges) {
                moa::BatchArgs a = batch_args(p, dir, in, out, r.first, r.second);
                if (moa::launch_batched(p->fp64, a, r.second, p->batch_threads, p->batch_lds, s) != hipSuccess)
                    return MOA_ERR_HIP;
            }
        } else {
            moa::BatchArgs a = batch_args(p, dir, in, out, 0, int(p->tasks.size()));
            if (moa::launch_batched(p->fp64, a, p->batch_grid, p->batch_threads, p->batch_lds, s) != hipSuccess)
                return MOA_ERR_HIP;
        }
        return MOA_OK;
    }
    moa::PassArgs args[moa::kMaxPasses];
    pass_args(p, dir, in, out, ws, args);
    for (size_t l = 0; l < p->passes.size(); ++l)
        if (moa::launch_pass(p->fp64, p->passes[l], args[l], s) != hipSuccess) return MOA_ERR_HIP;
    return MOA_OK;
}

moa_status_t add_node(hipGraph_t g, hipGraphNode_t* prev, const void* fn, dim3 grid, dim3 block, int lds,
                      void* argp)
{
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void*>(fn);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = unsigned(lds);
    void* params[1] = {argp};
    kp.kernelParams = params;
    kp.extra = nullptr;
    hipGraphNode_t node;
    if (hipGraphAddKernelNode(&node, g, *prev ? prev : nullptr, *prev ? 1 : 0, &kp) != hipSuccess)
        return MOA_ERR_HIP;
    *prev = node;
    return MOA_OK;
}

moa_status_t make_graph(moa_fft_plan_s* p, int dir, const void* in, void* out, GraphEntry& g)
{
    g.dir = dir;
    g.in = in;
    g.out = out;
    if (hipGraphCreate(&g.graph, 0) != hipSuccess) return MOA_ERR_HIP;
    hipGraphNode_t prev = nullptr;
    moa_status_t st = MOA_OK;
    if (p->batched) {
        if (p->flags & MOA_FFT_FLAG_PER_SIZE) {
            for (const auto& r : p->size_ranges) {
                moa::BatchArgs a = batch_args(p, dir, in, out, r.first, r.second);
                st = add_node(g.graph, &prev, moa::batched_kernel_fn(p->fp64, dir == MOA_FFT_FORWARD), dim3(unsigned(r.second)),
                              dim3(unsigned(p->batch_threads)), p->batch_lds, &a);
                if (st != MOA_OK) break;
            }
        } else {
            moa::BatchArgs a = batch_args(p, dir, in, out, 0, int(p->tasks.size()));
            st = add_node(g.graph, &prev, moa::batched_kernel_fn(p->fp64, dir == MOA_FFT_FORWARD), dim3(unsigned(p->batch_grid)),
                          dim3(unsigned(p->batch_threads)), p->batch_lds, &a);
        }
    } else {
        moa::PassArgs args[moa::kMaxPasses];
        pass_args(p, dir, in, out, p->d_ws, args);
        for (size_t l = 0; l < p->passes.size() && st == MOA_OK; ++l) {
            const PassDesc& d = p->passes[l];
            st = add_node(g.graph, &prev, moa::pass_kernel_fn(p->fp64, d, dir == MOA_FFT_FORWARD), dim3(unsigned(d.grid)),
                          dim3(unsigned(d.threads)), d.lds_bytes, &args[l]);
        }
    }
    if (st == MOA_OK && hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) != hipSuccess) st = MOA_ERR_HIP;
    if (st != MOA_OK) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        g.exec = nullptr;
        g.graph = nullptr;
    }
    return st;
}

// Validate the sizes and build the tasks of an uneven batch.
moa_status_t plan_uneven(moa_fft_plan_s* p, const moa_fft_tuning_t* tuning)
{
    const int maxlg = max_lg_block(p->fp64);
    const size_t eb = elem_bytes(p->fp64);
    // Tasks of up to 2^13 points on 512 threads, 16 points a thread (one
    // transform a thread when it is shorter than that), or one complex64
    // transform of 2^14 points as two halves of 2^13.  A tuned task size of
    // 2^11 or 2^12 points packs fewer of the shorter transforms a task.
    const int T = 512;
    const int task_lg = tuning && tuning->batch_task_lg ? tuning->batch_task_lg : 13;
    if (task_lg < 11 || task_lg > 13) return MOA_ERR_TUNING;
    p->batch_task_lg = task_lg;
    const int64_t count = int64_t(p->sizes.size());
    std::vector<int64_t> off(size_t(count) + 1, 0);
    std::vector<std::vector<int64_t>> by_lg(size_t(maxlg) + 1);
    for (int64_t i = 0; i < count; ++i) {
        const int64_t s = p->sizes[size_t(i)];
        if (!is_pow2(s) || lg2(s) > maxlg) return MOA_ERR_SIZE;
        off[size_t(i) + 1] = off[size_t(i)] + s;
        by_lg[size_t(lg2(s))].push_back(i);
    }
    p->total = off[size_t(count)];
    int lds_max = 0;
    p->tasks.clear();
    p->toff.clear();
    p->size_ranges.clear();
    for (int lg = maxlg; lg >= 0; --lg) {
        const auto& idx = by_lg[size_t(lg)];
        if (idx.empty()) continue;
        // A 2^14-point complex64 transform runs as its two 2^13-point halves
        // (even and odd samples) in one task, so its LDS tile is theirs.
        const bool split = !p->fp64 && lg == 14;
        const int lgt = split ? 13 : lg;
        const int tpc = 1 << (lgt - lgE(lgt, 4));
        const int cs = moa::lds_col_stride(1 << lgt, tpc);
        // 2^(13 - lg) transforms of 16 points or more, T shorter ones; a
        // smaller task size scales that down (at least one transform).
        const int per = split ? 1 : std::max(1, (T / tpc) >> (13 - task_lg));
        const bool uses_lds = lg > 4;  // a single register stage needs no exchange
        const int first_task = int(p->tasks.size());
        for (size_t k = 0; k < idx.size(); k += size_t(per)) {
            const int cnt = int(std::min<size_t>(size_t(per), idx.size() - k));
            BatchTask tk;
            tk.lgn = lg;
            tk.count = cnt;
            tk.first = int64_t(p->toff.size());
            tk.off0 = off[size_t(idx[k])];
            for (int w = 0; w < cnt; ++w) p->toff.push_back(off[size_t(idx[k + size_t(w)])]);
            p->tasks.push_back(tk);
            if (uses_lds) lds_max = std::max(lds_max, int(int64_t(cnt) * cs * int64_t(eb)));
        }
        p->size_ranges.push_back({first_task, int(p->tasks.size()) - first_task});
    }
    // Within a size the full tasks come first; sizes are already longest first.
    p->batch_threads = T;
    // LDS: exchange tile, then the in-block twiddle table.
    p->batch_data_elems = int(lds_max / int64_t(eb));
    p->batch_lds = lds_max + moa::kTwBlkEntries * int(eb);
    if (p->batch_lds > moa::kLdsBytes) return MOA_ERR_STATE;
    // Default grid: one workgroup per task.  The hardware dispatcher then
    // hands each freed slot the next task of the longest-first order, which
    // balances the CUs better than any static split of tasks this coarse
    // (at 8192 mixed transforms a 2^14-point task is over a quarter of what
    // each of the 512 resident workgroups moves).  A tuned grid smaller than that makes the launch
    // persistent: each workgroup walks tasks blockIdx.x, + grid, ...
    int grid = int(p->tasks.size());
    if (tuning && tuning->persistent_blocks < 0) return MOA_ERR_TUNING;
    if (tuning && tuning->persistent_blocks > 0) grid = std::min(grid, int(tuning->persistent_blocks));
    p->batch_grid = std::max(grid, 1);
    return MOA_OK;
}

// Paired-column levels move column pairs with 16-byte accesses on their
// unit-stride side; a caller buffer on that side must be 16-byte aligned.
bool pair_aligned(const PassDesc& d, const void* in, const void* out, bool reads_in, bool writes_out)
{
    if (d.kmode != 3) return true;
    if (reads_in && d.in_tile_fast && (reinterpret_cast<uintptr_t>(in) & 15u)) return false;
    if (writes_out && d.out_tile_fast && (reinterpret_cast<uintptr_t>(out) & 15u)) return false;
    return true;
}

// Every pass's caller buffers meet the paired-column alignment: a 1-D plan
// reads `in` on level 0 and writes `out` on its last level; a
// multi-dimensional plan reads `in` on its first pass and `out` after it,
// and writes `out` on every pass.
bool exec_aligned(const moa_fft_plan_s* p, const void* in, const void* out)
{
    const size_t P = p->passes.size();
    for (size_t l = 0; l < P; ++l) {
        const bool ok = p->dims.empty() ? pair_aligned(p->passes[l], in, out, l == 0, l + 1 == P)
                                        : pair_aligned(p->passes[l], l == 0 ? in : out, out, true, true);
        if (!ok) return false;
    }
    return true;
}

}  // namespace

// Execution on a workspace supplied by the caller of these two functions
// (the allocation-free entry point keeps it in a static device array).
moa_status_t moa::check_exec(moa_fft_plan_t p, int dir, const void* in, const void* out, size_t* ws_bytes)
{
    if (const moa_status_t hs = check_plan(p)) return hs;
    if (!in || !out || !ws_bytes) return MOA_ERR_NULL;
    if (dir != MOA_FFT_FORWARD && dir != MOA_FFT_ADJOINT) return MOA_ERR_ARG;
    *ws_bytes = p->ws_bytes;
    if (p->ws_bytes > MOA_FFT_SCRATCH_BYTES) return MOA_ERR_SCRATCH;
    if (p->host_only) return MOA_ERR_STATE;
    if (!exec_aligned(p, in, out)) return MOA_ERR_ARG;
    return MOA_OK;
}

moa_status_t moa::launch_on_workspace(moa_fft_plan_t p, int dir, const void* in, void* out, void* ws, hipStream_t s)
{
    return launch_all(p, dir, in, out, ws, s);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* moa_fft_status_string(moa_status_t s)
{
    switch (s) {
        case MOA_OK: return "MOA_OK";
        case MOA_ERR_NULL: return "MOA_ERR_NULL";
        case MOA_ERR_SIZE: return "MOA_ERR_SIZE";
        case MOA_ERR_LIFT: return "MOA_ERR_LIFT";
        case MOA_ERR_BATCH: return "MOA_ERR_BATCH";
        case MOA_ERR_DTYPE: return "MOA_ERR_DTYPE";
        case MOA_ERR_ALLOC: return "MOA_ERR_ALLOC";
        case MOA_ERR_HIP: return "MOA_ERR_HIP";
        case MOA_ERR_STATE: return "MOA_ERR_STATE";
        case MOA_ERR_ARG: return "MOA_ERR_ARG";
        case MOA_ERR_TUNING: return "MOA_ERR_TUNING";
        case MOA_ERR_SCRATCH: return "MOA_ERR_SCRATCH";
    }
    return "MOA_ERR_UNKNOWN";
}

int64_t moa_fft_max_block(moa_fft_dtype_t dtype)
{
    if (dtype == MOA_C64) return int64_t(1) << moa::kMaxLgBlockC64;
    if (dtype == MOA_C128) return int64_t(1) << moa::kMaxLgBlockC128;
    return 0;
}

moa_status_t moa_fft_plan_tuned(moa_fft_plan_t* out, int64_t n, int64_t batch, const int64_t* lift_shape,
                                int32_t lift_rank, moa_fft_dtype_t dtype, moa_fft_prec_t prec, uint32_t flags,
                                const moa_fft_tuning_t* tuning)
{
    if (!out) return MOA_ERR_NULL;
    if (lift_rank > 0 && !lift_shape) return MOA_ERR_NULL;
    moa_status_t st = check_common(dtype, prec, flags);
    if (st != MOA_OK) return st;
    if (flags & MOA_FFT_FLAG_PER_SIZE) return MOA_ERR_ARG;
    if (!is_pow2(n) || lg2(n) > kLgMaxN) return MOA_ERR_SIZE;
    if (batch < 1) return MOA_ERR_BATCH;
    if (n > (int64_t(1) << 40) / batch) return MOA_ERR_BATCH;
    if (lift_rank < 0 || lift_rank > 8) return MOA_ERR_LIFT;
    const bool fp64 = dtype == MOA_C128;
    const int maxlg = max_lg_block(fp64);
    std::vector<int64_t> lift;
    if (lift_rank > 0) {
        int64_t prod = 1;
        for (int i = 0; i < lift_rank; ++i) {
            const int64_t f = lift_shape[i];
            if (!is_pow2(f) || lg2(f) > maxlg) return MOA_ERR_LIFT;
            if (f < 2 && !(n == 1 && lift_rank == 1)) return MOA_ERR_LIFT;
            if (prod > (int64_t(1) << 40) / f) return MOA_ERR_LIFT;
            prod *= f;
            lift.push_back(f);
        }
        if (prod != n) return MOA_ERR_LIFT;
    } else {
        const int d = lg2(n);
        const int L = d <= maxlg ? 1 : (d + maxlg - 1) / maxlg;
        // Level sizes in pass order (innermost level first); lift is the reverse.
        std::vector<int> parts;
        if (prec != MOA_FFT_PREC_NATIVE && d <= 24) {
            // Split precisions up to 2^24 points: the fewest levels (HBM
            // passes), cut into whole radix-16 digits so that the levels run
            // on the matrix cores (2^4, 2^8 and 2^12 points).  The bits that
            // do not make a whole digit go to the first level, which runs in
            // FP32 and takes as few bits as the 12-bit levels after it allow.
            // The digits are spread evenly, the shorter levels first (2^20:
            // <4096 256>, 1.85-2.05 ms against 2.07-2.25 ms for <256 4096>
            // on 256 transforms).  From 2^25 points the FP32 default below,
            // <256 4096 2^(d-20)>, already has two matrix-core levels.
            const int r = d % 4;
            const int f = r == 0 && d <= 12 * L ? 0 : std::max(r, d - 12 * (L - 1));
            const int k = f ? L - 1 : L;  // levels of whole digits
            if (f <= maxlg && (k > 0 || f == d)) {
                const int q = (d - f) / 4;
                if (f) parts.push_back(f);
                for (int i = 0; i < k; ++i) parts.push_back(4 * (q / k + (i >= k - q % k ? 1 : 0)));
            }
        }
        if (parts.empty() && !fp64 && d == 23 && n * batch <= (int64_t(1) << 25)) {
            // Complex64 FP32, 2^23 points in batches of up to 2^25 points:
            // three levels <256 128 256>, 0.073 / 0.142 / 0.298 ms against
            // 0.075 / 0.158 / 0.365 ms for two (1, 2, 4 transforms); 8
            // transforms take the two levels below (0.660 against 0.676 ms).
            parts = {8, 7, 8};
        }
        if (parts.empty() && !fp64 && d >= 19 && d <= 23 && n * batch >= (int64_t(1) << 24)) {
            // Complex64 FP32, 2^19 .. 2^23 points, batches of 2^24 points or
            // more: two levels, one of 4096 points (the paired-column level,
            // 64-byte runs from 2^15-point tiles).  It runs first (<2^(d-12)
            // 4096>) while the batch holds 2^25 points or fewer, last (<4096
            // 2^(d-12)>) beyond, and first at 2^23 points either way.
            // Measured against the near-equal split, e.g. 16 x 2^20 0.110
            // against 0.138 ms, 4 x 2^22 0.129 against 0.169 ms, 32 x 2^20
            // 0.219 against 0.278 ms (<4096 256>: 0.277), 64 x 2^20 0.490
            // against 0.579 ms (<256 4096>: 0.513), 256 x 2^20 1.69 against
            // 2.24 ms, 32 x 2^23 2.05 against 2.38 ms.  Smaller batches keep
            // the near-equal split (a 4096-point level has too few of its
            // one-per-CU tiles there: 2^22 0.053 against 0.041 ms, 8 x 2^19
            // 0.046 against 0.035 ms).
            const bool fits = n * batch <= (int64_t(1) << 25);
            parts = (d == 23 || fits) ? std::vector<int>{12, d - 12} : std::vector<int>{d - 12, 12};
        }
        if (parts.empty() && !fp64 && d >= 25) {
            // Complex64 FP32, 2^25 points and more: three levels <256 4096
            // 2^(d-20)> rather than two with 2^13- or 2^14-point levels,
            // whose tiles read and write 16- or 32-byte runs: 2^25 0.315
            // against 0.473 ms, 2^26 0.721 against 0.920 ms, 2^27 1.39
            // against 1.84 ms, 2^28 2.96 against 4.12 ms, 2^29 5.86 against
            // 6.93 ms (<1024 1024 512>), 2^30 13.8 against 14.7 ms.
            parts = {d - 20, 12, 8};
        }
        if (parts.empty() && fp64 && d >= 23 && d <= 26) {
            // Complex128, 2^23 .. 2^26 points: three levels <256 256
            // 2^(d-16)> rather than two of 2^11 .. 2^13 points, whose tiles
            // of at most 2^13 points hold one to four columns: 2^23 0.159
            // against 0.208 ms, 4 x 2^23 0.646 against 0.871 ms, 8 x 2^24
            // 2.38 against 3.46 ms, 2^25 0.665 against 1.12 ms, 2 x 2^26
            // 2.53 against 4.29 ms.
            parts = {d - 16, 8, 8};
        }
        if (parts.empty()) {
            // near-equal split, the outer levels take the remainder first
            for (int i = L - 1; i >= 0; --i) parts.push_back(d / L + (i < d % L ? 1 : 0));
        }
        for (size_t i = parts.size(); i-- > 0;) lift.push_back(int64_t(1) << parts[i]);
    }
    moa_fft_plan_s* p = new (std::nothrow) moa_fft_plan_s();
    if (!p) return MOA_ERR_ALLOC;
    p->fp64 = fp64;
    p->prec = prec;
    p->flags = flags;
    p->host_only = (flags & MOA_FFT_FLAG_HOST_ONLY) != 0;
    p->n = n;
    p->batch = batch;
    p->total = n * batch;
    p->lift = lift;
    p->levels.assign(lift.rbegin(), lift.rend());
    if (!p->host_only) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            p->cus = cus;
    }
    st = lower(p, tuning);
    if (st == MOA_OK) st = stream_choice(tuning, size_t(p->total) * elem_bytes(fp64), p->stream);
    if (st != MOA_OK) {
        delete p;
        return st;
    }
    build_tables(p);
    p->ws_bytes = p->passes.size() > 1 ? size_t(p->total) * elem_bytes(fp64) : 0;
    return finalize(p, out);
}

moa_status_t moa_fft_plan(moa_fft_plan_t* out, int64_t n, int64_t batch, const int64_t* lift_shape,
                          int32_t lift_rank, moa_fft_dtype_t dtype, moa_fft_prec_t prec, uint32_t flags)
{
    return moa_fft_plan_tuned(out, n, batch, lift_shape, lift_rank, dtype, prec, flags, nullptr);
}

moa_status_t moa_fft_plan_nd_tuned(moa_fft_plan_t* out, int32_t rank, const int64_t* dims, int64_t batch,
                                   moa_fft_dtype_t dtype, moa_fft_prec_t prec, uint32_t flags,
                                   const moa_fft_tuning_t* tuning)
{
    if (!out || !dims) return MOA_ERR_NULL;
    moa_status_t st = check_common(dtype, prec, flags);
    if (st != MOA_OK) return st;
    if (flags & MOA_FFT_FLAG_PER_SIZE) return MOA_ERR_ARG;
    if (rank < 1 || rank > 8) return MOA_ERR_ARG;
    const bool fp64 = dtype == MOA_C128;
    const int maxlg = max_lg_block(fp64);
    int64_t n = 1;
    for (int i = 0; i < rank; ++i) {
        if (!is_pow2(dims[i]) || lg2(dims[i]) > maxlg) return MOA_ERR_SIZE;
        n *= dims[i];
        if (lg2(n) > kLgMaxN) return MOA_ERR_SIZE;
    }
    if (batch < 1) return MOA_ERR_BATCH;
    if (n > (int64_t(1) << 40) / batch) return MOA_ERR_BATCH;
    moa_fft_plan_s* p = new (std::nothrow) moa_fft_plan_s();
    if (!p) return MOA_ERR_ALLOC;
    p->fp64 = fp64;
    p->prec = prec;
    p->flags = flags;
    p->host_only = (flags & MOA_FFT_FLAG_HOST_ONLY) != 0;
    p->n = n;
    p->batch = batch;
    p->total = n * batch;
    p->dims.assign(dims, dims + rank);
    p->lift = p->dims;
    if (!p->host_only) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            p->cus = cus;
    }
    st = lower_nd(p, tuning);
    if (st == MOA_OK) st = stream_choice(tuning, size_t(p->total) * elem_bytes(fp64), p->stream);
    if (st != MOA_OK) {
        delete p;
        return st;
    }
    build_tables(p);
    p->ws_bytes = 0;
    return finalize(p, out);
}

moa_status_t moa_fft_plan_nd(moa_fft_plan_t* out, int32_t rank, const int64_t* dims, int64_t batch,
                             moa_fft_dtype_t dtype, moa_fft_prec_t prec, uint32_t flags)
{
    return moa_fft_plan_nd_tuned(out, rank, dims, batch, dtype, prec, flags, nullptr);
}

moa_status_t moa_fft_plan_batched_tuned(moa_fft_plan_t* out, const int64_t* sizes, int64_t count,
                                        moa_fft_dtype_t dtype, uint32_t flags, const moa_fft_tuning_t* tuning)
{
    if (!out || !sizes) return MOA_ERR_NULL;
    moa_status_t st = check_common(dtype, MOA_FFT_PREC_NATIVE, flags);
    if (st != MOA_OK) return st;
    if (count < 1 || count > (int64_t(1) << 28)) return MOA_ERR_BATCH;
    moa_fft_plan_s* p = new (std::nothrow) moa_fft_plan_s();
    if (!p) return MOA_ERR_ALLOC;
    p->batched = true;
    p->fp64 = dtype == MOA_C128;
    p->flags = flags;
    p->host_only = (flags & MOA_FFT_FLAG_HOST_ONLY) != 0;
    p->sizes.assign(sizes, sizes + count);
    p->batch = count;
    st = plan_uneven(p, tuning);
    if (st == MOA_OK) st = stream_choice(tuning, size_t(p->total) * elem_bytes(p->fp64), p->stream);
    if (st != MOA_OK) {
        delete p;
        return st;
    }
    p->tab_host.clear();
    p->tw_blk_off = add_block_table(p);
    return finalize(p, out);
}

moa_status_t moa_fft_plan_batched(moa_fft_plan_t* out, const int64_t* sizes, int64_t count, moa_fft_dtype_t dtype,
                                  uint32_t flags)
{
    return moa_fft_plan_batched_tuned(out, sizes, count, dtype, flags, nullptr);
}

moa_status_t moa_fft_exec(moa_fft_plan_t p, moa_fft_dir_t dir, const void* in, void* out, void* stream)
{
    if (const moa_status_t hs = check_plan(p)) return hs;
    if (!in || !out) return MOA_ERR_NULL;
    if (dir != MOA_FFT_FORWARD && dir != MOA_FFT_ADJOINT) return MOA_ERR_ARG;
    if (p->host_only) return MOA_ERR_STATE;
    if (p->ws_bytes && !p->d_ws) return MOA_ERR_STATE;  // planned without a workspace
    if (!exec_aligned(p, in, out)) return MOA_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!(p->flags & MOA_FFT_FLAG_GRAPH)) return launch_all(p, int(dir), in, out, p->d_ws, s);
    std::lock_guard<std::mutex> lock(p->mu);
    GraphEntry* hit = nullptr;
    for (GraphEntry& g : p->graphs)
        if (g.dir == int(dir) && g.in == in && g.out == out) hit = &g;
    if (!hit) {
        if (p->graphs.size() >= 8) {
            GraphEntry& old = p->graphs.front();
            if (old.exec) (void)hipGraphExecDestroy(old.exec);
            if (old.graph) (void)hipGraphDestroy(old.graph);
            p->graphs.erase(p->graphs.begin());
        }
        GraphEntry g;
        moa_status_t st = make_graph(p, int(dir), in, out, g);
        if (st != MOA_OK) return st;
        p->graphs.push_back(g);
        hit = &p->graphs.back();
    }
    return hipGraphLaunch(hit->exec, s) == hipSuccess ? MOA_OK : MOA_ERR_HIP;
}

moa_status_t moa_fft_exec_level(moa_fft_plan_t p, moa_fft_dir_t dir, int32_t level, const void* in, void* out,
                                void* stream)
{
    if (const moa_status_t hs = check_plan(p)) return hs;
    if (!in || !out) return MOA_ERR_NULL;
    if (dir != MOA_FFT_FORWARD && dir != MOA_FFT_ADJOINT) return MOA_ERR_ARG;
    if (p->host_only && !p->batched && level >= 0 && size_t(level) < p->passes.size()) return MOA_ERR_STATE;
    if (p->batched) {
        // An uneven batch: level = one size group of a per-size plan, or the
        // single fused launch (level 0).
        const bool per_size = (p->flags & MOA_FFT_FLAG_PER_SIZE) != 0;
        const int groups = per_size ? int(p->size_ranges.size()) : 1;
        if (level < 0 || level >= groups) return MOA_ERR_ARG;
        if (p->host_only) return MOA_ERR_STATE;
        const int task0 = per_size ? p->size_ranges[size_t(level)].first : 0;
        const int ntasks = per_size ? p->size_ranges[size_t(level)].second : int(p->tasks.size());
        moa::BatchArgs a = batch_args(p, int(dir), in, out, task0, ntasks);
        return moa::launch_batched(p->fp64, a, per_size ? ntasks : p->batch_grid, p->batch_threads, p->batch_lds,
                                   static_cast<hipStream_t>(stream)) == hipSuccess
                   ? MOA_OK
                   : MOA_ERR_HIP;
    }
    if (level < 0 || size_t(level) >= p->passes.size()) return MOA_ERR_ARG;
    if (p->host_only) return MOA_ERR_STATE;
    const PassDesc& d = p->passes[size_t(level)];
    if (!pair_aligned(d, in, out, true, true)) return MOA_ERR_ARG;
    // In place only where the level stores in its load pattern.
    const size_t P = p->passes.size();
    if (in == out && p->dims.empty() && P > 1) {
        const bool last = size_t(level) + 1 == P;
        const bool blocked = d.out_lgb != moa::kNoBlock || d.out_pair_s || d.out_tile_s;
        if (last || (level == 0 && blocked)) return MOA_ERR_ARG;
    }
    moa::PassArgs args[moa::kMaxPasses];
    pass_args(p, int(dir), in, out, p->d_ws, args);
    moa::PassArgs& a = args[size_t(level)];
    // One level runs from `in` to `out` whatever its position (the middle
    // levels of a whole execution read and write the workspace).
    a.in = in;
    a.out = out;
    return moa::launch_pass(p->fp64, p->passes[size_t(level)], a,
                            static_cast<hipStream_t>(stream)) == hipSuccess
               ? MOA_OK
               : MOA_ERR_HIP;
}

moa_status_t moa_fft_num_levels(moa_fft_plan_t p, int32_t* levels)
{
    if (const moa_status_t hs = check_plan(p)) return hs;
    if (!levels) return MOA_ERR_NULL;
    if (p->batched)
        *levels = (p->flags & MOA_FFT_FLAG_PER_SIZE) ? int32_t(p->size_ranges.size()) : 1;
    else
        *levels = int32_t(p->passes.size());
    return MOA_OK;
}

moa_status_t moa_fft_workspace_size(moa_fft_plan_t p, size_t* bytes)
{
    if (const moa_status_t hs = check_plan(p)) return hs;
    if (!bytes) return MOA_ERR_NULL;
    *bytes = p->ws_bytes;
    return MOA_OK;
}

moa_status_t moa_fft_describe_size(moa_fft_plan_t p, size_t* bytes)
{
    if (const moa_status_t hs = check_plan(p)) return hs;
    if (!bytes) return MOA_ERR_NULL;
    *bytes = describe_json(p).size() + 1;
    return MOA_OK;
}

moa_status_t moa_fft_describe(moa_fft_plan_t p, char* buf, size_t len)
{
    if (const moa_status_t hs = check_plan(p)) return hs;
    if (!buf) return MOA_ERR_NULL;
    const std::string s = describe_json(p);
    if (len == 0) return MOA_ERR_ARG;
    const size_t k = std::min(len - 1, s.size());
    memcpy(buf, s.data(), k);
    buf[k] = '\0';
    return (s.size() + 1 <= len) ? MOA_OK : MOA_ERR_ARG;
}

moa_status_t moa_fft_destroy(moa_fft_plan_t p)
{
    if (!p) return MOA_OK;
    {
        std::lock_guard<std::mutex> lock(registry_mutex());
        if (registry().erase(p) == 0) return MOA_ERR_STATE;
    }
    release(p);
    p->magic = 0;
    delete p;
    return MOA_OK;
}

}  // extern "C"
