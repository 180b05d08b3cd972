// Internal interfaces between the host planner (plan.cpp, psi.hpp) and the
// gfx950 kernels (fft_kernels.hip, fft_pair.hip, fft_batched.hip, fft_mfma.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/moa_fft.h"

namespace moa {

constexpr int kMaxDigits = 8;     // batch digits of one pass descriptor
constexpr int kMaxPasses = 8;     // passes of one plan (lift rank or array rank <= 8)
constexpr int kLgRadixDefault = 4;  // register stages of radix 16 unless tuned otherwise
constexpr int kMaxThreads = 512;  // level-kernel workgroup limit (1024: staged-store, paired-column and batch kernels)
constexpr int kLdsBytes = 160 * 1024;
constexpr int kNoBlock = 30;      // lgb of an axis with one plain stride
constexpr int kMaxLgBlockC64 = 14;  // 2^14 complex64 = 128 KiB (+pad) in LDS
constexpr int kMaxLgBlockC128 = 13; // 2^13 complex128
constexpr int kLgSmallMin = 4;      // one short transform: 2^4 .. 2^12 points
constexpr int kLgSmallMax = 12;     // on N / 4 threads (fft_small.hip)
constexpr int kLgSmallMaxC128 = 11; // complex128 2^12: the level kernel is faster
constexpr int kLgSmallDirect = 8;   // up to 2^8 points the kernel builds a table of omega_N
// A batch of short transforms runs one workgroup per transform while that
// beats the level kernel's tiles of several transforms: at most 2048
// transforms and 2^19 points in all (measured crossover 2^19 .. 2^21 points).
constexpr int64_t kSmallMaxBatch = 2048;
constexpr int kLgSmallMaxPoints = 19;

// Entries of the in-block twiddle table kept in LDS (two halves of 128).
constexpr int kTwBlkEntries = 256;
// LDS elements after the tables of a matrix-core level: 16 floats, the
// per-wave maxima from which an fp16 tile takes its scale.
constexpr int kMfmaScaleElems = 8;

// LDS twiddle entries of the short-transform kernel: omega_N^e for e < N up
// to 2^kLgSmallDirect points, else a copy of the in-block table.
__host__ __device__ constexpr inline int small_table_entries(int lgn)
{
    return lgn <= kLgSmallDirect ? (1 << lgn) : kTwBlkEntries;
}

// Elements each thread keeps in registers across a pass (the radix of the
// register-resident stages) is 2^lge, lge = 4 or 5; a transform shorter than
// that uses one thread.
constexpr int kLgE = 4;  // the default; tiles that would need more than 512 threads use 5

// Element index -> padded LDS slot: one spare slot after every 16 elements
// breaks the power-of-two strides of the butterfly exchanges across banks.
__host__ __device__ constexpr inline int lds_pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr inline int lds_padded_len(int n) { return n + (n >> 4); }

// Column stride (elements) of the LDS tile that holds several transforms side
// by side.  It is the padded length rounded up so that 16 consecutive lanes
// (the lanes served by one LDS cycle for 8-byte accesses) fall on distinct
// 8-byte bank pairs: lanes_per_col consecutive rows of each of the
// 16/lanes_per_col columns they cover.
__host__ __device__ constexpr inline int lds_col_stride(int n, int lanes_per_col)
{
    int base = lds_padded_len(n);
    int want = lanes_per_col >= 16 ? 0 : (lanes_per_col <= 0 ? 1 : lanes_per_col);
    if (want == 0) return base;
    int r = base & 31;
    int add = (want - r + 32) & 31;
    return base + add;
}

// One pass of a lifted plan in operational normal form: a DFT of length
// 2^lgn along one axis (in stride in_s_e, out stride out_s_k) for every
// combination of the batch digits.  Digit 0 is the tile digit: a workgroup
// takes 2^lgw consecutive values of it.  All digit sizes are powers of two,
// so block-index decoding is shifts and masks only -- except the last digit
// (the batch of transforms), which may have any size: it takes whatever is
// left of the block index.  A lone digit 0 is tiled by a width dividing it.
struct PassDesc {
    int lgn = 0;
    int64_t in_s_e = 0, out_s_k = 0;
    int nd = 0;
    int64_t size[kMaxDigits] = {0};
    int lg[kMaxDigits] = {0};
    int64_t in_s[kMaxDigits] = {0};
    int64_t out_s[kMaxDigits] = {0};
    int lgw = 0;                  // log2 transforms per workgroup (tile width)
    int lge = kLgE;               // log2 points per thread
    int kmode = 0;                // level kernel variant (fft_kernels.hip; 3 = paired columns, fft_pair.hip;
                                  // 4 = one short transform, fft_small.hip)
    // Inter-level twiddle omega_{2^tw_lgroot}^(d0 * k), d0 = value of digit 0.
    int tw = 0;
    int tw_lgroot = 0;
    int tw_parts = 0;             // byte-wise parts of the exponent (256-entry tables each)
    int64_t tw_inter_off = 0;     // offset (elements) of the part tables in the plan's table buffer
    // Launch shape (filled by the planner).
    bool in_tile_fast = false;    // digit 0 is the unit-stride input axis
    bool out_tile_fast = false;   // digit 0 is the unit-stride output axis
    int threads = 0;
    int col_stride = 0;           // LDS column stride in elements
    int64_t blocks = 0;           // tiles (logical workgroups)
    int64_t grid = 0;             // resident workgroups of the persistent launch
    int data_elems = 0;           // LDS elements of the data tile (tables follow)
    int lds_bytes = 0;
    int xcd_remap = 0;
    int mfma = 0;                 // 0 = VALU radix-16, 1 = split bf16 MFMA, 2 = split fp16 MFMA
    int pre_lg = 0;               // log2 of the points transformed by earlier levels
    int lgrad = 0;                // log2 of the largest register radix of the level kernel (0: 16)
    // Blocked layouts (paired-column kernel only).  Row k of the DFT axis
    // lies at (k mod 2^lgb) * s_e + (k >> lgb) * s_hi (lgb = kNoBlock: k * s_e);
    // column w of tile t of digit 0 at t * tile_s + (w / 2) * pair_s +
    // (w mod 2) * s[0].  The defaults make both plain strides.
    int in_lgb = kNoBlock, out_lgb = kNoBlock;
    int64_t in_s_hi = 0, out_s_hi = 0;
    int64_t in_pair_s = 0, out_pair_s = 0;  // 0: 2 * s[0]
    int64_t in_tile_s = 0, out_tile_s = 0;  // 0: tile width * s[0]
};

// Kernel argument block (passed by value).
struct PassArgs {
    const void* in;
    void* out;
    int64_t in_s_e, out_s_k;
    int64_t in_s[kMaxDigits];
    int64_t out_s[kMaxDigits];
    int lg[kMaxDigits];
    int nd;
    int lgw;
    int lg_tiles;                 // log2(size of digit 0 / tile width)
    int col_stride;
    int tw_parts;                 // 0: no inter-level twiddle
    int tw_lgroot;
    const void* tw_inter;         // tw_parts x 256 entries, part p = omega^(e 2^(8p))
    const void* tw_blk;           // 2 x 128 entries: omega_{2^14}^e and omega_{2^14}^(128 e)
    int64_t ntiles;               // tiles of the launch
    int data_elems;               // LDS elements of the data tile
    int xcd_remap;
    int pre_lg;                   // log2 of the points transformed by earlier levels
    float sign;                   // -1 forward, +1 adjoint
    int nt_in;                    // 1: `in` is the caller's input, read once (streaming loads)
    int nt_out;                   // 1: streaming stores of full-line output runs (complex64 k_pass)
    // Blocked layouts (see PassDesc); the tile strides are always set.
    int in_lgb, out_lgb;
    int64_t in_s_hi, out_s_hi;
    int64_t in_pair_s, out_pair_s;
    int64_t in_tile_s, out_tile_s;
};

// A task of the uneven batch: `count` transforms of length 2^lgn whose
// element offsets are toff[first .. first + count).
struct BatchTask {
    int32_t lgn;
    int32_t count;
    int64_t first;
    int64_t off0;                 // toff[first], so a one-transform task needs no offset load
};

struct BatchArgs {
    const void* in;
    void* out;
    const BatchTask* tasks;
    const int64_t* toff;
    const void* tw_blk;
    int ntasks;
    int task0;                    // first task of this launch
    int data_elems;               // LDS elements of the exchange tile (the twiddle table follows)
    float sign;
    int nt;                       // 1: streaming loads of `in` and stores of `out`
};

// Launchers (fft_kernels.hip / fft_batched.hip / fft_mfma.hip).  They return
// hipSuccess or the launch error; they never synchronise.
hipError_t launch_pass(bool fp64, const PassDesc& d, const PassArgs& a, hipStream_t s);
hipError_t prepare_pass_kernel(bool fp64, const PassDesc& d);  // sets LDS attributes
hipError_t launch_batched(bool fp64, const BatchArgs& a, int grid, int threads, int lds_bytes,
                          hipStream_t s);
hipError_t prepare_batched_kernel(bool fp64, int lds_bytes);
// Matrix-core levels (fft_mfma.hip): lgn in {4, 8, 12}, d.mfma = 1 (bf16) or 2 (fp16).
hipError_t launch_mfma(const PassDesc& d, const PassArgs& a, hipStream_t s);
hipError_t prepare_mfma_kernel(const PassDesc& d);
const void* mfma_kernel_fn(const PassDesc& d, bool fwd);
// Paired-column levels (fft_pair.hip): complex64, lgn in [12, 14], kmode 3.
hipError_t launch_pair(const PassDesc& d, const PassArgs& a, hipStream_t s);
hipError_t prepare_pair_kernel(const PassDesc& d);
const void* pair_kernel_fn(const PassDesc& d, bool fwd);
// One short transform (fft_small.hip): a single-level plan of batch one,
// unit strides, lgn in [kLgSmallMin, kLgSmallMax], kmode 4; N / 4 threads.
hipError_t launch_small(bool fp64, const PassDesc& d, const PassArgs& a, hipStream_t s);
hipError_t prepare_small_kernel(bool fp64, const PassDesc& d);
const void* small_kernel_fn(bool fp64, const PassDesc& d, bool fwd);
// Execution on a workspace the caller of these two supplies (the
// allocation-free entry point in scratch.hip).  check_exec validates like
// moa_fft_exec, host-side only, and reports the workspace bytes the plan's
// launches need; launch_on_workspace then launches them directly (never
// through the plan's graphs) with `ws` as the workspace.
moa_status_t check_exec(moa_fft_plan_t p, int dir, const void* in, const void* out, size_t* ws_bytes);
moa_status_t launch_on_workspace(moa_fft_plan_t p, int dir, const void* in, void* out, void* ws, hipStream_t s);
// The level kernel with register stages of radix 2^d.lgrad (fft_radix.hip;
// lgrad 2, 3 or 5, complex64 levels of 2^5 .. 2^14 points); nullptr where no
// such kernel exists.
const void* radix_pass_fn(const PassDesc& d);
// The kernel function pointers, used to build HIP graph nodes.
const void* pass_kernel_fn(bool fp64, const PassDesc& d, bool fwd);
const void* batched_kernel_fn(bool fp64, bool fwd);

}  // namespace moa
