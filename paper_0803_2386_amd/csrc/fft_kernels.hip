// Pass kernel of the dimension-lifted FFT for gfx950.
//
// One launch runs one level of the lift (Ch. 3, "The General Algorithm"):
// every workgroup loads a tile of 2^lgw transforms of length N = 2^LGN (the
// columns of the lifted <... r c> view that share this level), runs all of
// the level's butterflies in VGPRs and LDS, multiplies by the inter-level
// twiddle omega_{N_l}^(d0 * k), and stores the tile at the next level's
// address pattern -- the reshape-transpose, or on the last level the final
// transpose, folded into the store.  The paper spreads the inter-level factor
// over the stages of the next level as the transformed weights
// omega_L^(sigma + j c^l) ("General Weight Sub-Matrices"): there the stage-p
// weight is omega_{2^p c^l}^sigma * omega_{2^p}^j, i.e. the next level's
// plain DIT weight evaluated at the shifted frequency k + sigma / c^l; the
// product of those factors over the level is the single multiply by
// omega_{N_l}^(d0 k) applied here (the four-step identity).
//
// Template parameters: R (float/double), LGN, and whether digit 0 (the tile
// digit) is the unit-stride axis of the input (TIN) or output (TOUT).  The
// thread <-> (column, row) map is chosen so that the global loads coalesce;
// if the store wants the other map, the tile goes back through LDS first.
#include "fft_device.h"

namespace moa {

template <typename R, typename V>
__device__ __forceinline__ V inter_level_twiddle(const PassArgs& a, int64_t d0, int k, R sign)
{
    const uint64_t mask = (uint64_t(1) << a.tw_lgroot) - 1;
    const uint64_t e = (uint64_t(d0) * uint64_t(k)) & mask;
    const V* hi = reinterpret_cast<const V*>(a.tw_hi);
    const V* lo = reinterpret_cast<const V*>(a.tw_lo);
    V w = cmul(hi[e >> a.tw_lglo], lo[e & ((uint64_t(1) << a.tw_lglo) - 1)]);
    w.y = -sign * w.y;
    return w;
}

template <typename R, int LGN, bool TIN, bool TOUT>
__global__ void __launch_bounds__(max_threads_for<R>()) k_pass(PassArgs a)
{
    using V = typename cpx<R>::V;
    constexpr int LGE = lg_e(LGN);
    constexpr int E = 1 << LGE;
    constexpr int LGTPC = LGN - LGE;
    constexpr int TPC = 1 << LGTPC;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const R sign = (R)a.sign;
    const int lgw = a.lgw;
    const int t = threadIdx.x;
    int w, j;
    if constexpr (TIN) {
        w = t & ((1 << lgw) - 1);
        j = t >> lgw;
    } else {
        j = t & (TPC - 1);
        w = t >> LGTPC;
    }

    // Logical block: the dispatcher deals blocks round-robin over the 8 XCDs;
    // remapping gives each XCD a contiguous range of tiles, so tiles that
    // share cache lines meet in the same L2.
    uint32_t bid = blockIdx.x;
    if (a.xcd_remap) bid = (bid & 7u) * (gridDim.x >> 3) + (bid >> 3);
    // Digit 0 holds the tile (alone, it may have any size); the last digit
    // takes the rest of the block index; the ones between are powers of two.
    uint64_t tile, rest;
    if (a.nd == 1) {
        tile = bid;
        rest = 0;
    } else {
        tile = bid & ((uint64_t(1) << a.lg_tiles) - 1);
        rest = uint64_t(bid) >> a.lg_tiles;
    }
    const int64_t d0 = int64_t(tile << lgw);
    int64_t ib = d0 * a.in_s[0], ob = d0 * a.out_s[0];
    for (int d = 1; d < a.nd; ++d) {
        int64_t idx;
        if (d + 1 == a.nd) {
            idx = int64_t(rest);
        } else {
            idx = int64_t(rest & ((uint64_t(1) << a.lg[d]) - 1));
            rest >>= a.lg[d];
        }
        ib += idx * a.in_s[d];
        ob += idx * a.out_s[d];
    }

    V v[E];
    {
        const V* __restrict__ src = reinterpret_cast<const V*>(a.in) + ib + int64_t(w) * a.in_s[0];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = src[int64_t(j + m * TPC) * a.in_s_e];
    }
    const V* __restrict__ twb = reinterpret_cast<const V*>(a.tw_blk);
    V* col = lds + w * a.col_stride;
    run_stages<R, LGN, 0, false>(v, col, j, sign, twb, true);

    if constexpr (TIN == TOUT) {
        V* __restrict__ dst = reinterpret_cast<V*>(a.out) + ob + int64_t(w) * a.out_s[0];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int k = out_index_of_slot<LGN>(m, j);
            V y = v[m];
            if (a.tw) y = cmul(y, inter_level_twiddle<R, V>(a, d0 + w, k, sign));
            dst[int64_t(k) * a.out_s_k] = y;
        }
    } else {
        if constexpr (n_stages(LGN) > 1) __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) col[lds_pad(out_index_of_slot<LGN>(m, j))] = v[m];
        __syncthreads();
        int w2, j2;
        if constexpr (TOUT) {
            w2 = t & ((1 << lgw) - 1);
            j2 = t >> lgw;
        } else {
            j2 = t & (TPC - 1);
            w2 = t >> LGTPC;
        }
        const V* col2 = lds + w2 * a.col_stride;
        V* __restrict__ dst = reinterpret_cast<V*>(a.out) + ob + int64_t(w2) * a.out_s[0];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int k = j2 + m * TPC;
            V y = col2[lds_pad(k)];
            if (a.tw) y = cmul(y, inter_level_twiddle<R, V>(a, d0 + w2, k, sign));
            dst[int64_t(k) * a.out_s_k] = y;
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel table: [fp64][lgn][tin][tout]
// ---------------------------------------------------------------------------
using PassFn = void (*)(PassArgs);

#define MOA_PASS_ROW(R, L) \
    { &k_pass<R, L, false, false>, &k_pass<R, L, false, true>, &k_pass<R, L, true, false>, &k_pass<R, L, true, true> }

static const PassFn kPass32[kMaxLgBlockC64 + 1][4] = {
    MOA_PASS_ROW(float, 0),  MOA_PASS_ROW(float, 1),  MOA_PASS_ROW(float, 2),  MOA_PASS_ROW(float, 3),
    MOA_PASS_ROW(float, 4),  MOA_PASS_ROW(float, 5),  MOA_PASS_ROW(float, 6),  MOA_PASS_ROW(float, 7),
    MOA_PASS_ROW(float, 8),  MOA_PASS_ROW(float, 9),  MOA_PASS_ROW(float, 10), MOA_PASS_ROW(float, 11),
    MOA_PASS_ROW(float, 12), MOA_PASS_ROW(float, 13), MOA_PASS_ROW(float, 14)};

static const PassFn kPass64[kMaxLgBlockC128 + 1][4] = {
    MOA_PASS_ROW(double, 0),  MOA_PASS_ROW(double, 1),  MOA_PASS_ROW(double, 2),  MOA_PASS_ROW(double, 3),
    MOA_PASS_ROW(double, 4),  MOA_PASS_ROW(double, 5),  MOA_PASS_ROW(double, 6),  MOA_PASS_ROW(double, 7),
    MOA_PASS_ROW(double, 8),  MOA_PASS_ROW(double, 9),  MOA_PASS_ROW(double, 10), MOA_PASS_ROW(double, 11),
    MOA_PASS_ROW(double, 12), MOA_PASS_ROW(double, 13)};

static PassFn pass_fn_lookup(bool fp64, int lgn, bool tin, bool tout)
{
    const int mode = (tin ? 2 : 0) + (tout ? 1 : 0);
    if (lgn < 0) return nullptr;
    if (fp64) return lgn <= kMaxLgBlockC128 ? kPass64[lgn][mode] : nullptr;
    return lgn <= kMaxLgBlockC64 ? kPass32[lgn][mode] : nullptr;
}

const void* pass_kernel_fn(bool fp64, const PassDesc& d)
{
    if (d.mfma) return mfma_kernel_fn(d);
    return reinterpret_cast<const void*>(pass_fn_lookup(fp64, d.lgn, d.in_tile_fast, d.out_tile_fast));
}

hipError_t prepare_pass_kernel(bool fp64, const PassDesc& d)
{
    if (d.mfma) return prepare_mfma_kernel(d);
    PassFn f = pass_fn_lookup(fp64, d.lgn, d.in_tile_fast, d.out_tile_fast);
    if (!f) return hipErrorInvalidValue;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                               d.lds_bytes);
}

hipError_t launch_pass(bool fp64, const PassDesc& d, const PassArgs& a, hipStream_t s)
{
    if (d.mfma) return launch_mfma(d, a, s);
    PassFn f = pass_fn_lookup(fp64, d.lgn, d.in_tile_fast, d.out_tile_fast);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(unsigned(d.blocks)), dim3(unsigned(d.threads)), d.lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace moa
