// Pass kernel of the dimension-lifted FFT for gfx950 (k_pass), shared by the
// radix-16 instantiations (fft_kernels.hip) and the other register radices
// (fft_radix.hip).
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
//
// The grid is persistent: each workgroup walks a run of tiles and issues the
// loads of its next tile before it transforms the current one, so the HBM
// transfer of one tile overlaps the LDS/VALU work of the previous one.  All
// twiddles come from small LDS tables, leaving the in-order vector-memory
// counter to the data loads.  On each XCD the resident workgroups take
// consecutive tiles, so tiles that share cache lines meet in the same L2.
#pragma once

#include "fft_device.h"

namespace moa {

// Load the points of tile `tile_id` this thread owns (slot order of stage 0).
template <int LGN, int LGE, int LGRAD, typename V>
__device__ __forceinline__ void prefetch_now(const PassArgs& a, uint64_t tile_id, int64_t& d0, int64_t& ib,
                                             int64_t& ob, const V* gin, int w, int j, V* vn)
{
    constexpr int LE = lg_e(LGN, LGE);
    constexpr int TPC = 1 << (LGN - LE);
    tile_offsets(a, tile_id, d0, ib, ob);
    const V* src = gin + ib + int64_t(w) * a.in_s[0];
    // The caller's input streams past the caches (complex64; the complex128
    // kernels keep one load path, their registers are full).
    if (sizeof(V) == 8 && a.nt_in) {
#pragma unroll
        for (int m = 0; m < (1 << LE); ++m) vn[in_slot<LGN, LGE, LGRAD>(m)] = load_once(src + int64_t(j + m * TPC) * a.in_s_e);
    } else {
#pragma unroll
        for (int m = 0; m < (1 << LE); ++m) vn[in_slot<LGN, LGE, LGRAD>(m)] = src[int64_t(j + m * TPC) * a.in_s_e];
    }
}

// Kernel modes: 0 = 16 points a thread, <= 512 threads, next tile prefetched;
// 1 = 32 points a thread, <= 512 threads, prefetched (levels that store in
// their load pattern); 2 = 16 points a thread, <= 1024 threads, no prefetch
// (large tiles whose store goes through LDS: two tiles do not fit the VGPRs).
__host__ __device__ constexpr int mode_lge(int km) { return km == 1 ? 5 : 4; }
__host__ __device__ constexpr int mode_threads(int km) { return km == 2 ? 1024 : 512; }

// LGRAD: log2 of the largest radix of the level's register stages (the
// general-radix block of Ch. 1; 4 = radix 16 by default, 2..5 selectable
// through the tuning block, at most the points a thread holds).
template <typename R, int LGN, int KM, bool TIN, bool TOUT, int LGRAD = kLgRadix>
__global__ void __launch_bounds__(mode_threads(KM)) k_pass(PassArgs a)
{
    using V = typename cpx<R>::V;
    constexpr int LGE = mode_lge(KM);
    constexpr int LE = lg_e(LGN, LGE);
    constexpr int E = 1 << LE;
    constexpr int LGTPC = LGN - LE;
    constexpr int TPC = 1 << LGTPC;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    V* tl = lds + a.data_elems;          // in-block twiddles (256)
    V* tt = tl + kTwBlkEntries;          // inter-level twiddles (256 per part)
    const R sign = (R)a.sign;
    const int lgw = a.lgw;
    const int t = threadIdx.x, T = blockDim.x;
    int w, j;
    if constexpr (TIN) {
        w = t & ((1 << lgw) - 1);
        j = t >> lgw;
    } else {
        j = t & (TPC - 1);
        w = t >> LGTPC;
    }

    {
        // A level of one radix stage has no stage twiddles: it skips the
        // in-block table (a short level may run on a single thread).
        if constexpr (n_stages(LGN, LGRAD) > 1) {
            const V* g1 = reinterpret_cast<const V*>(a.tw_blk);
            for (int i = t; i < kTwBlkEntries; i += T) tl[i] = g1[i];
        }
        const V* g2 = reinterpret_cast<const V*>(a.tw_inter);
        for (int i = t; i < 256 * a.tw_parts; i += T) tt[i] = g2[i];
    }
    __syncthreads();

    // Tile run of this workgroup.
    uint64_t tile, end, step;
    if (a.xcd_remap) {
        const uint64_t per_xcd = gridDim.x >> 3;
        const uint64_t chunk = (uint64_t(a.ntiles) + 7) >> 3;
        const uint64_t x = blockIdx.x & 7u;
        tile = x * chunk + (blockIdx.x >> 3);
        end = min(uint64_t(a.ntiles), (x + 1) * chunk);
        step = per_xcd;
    } else {
        tile = blockIdx.x;
        end = uint64_t(a.ntiles);
        step = gridDim.x;
    }

    const V* __restrict__ gin = reinterpret_cast<const V*>(a.in);
    V* __restrict__ gout = reinterpret_cast<V*>(a.out);
    V v[E];
    int64_t d0 = 0, ib = 0, ob = 0;
    if (tile < end) {
        tile_offsets(a, tile, d0, ib, ob);
        const V* src = gin + ib + int64_t(w) * a.in_s[0];
        if (sizeof(V) == 8 && a.nt_in) {  // as in prefetch_now
#pragma unroll
            for (int m = 0; m < E; ++m) v[in_slot<LGN, LGE, LGRAD>(m)] = load_once(src + int64_t(j + m * TPC) * a.in_s_e);
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) v[in_slot<LGN, LGE, LGRAD>(m)] = src[int64_t(j + m * TPC) * a.in_s_e];
        }
    }
    // Mode 2 runs one tile per workgroup (grid = tiles): without a prefetch a
    // tile loop buys nothing and costs registers.
    constexpr bool kPersistent = KM != 2;
    for (int once = 0; kPersistent ? (tile < end) : (once == 0 && tile < end); ++once) {
        // Hide the thread coordinates from loop-invariant code motion: every
        // LDS address of the stages derives from them, and hoisting those
        // out of the tile loop would keep hundreds of addresses live.
        asm volatile("" : "+v"(j), "+v"(w));
        V* col = lds + w * a.col_stride;
        const uint64_t next = tile + step;
        int64_t nd0 = 0, nib = 0, nob = 0;
        V vn[E];
        // Prefetch the next tile of the run into registers: before the stages
        // when the store needs no LDS pass, else once the stage outputs have
        // left the registers for LDS (so both tiles never sit in VGPRs while
        // the stages run).
        // complex128 plans are for accuracy, not bandwidth: no prefetch there.
        constexpr bool kPrefetch = sizeof(R) == 4 && KM != 2;
        auto prefetch = [&]() {
            if (kPrefetch && next < end) prefetch_now<LGN, LGE, LGRAD>(a, next, nd0, nib, nob, gin, w, j, vn);
        };
        if constexpr (TIN == TOUT) prefetch();

        V tw[kMaxStageTw];
        run_stages<R, LGN, LGE, 0, false, LGRAD>(v, col, j, sign, tl, true, tw);

        // Store phase.  rank(m): the output row of slot m is jst + rank * TPC.
        int wst = w, jst = j;
        if constexpr (TIN != TOUT) {
            if constexpr (n_stages(LGN, LGRAD) > 1) __syncthreads();
#pragma unroll
            for (int m = 0; m < E; ++m) col[lds_pad(j + out_slot_rank<LGN, LGE, LGRAD>(m) * TPC)] = v[m];
            prefetch();
            __syncthreads();
            if constexpr (TOUT) {
                wst = t & ((1 << lgw) - 1);
                jst = t >> lgw;
            } else {
                jst = t & (TPC - 1);
                wst = t >> LGTPC;
            }
            const V* col2 = lds + wst * a.col_stride;
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = col2[lds_pad(jst + m * TPC)];
        }
        auto rank = [&](int m) {
            if constexpr (TIN == TOUT) return out_slot_rank<LGN, LGE, LGRAD>(m);
            else return m;
        };
        // The inter-level factor only occurs on levels that store in their
        // load pattern (every level but the last); the planner guarantees it.
        if (TIN == TOUT && a.tw_parts) {
            // omega^(dcol * (jst + rank * TPC)) = base * prod over the set bits
            // b of rank of omega^(dcol * TPC * 2^b).
            const uint64_t mask = (uint64_t(1) << a.tw_lgroot) - 1;
            const uint64_t dcol = uint64_t(d0 + wst);
            V base = tw_inter(tt, a.tw_parts, (dcol * uint64_t(jst)) & mask);
            base.y = -sign * base.y;
            V pw[LE > 0 ? LE : 1];
#pragma unroll
            for (int b = 0; b < LE; ++b) {
                pw[b] = tw_inter(tt, a.tw_parts, (dcol * (uint64_t(TPC) << b)) & mask);
                pw[b].y = -sign * pw[b].y;
            }
#pragma unroll
            for (int m = 0; m < E; ++m) {
                V f = base;
#pragma unroll
                for (int b = 0; b < LE; ++b)
                    if (rank(m) & (1 << b)) f = cmul(f, pw[b]);
                v[m] = cmul(v[m], f);
            }
        }
        V* dst = gout + ob + int64_t(wst) * a.out_s[0];
        if (sizeof(V) == 8 && a.nt_out) {  // output written once, in whole lines
#pragma unroll
            for (int m = 0; m < E; ++m) store_once(dst + int64_t(jst + rank(m) * TPC) * a.out_s_k, v[m]);
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) dst[int64_t(jst + rank(m) * TPC) * a.out_s_k] = v[m];
        }

        if constexpr (!kPersistent) break;
        __syncthreads();  // the next tile overwrites the LDS exchange buffer
        if (!kPrefetch && next < end) prefetch_now<LGN, LGE, LGRAD>(a, next, nd0, nib, nob, gin, w, j, vn);
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = vn[m];
        tile = next;
        d0 = nd0;
        ib = nib;
        ob = nob;
    }
}

}  // namespace moa
