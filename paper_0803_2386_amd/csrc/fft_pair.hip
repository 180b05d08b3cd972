// Paired-column level kernel for complex64 levels of 2^12 .. 2^14 points.
//
// A level whose tile digit is the unit-stride axis of its input or output
// (the column FFTs of the four-step view, Ch. 3 "The General Algorithm", and
// the final transpose of the last level) touches, per row of the tile, one
// run of W adjacent elements.  A tile held in LDS has at most 2^14 points,
// i.e. W = 16384 / N columns: 32-byte runs at N = 4096, and HBM serves those
// at about half the rate of 64-byte runs (partial bursts on reads, partial
// line writes on stores).  This kernel doubles W by keeping the tile in VGPRs:
// each of 1024 threads owns two adjacent columns, 16 points of each, and moves
// both with one 16-byte access on a unit-stride side.  LDS carries only the
// butterfly exchanges, one half of the tile at a time (the even columns, then
// the odd ones), so a tile of 2^15 points needs the LDS of 2^14.
//
// The thread map is the same on both sides (pair index fastest, then row), so
// a level whose other side is not unit-stride still reads or writes runs of
// 64 / P consecutive rows per column and needs no LDS pass before its store.
// The in-block stage twiddles depend on the row only and are shared by the
// two columns of a thread.  One tile per workgroup; the XCD-aware order gives
// each XCD a contiguous run of tiles, so neighbouring tiles meet in one L2.
#include "fft_device.h"

namespace moa {

namespace {

// Byte offset helpers: every offset inside one tile is below 2^32 (the
// planner checks the span), so per-element addresses are a uniform 64-bit
// base plus a 32-bit lane offset.
__device__ __forceinline__ const float2* at(const char* base, uint32_t off)
{
    return reinterpret_cast<const float2*>(base + size_t(off));
}
__device__ __forceinline__ float2* at(char* base, uint32_t off) { return reinterpret_cast<float2*>(base + size_t(off)); }

}  // namespace

// One tile of a paired-column level (the whole kernel body; 1024 threads).
template <int LGN, bool TIN, bool TOUT, bool FWD>
__device__ __forceinline__ void pair_tile(const PassArgs& a, uint64_t tile)
{
    using V = float2;
    constexpr int E = 16;
    constexpr int TPC = 1 << (LGN - 4);
    static_assert(LGN >= 12 && LGN <= 14, "paired-column kernel covers 2^12 .. 2^14 points");

    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    V* tl = lds + a.data_elems;  // in-block twiddles (256)
    V* tt = tl + kTwBlkEntries;  // inter-level twiddles (256 per part)
    const int lgp = a.lgw - 1;   // column pairs per tile: 2^lgp
    const int t = threadIdx.x;
    const int u = t & ((1 << lgp) - 1);
    const int j = t >> lgp;

    // Twiddle tables first: their loads then retire ahead of the data loads
    // (the planner keeps 256 (1 + tw_parts) <= 2048).
    V tab[2];
    const int nt = 256 * (1 + a.tw_parts);
    {
        const V* g1 = reinterpret_cast<const V*>(a.tw_blk);
        const V* g2 = reinterpret_cast<const V*>(a.tw_inter);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = t + 1024 * k;
            if (i < nt) tab[k] = i < 256 ? g1[i] : g2[i - 256];
        }
    }

    int64_t d0, ib, ob;
    tile_offsets(a, tile, d0, ib, ob);
    const char* gin = reinterpret_cast<const char*>(a.in) + ib * int64_t(sizeof(V));
    char* gout = reinterpret_cast<char*>(a.out) + ob * int64_t(sizeof(V));

    // 32-bit strides (bytes) and lane offsets; see at().  Row r of the DFT
    // axis lies at (r mod 2^lgb) s_e + (r >> lgb) s_hi: with TPC a multiple
    // of 2^lgb (planner), rows j + m TPC step by the uniform row(TPC).
    auto row = [](uint32_t r, int lgb, uint32_t se, uint32_t shi) {
        return (r & ((1u << lgb) - 1u)) * se + (r >> lgb) * shi;
    };
    const uint32_t ju = uint32_t(j), uu = uint32_t(u);
    V v0[E], v1[E];
    {
        const uint32_t se = uint32_t(a.in_s_e), shi = uint32_t(a.in_s_hi);
        const uint32_t s0 = uint32_t(a.in_s[0]) * 8u;
        const uint32_t step = row(uint32_t(TPC), a.in_lgb, se, shi) * 8u;
        const uint32_t o0 = (uu * uint32_t(a.in_pair_s) + row(ju, a.in_lgb, se, shi)) * 8u;
        // The caller's input (first level) streams past the caches.
        const bool once = a.nt_in != 0;
        if constexpr (TIN) {
            auto ld = [&](bool nt) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const float4* p = reinterpret_cast<const float4*>(at(gin, o0 + uint32_t(m) * step));
                    const float4 x = nt ? load_once(p) : *p;
                    v0[in_slot<LGN, 4>(m)] = make_float2(x.x, x.y);
                    v1[in_slot<LGN, 4>(m)] = make_float2(x.z, x.w);
                }
            };
            if (once) ld(true);
            else ld(false);
        } else {
            const uint32_t o1 = o0 + s0;
            auto ld = [&](bool nt) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const V* p0 = at(gin, o0 + uint32_t(m) * step);
                    const V* p1 = at(gin, o1 + uint32_t(m) * step);
                    v0[in_slot<LGN, 4>(m)] = nt ? load_once(p0) : *p0;
                    v1[in_slot<LGN, 4>(m)] = nt ? load_once(p1) : *p1;
                }
            };
            if (once) ld(true);
            else ld(false);
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = t + 1024 * k;
        if (i < nt) tl[i] = tab[k];
    }
    // Stage 0 needs no twiddles; the exchange barriers publish the tables.
    pair_stages<FWD, LGN, 0>(v0, v1, lds + u * a.col_stride, j, tl);

    // Inter-level factor omega^(dcol * (j + rank * TPC)): base times the
    // powers omega^(dcol * TPC * 2^b) of the set bits b of rank.  The root
    // is at most 2^32 (planner), so exponents wrap in 32-bit arithmetic.
    const uint32_t mask = uint32_t((uint64_t(1) << a.tw_lgroot) - 1);
    auto twiddle = [&](V* v, int c) {
        const uint32_t dcol = uint32_t(d0) + 2u * uu + uint32_t(c);
        V f[E];
        f[0] = tw_inter32(tt, a.tw_parts, (dcol * ju) & mask);
        V pw[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) pw[b] = tw_inter32(tt, a.tw_parts, (dcol * (uint32_t(TPC) << b)) & mask);
        power_tree<4, false>(f, pw);
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = cmul_dir<FWD>(v[m], f[out_slot_rank<LGN, 4>(m)]);
    };

    const uint32_t sk = uint32_t(a.out_s_k), shi = uint32_t(a.out_s_hi), s0 = uint32_t(a.out_s[0]) * 8u;
    const uint32_t step = row(uint32_t(TPC), a.out_lgb, sk, shi) * 8u;
    const uint32_t o0 = (uu * uint32_t(a.out_pair_s) + row(ju, a.out_lgb, sk, shi)) * 8u;
    if constexpr (TOUT) {
        if (a.tw_parts) {
            twiddle(v0, 0);
            twiddle(v1, 1);
        }
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const uint32_t o = o0 + uint32_t(out_slot_rank<LGN, 4>(m)) * step;
            *reinterpret_cast<float4*>(at(gout, o)) = make_float4(v0[m].x, v0[m].y, v1[m].x, v1[m].y);
        }
    } else {
        // One column at a time: its factors and stores, then the next.
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            V* v = c ? v1 : v0;
            if (a.tw_parts) twiddle(v, c);
            const uint32_t o = o0 + uint32_t(c) * s0;
#pragma unroll
            for (int m = 0; m < E; ++m) *at(gout, o + uint32_t(out_slot_rank<LGN, 4>(m)) * step) = v[m];
        }
    }
}

template <int LGN, bool TIN, bool TOUT, bool FWD>
__global__ void __launch_bounds__(1024) k_pass_pair(PassArgs a)
{
    uint64_t tile = blockIdx.x;
    if (a.xcd_remap) tile = uint64_t(blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    pair_tile<LGN, TIN, TOUT, FWD>(a, tile);
}

using PairFn = void (*)(PassArgs);

#define MOA_PAIR_ROW(L, F)                                                                              \
    {                                                                                                   \
        {nullptr, &k_pass_pair<L, false, true, F>}, { &k_pass_pair<L, true, false, F>, &k_pass_pair<L, true, true, F> } \
    }

// [direction][lgn - 12][tin][tout]; a paired level has at least one unit-stride side.
static const PairFn kPair[2][3][2][2] = {
    {MOA_PAIR_ROW(12, true), MOA_PAIR_ROW(13, true), MOA_PAIR_ROW(14, true)},
    {MOA_PAIR_ROW(12, false), MOA_PAIR_ROW(13, false), MOA_PAIR_ROW(14, false)},
};

static PairFn pair_lookup(const PassDesc& d, bool fwd)
{
    if (d.lgn < 12 || d.lgn > 14) return nullptr;
    return kPair[fwd ? 0 : 1][d.lgn - 12][d.in_tile_fast ? 1 : 0][d.out_tile_fast ? 1 : 0];
}

const void* pair_kernel_fn(const PassDesc& d, bool fwd) { return reinterpret_cast<const void*>(pair_lookup(d, fwd)); }

hipError_t prepare_pair_kernel(const PassDesc& d)
{
    for (bool fwd : {true, false}) {
        PairFn f = pair_lookup(d, fwd);
        if (!f) return hipErrorInvalidValue;
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, d.lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pair(const PassDesc& d, const PassArgs& a, hipStream_t s)
{
    PairFn f = pair_lookup(d, a.sign < 0.f);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(unsigned(d.grid)), dim3(1024u), d.lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace moa
