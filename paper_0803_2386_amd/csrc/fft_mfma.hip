// Split-precision matrix-core pass kernel: every radix-16 stage of a level is
// a dense 16-point DFT contraction on the gfx950 matrix cores.
//
// The general-radix butterfly of Ch. 1 (Fig. radnbutterfly) computes, for
// twiddled inputs c_l, the outputs z_k = sum_l c_l E^(k l mod 16) -- a dense
// 16 x 16 complex matrix-vector product.  A wave gathers 16 such butterflies
// as the 16 columns of the B operand of v_mfma_f32_16x16x32_{bf16,f16}: the
// 16 complex inputs of a butterfly are 32 real rows (re, im interleaved), and
// the real 32 x 32 form of the DFT matrix,
//     [Re y_q]   [ c  -s ] [Re x_p]
//     [Im y_q] = [ s   c ] [Im x_p],   c + i s = omega_16^(p q),
// is the A operand in two 16-row halves.  Each operand is split into a high
// and a low half-precision part (x = hi + lo); three products hi*hi + hi*lo +
// lo*hi are accumulated in float32 (the lo*lo term is below the accumulated
// rounding).  Twiddles, the inter-level factor and all other arithmetic stay
// float32.  For fp16 the data are scaled by an exact power of two before the
// split (the square root of the growth bound of the stages before it), so
// that both parts stay in the normal fp16 range, and unscaled after.
//
// Operand layouts of the 16x16x32 MFMA (lane l, 0 <= l < 64):
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + i], i < 8
//   B (32 x 16): lane l holds B[8 (l / 16) + i][l % 16], i < 8
//   D (16 x 16): lane l holds D[4 (l / 16) + i][l % 16], i < 4
// so lane l of a group owns points 4g..4g+3 (g = l / 16) of butterfly l % 16
// on input and frequencies {2g, 2g+1, 8+2g, 9+2g} on output.  A wave works
// on 8 groups of 16 butterflies per stage (32 points per thread).
#include "fft_device.h"

namespace moa {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

template <int PREC> struct SplitT;
template <> struct SplitT<1> {
    using S = __bf16;
    using V8 = bf16x8;
    static __device__ __forceinline__ floatx4 mma(V8 a, V8 b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct SplitT<2> {
    using S = _Float16;
    using V8 = half8;
    static __device__ __forceinline__ floatx4 mma(V8 a, V8 b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Entry (row, col) of the real 32 x 32 DFT matrix.
__device__ __forceinline__ double dft32_entry(int row, int col, float sign)
{
    const int q = row >> 1, p = col >> 1;
    const int e = (p * q) & 15;
    const double c = cos16(e), s = double(sign) * sin16(e);
    if ((row & 1) == 0) return (col & 1) == 0 ? c : -s;
    return (col & 1) == 0 ? s : c;
}

template <int LGN, int PREC>
__global__ void __launch_bounds__(kMaxThreads) k_pass_mfma(PassArgs a)
{
    using V = float2;
    using Sp = SplitT<PREC>;
    using S = typename Sp::S;
    using V8 = typename Sp::V8;
    constexpr int N = 1 << LGN;
    constexpr int NST = LGN / 4;  // radix-16 stages, all on the matrix cores
    static_assert(LGN % 4 == 0 && LGN >= 4, "matrix-core levels are powers of 16");
    constexpr int NB = N / 16;    // butterflies per column per stage
    constexpr int GPW = 8;        // butterfly groups per wave
    constexpr int PPT = 32;       // points per thread

    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    V* tl = lds + a.data_elems;   // in-block twiddles (256)
    V* tt = tl + kTwBlkEntries;   // inter-level twiddles (256 per part)
    const float sign = a.sign;
    const int lgw = a.lgw, W = 1 << lgw;
    const int t = threadIdx.x, T = blockDim.x;
    const int cs = a.col_stride;

    uint32_t bid = blockIdx.x;
    if (a.xcd_remap) bid = (bid & 7u) * (gridDim.x >> 3) + (bid >> 3);
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

    {
        const V* g1 = reinterpret_cast<const V*>(a.tw_blk);
        for (int i = threadIdx.x; i < kTwBlkEntries; i += blockDim.x) tl[i] = g1[i];
        const V* g2 = reinterpret_cast<const V*>(a.tw_inter);
        for (int i = threadIdx.x; i < 256 * a.tw_parts; i += blockDim.x) tt[i] = g2[i];
    }
    // Coalesced copy of the tile into LDS along whichever axis is unit-stride;
    // each thread moves PPT points (T = W N / PPT) and issues all its loads
    // before the first LDS store.
    {
        const V* __restrict__ src = reinterpret_cast<const V*>(a.in) + ib;
        const bool tf = a.in_s[0] == 1 && W > 1;
#pragma unroll
        for (int half = 0; half < PPT / 16; ++half) {
            V tmp[16];
            int slot[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int i = t + (half * 16 + m) * T;
                int w, e;
                if (tf) {
                    w = i & (W - 1);
                    e = i >> lgw;
                } else {
                    e = i & (N - 1);
                    w = i >> LGN;
                }
                slot[m] = w * cs + lds_pad(e);
                tmp[m] = src[int64_t(w) * a.in_s[0] + int64_t(e) * a.in_s_e];
            }
#pragma unroll
            for (int m = 0; m < 16; ++m) lds[slot[m]] = tmp[m];
        }
    }

    // A operand fragments of this lane: two 16-row halves, hi and lo parts.
    const int lane = t & 63, wave = t >> 6;
    const int g = lane >> 4;
    V8 ahi[2], alo[2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const double v = dft32_entry(16 * h + (lane & 15), 8 * g + i, sign);
            const S hi = S(float(v));
            ahi[h][i] = hi;
            alo[h][i] = S(float(v - double(float(hi))));
        }
    __syncthreads();

#pragma unroll
    for (int s = 0; s < NST; ++s) {
        const int lgns = 4 * s;
        const int ns = 1 << lgns;
        // Exact power-of-two scaling for fp16 (see the file comment).
        const int lgscale = PREC == 2 ? (a.pre_lg + lgns) / 2 : 0;
        const float down = __builtin_ldexpf(1.0f, -lgscale), up = __builtin_ldexpf(1.0f, lgscale);
        V y[GPW][4];
        int bidx[GPW], widx[GPW];
#pragma unroll
        for (int grp = 0; grp < GPW; ++grp) {
            const int bf = wave * (16 * GPW) + grp * 16 + (lane & 15);  // flat butterfly index
            const int w = bf >> (LGN - 4), b = bf & (NB - 1);
            bidx[grp] = b;
            widx[grp] = w;
            const V* col = lds + w * cs;
            V8 bhi, blo;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 4 * g + i;
                V x = col[lds_pad(b + r * NB)];
                if (s > 0) {
                    const int e = ((b & (ns - 1)) * r) << (kLgTwBlk - lgns - 4);
                    V tw = tw_blk(tl, e);
                    tw.y = -sign * tw.y;
                    x = cmul(x, tw);
                }
                const float xr = x.x * down, xi = x.y * down;
                const S hr = S(xr), hi_ = S(xi);
                bhi[2 * i] = hr;
                bhi[2 * i + 1] = hi_;
                blo[2 * i] = S(xr - float(hr));
                blo[2 * i + 1] = S(xi - float(hi_));
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = Sp::mma(ahi[h], bhi, acc);
                acc = Sp::mma(ahi[h], blo, acc);
                acc = Sp::mma(alo[h], bhi, acc);
                y[grp][2 * h] = mkc(acc[0] * up, acc[1] * up);
                y[grp][2 * h + 1] = mkc(acc[2] * up, acc[3] * up);
            }
        }
        __syncthreads();
#pragma unroll
        for (int grp = 0; grp < GPW; ++grp) {
            const int b = bidx[grp];
            V* col = lds + widx[grp] * cs;
            const int base = ((b >> lgns) << (lgns + 4)) + (b & (ns - 1));
            // outputs q = 2g, 2g+1, 8+2g, 9+2g
            col[lds_pad(base + (2 * g) * ns)] = y[grp][0];
            col[lds_pad(base + (2 * g + 1) * ns)] = y[grp][1];
            col[lds_pad(base + (8 + 2 * g) * ns)] = y[grp][2];
            col[lds_pad(base + (9 + 2 * g) * ns)] = y[grp][3];
        }
        __syncthreads();
    }

    // Copy out along the output's unit-stride axis, with the inter-level
    // twiddle; each thread's loads (LDS and twiddle tables) all precede its
    // stores.
    {
        V* __restrict__ dst = reinterpret_cast<V*>(a.out) + ob;
        const bool tf = a.out_s[0] == 1 && W > 1;
#pragma unroll
        for (int half = 0; half < PPT / 16; ++half) {
            V v[16];
            int wi[16], ki[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int i = t + (half * 16 + m) * T;
                if (tf) {
                    wi[m] = i & (W - 1);
                    ki[m] = i >> lgw;
                } else {
                    ki[m] = i & (N - 1);
                    wi[m] = i >> LGN;
                }
                v[m] = lds[wi[m] * cs + lds_pad(ki[m])];
            }
            if (a.tw_parts) {
                const uint64_t mask = (uint64_t(1) << a.tw_lgroot) - 1;
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    V tw = tw_inter(tt, a.tw_parts, (uint64_t(d0 + wi[m]) * uint64_t(ki[m])) & mask);
                    tw.y = -sign * tw.y;
                    v[m] = cmul(v[m], tw);
                }
            }
#pragma unroll
            for (int m = 0; m < 16; ++m) dst[int64_t(wi[m]) * a.out_s[0] + int64_t(ki[m]) * a.out_s_k] = v[m];
        }
    }
}

using PassFn = void (*)(PassArgs);

#define MOA_MFMA_ROW(L) \
    { &k_pass_mfma<L, 1>, &k_pass_mfma<L, 2> }

// Levels of 2^4 .. 2^12 points (powers of 16).
static const PassFn kMfma[4][2] = {MOA_MFMA_ROW(4), MOA_MFMA_ROW(8), MOA_MFMA_ROW(12), {nullptr, nullptr}};

static PassFn mfma_lookup(int lgn, int prec)
{
    if (lgn % 4 != 0 || lgn < 4 || lgn > 12 || prec < 1 || prec > 2) return nullptr;
    return kMfma[lgn / 4 - 1][prec - 1];
}

const void* mfma_kernel_fn(const PassDesc& d) { return reinterpret_cast<const void*>(mfma_lookup(d.lgn, d.mfma)); }

hipError_t prepare_mfma_kernel(const PassDesc& d)
{
    PassFn f = mfma_lookup(d.lgn, d.mfma);
    if (!f) return hipErrorInvalidValue;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                               d.lds_bytes);
}

hipError_t launch_mfma(const PassDesc& d, const PassArgs& a, hipStream_t s)
{
    PassFn f = mfma_lookup(d.lgn, d.mfma);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(unsigned(d.grid)), dim3(unsigned(d.threads)), d.lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace moa
