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
// is the A operand in two 16-row halves.  (The paired-column kernel further
// down swaps the roles: the butterflies are the 16 rows of A and the DFT
// matrix is B, so that one stage's accumulators are the next stage's
// operand; see there.)  Each operand is split into a high
// and a low half-precision part (x = hi + lo); three products hi*hi + hi*lo +
// lo*hi are accumulated in float32 (the lo*lo term is below the accumulated
// rounding).  Twiddles, the inter-level factor and all other arithmetic stay
// float32.  For fp16 every tile (in the paired-column kernel, every half
// tile) is scaled on entry by an exact power of two taken from its data,
// 2^-e with e the exponent of the largest |re| or |im| it holds, so that its
// values lie below 1 whatever the input's range, and unscaled by 2^e on exit.  A radix-16 stage grows the largest value by
// at most 16 (unit twiddles), so the input of stage s stays below 16^s
// (256 at the third stage of a 4096-point level), inside fp16's range, and
// values near the tile's largest keep their low part in the normal range.
//
// Operand layouts of the 16x16x32 MFMA (lane l, 0 <= l < 64):
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + i], i < 8
//   B (32 x 16): lane l holds B[8 (l / 16) + i][l % 16], i < 8
//   D (16 x 16): lane l holds D[4 (l / 16) + i][l % 16], i < 4
// so in k_pass_mfma lane l of a group owns points 4g..4g+3 (g = l / 16) of
// butterfly l % 16 on input and frequencies {2g, 2g+1, 8+2g, 9+2g} on output.
// A wave works on 8 groups of 16 butterflies per stage (32 points per thread).
#include "fft_device.h"
#include "fft_mfma_layout.h"

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

// Largest value of m over the 64 lanes of the wave.
__device__ __forceinline__ float wave_max(float m)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    return m;
}

// Exact powers of two down = 2^-e, up = 2^e with m < 2^e (m >= 0), so that
// m * down lies in [1/2, 1); e is clamped to [-100, 100] (a zero tile).  m is
// the same in every lane: it is taken as a scalar, so the two factors live in
// scalar registers (the vector registers are the kernels' limit).
__device__ __forceinline__ void tile_scale(float m, float& down, float& up)
{
    const uint32_t bits = uint32_t(__builtin_amdgcn_readfirstlane(int(__float_as_uint(m))));
    int e = int((bits >> 23) & 0xffu) - 126;
    e = e < -100 ? -100 : (e > 100 ? 100 : e);
    down = __uint_as_float(uint32_t(127 - e) << 23);
    up = __uint_as_float(uint32_t(127 + e) << 23);
}

__device__ __forceinline__ float abs_max(float2 v, float m) { return fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y))); }

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
    // before the first LDS store.  fp16: the largest |component| of the tile
    // goes through one slot per wave after the tables.
    float* wmax = reinterpret_cast<float*>(tt + 256 * a.tw_parts);
    float tmax = 0.f;
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
                const V* p = src + int64_t(w) * a.in_s[0] + int64_t(e) * a.in_s_e;
                tmp[m] = a.nt_in ? load_once(p) : *p;
            }
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                lds[slot[m]] = tmp[m];
                if constexpr (PREC == 2) tmax = abs_max(tmp[m], tmax);
            }
        }
    }
    if constexpr (PREC == 2) {
        tmax = wave_max(tmax);
        if ((t & 63) == 0) wmax[t >> 6] = tmax;
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
    // Exact power-of-two scaling of the tile for fp16 (see the file comment).
    float down = 1.f, up = 1.f;
    if constexpr (PREC == 2) {
        float m = 0.f;
        for (int w = 0; w < (T >> 6); ++w) m = fmaxf(m, wmax[w]);
        tile_scale(m, down, up);
    }

#pragma unroll
    for (int s = 0; s < NST; ++s) {
        const int lgns = 4 * s;
        const int ns = 1 << lgns;
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
                float xr = x.x, xi = x.y;
                if (PREC == 2 && s == 0) {
                    xr *= down;
                    xi *= down;
                }
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
                if (PREC == 2 && s + 1 == NST) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] *= up;
                }
                y[grp][2 * h] = mkc(acc[0], acc[1]);
                y[grp][2 * h + 1] = mkc(acc[2], acc[3]);
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

// ---------------------------------------------------------------------------
// Paired-column matrix-core level (LGN = 8 or 12).  The tile is the one of
// the paired-column FP32 kernel -- 2^(15 - LGN) columns, 1024 threads, each
// thread two adjacent columns x 16 points moved with 16-byte accesses on a
// unit-stride side -- so the HBM traffic is the same.  The radix-16 stages
// run on half of the tile at a time (the even columns, then the odd ones)
// in LDS: the half is written to LDS in digit-reversed order, every stage
// reads its B operands from LDS (twiddled and split), contracts them on the
// matrix cores and writes its outputs back in place, and the result is read
// back in natural order.  The other half waits in registers.
// Thread maps: on a unit-stride side the pair index runs fastest across the
// lanes (runs of adjacent columns), on the other side the row does (runs of
// one column); the two maps meet through LDS.
// ---------------------------------------------------------------------------
namespace {

// x * w (forward) or x * conj(w) (adjoint) for a forward table root w.
__device__ __forceinline__ float2 cmul_fwd_or_conj(float2 x, float2 w, bool fwd)
{
    return fwd ? cmul(x, w) : mkc(x.x * w.x + x.y * w.y, x.y * w.x - x.x * w.y);
}

// Base-16 digit reversal of an index of NST digits.
template <int NST>
__device__ __forceinline__ int rev16(int p)
{
    int r = 0;
#pragma unroll
    for (int d = 0; d < NST; ++d) {
        r = (r << 4) | (p & 15);
        p >>= 4;
    }
    return r;
}

// hi + lo split of one complex value into two packed 32-bit words (re in the
// low half, im in the high half), as the operands of the contraction hold them.
template <int PREC>
__device__ __forceinline__ void split_pack(float xr, float xi, uint32_t& hw, uint32_t& lw)
{
    typedef float f2v __attribute__((ext_vector_type(2)));
    if constexpr (PREC == 1) {
        typedef __bf16 h2v __attribute__((ext_vector_type(2)));
        hw = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){xr, xi}, h2v));
        const float hr = __uint_as_float(hw << 16), hi = __uint_as_float(hw & 0xffff0000u);
        lw = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){xr - hr, xi - hi}, h2v));
    } else {
        typedef _Float16 h2v __attribute__((ext_vector_type(2)));
        hw = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){xr, xi}, h2v));
        // x - hi (exact) with the fp16 half read in place by one mixed-precision
        // fused multiply-add a component: x + (-1) * hi
        float lr, li;
        asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(lr) : "v"(hw), "v"(xr));
        asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(li) : "v"(hw), "v"(xi));
        lw = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){lr, li}, h2v));
    }
}

// The data of a stage are the A operand of the contraction (row c: the
// butterfly, 32 columns: its 16 complex inputs, re and im interleaved; lane
// (g, c) holds inputs 4g .. 4g+3 of butterfly c), the DFT matrix is the B
// operand in two halves (columns: the real parts of the 16 outputs, then
// their imaginary parts).  So lane (g, q) receives output q of butterflies
// 4g .. 4g+3, real part from half 0 and imaginary part from half 1 -- which
// is the A-operand layout of the next radix-16 stage when that stage's
// butterfly q combines output q of these 16 butterflies: stages 0 and 1 of a
// level run back to back in registers, with no exchange between them.

// hi + lo split of a lane's four inputs into the A operand.
template <int PREC, bool SCALE, typename V8>
__device__ __forceinline__ void split_inputs(const float2 (&x)[4], float mul, V8& dhi, V8& dlo)
{
    union Op {
        V8 v;
        uint32_t w[4];
    } hi, lo;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float xr = x[i].x, xi = x[i].y;
        if constexpr (SCALE) {
            xr *= mul;
            xi *= mul;
        }
        split_pack<PREC>(xr, xi, hi.w[i], lo.w[i]);
    }
    dhi = hi.v;
    dlo = lo.v;
}

// Three split products per half: acc[h][i] = half h (re / im) of output q of
// the lane's butterfly group rows 4g + i.
template <int PREC, typename V8>
__device__ __forceinline__ void contract(const V8& dhi, const V8& dlo, const V8 (&fhi)[2], const V8 (&flo)[2],
                                         floatx4 (&acc)[2])
{
    using Sp = SplitT<PREC>;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        floatx4 a = {0.f, 0.f, 0.f, 0.f};
        a = Sp::mma(dhi, fhi[h], a);
        a = Sp::mma(dhi, flo[h], a);
        a = Sp::mma(dlo, fhi[h], a);
        acc[h] = a;
    }
}

// x[i] * omega^(j (4g + i) 2^tsh), i < 4, from two table lookups:
// omega^(4 g j) * omega^(i j).
template <bool FWD>
__device__ __forceinline__ void twiddle4(float2 (&x)[4], const float2* tl, int j, int g, int tsh)
{
    const float2 w4 = tw_blk(tl, (j * 4 * g) << tsh), w1 = tw_blk(tl, j << tsh);
    float2 f = w4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[i] = cmul_fwd_or_conj(x[i], f, FWD);
        if (i < 3) f = cmul(f, w1);
    }
}

// Stages 0 and 1 of the P columns held in LDS (entered in base-16
// digit-reversed order): each group of 16 consecutive stage-0 butterflies is
// one block of stage 1.  Stage 0 reads the block's 256 slots (slot 16 b + r,
// input r of butterfly b; fp16: times the tile scale `mul`), contracts,
// stage 1 twiddles its inputs (omega_256^(j r), j = c and r = 4g + i for
// every group: the lane's four entries of the LDS table t1) and contracts again, and the
// outputs go back to the same 256 slots (output k of stage-1 butterfly j at
// j + 16 k), all within one wave.
template <int LGN, int PREC, bool FWD, typename V8>
__device__ __forceinline__ void mfma_stages01(float2* lds, int cs, const float2* t1, float mul, int t,
                                              const V8 (&fhi)[2], const V8 (&flo)[2])
{
    constexpr int N = 1 << LGN;
    constexpr int NB = N / 16;  // butterflies per column per stage
    constexpr int GPW = 4;      // 16-butterfly groups per wave: 1024 butterflies, 16 waves
    const int lane = t & 63, wave = t >> 6, g = lane >> 4, c = lane & 15;
#pragma unroll 2
    for (int grp = 0; grp < GPW; ++grp) {
        const int gb = (wave * GPW + grp) * 16;  // first butterfly of the group (flat)
        const int w = gb >> (LGN - 4), b0 = gb & (NB - 1);
        float2* col = lds + w * cs;
        // stage 0: row c = butterfly b0 + c, inputs 4g .. 4g+3
        float2 x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = col[mfma_lds_pad(16 * (b0 + c) + 4 * g + i)];
        V8 dhi, dlo;
        split_inputs<PREC, PREC == 2>(x, mul, dhi, dlo);
        floatx4 acc[2];
        contract<PREC>(dhi, dlo, fhi, flo, acc);
        // stage 1: row c = butterfly j = c of the block, inputs r = 4g + i
        {
            const float4* tw = reinterpret_cast<const float4*>(t1) + 2 * lane;
            const float4 w01 = tw[0], w23 = tw[1];
            x[0] = cmul_fwd_or_conj(mkc(acc[0][0], acc[1][0]), mkc(w01.x, w01.y), FWD);
            x[1] = cmul_fwd_or_conj(mkc(acc[0][1], acc[1][1]), mkc(w01.z, w01.w), FWD);
            x[2] = cmul_fwd_or_conj(mkc(acc[0][2], acc[1][2]), mkc(w23.x, w23.y), FWD);
            x[3] = cmul_fwd_or_conj(mkc(acc[0][3], acc[1][3]), mkc(w23.z, w23.w), FWD);
        }
        split_inputs<PREC, false>(x, 1.0f, dhi, dlo);
        contract<PREC>(dhi, dlo, fhi, flo, acc);
        // output k = c of stage-1 butterflies j = 4g + i: slot 16 b0 + j + 16 k
        float2* ob = col + mfma_lds_pad(16 * b0);
#pragma unroll
        for (int i = 0; i < 4; ++i) ob[4 * g + i + c * 17] = mkc(acc[0][i], acc[1][i]);
    }
}

// One radix-16 stage s >= 2 of the P columns held in LDS, in place by
// decimation in time: butterfly j of a block of 16^(s+1) slots reads slots
// base + j + r 16^s, multiplies input r by omega_{16^(s+1)}^(j r), contracts
// and writes output k back to slot base + j + k 16^s.  Padded slot
// base + r 16^s is pad(base) + r * pstep, pstep = 16^s (1 + 1/16 + 1/256)
// (16^s is a multiple of 256 from s = 2 on).  A lane
// reads its four inputs (those of butterfly c of its group) and writes
// output q = c of butterflies 4g .. 4g+3 of the group.
template <int LGN, int PREC, bool FWD, typename V8>
__device__ __forceinline__ void mfma_stage(float2* lds, int cs, const float2* tl, int s, int t,
                                           const V8 (&fhi)[2], const V8 (&flo)[2])
{
    constexpr int N = 1 << LGN;
    constexpr int NB = N / 16;
    constexpr int GPW = 4;
    const int lane = t & 63, wave = t >> 6, g = lane >> 4, c = lane & 15;
    const int lgns = 4 * s, ns = 1 << lgns;
    const int pstep = ns + (ns >> 4) + (ns >> 8);
    const int tsh = kLgTwBlk - lgns - 4;
#pragma unroll 2
    for (int grp = 0; grp < GPW; ++grp) {
        const int gb = (wave * GPW + grp) * 16;
        const int w = gb >> (LGN - 4);
        float2* col = lds + w * cs;
        auto base = [&](int bf) {
            const int b = bf & (NB - 1);
            return mfma_lds_pad(((b >> lgns) << (lgns + 4)) + (b & (ns - 1)));
        };
        const int bin = gb + c;
        float2 x[4];
        const float2* pin = col + base(bin);
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = pin[(4 * g + i) * pstep];
        twiddle4<FWD>(x, tl, bin & (ns - 1), g, tsh);
        V8 dhi, dlo;
        split_inputs<PREC, false>(x, 1.0f, dhi, dlo);
        floatx4 acc[2];
        contract<PREC>(dhi, dlo, fhi, flo, acc);
        // the other rows' butterflies of the group are written only by this
        // wave, and read by it before: a wave's LDS accesses keep their order
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // real and imaginary parts stored separately: no register pairing
            float* o = reinterpret_cast<float*>(col + base(gb + 4 * g + i) + c * pstep);
            o[0] = acc[0][i];
            o[1] = acc[1][i];
        }
    }
}

// The NST radix-16 stages of the P columns held in LDS: the columns enter in
// base-16 digit-reversed order and leave in natural order.  Stages 0 and 1
// run together in registers; the others (the 4096-point level's third) read
// and write LDS.  The loop over those is not unrolled (register budget).
template <int LGN, int PREC, bool FWD, typename V8>
__device__ __forceinline__ void mfma_half_stages(float2* lds, int cs, const float2* tl, const float2* t1, float down,
                                                 int t, const V8 (&fhi)[2], const V8 (&flo)[2])
{
    constexpr int NST = LGN / 4;
    static_assert(NST >= 2, "the matrix-core pair levels have at least two radix-16 stages");
    mfma_stages01<LGN, PREC, FWD>(lds, cs, t1, down, t, fhi, flo);
    __syncthreads();
#pragma unroll 1
    for (int s = 2; s < NST; ++s) {
        mfma_stage<LGN, PREC, FWD>(lds, cs, tl, s, t, fhi, flo);
        __syncthreads();
    }
}

__device__ __forceinline__ const float2* mat(const char* base, uint32_t off)
{
    return reinterpret_cast<const float2*>(base + size_t(off));
}
__device__ __forceinline__ float2* mat(char* base, uint32_t off) { return reinterpret_cast<float2*>(base + size_t(off)); }

}  // namespace

// One tile of a paired-column matrix-core level.  NTM picks the input load
// policy: 0 = by a.nt_in at run time, 1 = streaming, 2 = cached.  With a
// fixed policy the loads and their first uses share one straight-line path,
// so each wait covers only the loads it needs: on a strided input the even
// columns load first and the first half's LDS scatter and stages start while
// the odd columns are still in flight.
template <int LGN, int PREC, bool TIN, bool TOUT, bool FWD, int NTM>
__device__ __forceinline__ void mfma_pair_tile(const PassArgs& a)
{
    using V = float2;
    using Sp = SplitT<PREC>;
    using S = typename Sp::S;
    using V8 = typename Sp::V8;
    constexpr int N = 1 << LGN;
    constexpr int E = 16;  // points of each column a thread
    constexpr int LGTPC = LGN - 4, TPC = 1 << LGTPC;
    constexpr int LGP = 14 - LGN, P = 1 << LGP;  // column pairs of the tile
    static_assert(LGN == 8 || LGN == 12, "paired-column matrix-core levels of 2^8 or 2^12 points");

    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    V* tl = lds + a.data_elems;
    V* tt = tl + kTwBlkEntries;
    const int t = threadIdx.x;
    const int cs = a.col_stride;
    // (pair, row) of this thread on the input and on the output side.
    const int ui = TIN ? (t & (P - 1)) : (t >> LGTPC), ji = TIN ? (t >> LGP) : (t & (TPC - 1));
    const int uo = TOUT ? (t & (P - 1)) : (t >> LGTPC), jo = TOUT ? (t >> LGP) : (t & (TPC - 1));

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
    // The stage-1 twiddle of operand slot (lane, i): omega_256^(c (4g + i)) =
    // omega_{2^14}^e, e = 64 (c (4g + i) mod 256), the same for every group
    // and both halves (a forward root; the adjoint conjugates it on use).
    V t1v[2];
    if (t < 256) {
        const V* g1 = reinterpret_cast<const V*>(a.tw_blk);
        const int l = t >> 2, i = t & 3;
        const int e = 64 * (((l & 15) * (4 * (l >> 4) + i)) & 255);
        t1v[0] = g1[e & 127];
        t1v[1] = g1[128 + (e >> 7)];
    }
    uint64_t tile = blockIdx.x;
    if (a.xcd_remap) tile = uint64_t(blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    int64_t d0, ib, ob;
    tile_offsets(a, tile, d0, ib, ob);
    const char* gin = reinterpret_cast<const char*>(a.in) + ib * int64_t(sizeof(V));
    char* gout = reinterpret_cast<char*>(a.out) + ob * int64_t(sizeof(V));

    V v0[E], v1[E];
    {
        const uint32_t se = uint32_t(a.in_s_e) * 8u, s0 = uint32_t(a.in_s[0]) * 8u;
        const uint32_t step = uint32_t(TPC) * se;
        // The caller's input (first level) streams past the caches.
        const bool once = a.nt_in != 0;
        if constexpr (TIN) {
            const uint32_t off = 16u * uint32_t(ui) + uint32_t(ji) * se;
            auto ld = [&](bool nt) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const float4* p = reinterpret_cast<const float4*>(mat(gin, off + uint32_t(m) * step));
                    const float4 x = nt ? load_once(p) : *p;
                    v0[m] = make_float2(x.x, x.y);
                    v1[m] = make_float2(x.z, x.w);
                }
            };
            if (once) ld(true);
            else ld(false);
        } else {
            // The even column first, then the odd one; the scheduling
            // barriers keep that issue order.
            const uint32_t o0 = 2u * uint32_t(ui) * s0 + uint32_t(ji) * se, o1 = o0 + s0;
            auto ld = [&](bool nt) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const V* p0 = mat(gin, o0 + uint32_t(m) * step);
                    v0[m] = nt ? load_once(p0) : *p0;
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const V* p1 = mat(gin, o1 + uint32_t(m) * step);
                    v1[m] = nt ? load_once(p1) : *p1;
                }
                __builtin_amdgcn_sched_barrier(0);
            };
            if constexpr (NTM == 0) {
                if (once) ld(true);
                else ld(false);
            } else {
                (void)once;
                ld(NTM == 1);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = t + 1024 * k;
        if (i < nt) tl[i] = tab[k];
    }
    // fp16: the largest |component| of each half tile, one slot per wave
    // after the tables (see the file comment); then the stage-1 twiddles,
    // lane-major.
    float* wmax = reinterpret_cast<float*>(tl + nt);
    V* t1 = tl + nt + kMfmaScaleElems;
    if (t < 256) t1[t] = cmul(t1v[0], t1v[1]);
    float down = 1.f, up = 1.f;
    V8 ahi[2], alo[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        V* vh = h ? v1 : v0;
        // (The second half's slots are written after the stage barriers of
        // the first, which every wave passes only after reading them.)
        if constexpr (PREC == 2) {
            float m = 0.f;
#pragma unroll
            for (int k = 0; k < E; ++k) m = abs_max(vh[k], m);
            m = wave_max(m);
            if ((t & 63) == 0) wmax[t >> 6] = m;
        }
        if (h) __syncthreads();  // the first half has been read back everywhere
        // Row ji + m TPC enters at padded slot pad(rev16(ji)) + m: m is the
        // top base-16 digit, which reverses to the lowest, below any padding.
        V* cin = lds + ui * cs + mfma_lds_pad(rev16<LGN / 4>(ji));
#pragma unroll
        for (int m = 0; m < E; ++m) cin[m] = vh[m];
        __syncthreads();
        if constexpr (PREC == 2) {
            float m = 0.f;
#pragma unroll
            for (int w = 0; w < 16; ++w) m = fmaxf(m, wmax[w]);
            tile_scale(m, down, up);
        }
        if (h == 0) {
            // B operand fragments of this lane (the DFT matrix, hi and lo
            // parts): half 0 maps input (re, im) of point r to the real part
            // of output q (c, -s), half 1 to its imaginary part (s, c), with
            // c + i s = omega_16^(q r) from the in-block table:
            // tl[128 + 8 e] = omega_{2^14}^(1024 e).  Lane (g, q) holds rows
            // 8g .. 8g+7 (points 4g .. 4g+3) of column q.
            const int lane = t & 63, g = lane >> 4, q = lane & 15;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int r = 4 * g + (i >> 1), comp = i & 1;
                    const V w = tl[128 + 8 * ((q * r) & 15)];
                    const float c = w.x, sn = FWD ? w.y : -w.y;  // forward table: w.y = -sin
                    const float v = hh == 0 ? (comp == 0 ? c : -sn) : (comp == 0 ? sn : c);
                    const S hi = S(v);
                    ahi[hh][i] = hi;
                    alo[hh][i] = S(v - float(hi));
                }
        }
        mfma_half_stages<LGN, PREC, FWD>(lds, cs, tl, t1, down, t, ahi, alo);
        // Read back in natural order (fp16: undoing the tile scale): row
        // jo + m TPC sits at padded slot pad(jo) + m TPC (1 + 1/16 + 1/256).
        constexpr int RSTEP = TPC + TPC / 16 + TPC / 256;
        const V* cout = lds + uo * cs + mfma_lds_pad(jo);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            vh[m] = cout[m * RSTEP];
            if constexpr (PREC == 2) vh[m] = mkc(vh[m].x * up, vh[m].y * up);
        }
    }

    const uint32_t ju = uint32_t(jo), uu = uint32_t(uo);
    if (a.tw_parts) {
        const uint32_t mask = uint32_t((uint64_t(1) << a.tw_lgroot) - 1);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            V* v = c ? v1 : v0;
            const uint32_t dcol = uint32_t(d0) + 2u * uu + uint32_t(c);
            V f[E];
            f[0] = tw_inter32(tt, a.tw_parts, (dcol * ju) & mask);
            V pw[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) pw[b] = tw_inter32(tt, a.tw_parts, (dcol * (uint32_t(TPC) << b)) & mask);
            power_tree<4, false>(f, pw);
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = cmul_fwd_or_conj(v[m], f[m], FWD);
        }
    }
    const uint32_t sk = uint32_t(a.out_s_k) * 8u, s0 = uint32_t(a.out_s[0]) * 8u;
    const uint32_t step = uint32_t(TPC) * sk;
    if constexpr (TOUT) {
        const uint32_t off = 16u * uu + ju * sk;
#pragma unroll
        for (int m = 0; m < E; ++m)
            *reinterpret_cast<float4*>(mat(gout, off + uint32_t(m) * step)) =
                make_float4(v0[m].x, v0[m].y, v1[m].x, v1[m].y);
    } else {
        const uint32_t o0 = 2u * uu * s0 + ju * sk, o1 = o0 + s0;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            *mat(gout, o0 + uint32_t(m) * step) = v0[m];
            *mat(gout, o1 + uint32_t(m) * step) = v1[m];
        }
    }
}

template <int LGN, int PREC, bool TIN, bool TOUT, bool FWD>
__global__ void __launch_bounds__(1024) k_pass_mfma_pair(PassArgs a)
{
    if constexpr (TIN) {
        mfma_pair_tile<LGN, PREC, TIN, TOUT, FWD, 0>(a);
    } else {
        if (a.nt_in) mfma_pair_tile<LGN, PREC, TIN, TOUT, FWD, 1>(a);
        else mfma_pair_tile<LGN, PREC, TIN, TOUT, FWD, 2>(a);
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

#define MOA_MP(L, PR, F) \
    { {&k_pass_mfma_pair<L, PR, false, false, F>, &k_pass_mfma_pair<L, PR, false, true, F>}, \
      {&k_pass_mfma_pair<L, PR, true, false, F>, &k_pass_mfma_pair<L, PR, true, true, F>} }
// [lgn 8 / 12][prec - 1][direction][tin][tout]
static const PassFn kMfmaPair[2][2][2][2][2] = {
    {{MOA_MP(8, 1, true), MOA_MP(8, 1, false)}, {MOA_MP(8, 2, true), MOA_MP(8, 2, false)}},
    {{MOA_MP(12, 1, true), MOA_MP(12, 1, false)}, {MOA_MP(12, 2, true), MOA_MP(12, 2, false)}},
};

static PassFn mfma_pair_lookup(const PassDesc& d, bool fwd)
{
    if ((d.lgn != 8 && d.lgn != 12) || d.mfma < 1 || d.mfma > 2) return nullptr;
    return kMfmaPair[d.lgn == 12][d.mfma - 1][fwd ? 0 : 1][d.in_tile_fast][d.out_tile_fast];
}

static PassFn mfma_fn(const PassDesc& d, bool fwd)
{
    return d.kmode == 3 ? mfma_pair_lookup(d, fwd) : mfma_lookup(d.lgn, d.mfma);
}

const void* mfma_kernel_fn(const PassDesc& d, bool fwd) { return reinterpret_cast<const void*>(mfma_fn(d, fwd)); }

hipError_t prepare_mfma_kernel(const PassDesc& d)
{
    for (bool fwd : {true, false}) {
        PassFn f = mfma_fn(d, fwd);
        if (!f) return hipErrorInvalidValue;
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, d.lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_mfma(const PassDesc& d, const PassArgs& a, hipStream_t s)
{
    PassFn f = mfma_fn(d, a.sign < 0.f);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(unsigned(d.grid)), dim3(unsigned(d.threads)), d.lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace moa
