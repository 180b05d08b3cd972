// Device building blocks shared by the gfx950 FFT kernels: complex helpers,
// the register-resident radix-2^k butterflies and the Stockham stage sequence
// that runs one workgroup-resident transform through VGPRs and LDS.
//
// A transform of length N = 2^LGN inside one workgroup is split over
// TPC = N / E threads that each keep E = 16 elements in registers.  The
// radix-2 stages of the method (Ch. 3, Fig. rad2_fft, and the hyper-cube
// butterfly of Ch. 5) are grouped four at a time into register-resident
// radix-16 blocks; between groups the data crosses LDS once, which is the
// GPU form of the paper's in-cache reshape: the index bits a thread owns
// change, the data never leaves the workgroup.  Stages use the self-sorting
// (Stockham) order, so input and output of every level are in natural order
// and the bit-reversal permutation P_n of Fig. vanloan_fft is absorbed into
// the addressing.
#pragma once

#include "fft_internal.h"

namespace moa {

template <typename R> struct cpx;
template <> struct cpx<float> { using V = float2; };
template <> struct cpx<double> { using V = double2; };

__device__ __forceinline__ float2 mkc(float a, float b) { return make_float2(a, b); }
__device__ __forceinline__ double2 mkc(double a, double b) { return make_double2(a, b); }

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return mkc(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return mkc(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b)
{
    return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// cos(2 pi k / 16) for k = 0..4; the rest follow by symmetry.
__host__ __device__ constexpr double cos16_base(int k)
{
    return k == 0 ? 1.0
         : k == 1 ? 0.92387953251128675612818318939678828682
         : k == 2 ? 0.70710678118654752440084436210484903928
         : k == 3 ? 0.38268343236508977172845998403039886676
                  : 0.0;
}
__host__ __device__ constexpr double cos16(int k)
{
    k &= 15;
    return k <= 4 ? cos16_base(k) : k <= 8 ? -cos16_base(8 - k) : k <= 12 ? -cos16_base(k - 8) : cos16_base(16 - k);
}
__host__ __device__ constexpr double sin16(int k) { return cos16((k + 12) & 15); }

// d * omega_16^K with omega = exp(sign * 2 pi i / 16); K is a constant after
// unrolling, so the trivial factors 1 and -+i cost no multiplies.
template <typename R, typename V>
__device__ __forceinline__ V rot16(V d, int K, R sign)
{
    if (K == 0) return d;
    if (K == 4) return mkc(-sign * d.y, sign * d.x);
    const R c = (R)cos16(K), s = sign * (R)sin16(K);
    return mkc(d.x * c - d.y * s, d.x * s + d.y * c);
}

__host__ __device__ constexpr int bitrev_small(int k, int lg)
{
    int r = 0;
    for (int b = 0; b < lg; ++b)
        if (k & (1 << b)) r |= 1 << (lg - 1 - b);
    return r;
}

// In-register DFT of length 2^LGR (<= 16) on v[0..RS): radix-2 stages by
// decimation in frequency, then the bit-reversal folded into register names.
template <typename R, int LGR, typename V>
__device__ __forceinline__ void dft_reg(V* v, R sign)
{
    constexpr int RS = 1 << LGR;
    if constexpr (RS > 1) {
#pragma unroll
        for (int h = RS / 2; h >= 1; h >>= 1) {
#pragma unroll
            for (int blk = 0; blk < RS; blk += 2 * h) {
#pragma unroll
                for (int i = 0; i < h; ++i) {
                    V a = v[blk + i], b = v[blk + i + h];
                    v[blk + i] = cadd(a, b);
                    v[blk + i + h] = rot16<R>(csub(a, b), i * (8 / h), sign);
                }
            }
        }
        V tmp[RS];
#pragma unroll
        for (int k = 0; k < RS; ++k) tmp[k] = v[bitrev_small(k, LGR)];
#pragma unroll
        for (int k = 0; k < RS; ++k) v[k] = tmp[k];
    }
}

// Stage schedule of a length-2^lgn transform: radix-16 stages, then one
// stage with the remaining radix.
__host__ __device__ constexpr int lg_e(int lgn) { return lgn < kLgE ? lgn : kLgE; }
__host__ __device__ constexpr int n_stages(int lgn)
{
    return lgn <= kLgE ? 1 : lgn / kLgE + ((lgn % kLgE) ? 1 : 0);
}
__host__ __device__ constexpr int stage_lgr(int lgn, int s)
{
    return lgn <= kLgE ? lgn : (s < lgn / kLgE ? kLgE : lgn % kLgE);
}
__host__ __device__ constexpr int stage_lgns(int lgn, int s)
{
    int acc = 0;
    for (int i = 0; i < s; ++i) acc += stage_lgr(lgn, i);
    return acc;
}

// Workgroup size limit per element type: complex128 blocks are at most 2^13
// points, i.e. 512 threads of 16 elements, which leaves 256 VGPRs a lane.
template <typename R>
__host__ __device__ constexpr int max_threads_for() { return sizeof(R) == 8 ? 512 : kMaxThreads; }

// Root of the in-block twiddle table: omega_{2^14}^e for e < 2^14.
constexpr int kLgTwBlk = 14;

// Run stages S.. of a length-2^LGN transform held by this thread.
// Register v[q*RS + r] is input r of the thread's q-th butterfly of the
// stage.  On entry to stage 0, v[m] holds element j + m*TPC (loaded from
// global memory) unless FROM_LDS, in which case the stage reads it from
// `col` like every later stage.  Every stage but the last leaves its output
// in `col` (padded, natural Stockham positions); the last leaves it in v,
// with v[q*RS + r] = output element j + (q + r*NB)*TPC, NB = E/RS.
// Threads with active == false only take part in the barriers.
template <typename R, int LGN, int S, bool FROM_LDS, typename V>
__device__ __forceinline__ void run_stages(V* v, V* col, int j, R sign, const V* __restrict__ twb,
                                           bool active)
{
    constexpr int NST = n_stages(LGN);
    if constexpr (S < NST) {
        constexpr int N = 1 << LGN;
        constexpr int LGR = stage_lgr(LGN, S);
        constexpr int RS = 1 << LGR;
        constexpr int LGNS = stage_lgns(LGN, S);
        constexpr int NS = 1 << LGNS;
        constexpr int E = 1 << lg_e(LGN);
        constexpr int TPC = N / E;
        constexpr int NB = E / RS;
        constexpr bool READS_LDS = (S > 0) || FROM_LDS;
        if constexpr (READS_LDS) {
            if (active) {
#pragma unroll
                for (int q = 0; q < NB; ++q)
#pragma unroll
                    for (int r = 0; r < RS; ++r) v[q * RS + r] = col[lds_pad(j + q * TPC + r * (N / RS))];
            }
        }
        if (active) {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                if constexpr (NS > 1) {
                    const int bm = (j + q * TPC) & (NS - 1);
#pragma unroll
                    for (int r = 1; r < RS; ++r) {
                        // omega_{NS*RS}^(bm*r) = omega_{2^14}^(bm*r*2^(14-LGNS-LGR))
                        const int e = (bm * r) << (kLgTwBlk - LGNS - LGR);
                        V w = twb[e];
                        w.y = -sign * w.y;  // table holds forward roots
                        v[q * RS + r] = cmul(v[q * RS + r], w);
                    }
                }
                dft_reg<R, LGR>(v + q * RS, sign);
            }
        }
        if constexpr (S + 1 < NST) {
            if constexpr (READS_LDS) __syncthreads();
            if (active) {
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    const int b = j + q * TPC;
                    const int base = ((b >> LGNS) << (LGNS + LGR)) + (b & (NS - 1));
#pragma unroll
                    for (int r = 0; r < RS; ++r) col[lds_pad(base + r * NS)] = v[q * RS + r];
                }
            }
            __syncthreads();
            run_stages<R, LGN, S + 1, FROM_LDS>(v, col, j, sign, twb, active);
        }
    }
}

// Output element held in register slot m after the last stage.
template <int LGN>
__device__ __forceinline__ constexpr int out_index_of_slot(int m, int j)
{
    constexpr int LAST = n_stages(LGN) - 1;
    constexpr int LGR = stage_lgr(LGN, LAST);
    constexpr int RS = 1 << LGR;
    constexpr int E = 1 << lg_e(LGN);
    constexpr int NB = E / RS;
    constexpr int TPC = (1 << LGN) / E;
    const int q = m / RS, r = m % RS;
    return j + (q + r * NB) * TPC;
}

}  // namespace moa
