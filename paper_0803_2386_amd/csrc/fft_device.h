// Device building blocks shared by the gfx950 FFT kernels: complex helpers,
// the register-resident radix-2^k butterflies and the Stockham stage sequence
// that runs one workgroup-resident transform through VGPRs and LDS.
//
// A transform of length N = 2^LGN inside one workgroup is split over
// TPC = N / E threads that each keep E = 2^LGE elements (16 or 32) in
// registers.  The radix-2 stages of the method (Ch. 3, Fig. rad2_fft, and the
// hyper-cube butterfly of Ch. 5) are grouped LGE at a time into
// register-resident radix-2^LGE blocks; between groups the data cross LDS
// once, which is the GPU form of the paper's in-cache reshape: the index bits
// a thread owns change, the data never leave the workgroup.  Stages use the
// self-sorting (Stockham) order, so input and output of every level are in
// natural order and the bit-reversal permutation P_n of Fig. vanloan_fft is
// absorbed into the addressing.
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

// cos(2 pi k / 32) for k = 0..8; the rest follow by symmetry.
__host__ __device__ constexpr double cos32_base(int k)
{
    return k == 0 ? 1.0
         : k == 1 ? 0.98078528040323044912618223613424
         : k == 2 ? 0.92387953251128675612818318939679
         : k == 3 ? 0.83146961230254523707878837761791
         : k == 4 ? 0.70710678118654752440084436210485
         : k == 5 ? 0.55557023301960222474283081394853
         : k == 6 ? 0.38268343236508977172845998403040
         : k == 7 ? 0.19509032201612826784828486847702
                  : 0.0;
}
__host__ __device__ constexpr double cos32(int k)
{
    k &= 31;
    return k <= 8 ? cos32_base(k) : k <= 16 ? -cos32_base(16 - k) : k <= 24 ? -cos32_base(k - 16) : cos32_base(32 - k);
}
__host__ __device__ constexpr double sin32(int k) { return cos32((k + 24) & 31); }
__host__ __device__ constexpr double cos16(int k) { return cos32(2 * k); }
__host__ __device__ constexpr double sin16(int k) { return sin32(2 * k); }

// d * omega_32^K with omega = exp(sign * 2 pi i / 32); K is a constant after
// unrolling, so the trivial factors 1 and -+i cost no multiplies.
template <typename R, typename V>
__device__ __forceinline__ V rot32(V d, int K, R sign)
{
    if (K == 0) return d;
    if (K == 8) return mkc(-sign * d.y, sign * d.x);
    const R c = (R)cos32(K), s = sign * (R)sin32(K);
    return mkc(d.x * c - d.y * s, d.x * s + d.y * c);
}

__host__ __device__ constexpr int bitrev_small(int k, int lg)
{
    int r = 0;
    for (int b = 0; b < lg; ++b)
        if (k & (1 << b)) r |= 1 << (lg - 1 - b);
    return r;
}

// In-register DFT of length 2^LGR (<= 32) on v[0..RS): radix-2 stages by
// decimation in frequency, then the bit-reversal folded into register names.
template <typename R, int LGR, typename V>
__device__ __forceinline__ void dft_reg(V* v, R sign)
{
    constexpr int RS = 1 << LGR;
    static_assert(RS <= 32, "register DFT up to 32 points");
    if constexpr (RS > 1) {
#pragma unroll
        for (int h = RS / 2; h >= 1; h >>= 1) {
#pragma unroll
            for (int blk = 0; blk < RS; blk += 2 * h) {
#pragma unroll
                for (int i = 0; i < h; ++i) {
                    V a = v[blk + i], b = v[blk + i + h];
                    v[blk + i] = cadd(a, b);
                    v[blk + i + h] = rot32<R>(csub(a, b), i * (16 / h), sign);
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

// Highest set bit of r > 0 (a constant after unrolling).
__host__ __device__ constexpr int hibit(int r)
{
    int b = 0;
    while ((r >> (b + 1)) != 0) ++b;
    return b;
}

// Products of powers: f[r] = f0 * prod over the set bits b of r of pw[b],
// for 0 < r < 2^LG.  Each entry is one product of an earlier entry with one
// power, so f[r] carries popcount(r) roundings past f0 -- the same as
// multiplying the powers in one at a time -- for RS - 1 products in all.
// With unit f0 (ONE_BASE) the first product of each chain is skipped.
template <int LG, bool ONE_BASE, typename V>
__device__ __forceinline__ void power_tree(V (&f)[1 << LG], const V* pw)
{
#pragma unroll
    for (int r = 1; r < (1 << LG); ++r) {
        const int hb = hibit(r);
        const int rest = r - (1 << hb);
        if (ONE_BASE && rest == 0) f[r] = pw[hb];
        else f[r] = cmul(f[rest], pw[hb]);
    }
}

// ---------------------------------------------------------------------------
// Direction-specialised butterflies: FWD uses omega = exp(-2 pi i / n), the
// adjoint its conjugate.  With the direction a template parameter the
// factors -+i become swaps folded into the adds, and conjugated twiddles cost
// nothing (cmul_dir flips the signs of the product instead).
// ---------------------------------------------------------------------------

// x * omega_4 = x * (-i) forward, x * (+i) adjoint.
template <bool FWD, typename V>
__device__ __forceinline__ V mul_w4(V x)
{
    return FWD ? mkc(x.y, -x.x) : mkc(-x.y, x.x);
}

// x * w (forward) or x * conj(w) (adjoint), w a forward root from a table.
template <bool FWD, typename V>
__device__ __forceinline__ V cmul_dir(V x, V w)
{
    if constexpr (FWD) return cmul(x, w);
    else return mkc(x.x * w.x + x.y * w.y, x.y * w.x - x.x * w.y);
}

// x * omega_16^P for a constant P.
template <bool FWD, int P, typename R, typename V>
__device__ __forceinline__ V rot16(V x)
{
    constexpr int p = P & 15;
    if constexpr (p == 0) return x;
    else if constexpr (p == 4) return mul_w4<FWD>(x);
    else if constexpr (p == 8) return mkc(-x.x, -x.y);
    else if constexpr (p == 12) return mul_w4<!FWD>(x);
    else {
        const R c = (R)cos16(p), s = FWD ? -(R)sin16(p) : (R)sin16(p);
        return mkc(x.x * c - x.y * s, x.x * s + x.y * c);
    }
}

// In-place 4-point DFT, natural order in and out.
template <bool FWD, typename V>
__device__ __forceinline__ void dft4(V& a0, V& a1, V& a2, V& a3)
{
    const V t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_w4<FWD>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// In-place 16-point DFT as 4 x 4 (n = 4 n1 + n2, k = k1 + 4 k2): 4-point
// DFTs over n1, the factors omega_16^(n2 k1), 4-point DFTs over n2.
template <bool FWD, typename R, typename V>
__device__ __forceinline__ void dft16(V* v)
{
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<FWD>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // v[4 k1 + n2] now holds Y[n2][k1].
    v[5] = rot16<FWD, 1, R>(v[5]);
    v[6] = rot16<FWD, 2, R>(v[6]);
    v[7] = rot16<FWD, 3, R>(v[7]);
    v[9] = rot16<FWD, 2, R>(v[9]);
    v[10] = rot16<FWD, 4, R>(v[10]);
    v[11] = rot16<FWD, 6, R>(v[11]);
    v[13] = rot16<FWD, 3, R>(v[13]);
    v[14] = rot16<FWD, 6, R>(v[14]);
    v[15] = rot16<FWD, 9, R>(v[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<FWD>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 register grid.
    V x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = v[4 * (k & 3) + (k >> 2)];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = x[k];
}

// In-register DFT of length 2^LGR (natural order), direction-specialised.
template <bool FWD, typename R, int LGR, typename V>
__device__ __forceinline__ void dft_dir(V* v)
{
    if constexpr (LGR == 0) {
    } else if constexpr (LGR == 1) {
        const V a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (LGR == 2) {
        dft4<FWD>(v[0], v[1], v[2], v[3]);
    } else if constexpr (LGR == 4) {
        dft16<FWD, R>(v);
    } else {
        dft_reg<R, LGR>(v, FWD ? R(-1) : R(1));
    }
}

// Stage schedule of a length-2^lgn transform: stages of radix 2^lgrad (the
// general-radix block of Ch. 1, Fig. radnbutterfly; 16 by default), then one
// stage with the remaining radix.  A thread holds 2^lge points (16 or 32),
// i.e. NB = 2^lge / radix butterflies of each stage, so lgrad <= lge.
constexpr int kLgRadix = 4;
__host__ __device__ constexpr int lg_e(int lgn, int lge) { return lgn < lge ? lgn : lge; }
__host__ __device__ constexpr int n_stages(int lgn, int lgrad = kLgRadix)
{
    return lgn <= lgrad ? 1 : lgn / lgrad + ((lgn % lgrad) ? 1 : 0);
}
__host__ __device__ constexpr int stage_lgr(int lgn, int s, int lgrad = kLgRadix)
{
    return lgn <= lgrad ? lgn : (s < lgn / lgrad ? lgrad : lgn % lgrad);
}
__host__ __device__ constexpr int stage_lgns(int lgn, int s, int lgrad = kLgRadix)
{
    int acc = 0;
    for (int i = 0; i < s; ++i) acc += stage_lgr(lgn, i, lgrad);
    return acc;
}

// Root of the in-block twiddle table: omega_{2^14}^e for e < 2^14.  Kernels
// keep it in LDS as two 128-entry halves, lo[e] = omega^e and
// hi[e] = omega^(128 e), so omega^e = lo[e mod 128] * hi[e / 128] (one extra
// rounding); reading twiddles from LDS keeps the in-order vector-memory
// counter free for the data loads of the next tile.
constexpr int kLgTwBlk = 14;

template <typename V>
__device__ __forceinline__ V tw_blk(const V* tl, int e)
{
    return cmul(tl[e & 127], tl[128 + (e >> 7)]);
}

// Inter-level twiddle omega_{2^R}^e from `parts` 256-entry LDS tables,
// part p holding omega^(e_p 2^(8p)) for the p-th byte e_p of e.
template <typename V>
__device__ __forceinline__ V tw_inter(const V* tt, int parts, uint64_t e)
{
    V w = tt[e & 255];
    for (int p = 1; p < parts; ++p) w = cmul(w, tt[256 * p + ((e >> (8 * p)) & 255)]);
    return w;
}

// tw_inter for exponents below 2^32.
template <typename V>
__device__ __forceinline__ V tw_inter32(const V* tt, int parts, uint32_t e)
{
    V w = tt[e & 255u];
    for (int p = 1; p < parts; ++p) w = cmul(w, tt[256 * p + ((e >> (8 * p)) & 255u)]);
    return w;
}

// Loads of the caller's input, which a transform reads exactly once (its
// first level; every task of an uneven batch): non-temporal (streaming)
// loads leave the caches to the data that is read again -- the workspace a
// level has just written and the next level reads.  On the 2^24-point
// transform the first level runs in 79 us with them against 108 us without.
__device__ __forceinline__ float2 load_once(const float2* p)
{
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 x = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return make_float2(x.x, x.y);
}
__device__ __forceinline__ double2 load_once(const double2* p)
{
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 x = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return make_double2(x.x, x.y);
}
__device__ __forceinline__ float4 load_once(const float4* p)
{
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 x = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
    return make_float4(x.x, x.y, x.z, x.w);
}

// Stores of output a transform writes once and does not read back (an
// uneven batch's full-line stores): non-temporal.
__device__ __forceinline__ void store_once(float2* p, float2 v)
{
    typedef float v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store((v2){v.x, v.y}, reinterpret_cast<v2*>(p));
}
__device__ __forceinline__ void store_once(double2* p, double2 v)
{
    typedef double v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store((v2){v.x, v.y}, reinterpret_cast<v2*>(p));
}

template <int LGN, int LGE, int S, int LGRAD = kLgRadix>
struct StageTw {
    static_assert(LGRAD <= LGE || LGN <= LGE, "a stage's radix must fit the points of a thread");
    static constexpr int N = 1 << LGN;
    static constexpr int LGR = stage_lgr(LGN, S, LGRAD);
    static constexpr int RS = 1 << LGR;
    static constexpr int LGNS = stage_lgns(LGN, S, LGRAD);
    static constexpr int NS = 1 << LGNS;
    static constexpr int E = 1 << lg_e(LGN, LGE);
    static constexpr int TPC = N / E;
    static constexpr int NB = E / RS;
};

// Register slot of the point j + m*TPC a thread loads before stage 0: input r
// of butterfly q sits in slot q*RS + r and is point j + (q + r*NB)*TPC.
template <int LGN, int LGE, int LGRAD = kLgRadix>
__host__ __device__ constexpr int in_slot(int m)
{
    using I = StageTw<LGN, LGE, 0, LGRAD>;
    return (m % I::NB) * I::RS + m / I::NB;
}

// Twiddles of stage S: input r of the thread's butterfly q is multiplied by
// omega_{NS*RS}^(bm*r), bm = butterfly index mod NS.  Only the powers
// r = 2^b are read from the table, tw[q * LGR + b]; input r is multiplied by
// the powers of its set bits in turn (at most five roundings).
constexpr int kMaxStageTw = 16;

template <typename R, int LGN, int LGE, int S, int LGRAD = kLgRadix, typename V>
__device__ __forceinline__ void load_stage_twiddles(V (&tw)[kMaxStageTw], int j, R sign, const V* tl)
{
    using I = StageTw<LGN, LGE, S, LGRAD>;
    if constexpr (S < n_stages(LGN, LGRAD) && I::NS > 1) {
        static_assert(I::NB * I::LGR <= kMaxStageTw, "stage twiddle buffer too small");
#pragma unroll
        for (int q = 0; q < I::NB; ++q) {
            const int bm = (j + q * I::TPC) & (I::NS - 1);
            const int e1 = bm << (kLgTwBlk - I::LGNS - I::LGR);
#pragma unroll
            for (int b = 0; b < I::LGR; ++b) {
                V w = tw_blk(tl, e1 << b);
                w.y = -sign * w.y;  // the table holds forward roots
                tw[q * I::LGR + b] = w;
            }
        }
    }
}

// Run stages S.. of a length-2^LGN transform held by this thread.
// Register v[q*RS + r] is input r of the thread's q-th butterfly of the
// stage.  On entry to stage 0, v[in_slot(m)] holds element j + m*TPC (loaded
// from global memory) unless FROM_LDS, in which case the stage reads it from
// `col` like every later stage.  Every stage but the last leaves its output
// in `col` (padded, natural Stockham positions); the last leaves it in v,
// with v[q*RS + r] = output element j + (q + r*NB)*TPC, NB = E/RS.  `tw`
// holds the stage's twiddle powers, read one stage ahead from the LDS table
// `twb` (see tw_blk).  Threads with active == false only take part in the
// barriers.
template <typename R, int LGN, int LGE, int S, bool FROM_LDS, int LGRAD = kLgRadix, typename V>
__device__ __forceinline__ void run_stages(V* v, V* col, int j, R sign, const V* twb, bool active,
                                           V (&tw)[kMaxStageTw])
{
    constexpr int NST = n_stages(LGN, LGRAD);
    if constexpr (S < NST) {
        using I = StageTw<LGN, LGE, S, LGRAD>;
        constexpr int N = I::N, LGR = I::LGR, RS = I::RS, LGNS = I::LGNS, NS = I::NS, TPC = I::TPC, NB = I::NB;
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
#pragma unroll
                    for (int r = 1; r < RS; ++r) {
                        V x = v[q * RS + r];
#pragma unroll
                        for (int b = 0; b < LGR; ++b)
                            if (r & (1 << b)) x = cmul(x, tw[q * LGR + b]);
                        v[q * RS + r] = x;
                    }
                }
                dft_reg<R, LGR>(v + q * RS, sign);
            }
        }
        if constexpr (S + 1 < NST) {
            // After a stage read from LDS the next stage's factors load while
            // the barrier drains; after the register-only first stage they
            // load behind the exchange barrier, which also publishes a table
            // stored just before the stages (a batched task stores it with
            // its data loads in flight).
            if constexpr (READS_LDS) {
                if (active) load_stage_twiddles<R, LGN, LGE, S + 1, LGRAD>(tw, j, sign, twb);
                __syncthreads();
            }
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
            if constexpr (!READS_LDS) {
                if (active) load_stage_twiddles<R, LGN, LGE, S + 1, LGRAD>(tw, j, sign, twb);
            }
            run_stages<R, LGN, LGE, S + 1, FROM_LDS, LGRAD>(v, col, j, sign, twb, active, tw);
        }
    }
}

// Element offsets of tile `tile`: its first value of digit 0 and the input and
// output offsets of the remaining digits.
__device__ __forceinline__ void tile_offsets(const PassArgs& a, uint64_t tile_id, int64_t& d0, int64_t& ib,
                                             int64_t& ob)
{
    uint64_t tile, rest;
    if (a.nd == 1) {
        tile = tile_id;
        rest = 0;
    } else {
        tile = tile_id & ((uint64_t(1) << a.lg_tiles) - 1);
        rest = tile_id >> a.lg_tiles;
    }
    d0 = int64_t(tile << a.lgw);
    ib = int64_t(tile) * a.in_tile_s;
    ob = int64_t(tile) * a.out_tile_s;
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
}

// Stage S of two 16-point-per-thread transforms of 2^LGN points held side by
// side (v0 and v1: the even and odd column of a paired-column tile, or the
// even and odd samples of one longer transform); slot layout as in
// run_stages (LGE = 4).  The two share the stage twiddles and one LDS
// column: each exchange runs v0 through it, then v1.  Every stage
// but the last is radix 16 with one butterfly a thread (NB = 1), so each LDS
// slot a thread touches is its padded base slot plus a constant.
template <bool FWD, int LGN, int S>
__device__ __forceinline__ void pair_stages(float2* v0, float2* v1, float2* col, int j, const float2* twb)
{
    constexpr int NST = n_stages(LGN);
    using I = StageTw<LGN, 4, S>;
    constexpr int N = I::N, LGR = I::LGR, RS = I::RS, LGNS = I::LGNS, NS = I::NS, TPC = I::TPC, NB = I::NB;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if constexpr (NS > 1) {
            // omega_{NS RS}^(bm r) for r < RS from the table powers r = 2^b.
            const int bm = (j + q * TPC) & (NS - 1);
            const int e1 = bm << (kLgTwBlk - LGNS - LGR);
            float2 pw[LGR];
#pragma unroll
            for (int b = 0; b < LGR; ++b) pw[b] = tw_blk(twb, e1 << b);
            float2 f[RS];
            power_tree<LGR, true>(f, pw);
#pragma unroll
            for (int r = 1; r < RS; ++r) {
                v0[q * RS + r] = cmul_dir<FWD>(v0[q * RS + r], f[r]);
                v1[q * RS + r] = cmul_dir<FWD>(v1[q * RS + r], f[r]);
            }
        }
        dft_dir<FWD, float, LGR>(v0 + q * RS);
        dft_dir<FWD, float, LGR>(v1 + q * RS);
    }
    if constexpr (S + 1 < NST) {
        static_assert(NB == 1 && RS == 16, "inner stages are radix 16");
        using J = StageTw<LGN, 4, S + 1>;
        // Output r of the butterfly goes to Stockham slot base + r NS.
        const int base = ((j >> LGNS) << (LGNS + LGR)) + (j & (NS - 1));
        float2* wp = col + lds_pad(base);
        auto put = [&](const float2* v) {
#pragma unroll
            for (int r = 0; r < RS; ++r) wp[NS == 1 ? r : lds_pad(r * NS)] = v[r];
        };
        // Input r of butterfly q of the next stage is row j + q TPC + r N / RS'.
        float2* rp = col + lds_pad(j);
        auto get = [&](float2* v) {
#pragma unroll
            for (int q = 0; q < J::NB; ++q)
#pragma unroll
                for (int r = 0; r < J::RS; ++r) v[q * J::RS + r] = rp[lds_pad(q * TPC + r * (N / J::RS))];
        };
        if constexpr (S > 0) __syncthreads();  // the last exchange has been read everywhere
        put(v0);
        __syncthreads();
        get(v0);
        __syncthreads();
        put(v1);
        __syncthreads();
        get(v1);
        pair_stages<FWD, LGN, S + 1>(v0, v1, col, j, twb);
    }
}

// Position, in units of TPC past the thread's row j, of the output element
// held in register slot m after the last stage.
template <int LGN, int LGE, int LGRAD = kLgRadix>
__host__ __device__ constexpr int out_slot_rank(int m)
{
    using I = StageTw<LGN, LGE, n_stages(LGN, LGRAD) - 1, LGRAD>;
    return m / I::RS + (m % I::RS) * I::NB;
}

}  // namespace moa
