/*
 * FP64 CPU oracle for the MoA dimension-lifted radix-2 FFT.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may include, link, load or call this file.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code, header, table or helper with the GPU path.
 *
 * Everything here is written for obviousness, not speed:
 *
 *  - moa_or_fft          : the result oracle.  The DFT of the problem
 *                          statement of Ch. 3 ("Traditional FFT Algorithm":
 *                          input x in C^n, n = 2^t, output the DFT of x),
 *                          evaluated by the even/odd split of the definition
 *                          itself: with E and O the half-length DFTs of the
 *                          even and odd samples, X_k = E_k + w^k O_k and
 *                          X_{k+n/2} = E_k - w^k O_k, applied recursively,
 *                          out of place, natural order in and out (no
 *                          bit-reversal table, no in-place loop nest).
 *  - moa_or_dft_brute    : the plain O(n^2) definition of the DFT, in long
 *                          double, used to pin moa_or_fft for small n.
 *  - moa_or_fft_lifted   : the method oracle.  The cache-optimized FFT of
 *                          Ch. 3 ("Cache-Optimized FFT: Key Elements",
 *                          "The General Algorithm"): in-row stages with the
 *                          transformed weights omega_L^(sigma + j c^l),
 *                          reshape-transposes between levels, and the final
 *                          transpose (Eq. xihyper).
 *  - moa_or_trans_rshp   : the reshape-transpose <r c> rho^ (transpose
 *                          (<r c> rho^ x)) (Eqs. reversed/trans).
 *  - moa_or_final_trans  : X[t 2^s + s'] = x[s' 2^(d-s) + t] (Eq. xihyper).
 *
 * Conventions (readings where the paper is silent or inconsistent):
 *  - sign = -1 is the forward transform, omega_L = exp(-2 pi i / L);
 *    sign = +1 is the adjoint (unnormalised conjugate transform).  The paper
 *    prints +2 pi i in Fig. fftpsirad2 and -2 pi i in Fig. radnbutterfly.
 *  - Neither direction is normalised.
 *  - The reshape-transpose outer loop runs over all c columns (the printed
 *    fragment of Fig. trans_rshp_code bounds it by n/c^2 - 1, which moves only
 *    n^2/c^3 of the n elements; Eqs. reversed/transsimp and the worked
 *    example x^(c) fix the full range).
 *  - The number of reshape-transposes is l_max = ceil(d / log2 c) - 1, so that
 *    n = 2^p_max c^l_max with 1 <= p_max <= log2 c ("Number of Different
 *    Weight Matrices"); c >= n gives l_max = 0, the plain FFT.
 *
 * Complex numbers are interleaved (re, im) doubles, the layout of numpy's
 * complex128.  Twiddles are computed from exact integer exponents: the
 * exponent is reduced modulo L in integers and folded into [0, pi/4] by the
 * octant symmetries before cos/sin are called, so each twiddle is within
 * about one ulp.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double re, im;
} or_cplx;

static int or_log2(int64_t n)
{
    int t = 0;
    while (((int64_t)1 << t) < n) ++t;
    return t;
}

static int or_is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

/* omega_L^e = exp(sign * 2 pi i e / L) for an integer exponent e and L >= 1. */
void moa_or_root(int64_t e, int64_t L, int sign, double* re, double* im)
{
    /* Work in units of 1/(8L) of a turn so every fold below stays integral. */
    int64_t M = 8 * L;
    int64_t E = e % L;
    if (E < 0) E += L;
    E *= 8;
    int neg_s = 0, neg_c = 0, swap = 0;
    if (2 * E > M) { E = M - E; neg_s = 1; }          /* angle -> 2pi - angle  */
    if (4 * E > M) { E = M / 2 - E; neg_c = 1; }      /* angle -> pi - angle   */
    if (8 * E > M) { E = M / 4 - E; swap = 1; }       /* angle -> pi/2 - angle */
    double a = (2.0 * M_PI) * (double)E / (double)M;  /* in [0, pi/4] */
    double c = cos(a), s = sin(a);
    if (swap) { double t = c; c = s; s = t; }
    if (neg_c) c = -c;
    if (neg_s) s = -s;
    *re = c;
    *im = (sign < 0) ? -s : s;
}

/* P_n: the bit-reversal permutation that opens the radix-2 program of
 * Fig. vanloan_fft (used by the method oracle). */
void moa_or_bitrev(or_cplx* x, int64_t n)
{
    int t = or_log2(n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = 0;
        for (int b = 0; b < t; ++b)
            if (i & ((int64_t)1 << b)) j |= (int64_t)1 << (t - 1 - b);
        if (j > i) {
            or_cplx tmp = x[i];
            x[i] = x[j];
            x[j] = tmp;
        }
    }
}

static void or_butterfly(or_cplx* a, or_cplx* b, double wr, double wi)
{
    /* c = w * b; (a, b) <- (a + c, a - c): the radix-2 butterfly of the
       method's in-row stages (Ch. 3, Fig. rad2_fft) */
    double cr = wr * b->re - wi * b->im;
    double ci = wr * b->im + wi * b->re;
    double dr = a->re, di = a->im;
    a->re = dr + cr;
    a->im = di + ci;
    b->re = dr - cr;
    b->im = di - ci;
}

/* DFT of the m samples src[0], src[st], ..., src[(m-1) st] into dst[0..m),
 * by the even/odd split of the definition: the m/2-point DFTs of the even
 * samples (into dst[0..m/2)) and of the odd samples (into dst[m/2..m)),
 * then X_k = E_k + w_m^k O_k, X_{k+m/2} = E_k - w_m^k O_k.  w_m^k is read
 * from the table of the full length n as w_n^(k n/m), exact in the integer
 * exponent. */
static void or_dft_split(const or_cplx* src, int64_t st, or_cplx* dst, int64_t m, int64_t n,
                         const or_cplx* w)
{
    if (m == 1) {
        dst[0] = src[0];
        return;
    }
    const int64_t h = m / 2;
    or_dft_split(src, 2 * st, dst, h, n, w);
    or_dft_split(src + st, 2 * st, dst + h, h, n, w);
    const int64_t step = n / m;
    for (int64_t k = 0; k < h; ++k) {
        const or_cplx e = dst[k], o = dst[k + h], f = w[k * step];
        const double tr = f.re * o.re - f.im * o.im;
        const double ti = f.re * o.im + f.im * o.re;
        dst[k].re = e.re + tr;
        dst[k].im = e.im + ti;
        dst[k + h].re = e.re - tr;
        dst[k + h].im = e.im - ti;
    }
}

/* Result oracle: the DFT of one vector of length n = 2^t (in place; sign -1
 * forward, +1 the conjugate transform).  Returns 0 on success, -1 if n is
 * not a power of two or memory runs out. */
int moa_or_fft(or_cplx* x, int64_t n, int sign)
{
    if (!or_is_pow2(n)) return -1;
    if (n == 1) return 0;
    or_cplx* w = (or_cplx*)malloc(sizeof(or_cplx) * (size_t)(n / 2));
    or_cplx* y = (or_cplx*)malloc(sizeof(or_cplx) * (size_t)n);
    if (!w || !y) {
        free(w);
        free(y);
        return -1;
    }
    for (int64_t k = 0; k < n / 2; ++k) moa_or_root(k, n, sign, &w[k].re, &w[k].im);
    or_dft_split(x, 1, y, n, n, w);
    memcpy(x, y, sizeof(or_cplx) * (size_t)n);
    free(w);
    free(y);
    return 0;
}

/* Batch of contiguous length-n transforms, optionally over OpenMP threads. */
int moa_or_fft_batch(or_cplx* x, int64_t n, int64_t batch, int sign, int threads)
{
    if (!or_is_pow2(n) || batch < 0) return -1;
#ifdef _OPENMP
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
#endif
    for (int64_t b = 0; b < batch; ++b) moa_or_fft(x + b * n, n, sign);
    (void)threads;
    return 0;
}

/* Packed uneven batch: transform i has length sizes[i] and starts where
 * transform i-1 ends. */
int moa_or_fft_packed(or_cplx* x, const int64_t* sizes, int64_t count, int sign, int threads)
{
    for (int64_t i = 0; i < count; ++i)
        if (!or_is_pow2(sizes[i])) return -1;
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(count + 1));
    off[0] = 0;
    for (int64_t i = 0; i < count; ++i) off[i + 1] = off[i] + sizes[i];
#ifdef _OPENMP
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
#endif
    for (int64_t i = 0; i < count; ++i) moa_or_fft(x + off[i], sizes[i], sign);
    (void)threads;
    free(off);
    return 0;
}

/* Plain definition X_k = sum_j x_j exp(sign 2 pi i j k / n), O(n^2), long
 * double accumulation and long double twiddles (an independent route from
 * moa_or_root).  Any n >= 1 is accepted. */
int moa_or_dft_brute(const or_cplx* x, or_cplx* y, int64_t n, int sign)
{
    if (n < 1) return -1;
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int64_t k = 0; k < n; ++k) {
        long double sr = 0.0L, si = 0.0L;
        for (int64_t j = 0; j < n; ++j) {
            int64_t e = (j * k) % n;
            long double a = two_pi * (long double)e / (long double)n;
            long double c = cosl(a), s = sinl(a) * (sign < 0 ? -1.0L : 1.0L);
            sr += c * (long double)x[j].re - s * (long double)x[j].im;
            si += c * (long double)x[j].im + s * (long double)x[j].re;
        }
        y[k].re = (double)sr;
        y[k].im = (double)si;
    }
    return 0;
}

/* Number of levels of the lift of n = 2^d by a block c = 2^lam:
 * l_max = ceil(d / lam) - 1 and p_max = d - l_max lam ("Numbering",
 * "Number of Different Weight Matrices").  c >= n means no lifting. */
void moa_or_lift_levels(int64_t n, int64_t c, int* l_max, int* p_max)
{
    int d = or_log2(n), lam = or_log2(c);
    if (d == 0) { *l_max = 0; *p_max = 0; return; }
    if (lam >= d) { *l_max = 0; *p_max = d; return; }
    int l = (d + lam - 1) / lam - 1;
    *l_max = l;
    *p_max = d - l * lam;
}

/* Reshape-transpose <r c> rho^ (transpose (<r c> rho^ x)), r = n / c, with
 * the outer index over all c columns.  temp must hold n elements. */
int moa_or_trans_rshp(or_cplx* x, or_cplx* temp, int64_t n, int64_t c)
{
    if (!or_is_pow2(n) || !or_is_pow2(c) || c > n) return -1;
    int64_t r = n / c, idx = 0;
    for (int64_t jp = 0; jp < c; ++jp)
        for (int64_t i = 0; i < r; ++i) temp[idx++] = x[jp + c * i];
    memcpy(x, temp, sizeof(or_cplx) * (size_t)n);
    return 0;
}

/* Final transpose: with s = l_max log2 c and d = log2 n,
 * result[t 2^s + s'] = x[s' 2^(d-s) + t] (Eq. xihyper; the order of s' and t
 * follows the equation and the code fragment of Fig. final_trans_code). */
int moa_or_final_trans(or_cplx* x, or_cplx* temp, int64_t n, int l_max, int64_t c)
{
    if (!or_is_pow2(n) || !or_is_pow2(c)) return -1;
    int d = or_log2(n), sig = l_max * or_log2(c);
    if (sig > d) return -1;
    int64_t smax = (int64_t)1 << sig, tmax = (int64_t)1 << (d - sig), idx = 0;
    for (int64_t t = 0; t < tmax; ++t)
        for (int64_t s = 0; s < smax; ++s) temp[idx++] = x[s * tmax + t];
    memcpy(x, temp, sizeof(or_cplx) * (size_t)n);
    return 0;
}

/* The exponent e of the transformed weight omega_L^e used by the butterfly
 * whose upper element sits at position P, at level l and in-row stage p,
 * L = 2^p c^l ("General Weight Sub-Matrices").  The weight type sigma is the
 * value of the top l log2 c bits of P (the index bits that earlier
 * reshape-transposes rotated to the top) and j = P mod 2^(p-1).  Exponents
 * are returned for the n/2 upper positions in increasing order of P. */
int moa_or_lifted_exponents(int64_t n, int64_t c, int l, int p, int64_t* exps, int64_t* Lout)
{
    if (!or_is_pow2(n) || !or_is_pow2(c) || c < 2) return -1;
    int d = or_log2(n), lam = or_log2(c);
    int64_t half = (int64_t)1 << (p - 1);
    int64_t cl = (int64_t)1 << (l * lam);
    int shift = d - l * lam;
    int64_t k = 0;
    for (int64_t P = 0; P < n; ++P) {
        if (P & half) continue; /* P is the lower partner of P + half */
        int64_t sigma = (l == 0) ? 0 : (P >> shift);
        int64_t j = P & (half - 1);
        exps[k++] = sigma + j * cl;
    }
    *Lout = ((int64_t)1 << p) * cl;
    return 0;
}

/* Method oracle: the cache-optimized FFT of Ch. 3 on one vector, in place.
 * stop_level < 0 runs to completion (natural-order output); otherwise the
 * routine returns right after the in-row stages of level stop_level and,
 * when stop_level < l_max, that level's reshape-transpose, exposing the
 * intermediate array. */
int moa_or_fft_lifted(or_cplx* x, int64_t n, int64_t c, int sign, int stop_level)
{
    if (!or_is_pow2(n) || !or_is_pow2(c) || c < 2) return -1;
    int d = or_log2(n), lam = or_log2(c), l_max, p_max;
    moa_or_lift_levels(n, c, &l_max, &p_max);
    int64_t row_len = (c < n) ? c : n;
    or_cplx* temp = (or_cplx*)malloc(sizeof(or_cplx) * (size_t)n);
    moa_or_bitrev(x, n);
    for (int l = 0; l <= l_max; ++l) {
        int np = (l < l_max) ? lam : p_max;
        int64_t cl = (int64_t)1 << (l * lam);
        int shift = d - l * lam;
        for (int64_t row = 0; row < n; row += row_len) {      /* outer loop over data blocks */
            for (int p = 1; p <= np; ++p) {                     /* in-row stages, stride 2^(p-1) */
                int64_t half = (int64_t)1 << (p - 1);
                int64_t L = ((int64_t)1 << p) * cl;
                for (int64_t blk = 0; blk < row_len; blk += 2 * half)
                    for (int64_t j = 0; j < half; ++j) {
                        int64_t P = row + blk + j;
                        int64_t sigma = (l == 0) ? 0 : (P >> shift);
                        double wr, wi;
                        moa_or_root(sigma + j * cl, L, sign, &wr, &wi);
                        or_butterfly(&x[P], &x[P + half], wr, wi);
                    }
            }
        }
        if (l < l_max) moa_or_trans_rshp(x, temp, n, c);
        if (l == stop_level) {
            free(temp);
            return 0;
        }
    }
    moa_or_final_trans(x, temp, n, l_max, c);
    free(temp);
    return 0;
}

/* Loss of the differentiable workload: L = sum_k w_k |X_k|^2 with X = F x
 * (forward), summed over a batch of contiguous length-n vectors that share
 * the weight vector w.  grad (may be NULL) receives dL/d(conj x) * 2 =
 * 2 F^H (w . X), the gradient convention of torch for real losses of complex
 * inputs.  Returns the loss. */
double moa_or_weighted_power_loss(const or_cplx* x, const double* w, int64_t n, int64_t batch,
                                  or_cplx* grad, int threads)
{
    double total = 0.0;
#ifdef _OPENMP
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(+ : total)
#endif
    for (int64_t b = 0; b < batch; ++b) {
        or_cplx* X = (or_cplx*)malloc(sizeof(or_cplx) * (size_t)n);
        memcpy(X, x + b * n, sizeof(or_cplx) * (size_t)n);
        moa_or_fft(X, n, -1);
        double s = 0.0;
        for (int64_t k = 0; k < n; ++k) s += w[k] * (X[k].re * X[k].re + X[k].im * X[k].im);
        total += s;
        if (grad) {
            for (int64_t k = 0; k < n; ++k) {
                X[k].re *= 2.0 * w[k];
                X[k].im *= 2.0 * w[k];
            }
            moa_or_fft(X, n, +1);
            memcpy(grad + b * n, X, sizeof(or_cplx) * (size_t)n);
        }
        free(X);
    }
    (void)threads;
    return total;
}

int moa_or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
