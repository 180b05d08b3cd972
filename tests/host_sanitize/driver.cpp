// Host driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of
// the planner (plan.cpp: validation, lowering, tables, describe, the live-plan
// registry) and of the FP64 oracle (oracle.c).  Only host paths run: plans
// are host-only, so no HIP call is made (the stubs abort if one is).  Exit
// status 0 and no sanitizer report means every path below is free of
// out-of-bounds accesses, use after free, leaks and undefined behaviour.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>
#include <vector>

#include "moa_fft.h"
#include "fft_internal.h"

extern "C" {
typedef struct { double re, im; } or_cplx;
int moa_or_fft(or_cplx* x, int64_t n, int sign);
int moa_or_fft_batch(or_cplx* x, int64_t n, int64_t batch, int sign, int threads);
int moa_or_fft_packed(or_cplx* x, const int64_t* sizes, int64_t count, int sign, int threads);
int moa_or_dft_brute(const or_cplx* x, or_cplx* y, int64_t n, int sign);
void moa_or_bitrev(or_cplx* x, int64_t n);
void moa_or_lift_levels(int64_t n, int64_t c, int* l_max, int* p_max);
int moa_or_trans_rshp(or_cplx* x, or_cplx* temp, int64_t n, int64_t c);
int moa_or_final_trans(or_cplx* x, or_cplx* temp, int64_t n, int l_max, int64_t c);
int moa_or_lifted_exponents(int64_t n, int64_t c, int l, int p, int64_t* exps, int64_t* Lout);
int moa_or_fft_lifted(or_cplx* x, int64_t n, int64_t c, int sign, int stop_level);
double moa_or_weighted_power_loss(const or_cplx* x, const double* w, int64_t n, int64_t batch, or_cplx* grad,
                                  int threads);
}

static int failures = 0;
#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static const uint32_t HOST = MOA_FFT_FLAG_HOST_ONLY;

// Every query on a live host-only plan, then destroy, then the same calls on
// the stale handle.
static void exercise(moa_fft_plan_t p)
{
    size_t bytes = 0, ws = 0;
    int32_t levels = 0;
    EXPECT(moa_fft_describe_size(p, &bytes) == MOA_OK && bytes > 2);
    std::vector<char> buf(bytes + 0);
    EXPECT(moa_fft_describe(p, buf.data(), bytes) == MOA_OK);
    EXPECT(strlen(buf.data()) + 1 == bytes);
    char small[7];
    EXPECT(moa_fft_describe(p, small, sizeof(small)) == MOA_ERR_ARG && strlen(small) == 6);
    EXPECT(moa_fft_describe(p, small, 0) == MOA_ERR_ARG);
    EXPECT(moa_fft_workspace_size(p, &ws) == MOA_OK);
    EXPECT(moa_fft_num_levels(p, &levels) == MOA_OK && levels >= 1);
    char dummy[64];
    EXPECT(moa_fft_exec(p, MOA_FFT_FORWARD, dummy, dummy, nullptr) == MOA_ERR_STATE);
    EXPECT(moa_fft_exec(p, (moa_fft_dir_t)7, dummy, dummy, nullptr) == MOA_ERR_ARG);
    EXPECT(moa_fft_exec_level(p, MOA_FFT_ADJOINT, 0, dummy, dummy, nullptr) == MOA_ERR_STATE);
    EXPECT(moa_fft_exec_level(p, MOA_FFT_ADJOINT, levels, dummy, dummy, nullptr) == MOA_ERR_ARG);
    size_t need = 0;
    const moa_status_t st = moa::check_exec(p, 0, dummy, dummy, &need);
    EXPECT(need == ws);
    EXPECT(st == (ws > MOA_FFT_SCRATCH_BYTES ? MOA_ERR_SCRATCH : MOA_ERR_STATE));
    EXPECT(moa_fft_destroy(p) == MOA_OK);
    // stale handle: every call refuses it without reading the freed plan
    EXPECT(moa_fft_destroy(p) == MOA_ERR_STATE);
    EXPECT(moa_fft_describe_size(p, &bytes) == MOA_ERR_STATE);
    EXPECT(moa_fft_workspace_size(p, &ws) == MOA_ERR_STATE);
    EXPECT(moa_fft_num_levels(p, &levels) == MOA_ERR_STATE);
    EXPECT(moa_fft_exec(p, MOA_FFT_FORWARD, dummy, dummy, nullptr) == MOA_ERR_STATE);
    EXPECT(moa::check_exec(p, 0, dummy, dummy, &need) == MOA_ERR_STATE);
}

static void planner()
{
    std::mt19937_64 rng(12345);
    moa_fft_plan_t p = nullptr;
    // every length, default lifts, both dtypes and all precisions
    for (int t = 0; t <= 30; ++t)
        for (int dt = 0; dt < 2; ++dt)
            for (int prec = 0; prec < 3; ++prec) {
                const int64_t n = int64_t(1) << t;
                const int64_t batch = t < 20 ? 1 + int64_t(rng() % 5) : 1;
                const moa_status_t st = moa_fft_plan(&p, n, batch, nullptr, 0, (moa_fft_dtype_t)dt,
                                                     (moa_fft_prec_t)prec, HOST);
                if (dt == 1 && prec != 0) {
                    EXPECT(st == MOA_ERR_DTYPE);
                    continue;
                }
                if (st == MOA_OK) exercise(p);
                else EXPECT(st == MOA_ERR_LIFT);  // a split level with too few columns
            }
    // random lifts of rank 1..8 with random tuning
    for (int it = 0; it < 3000; ++it) {
        const int rank = 1 + int(rng() % 8);
        int64_t lift[8];
        int64_t n = 1;
        int lg = 0;
        for (int i = 0; i < rank; ++i) {
            const int f = 1 + int(rng() % 14);
            if (lg + f > 30) {
                lift[i] = 2;
                ++lg;
            } else {
                lift[i] = int64_t(1) << f;
                lg += f;
            }
            n *= lift[i];
        }
        if (lg > 30) continue;
        moa_fft_tuning_t tu;
        memset(&tu, 0, sizeof(tu));
        const bool tuned = rng() % 2;
        if (tuned)
            for (int i = 0; i < rank; ++i) tu.cols_per_block[i] = (rng() % 3) ? 0 : int32_t(1) << (rng() % 6);
        tu.stream = int32_t(rng() % 3) - 1;
        const int dt = int(rng() % 2);
        const int prec = dt ? 0 : int(rng() % 3);
        const int64_t batch = 1 + int64_t(rng() % 3);
        const uint32_t flags = HOST | ((rng() % 2) ? MOA_FFT_FLAG_NO_WORKSPACE : 0) |
                               ((rng() % 2) ? MOA_FFT_FLAG_GRAPH : 0);
        const moa_status_t st = moa_fft_plan_tuned(&p, n, batch, lift, rank, (moa_fft_dtype_t)dt,
                                                   (moa_fft_prec_t)prec, flags, tuned ? &tu : nullptr);
        if (st == MOA_OK) exercise(p);
        else EXPECT(st == MOA_ERR_LIFT || st == MOA_ERR_TUNING || st == MOA_ERR_BATCH);
    }
    // multi-dimensional plans
    for (int it = 0; it < 1000; ++it) {
        const int rank = 1 + int(rng() % 8);
        int64_t dims[8];
        int lg = 0;
        for (int i = 0; i < rank; ++i) {
            int f = int(rng() % 15);
            if (lg + f > 30) f = 0;
            dims[i] = int64_t(1) << f;
            lg += f;
        }
        const int dt = int(rng() % 2);
        const moa_status_t st = moa_fft_plan_nd(&p, rank, dims, 1 + int64_t(rng() % 4), (moa_fft_dtype_t)dt,
                                                MOA_FFT_PREC_NATIVE, HOST);
        if (st == MOA_OK) exercise(p);
        else EXPECT(st == MOA_ERR_SIZE || st == MOA_ERR_LIFT || st == MOA_ERR_BATCH);
    }
    // uneven batches
    for (int it = 0; it < 40; ++it) {
        const int64_t count = 1 + int64_t(rng() % 9000);
        std::vector<int64_t> sizes(static_cast<size_t>(count));
        const int dt = int(rng() % 2);
        for (auto& s : sizes) s = int64_t(1) << (rng() % (dt ? 14 : 15));
        moa_fft_tuning_t tu;
        memset(&tu, 0, sizeof(tu));
        tu.persistent_blocks = int32_t(rng() % 2048);
        const uint32_t flags = HOST | ((rng() % 2) ? MOA_FFT_FLAG_PER_SIZE : 0);
        const moa_status_t st = moa_fft_plan_batched_tuned(&p, sizes.data(), count, (moa_fft_dtype_t)dt, flags, &tu);
        EXPECT(st == MOA_OK);
        if (st == MOA_OK) exercise(p);
    }
    // invalid arguments
    int64_t bad_lift[2] = {4, 6};
    EXPECT(moa_fft_plan(nullptr, 16, 1, nullptr, 0, MOA_C64, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_NULL);
    EXPECT(moa_fft_plan(&p, 3, 1, nullptr, 0, MOA_C64, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_SIZE);
    EXPECT(moa_fft_plan(&p, int64_t(1) << 31, 1, nullptr, 0, MOA_C64, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_SIZE);
    EXPECT(moa_fft_plan(&p, 24, 1, bad_lift, 2, MOA_C64, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_SIZE);
    EXPECT(moa_fft_plan(&p, 32, 1, bad_lift, 2, MOA_C64, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_LIFT);
    EXPECT(moa_fft_plan(&p, 16, 0, nullptr, 0, MOA_C64, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_BATCH);
    EXPECT(moa_fft_plan(&p, 16, int64_t(1) << 40, nullptr, 0, MOA_C64, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_BATCH);
    EXPECT(moa_fft_plan(&p, 16, 1, nullptr, 0, (moa_fft_dtype_t)9, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_DTYPE);
    EXPECT(moa_fft_plan(&p, 16, 1, nullptr, 0, MOA_C64, MOA_FFT_PREC_NATIVE, HOST | 0x80u) == MOA_ERR_ARG);
    int64_t sizes_bad[3] = {64, 3, 16};
    EXPECT(moa_fft_plan_batched(&p, sizes_bad, 3, MOA_C64, HOST) == MOA_ERR_SIZE);
    EXPECT(moa_fft_plan_batched(&p, sizes_bad, 0, MOA_C64, HOST) == MOA_ERR_BATCH);
    int64_t dims_bad[2] = {16, 12};
    EXPECT(moa_fft_plan_nd(&p, 2, dims_bad, 1, MOA_C64, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_SIZE);
    EXPECT(moa_fft_plan_nd(&p, 9, dims_bad, 1, MOA_C64, MOA_FFT_PREC_NATIVE, HOST) == MOA_ERR_ARG);
    EXPECT(moa_fft_destroy(nullptr) == MOA_OK);
    int on_stack = 0;
    EXPECT(moa_fft_destroy(reinterpret_cast<moa_fft_plan_t>(&on_stack)) == MOA_ERR_STATE);
    for (int s = -1; s <= 12; ++s) EXPECT(moa_fft_status_string((moa_status_t)s) != nullptr);
}

static double rel_err(const or_cplx* a, const or_cplx* b, int64_t n)
{
    double num = 0, den = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double dr = a[i].re - b[i].re, di = a[i].im - b[i].im;
        num += dr * dr + di * di;
        den += b[i].re * b[i].re + b[i].im * b[i].im;
    }
    return sqrt(num / (den > 0 ? den : 1));
}

static void oracle_paths()
{
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    for (int t = 0; t <= 12; ++t) {
        const int64_t n = int64_t(1) << t;
        const size_t un = static_cast<size_t>(n);
        std::vector<or_cplx> x(un), y(un), z(un), tmp(un);
        for (auto& v : x) v = {u(rng), u(rng)};
        for (int sign = -1; sign <= 1; sign += 2) {
            y = x;
            EXPECT(moa_or_fft(y.data(), n, sign) == 0);
            if (n <= 256) {
                EXPECT(moa_or_dft_brute(x.data(), z.data(), n, sign) == 0);
                EXPECT(rel_err(y.data(), z.data(), n) < 1e-13);
            }
            for (int64_t c = 2; c <= n; c *= 2) {
                int l_max = 0, p_max = 0;
                moa_or_lift_levels(n, c, &l_max, &p_max);
                for (int stop = -1; stop <= l_max; ++stop) {
                    z = x;
                    EXPECT(moa_or_fft_lifted(z.data(), n, c, sign, stop) == 0);
                }
                z = x;
                EXPECT(moa_or_fft_lifted(z.data(), n, c, sign, -1) == 0);
                EXPECT(rel_err(z.data(), y.data(), n) < 1e-13);
                z = x;
                EXPECT(moa_or_trans_rshp(z.data(), tmp.data(), n, c) == 0);
                EXPECT(moa_or_final_trans(z.data(), tmp.data(), n, l_max, c) == 0);
                const int lam = int(log2(double(c)));
                for (int l = 0; l <= l_max; ++l)
                    for (int p = 1; p <= (l < l_max ? lam : p_max); ++p) {
                        std::vector<int64_t> e(static_cast<size_t>(n / 2 > 0 ? n / 2 : 1));
                        int64_t L = 0;
                        EXPECT(moa_or_lifted_exponents(n, c, l, p, e.data(), &L) == 0);
                        for (int64_t i = 0; i < n / 2; ++i) EXPECT(e[size_t(i)] >= 0);
                    }
            }
        }
        z = x;
        moa_or_bitrev(z.data(), n);
        moa_or_bitrev(z.data(), n);
        EXPECT(rel_err(z.data(), x.data(), n) == 0.0);
    }
    // batches, packed uneven batches, the loss and its gradient (threads)
    std::vector<int64_t> sizes;
    int64_t total = 0;
    for (int i = 0; i < 200; ++i) {
        sizes.push_back(int64_t(1) << (rng() % 11));
        total += sizes.back();
    }
    std::vector<or_cplx> pk(static_cast<size_t>(total));
    for (auto& v : pk) v = {u(rng), u(rng)};
    EXPECT(moa_or_fft_packed(pk.data(), sizes.data(), int64_t(sizes.size()), -1, 4) == 0);
    std::vector<or_cplx> bt(static_cast<size_t>(64 * 7));
    for (auto& v : bt) v = {u(rng), u(rng)};
    EXPECT(moa_or_fft_batch(bt.data(), 64, 7, 1, 3) == 0);
    std::vector<double> w(64);
    for (auto& v : w) v = 0.5 * (u(rng) + 1.0);
    std::vector<or_cplx> g(bt.size());
    EXPECT(moa_or_weighted_power_loss(bt.data(), w.data(), 64, 7, g.data(), 2) > 0.0);
    EXPECT(moa_or_weighted_power_loss(bt.data(), w.data(), 64, 7, nullptr, 1) > 0.0);
    // invalid arguments are refused, not read
    or_cplx one[4] = {};
    EXPECT(moa_or_fft(one, 3, -1) != 0);
    EXPECT(moa_or_fft_lifted(one, 4, 3, -1, -1) != 0);
    EXPECT(moa_or_trans_rshp(one, one, 4, 8) != 0);
    EXPECT(moa_or_dft_brute(one, one, 0, -1) != 0);
}

int main()
{
    planner();
    oracle_paths();
    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("host sanitizer driver: all paths clean\n");
    return 0;
}
