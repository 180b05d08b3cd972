// Latency kernel for one short transform (2^4 .. 2^12 points, batch of one).
//
// A single transform of a few thousand points is one workgroup, so its time
// is the length of the critical path through that workgroup rather than
// bandwidth.  The level kernels hold 16 points a thread, which leaves such a
// transform on one or a few waves, i.e. on one or a few SIMDs, with long
// radix-16 butterflies and twiddle chains in sequence.  Here each of N / 4
// threads holds 4 points: the stages are radix 4 (and one radix-2 stage when
// log2 N is odd), every SIMD of the CU takes part, and each stage is a short
// dependent chain.  The stages run in Stockham order through LDS, the same
// decimation as the level kernels (input r of butterfly b of a stage that
// follows NS points' worth of earlier radices is row b + r N / R; its output
// r goes to (b / NS) NS R + (b mod NS) + r NS), so the last stage writes the
// natural-order result straight to global memory.  The stage twiddles come
// from LDS tables filled behind the data loads.
#include "fft_device.h"

namespace moa {

template <typename R, int LGN, bool FWD>
__global__ void __launch_bounds__(1024) k_small(PassArgs a)
{
    using V = typename cpx<R>::V;
    constexpr int N = 1 << LGN, Q = N / 4;
    constexpr int NR4 = LGN / 2;           // radix-4 stages
    constexpr bool R2 = (LGN & 1) != 0;    // a final radix-2 stage
    static_assert(LGN >= kLgSmallMin && LGN <= kLgSmallMax, "short-transform kernel range");

    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* col = reinterpret_cast<V*>(smem_raw);
    V* tab = col + lds_padded_len(N);  // small_table_entries(LGN) twiddles
    constexpr bool DIRECT = LGN <= kLgSmallDirect;
    // Workgroup k transforms the k-th of a batch of contiguous transforms.
    const V* in = static_cast<const V*>(a.in) + int64_t(blockIdx.x) * a.in_s[0];
    V* out = static_cast<V*>(a.out) + int64_t(blockIdx.x) * a.out_s[0];
    const V* tb = static_cast<const V*>(a.tw_blk);
    const int b = threadIdx.x;

    V v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = in[b + r * Q];
    // Every twiddle of the transform is a power of omega_N.  A short one
    // builds that table in LDS from the in-block table (four entries a
    // thread, one product each: the rounding the level kernels' twiddles
    // carry); a longer one copies the 256-entry in-block table itself (at
    // most two entries a thread) and forms each twiddle as one product.
    // Either goes to LDS behind the data loads, and the first exchange
    // barrier publishes it before any stage reads it.
    if constexpr (DIRECT) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tab[b + r * Q] = tw_blk(tb, (b + r * Q) << (kLgTwBlk - LGN));
    } else {
#pragma unroll
        for (int i = b; i < kTwBlkEntries; i += Q) tab[i] = tb[i];
    }
    // omega_N^e for e < N.
    auto tw = [&](int e) { return DIRECT ? tab[e] : tw_blk(tab, e << (kLgTwBlk - LGN)); };

#pragma unroll
    for (int s = 0; s < NR4; ++s) {
        const int NS = 1 << (2 * s);
        if (s > 0) {
            // Input r times omega_{4 NS}^((b mod NS) r) = omega_N^((b mod NS) r N / (4 NS)).
            const int e1 = (b & (NS - 1)) << (LGN - 2 * s - 2);
#pragma unroll
            for (int r = 1; r < 4; ++r) v[r] = cmul_dir<FWD>(v[r], tw(e1 * r));
        }
        dft4<FWD>(v[0], v[1], v[2], v[3]);
        if (s + 1 == NR4 && !R2) {
            // NS = Q here, so the output slots b + r Q are the natural order.
#pragma unroll
            for (int r = 0; r < 4; ++r) out[b + r * Q] = v[r];
        } else {
            const int base = ((b >> (2 * s)) << (2 * s + 2)) + (b & (NS - 1));
            if (s > 0) __syncthreads();  // the last stage's reads are done everywhere
#pragma unroll
            for (int r = 0; r < 4; ++r) col[lds_pad(base + r * NS)] = v[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = col[lds_pad(b + r * Q)];
        }
    }
    if constexpr (R2) {
        // Butterflies b and b + Q take rows (b, b + 2Q) and (b + Q, b + 3Q),
        // i.e. v[0], v[2] and v[1], v[3]; the second input of butterfly c is
        // multiplied by omega_N^c; outputs c and c + N / 2.
        const V x = cmul_dir<FWD>(v[2], tw(b));
        const V y = cmul_dir<FWD>(v[3], tw(b + Q));
        out[b] = cadd(v[0], x);
        out[b + 2 * Q] = csub(v[0], x);
        out[b + Q] = cadd(v[1], y);
        out[b + 3 * Q] = csub(v[1], y);
    }
}

using SmallFn = void (*)(PassArgs);

#define MOA_SMALL_ROW(L) \
    {{&k_small<float, L, true>, &k_small<float, L, false>}, {&k_small<double, L, true>, &k_small<double, L, false>}}

// [lgn - kLgSmallMin][fp64][adjoint]
static const SmallFn kSmall[kLgSmallMax - kLgSmallMin + 1][2][2] = {
    MOA_SMALL_ROW(4),  MOA_SMALL_ROW(5),  MOA_SMALL_ROW(6), MOA_SMALL_ROW(7), MOA_SMALL_ROW(8),
    MOA_SMALL_ROW(9),  MOA_SMALL_ROW(10), MOA_SMALL_ROW(11), MOA_SMALL_ROW(12)};

static SmallFn small_lookup(bool fp64, const PassDesc& d, bool fwd)
{
    if (d.lgn < kLgSmallMin || d.lgn > kLgSmallMax) return nullptr;
    return kSmall[d.lgn - kLgSmallMin][fp64 ? 1 : 0][fwd ? 0 : 1];
}

const void* small_kernel_fn(bool fp64, const PassDesc& d, bool fwd)
{
    return reinterpret_cast<const void*>(small_lookup(fp64, d, fwd));
}

hipError_t prepare_small_kernel(bool fp64, const PassDesc& d)
{
    for (bool fwd : {true, false}) {
        SmallFn f = small_lookup(fp64, d, fwd);
        if (!f) return hipErrorInvalidValue;
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, d.lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_small(bool fp64, const PassDesc& d, const PassArgs& a, hipStream_t s)
{
    SmallFn f = small_lookup(fp64, d, a.sign < 0.f);
    if (!f || d.threads != (1 << (d.lgn - 2)) || d.grid != d.blocks || d.grid < 1 || d.grid > kSmallMaxBatch)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(unsigned(d.grid)), dim3(unsigned(d.threads)), d.lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace moa
