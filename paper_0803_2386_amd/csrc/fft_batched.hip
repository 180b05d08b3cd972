// Uneven batch: thousands of independent transforms of power-of-two lengths
// (2^0 .. 2^14 points) in one persistent launch.
//
// The host groups transforms of equal length into tasks that fill one
// workgroup (up to 2^14 points, several short transforms side by side as the
// columns of an LDS tile) and orders the tasks longest first; each resident
// workgroup walks the task list with a grid stride.  A task is one level of
// the method (Ch. 3): every butterfly of every transform in it runs inside
// the workgroup (VGPRs and LDS), so each element crosses HBM exactly once in
// each direction.  Loads and stores go through LDS so that they are
// coalesced along each transform whatever its length.
#include "fft_device.h"

namespace moa {

template <typename R, int LGN>
__device__ __forceinline__ void batched_task(const BatchArgs& a, const BatchTask& tk,
                                             typename cpx<R>::V* lds, R sign)
{
    using V = typename cpx<R>::V;
    constexpr int N = 1 << LGN;
    constexpr int LGE = lg_e(LGN);
    constexpr int E = 1 << LGE;
    constexpr int LGTPC = LGN - LGE;
    constexpr int TPC = 1 << LGTPC;
    constexpr int CS = lds_col_stride(N, TPC);

    const int count = tk.count;
    const int t = threadIdx.x, T = blockDim.x;
    const V* __restrict__ in = reinterpret_cast<const V*>(a.in);
    V* __restrict__ out = reinterpret_cast<V*>(a.out);
    const int64_t* __restrict__ toff = a.toff + tk.first;
    const int total = count << LGN;

    for (int i = t; i < total; i += T) {
        const int w = i >> LGN, e = i & (N - 1);
        lds[w * CS + lds_pad(e)] = in[toff[w] + e];
    }
    __syncthreads();

    const int j = t & (TPC - 1), w = t >> LGTPC;
    const bool active = w < count;
    V* col = lds + w * CS;
    V v[E];
    run_stages<R, LGN, 0, true>(v, col, j, sign, reinterpret_cast<const V*>(a.tw_blk), active);
    __syncthreads();
    if (active) {
#pragma unroll
        for (int m = 0; m < E; ++m) col[lds_pad(out_index_of_slot<LGN>(m, j))] = v[m];
    }
    __syncthreads();
    for (int i = t; i < total; i += T) {
        const int ww = i >> LGN, e = i & (N - 1);
        out[toff[ww] + e] = lds[ww * CS + lds_pad(e)];
    }
    __syncthreads();
}

template <typename R>
__global__ void __launch_bounds__(max_threads_for<R>()) k_batched(BatchArgs a)
{
    using V = typename cpx<R>::V;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const R sign = (R)a.sign;
    const int end = a.task0 + a.ntasks;
    for (int ti = a.task0 + int(blockIdx.x); ti < end; ti += int(gridDim.x)) {
        const BatchTask tk = a.tasks[ti];
        switch (tk.lgn) {
#define MOA_CASE(L) \
    case L: batched_task<R, (L <= (sizeof(R) == 8 ? kMaxLgBlockC128 : kMaxLgBlockC64) ? L : 0)>(a, tk, lds, sign); break;
            MOA_CASE(0) MOA_CASE(1) MOA_CASE(2) MOA_CASE(3) MOA_CASE(4) MOA_CASE(5) MOA_CASE(6) MOA_CASE(7)
            MOA_CASE(8) MOA_CASE(9) MOA_CASE(10) MOA_CASE(11) MOA_CASE(12) MOA_CASE(13) MOA_CASE(14)
#undef MOA_CASE
            default: break;
        }
    }
}

const void* batched_kernel_fn(bool fp64)
{
    return fp64 ? reinterpret_cast<const void*>(&k_batched<double>)
                : reinterpret_cast<const void*>(&k_batched<float>);
}

hipError_t prepare_batched_kernel(bool fp64, int lds_bytes)
{
    return hipFuncSetAttribute(batched_kernel_fn(fp64), hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t launch_batched(bool fp64, const BatchArgs& a, int grid, int threads, int lds_bytes, hipStream_t s)
{
    if (fp64)
        hipLaunchKernelGGL(k_batched<double>, dim3(grid), dim3(threads), lds_bytes, s, a);
    else
        hipLaunchKernelGGL(k_batched<float>, dim3(grid), dim3(threads), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace moa
