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

// Issue the loads of this thread's points of a task: point i = t + m T of
// the task's count x 2^lgn points, transform i >> lgn at offset offs[...].
// A task holds at most 2^13 points as 16 points a thread, or one 2^14-point
// transform as 32 points a thread (512 threads).  While a task of the first
// kind is transformed, the next task's points are already loading into
// registers; a 2^14-point task needs those registers itself and loads its
// successor after its stores.
__host__ __device__ constexpr int task_lge(int lgn) { return lgn >= 14 ? 5 : 4; }

template <int P, typename V>
__device__ __forceinline__ void issue_task_loads(V (&tmp)[P], const V* __restrict__ in, const BatchTask& tk,
                                                 const int64_t* offs, int t, int T)
{
    const int total = tk.count << tk.lgn;
    const int nmask = (1 << tk.lgn) - 1;
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const int i = t + m * T;
        if (i < total) tmp[m] = in[offs[i >> tk.lgn] + (i & nmask)];
    }
}

template <typename R, int LGN>
__device__ __forceinline__ void batched_stages(const BatchTask& tk, typename cpx<R>::V* lds,
                                               const typename cpx<R>::V* tl, R sign, int t)
{
    using V = typename cpx<R>::V;
    constexpr int kTaskLge = task_lge(LGN);
    constexpr int LE = lg_e(LGN, kTaskLge);
    constexpr int E = 1 << LE;
    constexpr int LGTPC = LGN - LE;
    constexpr int TPC = 1 << LGTPC;
    constexpr int CS = lds_col_stride(1 << LGN, TPC);
    const int j = t & (TPC - 1), w = t >> LGTPC;
    const bool active = w < tk.count;
    V* col = lds + w * CS;
    V v[E];
    V tw[kMaxStageTw];
    run_stages<R, LGN, kTaskLge, 0, true>(v, col, j, sign, tl, active, tw);
    __syncthreads();
    if (active) {
#pragma unroll
        for (int m = 0; m < E; ++m) col[lds_pad(j + out_slot_rank<LGN, kTaskLge>(m) * TPC)] = v[m];
    }
}

__device__ __forceinline__ int batched_col_stride(int lgn)
{
    const int n = 1 << lgn;
    const int tpc = n >> lg_e(lgn, task_lge(lgn));
    return lds_col_stride(n, tpc);
}

// Persistent uneven batch.  Each workgroup walks the tasks blockIdx.x,
// blockIdx.x + G, ...  While it transforms a task of at most 2^13 points it
// already has the loads of its next such task in flight (16 points a thread,
// into registers) and the offsets of the task after that on their way into
// LDS, so the HBM traffic of one task overlaps the work of the previous one.
// A 2^14-point task needs the registers itself: it loads its own points when
// it starts and prefetches nothing.  Task offsets live in two LDS buffers.
template <typename R>
__global__ void __launch_bounds__(kMaxThreads) k_batched(BatchArgs a)
{
    using V = typename cpx<R>::V;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    V* tl = lds + a.data_elems;
    int64_t* offb = reinterpret_cast<int64_t*>(tl + kTwBlkEntries);  // [2][kMaxTaskCols]
    const R sign = (R)a.sign;
    const int t = threadIdx.x, T = blockDim.x;
    const int G = gridDim.x;
    const int end = a.task0 + a.ntasks;
    const V* __restrict__ in = reinterpret_cast<const V*>(a.in);
    V* __restrict__ out = reinterpret_cast<V*>(a.out);
    constexpr int P = 16;  // prefetched points per thread (tasks of <= 2^13 points)
    constexpr bool kPF = sizeof(R) == 4;  // complex128 batches are for accuracy: no prefetch

    {
        const V* g1 = reinterpret_cast<const V*>(a.tw_blk);
        for (int i = t; i < kTwBlkEntries; i += T) tl[i] = g1[i];
    }
    int ti = a.task0 + int(blockIdx.x);
    if (ti < end) {
        const BatchTask tk = a.tasks[ti];
        for (int w = t; w < tk.count; w += T) offb[w] = a.toff[tk.first + w];
    }
    __syncthreads();
    V tmp[P];
    int64_t noff = 0;  // offset of column t of the task after next
    bool have = false;  // tmp holds this task's points
    {
        const int nti = ti + G;
        if (nti < end) {
            const BatchTask ntk = a.tasks[nti];
            if (t < ntk.count) noff = a.toff[ntk.first + t];
        }
        if (kPF && ti < end && a.tasks[ti].lgn < 14) {
            issue_task_loads(tmp, in, a.tasks[ti], offb, t, T);
            have = true;
        }
        __syncthreads();
        if (nti < end && t < a.tasks[nti].count) offb[kMaxTaskCols + t] = noff;
    }
    int buf = 0;
    int tt = t;
    while (ti < end) {
        // Keep the stage addresses (all derived from the thread index) out of
        // reach of loop-invariant code motion, which would hold them in VGPRs.
        asm volatile("" : "+v"(tt));
        const BatchTask tk = a.tasks[ti];
        const int lgn = tk.lgn;
        const int total = tk.count << lgn;
        const int cs = batched_col_stride(lgn);
        const int64_t* offs = offb + buf * kMaxTaskCols;
        // Park this task's points in LDS (loading them now if not prefetched).
        for (int part = 0; part * P * T < total; ++part) {
            if (!have) {
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const int i = t + (part * P + m) * T;
                    if (i < total) tmp[m] = in[offs[i >> lgn] + (i & ((1 << lgn) - 1))];
                }
            }
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int i = t + (part * P + m) * T;
                if (i < total) lds[(i >> lgn) * cs + lds_pad(i & ((1 << lgn) - 1))] = tmp[m];
            }
            have = false;
        }
        __syncthreads();
        // Loads of the next task (offsets already in LDS) and the offsets of
        // the one after it.
        const int nti = ti + G, nnti = ti + 2 * G;
        const bool big = lgn >= 14;
        noff = 0;
        if (nnti < end) {
            const BatchTask k2 = a.tasks[nnti];
            if (t < k2.count) noff = a.toff[k2.first + t];
        }
        if (kPF && !big && nti < end && a.tasks[nti].lgn < 14) {
            issue_task_loads(tmp, in, a.tasks[nti], offb + (buf ^ 1) * kMaxTaskCols, t, T);
            have = true;
        }
        if (big) {
            if constexpr (sizeof(R) == 4) batched_stages<R, 14>(tk, lds, tl, sign, tt);
        } else {
            switch (lgn) {
#define MOA_CASE(L) \
    case L: batched_stages<R, L>(tk, lds, tl, sign, tt); break;
                MOA_CASE(0) MOA_CASE(1) MOA_CASE(2) MOA_CASE(3) MOA_CASE(4) MOA_CASE(5) MOA_CASE(6)
                MOA_CASE(7) MOA_CASE(8) MOA_CASE(9) MOA_CASE(10) MOA_CASE(11) MOA_CASE(12) MOA_CASE(13)
#undef MOA_CASE
                default: break;
            }
        }
        __syncthreads();
        // Store this task from LDS (offsets from LDS: no global load between
        // the stores).
        for (int i = t; i < total; i += T)
            out[offs[i >> lgn] + (i & ((1 << lgn) - 1))] = lds[(i >> lgn) * cs + lds_pad(i & ((1 << lgn) - 1))];
        __syncthreads();  // the data area and this offset buffer are free again
        if (nnti < end && t < a.tasks[nnti].count) offb[buf * kMaxTaskCols + t] = noff;
        buf ^= 1;
        ti = nti;
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
