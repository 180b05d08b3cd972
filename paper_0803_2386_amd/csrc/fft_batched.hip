// Uneven batch: thousands of independent transforms of power-of-two lengths
// (2^0 .. 2^14 points) in one fused launch.
//
// The host groups transforms of equal length into tasks that fill one
// workgroup (up to 2^14 points, several short transforms side by side as the
// columns of the LDS exchange tile) and orders the tasks longest first.  By
// default the grid has one workgroup per task and the dispatcher hands out
// the tasks in that order; with a smaller grid each workgroup walks the task
// list with a grid stride (persistent form).  A task is one
// level of the method (Ch. 3): every butterfly of every transform in it runs
// inside the workgroup (VGPRs and LDS), so each element crosses HBM exactly
// once in each direction.
#include "fft_device.h"

namespace moa {

// A task is up to 2^13 points: count transforms of 2^lgn points side by side
// on 512 threads, 16 points a thread, or one whole transform a thread when it
// is shorter than that.  A complex64 transform of 2^14 points is one task
// too: the DFTs of its even and of its odd samples (2^13 points each, one
// after the other in the same LDS tile) and one radix-2 step in registers,
// the first decimation-in-time split of Fig. vanloan_fft.  So every task
// fits half of the LDS and two workgroups share each CU, one moving data
// while the other computes.
// Thread t owns column w = t / TPC, rows j + m TPC (j = t mod TPC): the
// stage-0 register layout of the level kernel, which also reads and writes
// each transform in runs of consecutive elements, so no LDS pass is needed
// around the stages.
template <typename R, int LGN>
__host__ __device__ constexpr int task_lge() { return 4; }
constexpr int kTaskPts = 16;  // register slots per thread

// Loads of this thread's points of a task of 2^LGN-point transforms (slot
// order of stage 0); `off` is the element offset of the thread's transform.
// ONCE: streaming loads (a batch reads each input element once).
template <typename R, int LGN, bool ONCE, typename V>
__device__ __forceinline__ void task_load(V (&v)[kTaskPts], const V* __restrict__ in, int64_t off, int t)
{
    constexpr int LGE = task_lge<R, LGN>();
    constexpr int LE = lg_e(LGN, LGE);
    constexpr int TPC = 1 << (LGN - LE);
    const int j = t & (TPC - 1);
    const V* src = in + off + j;
#pragma unroll
    for (int m = 0; m < (1 << LE); ++m) v[in_slot<LGN, LGE>(m)] = ONCE ? load_once(src + m * TPC) : src[m * TPC];
}

// Stages of one task (loads already in v).
template <typename R, int LGN>
__device__ __forceinline__ void task_stages(typename cpx<R>::V (&v)[kTaskPts], bool active,
                                            typename cpx<R>::V* lds, const typename cpx<R>::V* tl, R sign, int t)
{
    using V = typename cpx<R>::V;
    constexpr int LGE = task_lge<R, LGN>();
    constexpr int LGTPC = LGN - lg_e(LGN, LGE);
    constexpr int TPC = 1 << LGTPC;
    constexpr int CS = lds_col_stride(1 << LGN, TPC);
    const int j = t & (TPC - 1), w = t >> LGTPC;
    V tw[kMaxStageTw];
    run_stages<R, LGN, LGE, 0, false>(v, lds + w * CS, j, sign, tl, active, tw);
}

// Stores of one task (ONCE: streaming stores).
template <typename R, int LGN, bool ONCE, typename V>
__device__ __forceinline__ void task_store(const V (&v)[kTaskPts], V* __restrict__ out, int64_t off, int t)
{
    constexpr int LGE = task_lge<R, LGN>();
    constexpr int LE = lg_e(LGN, LGE);
    constexpr int TPC = 1 << (LGN - LE);
    V* dst = out + off + (t & (TPC - 1));
#pragma unroll
    for (int m = 0; m < (1 << LE); ++m) {
        V* q = dst + out_slot_rank<LGN, LGE>(m) * TPC;
        if (ONCE) store_once(q, v[m]);
        else *q = v[m];
    }
}

#define MOA_TASK_SWITCH(LG, EXPR)  \
    switch (LG) {                  \
        case 0: EXPR(0); break;    \
        case 1: EXPR(1); break;    \
        case 2: EXPR(2); break;    \
        case 3: EXPR(3); break;    \
        case 4: EXPR(4); break;    \
        case 5: EXPR(5); break;    \
        case 6: EXPR(6); break;    \
        case 7: EXPR(7); break;    \
        case 8: EXPR(8); break;    \
        case 9: EXPR(9); break;    \
        case 10: EXPR(10); break;  \
        case 11: EXPR(11); break;  \
        case 12: EXPR(12); break;  \
        case 13: EXPR(13); break;  \
        case 14: EXPR(14); break;  \
        default: break;            \
    }

// The in-block twiddle table (kTwBlkEntries <= 512 entries, one a thread):
// each thread loads its entry once, ahead of any data, and every task stores
// it to LDS after issuing its data loads, so a workgroup's first task waits
// for one memory round trip instead of two.  The stages read the table only
// behind their first exchange barrier, which publishes it.
// Complex128 stores the table up front instead: the per-task store costs that
// kernel its register-resident task array (the compiler moves it to scratch).
template <typename R>
constexpr bool kTableWithTask = sizeof(R) == 4;

template <typename V>
__device__ __forceinline__ void store_table(V* tl, const V& tab, int t)
{
    if (t < kTwBlkEntries) tl[t] = tab;
}

// One 2^14-point complex64 transform at element offset `off` (512 threads):
// e = its even samples, o = its odd samples, 16 points of each a thread,
// transformed together as the two columns of a paired tile (their exchanges
// take turns in the one LDS column), then
// X[k] = E[k] + w^k O[k], X[k + 2^13] = E[k] - w^k O[k], w = omega_{2^14}.
template <bool FWD>
__device__ __forceinline__ void split14_run(const BatchArgs& a, int64_t off, float2* lds, float2* tl,
                                            const float2& tab, int t)
{
    using V = float2;
    constexpr int LGH = 13, TPC = 512, E = 16;
    const V* __restrict__ src = reinterpret_cast<const V*>(a.in) + off;
    V* __restrict__ dst = reinterpret_cast<V*>(a.out) + off;
    V e[E], o[E];
    auto ld = [&](auto once) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i = 2 * (t + m * TPC);
            e[in_slot<LGH, 4>(m)] = once ? load_once(src + i) : src[i];
            o[in_slot<LGH, 4>(m)] = once ? load_once(src + i + 1) : src[i + 1];
        }
    };
    if (a.nt) ld(std::true_type{});
    else ld(std::false_type{});
    store_table(tl, tab, t);
    pair_stages<FWD, LGH, 0>(e, o, lds, t, tl);
    // w^k for k = t + rank * TPC: base w^t times the powers w^(TPC 2^b) of
    // the set bits b of rank.
    V f[E], pw[4];
    f[0] = tw_blk(tl, t);
#pragma unroll
    for (int b = 0; b < 4; ++b) pw[b] = tw_blk(tl, TPC << b);
    power_tree<4, false>(f, pw);
    auto st = [&](auto once) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int rank = out_slot_rank<LGH, 4>(m);
            const V p = cmul_dir<FWD>(o[m], f[rank]);
            V* q = dst + t + rank * TPC;
            if (once) {
                store_once(q, cadd(e[m], p));
                store_once(q + (1 << LGH), csub(e[m], p));
            } else {
                q[0] = cadd(e[m], p);
                q[1 << LGH] = csub(e[m], p);
            }
        }
    };
    if (a.nt) st(std::true_type{});
    else st(std::false_type{});
}

// The run of this workgroup's tasks (ti, ti + G, ...) that hold transforms
// of 2^LGN points; returns the first task of the run's end.  The
// longest-first task order makes each workgroup's walk a few such runs.
// No register prefetch of the next task: the second resident workgroup of
// the CU overlaps this one's memory phases, and the registers a prefetch
// would need are what let two workgroups fit.
template <typename R, bool FWD, int LGN>
__device__ __forceinline__ int batch_run(const BatchArgs& a, int ti, typename cpx<R>::V* lds,
                                         typename cpx<R>::V* tl, const typename cpx<R>::V& tab, int t)
{
    using V = typename cpx<R>::V;
    constexpr int LGE = task_lge<R, LGN>();
    constexpr int LGTPC = LGN - lg_e(LGN, LGE);
    const int end = a.task0 + a.ntasks;
    const int G = gridDim.x;
    auto same = [&](int task) { return task < end && a.tasks[task].lgn == LGN; };
    int tt = t;
    if constexpr (LGN == 14 && sizeof(R) == 4) {
        for (; same(ti); ti += G) {
            asm volatile("" : "+v"(tt));
            split14_run<FWD>(a, a.tasks[ti].off0, lds, tl, tab, tt);
            __syncthreads();  // the next task overwrites the LDS exchange area
        }
        return ti;
    } else {
        const V* __restrict__ in = reinterpret_cast<const V*>(a.in);
        V* __restrict__ out = reinterpret_cast<V*>(a.out);
        V v[kTaskPts];
        for (; same(ti); ti += G) {
            // Keep the stage addresses (all derived from the thread index) out
            // of reach of loop-invariant code motion, which would hold them in
            // VGPRs (and spill them) across every size's loop.
            asm volatile("" : "+v"(tt));
            const BatchTask tk = a.tasks[ti];
            const int w = tt >> LGTPC;
            const bool active = w < tk.count;
            // A 2^13-point task holds one transform: its offset comes with the
            // descriptor, one dependent load fewer before the data loads.
            int64_t off = 0;
            if constexpr (LGN == 13) {
                off = tk.off0;
            } else {
                if (active) off = a.toff[tk.first + w];
            }
            if (active) {
                if (a.nt) task_load<R, LGN, true>(v, in, off, tt);
                else task_load<R, LGN, false>(v, in, off, tt);
            }
            if constexpr (kTableWithTask<R>) store_table(tl, tab, tt);
            task_stages<R, LGN>(v, active, lds, tl, R(a.sign), tt);
            if (active) {
                if (a.nt) task_store<R, LGN, true>(v, out, off, tt);
                else task_store<R, LGN, false>(v, out, off, tt);
            }
            __syncthreads();  // the next task overwrites the LDS exchange area
        }
        return ti;
    }
}

// Uneven batch: each workgroup runs the tasks blockIdx.x, blockIdx.x + G, ...
// (one task when the grid has one workgroup per task) as runs of equal
// transform length; two workgroups are resident on each CU (complex64).
template <typename R, bool FWD>
__global__ void __launch_bounds__(512, sizeof(R) == 4 ? 4 : 2) k_batched(BatchArgs a)
{
    using V = typename cpx<R>::V;
    constexpr int kMaxLg = sizeof(R) == 8 ? kMaxLgBlockC128 : kMaxLgBlockC64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    V* tl = lds + a.data_elems;
    static_assert(kTwBlkEntries <= 512, "one table entry a thread");
    const int t = threadIdx.x;
    const int end = a.task0 + a.ntasks;
    V tab{};
    if (t < kTwBlkEntries) tab = reinterpret_cast<const V*>(a.tw_blk)[t];
    if constexpr (!kTableWithTask<R>) {
        store_table(tl, tab, t);
        __syncthreads();
    }
    int ti = a.task0 + int(blockIdx.x);
    while (ti < end) {
        const int lgn = a.tasks[ti].lgn;
        int nti = end;
#define MOA_RUN(L) \
    if constexpr (L <= kMaxLg) nti = batch_run<R, FWD, L>(a, ti, lds, tl, tab, t)
        MOA_TASK_SWITCH(lgn, MOA_RUN)
#undef MOA_RUN
        ti = nti;
    }
}

using BatchFn = void (*)(BatchArgs);
static BatchFn batched_lookup(bool fp64, bool fwd)
{
    if (fp64) return fwd ? &k_batched<double, true> : &k_batched<double, false>;
    return fwd ? &k_batched<float, true> : &k_batched<float, false>;
}

const void* batched_kernel_fn(bool fp64, bool fwd) { return reinterpret_cast<const void*>(batched_lookup(fp64, fwd)); }

hipError_t prepare_batched_kernel(bool fp64, int lds_bytes)
{
    for (bool fwd : {true, false}) {
        const hipError_t e = hipFuncSetAttribute(batched_kernel_fn(fp64, fwd),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batched(bool fp64, const BatchArgs& a, int grid, int threads, int lds_bytes, hipStream_t s)
{
    hipLaunchKernelGGL(batched_lookup(fp64, a.sign < 0.f), dim3(grid), dim3(threads), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace moa
