// Hyper-cube kernels (Ch. 6, "Density Matrix Operations for a Quantum
// Computer"; Ch. 4, "Reordering the Data"): the generalized transpose of an
// array viewed as a hyper-cube of 2-element axes, and the gating of a
// density matrix through the block-diagonal view of that transpose.
//
// Both kernels move tiles through LDS.  An element's offset is a string of
// bits; a transpose of the hyper-cube permutes those bits.  A tile is the set
// of elements whose offsets differ only in a chosen set of bit positions
// (the tile bits); the other bits, taken from the workgroup index, fix the
// tile.  The tile bits include the low bits of the source offset (so the
// tile's loads are runs of 256 contiguous bytes or more) and the low bits of
// the destination offset (so are its stores); the tile waits in LDS between
// the two.  Bit-deposit maps (tile bit j -> offset bit) come in the kernel
// arguments: per thread, the deposit of its thread index is computed once,
// and the deposit of each of its repeat indices is a table entry.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "../../include/moa_hypercube.h"
#include "hypercube_plan.h"

namespace moa_hc {

__device__ __forceinline__ int pad(int i) { return i + (i >> 5); }  // pad_slot on the device

// ---------------------------------------------------------------------------
// Transpose: out[o] = in[src(o)], src permuting the bits of o.
// ---------------------------------------------------------------------------

// PER elements of the tile per thread (PER * threads = tile elements).
template <typename T, int PER>
__global__ void __launch_bounds__(kThreads) k_hc_transpose(TransArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    const T* __restrict__ in = reinterpret_cast<const T*>(a.in);
    T* __restrict__ out = reinterpret_cast<T*>(a.out);
    const uint32_t t = threadIdx.x;
    // Tile offsets (uniform).
    const uint64_t tile = blockIdx.x;
    uint64_t ob = 0, ib = 0;
#pragma unroll
    for (int j = 0; j < kMaxRankBits; ++j) {
        if (j < a.nt_bits) {
            const uint64_t bit = (tile >> j) & 1u;
            ob |= bit << a.nt_out[j];
            ib |= bit << a.nt_in[j];
        }
    }
    // Deposits of the thread index.
    uint64_t in_lo = 0, out_lo = 0;
    uint32_t lds_lo = 0;
#pragma unroll
    for (int j = 0; j < kLgThreads; ++j) {
        if (j < a.lg_threads) {
            const uint32_t bit = (t >> j) & 1u;
            in_lo |= uint64_t(bit) << a.ld_in_lo[j];
            lds_lo |= bit << a.ld_lds_lo[j];
            out_lo |= uint64_t(bit) << a.st_out_lo[j];
        }
    }
    // Load the tile (all loads in flight before the LDS stores).
    T v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) v[r] = in[ib + in_lo + uint64_t(a.ld_in_hi[r])];
#pragma unroll
    for (int r = 0; r < PER; ++r) lds[pad(int(lds_lo) + a.ld_lds_hi[r])] = v[r];
    __syncthreads();
    // Store it in the destination's order.
#pragma unroll
    for (int r = 0; r < PER; ++r) v[r] = lds[pad(int(t) + (r << a.lg_threads))];
#pragma unroll
    for (int r = 0; r < PER; ++r) out[ob + out_lo + uint64_t(a.st_out_hi[r])] = v[r];
}

// ---------------------------------------------------------------------------
// Density-matrix gate: every 2^q x 2^q block B of the block-diagonal view
// becomes U B U^H, read and written in place through the normal form.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float2 cmadd(float2 acc, float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}
__device__ __forceinline__ double2 cmadd(double2 acc, double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// acc + a conj(b)
__device__ __forceinline__ float2 cmadd_conj(float2 acc, float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x)), fmaf(a.y, b.x, fmaf(-a.x, b.y, acc.y)));
}
__device__ __forceinline__ double2 cmadd_conj(double2 acc, double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.y, b.x, fma(-a.x, b.y, acc.y)));
}

// The vector kernel (one to three qubits).  A task is NC columns (phase 1)
// or rows (phase 2) of one block, so each entry of U read serves NC
// elements: two for three complex64 qubits, whose U lives in LDS (complex128
// keeps one: its register budget); one and two qubits read U (at most 16
// values) at uniform addresses straight from global memory, which the
// compiler keeps in scalar registers.
template <typename C, int Q, int PER>
__global__ void __launch_bounds__(kThreads) k_density_gate(GateArgs a)
{
    constexpr int D = 1 << Q;
    constexpr int NC = Q == 3 && sizeof(C) == 8 ? 2 : 1;  // columns (rows) a task
    constexpr bool ULDS = Q >= 3;       // U from LDS (else from global memory, uniform)
    extern __shared__ __align__(16) unsigned char smem[];
    C* lds = reinterpret_cast<C*>(smem);
    const int tile_elems = 1 << a.tile_bits;
    C* ul = lds + pad(tile_elems);   // U, D x D
    const C* __restrict__ ug = reinterpret_cast<const C*>(a.gate);
    C* __restrict__ rho = reinterpret_cast<C*>(a.rho);
    const uint32_t t = threadIdx.x;
    const int nthr = 1 << a.lg_threads;
    const uint64_t tile = blockIdx.x;
    uint64_t base = 0;
#pragma unroll
    for (int j = 0; j < 2 * 15; ++j)
        if (j < a.nt_bits) base |= ((tile >> j) & 1u) << a.nt_addr[j];
    uint64_t lo = 0;
#pragma unroll
    for (int j = 0; j < kLgThreads; ++j)
        if (j < a.lg_threads) lo |= uint64_t((t >> j) & 1u) << a.lo_addr[j];
    C v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) v[r] = rho[base + lo + uint64_t(a.hi_addr[r])];
    if constexpr (ULDS)
        for (int i = int(t); i < D * D; i += nthr) ul[i] = ug[i];
    auto U = [&](int i, int k) { return ULDS ? ul[i * D + k] : ug[i * D + k]; };
#pragma unroll
    for (int r = 0; r < PER; ++r) lds[pad(int(t) + (r << a.lg_threads))] = v[r];
    // LDS offsets of U's row and column indices (uniform).
    int roff[D], coff[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        int ro = 0, co = 0;
#pragma unroll
        for (int b = 0; b < Q; ++b) {
            if ((k >> b) & 1) {
                ro |= 1 << a.row_lds[b];
                co |= 1 << a.col_lds[b];
            }
        }
        roff[k] = ro;
        coff[k] = co;
    }
    __syncthreads();
    const int nblk = 1 << a.blk_bits;
    const int tasks = nblk * (D / NC);
    // Phase 1: columns l + c D / NC of block beta: B[., l] <- U B[., l].
    for (int task = int(t); task < tasks; task += nthr) {
        const int beta = task & (nblk - 1), l = task >> a.blk_bits;
        int bo = 0;
#pragma unroll
        for (int j = 0; j < kMaxTileBits; ++j)
            if (j < a.blk_bits) bo |= ((beta >> j) & 1) << a.blk_lds[j];
        int c0[NC];
        C x[NC][D];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            c0[c] = bo + coff[l + c * (D / NC)];
#pragma unroll
            for (int k = 0; k < D; ++k) x[c][k] = lds[pad(c0[c] + roff[k])];
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            C acc[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c].x = acc[c].y = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const C w = U(i, k);
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] = cmadd(acc[c], w, x[c][k]);
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) lds[pad(c0[c] + roff[i])] = acc[c];
        }
    }
    __syncthreads();
    // Phase 2: rows i + c D / NC of block beta: T[i, .] <- T[i, .] U^H.
    for (int task = int(t); task < tasks; task += nthr) {
        const int beta = task & (nblk - 1), i = task >> a.blk_bits;
        int bo = 0;
#pragma unroll
        for (int j = 0; j < kMaxTileBits; ++j)
            if (j < a.blk_bits) bo |= ((beta >> j) & 1) << a.blk_lds[j];
        int r0[NC];
        C x[NC][D];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            r0[c] = bo + roff[i + c * (D / NC)];
#pragma unroll
            for (int l = 0; l < D; ++l) x[c][l] = lds[pad(r0[c] + coff[l])];
        }
#pragma unroll
        for (int b = 0; b < D; ++b) {
            C acc[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c].x = acc[c].y = 0;
#pragma unroll
            for (int l = 0; l < D; ++l) {
                const C w = U(b, l);
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] = cmadd_conj(acc[c], x[c][l], w);
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) lds[pad(r0[c] + coff[b])] = acc[c];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) v[r] = lds[pad(int(t) + (r << a.lg_threads))];
#pragma unroll
    for (int r = 0; r < PER; ++r) rho[base + lo + uint64_t(a.hi_addr[r])] = v[r];
}

// Four-qubit gate of a density matrix on the matrix cores.  One wave takes a
// 16 x 16 block B of the tile at a time and forms C = B U^H, then
// E = U C = U B U^H, with v_mfma_f32_16x16x4_f32 for complex64 and
// v_mfma_f64_16x16x4_f64 for complex128 (operands and accumulation in the
// element's precision, as the vector kernel), four real products per
// complex one:
//   C = B U^H:  m = row i of B, n = row b of U, K = column l;
//   E = U C:    m = row a of U, n = column b of C, K = row i of C.
// Lane (g, x) = (lane / 16, lane % 16) holds, in K step s, the operand of K
// index k(g, s), where k(g, j) is also the row of the accumulator register j
// of lane (g, n): 4g + j for the f32 instruction, g + 4j for the f64 one
// (measured lane layouts).  In that K order the first product's
// accumulators (lane (g, n): C[k(g, j)][n]) are the second's B operand as
// they stand, and both products take the same U fragments U[x][k(g, s)]: a
// block leaves LDS once and returns once.  (The vector kernel reads 16 entries of U from
// LDS for every element of each product, which bounds it.)
template <typename C> struct GateMfma;
template <> struct GateMfma<float2> {
    using R = float;
    typedef float R4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ int k(int g, int s) { return 4 * g + s; }
    static __device__ __forceinline__ R4 mma(float x, float y, R4 acc)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc, 0, 0, 0);
    }
};
template <> struct GateMfma<double2> {
    using R = double;
    typedef double R4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ int k(int g, int s) { return g + 4 * s; }
    static __device__ __forceinline__ R4 mma(double x, double y, R4 acc)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
    }
};

template <typename C, int PER>
__global__ void __launch_bounds__(kThreads) k_density_gate4_mfma(GateArgs a)
{
    using M = GateMfma<C>;
    using R = typename M::R;
    using R4 = typename M::R4;
    extern __shared__ __align__(16) unsigned char smem[];
    C* lds = reinterpret_cast<C*>(smem);
    C* __restrict__ rho = reinterpret_cast<C*>(a.rho);
    const uint32_t t = threadIdx.x;
    const int nthr = 1 << a.lg_threads;
    const uint64_t tile = blockIdx.x;
    uint64_t base = 0;
#pragma unroll
    for (int j = 0; j < 2 * 15; ++j)
        if (j < a.nt_bits) base |= ((tile >> j) & 1u) << a.nt_addr[j];
    uint64_t lo = 0;
#pragma unroll
    for (int j = 0; j < kLgThreads; ++j)
        if (j < a.lg_threads) lo |= uint64_t((t >> j) & 1u) << a.lo_addr[j];
    C v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) v[r] = rho[base + lo + uint64_t(a.hi_addr[r])];
    // U fragments of this lane, behind the tile's loads.
    const int lane = int(t & 63u), g = lane >> 4, x = lane & 15;
    const C* __restrict__ u = reinterpret_cast<const C*>(a.gate);
    R ur[4], ui[4], nui[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const C w = u[x * 16 + M::k(g, s)];
        ur[s] = w.x;
        ui[s] = w.y;
        nui[s] = -w.y;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) lds[pad(int(t) + (r << a.lg_threads))] = v[r];
    // LDS offsets of U's row and column indices: x, and k(g, s).
    auto dep = [&](int k, const int8_t* pos) {
        int o = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((k >> b) & 1) o |= 1 << pos[b];
        return o;
    };
    const int rx = dep(x, a.row_lds), cx = dep(x, a.col_lds);
    int ca[4], rb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        ca[s] = dep(M::k(g, s), a.col_lds);
        rb[s] = dep(M::k(g, s), a.row_lds);
    }
    __syncthreads();
    const int nblk = 1 << a.blk_bits;
    for (int beta = int(t >> 6); beta < nblk; beta += nthr >> 6) {
        int bo = 0;
#pragma unroll
        for (int j = 0; j < kMaxTileBits; ++j)
            if (j < a.blk_bits) bo |= ((beta >> j) & 1) << a.blk_lds[j];
        C bv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) bv[s] = lds[pad(bo + rx + ca[s])];  // B[x][k(g, s)]
        // C = B U^H: Re = Br Ur^T + Bi Ui^T, Im = Bi Ur^T - Br Ui^T.
        R4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            cr = M::mma(bv[s].x, ur[s], cr);
            ci = M::mma(bv[s].y, ur[s], ci);
            cr = M::mma(bv[s].y, ui[s], cr);
            ci = M::mma(bv[s].x, nui[s], ci);
        }
        // E = U C: Re = Ur Cr - Ui Ci, Im = Ur Ci + Ui Cr.
        R4 er = {0, 0, 0, 0}, ei = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            er = M::mma(ur[s], cr[s], er);
            ei = M::mma(ur[s], ci[s], ei);
            er = M::mma(nui[s], ci[s], er);
            ei = M::mma(ui[s], cr[s], ei);
        }
        // The whole block was read by this wave above: in place.
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            C e;
            e.x = er[j];
            e.y = ei[j];
            lds[pad(bo + rb[j] + cx)] = e;  // E[k(g, j)][x]
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) v[r] = lds[pad(int(t) + (r << a.lg_threads))];
#pragma unroll
    for (int r = 0; r < PER; ++r) rho[base + lo + uint64_t(a.hi_addr[r])] = v[r];
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_transpose(const TransArgs& a, int64_t tiles, int lds_bytes, hipStream_t s)
{
    const dim3 g(static_cast<unsigned>(tiles)), b(1u << a.lg_threads);
    switch (a.tile_bits - a.lg_threads) {
        case 0: hipLaunchKernelGGL((k_hc_transpose<T, 1>), g, b, lds_bytes, s, a); break;
        case 1: hipLaunchKernelGGL((k_hc_transpose<T, 2>), g, b, lds_bytes, s, a); break;
        case 2: hipLaunchKernelGGL((k_hc_transpose<T, 4>), g, b, lds_bytes, s, a); break;
        case 3: hipLaunchKernelGGL((k_hc_transpose<T, 8>), g, b, lds_bytes, s, a); break;
        case 4: hipLaunchKernelGGL((k_hc_transpose<T, 16>), g, b, lds_bytes, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename C, int PER>
void launch_gate4_mfma(const GateArgs& a, dim3 g, dim3 b, int lds_bytes, hipStream_t s)
{
    hipLaunchKernelGGL((k_density_gate4_mfma<C, PER>), g, b, lds_bytes, s, a);
}

template <typename C, int Q>
hipError_t launch_gate_q(const GateArgs& a, dim3 g, dim3 b, int lds_bytes, hipStream_t s)
{
    // Four qubits: the matrix-core kernel (256 threads, blocks of 16 x 16,
    // at least one a tile).
    if constexpr (Q == 4) {
        switch (a.tile_bits - a.lg_threads) {
            case 0: launch_gate4_mfma<C, 1>(a, g, b, lds_bytes, s); break;
            case 1: launch_gate4_mfma<C, 2>(a, g, b, lds_bytes, s); break;
            case 2: launch_gate4_mfma<C, 4>(a, g, b, lds_bytes, s); break;
            case 3: launch_gate4_mfma<C, 8>(a, g, b, lds_bytes, s); break;
            case 4: launch_gate4_mfma<C, 16>(a, g, b, lds_bytes, s); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    } else {
        switch (a.tile_bits - a.lg_threads) {
            case 0: hipLaunchKernelGGL((k_density_gate<C, Q, 1>), g, b, lds_bytes, s, a); break;
            case 1: hipLaunchKernelGGL((k_density_gate<C, Q, 2>), g, b, lds_bytes, s, a); break;
            case 2: hipLaunchKernelGGL((k_density_gate<C, Q, 4>), g, b, lds_bytes, s, a); break;
            case 3: hipLaunchKernelGGL((k_density_gate<C, Q, 8>), g, b, lds_bytes, s, a); break;
            case 4: hipLaunchKernelGGL((k_density_gate<C, Q, 16>), g, b, lds_bytes, s, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

template <typename C>
hipError_t launch_gate(int q, const GateArgs& a, int64_t tiles, int lds_bytes, hipStream_t s)
{
    const dim3 g(static_cast<unsigned>(tiles)), b(1u << a.lg_threads);
    switch (q) {
        case 1: return launch_gate_q<C, 1>(a, g, b, lds_bytes, s);
        case 2: return launch_gate_q<C, 2>(a, g, b, lds_bytes, s);
        case 3: return launch_gate_q<C, 3>(a, g, b, lds_bytes, s);
        default: return launch_gate_q<C, 4>(a, g, b, lds_bytes, s);
    }
}

}  // namespace moa_hc

using namespace moa_hc;

extern "C" moa_status_t moa_hypercube_transpose(int32_t rank, const int32_t* t, int32_t elem_bytes, const void* in,
                                                void* out, void* stream)
{
    TransArgs a;
    Launch L;
    if (const moa_status_t st = plan_transpose(rank, t, elem_bytes, in, out, a, L)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (elem_bytes == 4) e = launch_transpose<uint32_t>(a, L.tiles, L.lds_bytes, s);
    else if (elem_bytes == 8) e = launch_transpose<uint2>(a, L.tiles, L.lds_bytes, s);
    else e = launch_transpose<uint4>(a, L.tiles, L.lds_bytes, s);
    return e == hipSuccess ? MOA_OK : MOA_ERR_HIP;
}

extern "C" moa_status_t moa_density_gate(int32_t n_qubits, int32_t q, const int32_t* gated_bits, const void* gate,
                                         moa_fft_dtype_t dtype, void* rho, void* stream)
{
    GateArgs a;
    Launch L;
    if (const moa_status_t st = plan_gate(n_qubits, q, gated_bits, gate, dtype, rho, a, L)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = dtype == MOA_C128 ? launch_gate<double2>(q, a, L.tiles, L.lds_bytes, s)
                                           : launch_gate<float2>(q, a, L.tiles, L.lds_bytes, s);
    return e == hipSuccess ? MOA_OK : MOA_ERR_HIP;
}
