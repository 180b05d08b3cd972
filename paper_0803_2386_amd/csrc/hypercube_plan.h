// Host planning of the hyper-cube kernels (hypercube.hip): validation and
// the bit-deposit maps of the tiles.  Plain C++ with no HIP types, so the
// CPU tests can build it and check every address the kernels form.
#pragma once

#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "../../include/moa_fft.h"

namespace moa_hc {

constexpr int kThreads = 256;
constexpr int kLgThreads = 8;
constexpr int kMaxTileBits = 12;     // 4096 elements
constexpr int kMaxRepeat = 1 << (kMaxTileBits - kLgThreads);  // per-thread elements of a tile
constexpr int kMaxRankBits = 34;     // offset bits of an array

// LDS slot of tile element i: one spare slot after every 32 elements.
constexpr inline int pad_slot(int i) { return i + (i >> 5); }

// Transpose: out[o] = in[src(o)], src permuting the bits of o.
struct TransArgs {
    const void* in;
    void* out;
    int tile_bits;                  // bits of the tile (LDS index bits)
    int lg_threads;                 // log2 threads of the workgroup
    int nt_bits;                    // bits of the tile index
    int8_t nt_out[kMaxRankBits];    // tile-index bit j -> out offset bit
    int8_t nt_in[kMaxRankBits];     // tile-index bit j -> in offset bit
    // load order: element e of the tile, low bits = in offset bits 0.. (runs)
    int8_t ld_in_lo[kLgThreads];    // bit j of e (j < lg_threads) -> in offset bit
    int8_t ld_lds_lo[kLgThreads];   // bit j of e -> LDS index bit
    int64_t ld_in_hi[kMaxRepeat];   // in-offset deposit of r << lg_threads
    int32_t ld_lds_hi[kMaxRepeat];  // LDS deposit of r << lg_threads
    // store order: LDS index e (low bits = out offset bits 0..)
    int8_t st_out_lo[kLgThreads];
    int64_t st_out_hi[kMaxRepeat];
};

// Density-matrix gate: every 2^q x 2^q block B of the block-diagonal view
// becomes U B U^H, read and written in place through the normal form.
struct GateArgs {
    void* rho;
    const void* gate;
    int tile_bits;
    int lg_threads;
    int nt_bits;
    int blk_bits;                   // block-index bits of the tile
    int8_t nt_addr[2 * 15];         // tile-index bit j -> offset bit of rho
    int8_t lo_addr[kLgThreads];     // LDS index bit j (j < lg_threads) -> offset bit
    int64_t hi_addr[kMaxRepeat];    // offset deposit of r << lg_threads
    int8_t blk_lds[kMaxTileBits];   // block-index bit -> LDS index bit
    int8_t row_lds[4];              // bit r of U's row index -> LDS index bit
    int8_t col_lds[4];              // bit r of U's column index -> LDS index bit
};

struct Launch {
    int64_t tiles = 0;   // workgroups
    int threads = 0;
    int lds_bytes = 0;
};

inline int lg2i(int64_t x)
{
    int r = 0;
    while ((int64_t(1) << r) < x) ++r;
    return r;
}

inline bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + nb && pb < pa + na;
}

// Validate a transpose and fill its kernel arguments and launch shape.
inline moa_status_t plan_transpose(int32_t rank, const int32_t* t, int32_t elem_bytes, const void* in, void* out,
                                   TransArgs& a, Launch& L)
{
    if (!t || !in || !out) return MOA_ERR_NULL;
    if (rank < 1 || rank > kMaxRankBits) return MOA_ERR_SIZE;
    if (elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16) return MOA_ERR_ARG;
    const int lge = lg2i(elem_bytes);
    if (rank + lge > 38) return MOA_ERR_SIZE;
    const int m = rank;
    bool seen[kMaxRankBits] = {false};
    for (int k = 0; k < m; ++k) {
        if (t[k] < 0 || t[k] >= m || seen[t[k]]) return MOA_ERR_ARG;
        seen[t[k]] = true;
    }
    const size_t bytes = size_t(elem_bytes) << m;
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) return MOA_ERR_ARG;
    if (overlap(in, bytes, out, bytes)) return MOA_ERR_ARG;
    // in offset bit of each out offset bit: axis k of the source takes the
    // value of axis t_k of the result (i[t]); axis k is offset bit m-1-k.
    int src_of[kMaxRankBits];
    for (int k = 0; k < m; ++k) src_of[m - 1 - t[k]] = m - 1 - k;
    int out_of[kMaxRankBits];
    for (int b = 0; b < m; ++b) out_of[src_of[b]] = b;
    // Tile: out bits 0..K-1 and the out bits fed by in bits 0..K-1, so that
    // both sides move runs of at least 2^K elements (256 bytes at the
    // smallest K = 8 - log2 elem_bytes).  K grows until the tile holds 2^10
    // elements (or the whole array): where the permutation keeps the low
    // bits low, the smallest K would leave tiles of a few dozen elements and
    // millions of tiny workgroups.  Each step of K adds at most two tile bits,
    // so the tile stays within max(2^11, 2^(2 K0)) <= 2^12 elements.
    auto tile_size = [&](int k) {
        bool tt[kMaxRankBits] = {false};
        int c = 0;
        for (int b = 0; b < k; ++b) tt[b] = true;
        for (int j = 0; j < k; ++j) tt[out_of[j]] = true;
        for (int b = 0; b < m; ++b) c += tt[b];
        return c;
    };
    int K = std::min(m, 8 - lge);
    while (K < m && tile_size(K) < 10) ++K;
    bool in_tile[kMaxRankBits] = {false};
    for (int b = 0; b < K; ++b) in_tile[b] = true;
    for (int j = 0; j < K; ++j) in_tile[out_of[j]] = true;
    int lds_of[kMaxRankBits];   // out bit -> LDS bit (tile bits only)
    int tb = 0;
    for (int b = 0; b < K; ++b) lds_of[b] = tb++;
    for (int b = K; b < m; ++b)
        if (in_tile[b]) lds_of[b] = tb++;
    memset(&a, 0, sizeof(a));
    a.in = in;
    a.out = out;
    a.tile_bits = tb;
    a.lg_threads = std::min(tb, kLgThreads);
    int nt = 0;
    for (int b = 0; b < m; ++b)
        if (!in_tile[b]) {
            a.nt_out[nt] = int8_t(b);
            a.nt_in[nt] = int8_t(src_of[b]);
            ++nt;
        }
    a.nt_bits = nt;
    // Load order: e bits 0..K-1 = in bits 0..K-1 (out bit out_of[j]); the
    // higher e bits = the tile's out bits whose in bit is >= K, increasing.
    int ld_in[kMaxTileBits], ld_lds[kMaxTileBits];
    int nb = 0;
    for (int j = 0; j < K; ++j) {
        ld_in[nb] = j;
        ld_lds[nb] = lds_of[out_of[j]];
        ++nb;
    }
    for (int b = 0; b < m; ++b)
        if (in_tile[b] && src_of[b] >= K) {
            ld_in[nb] = src_of[b];
            ld_lds[nb] = lds_of[b];
            ++nb;
        }
    // Store order: LDS bit j -> out bit.
    int st_out[kMaxTileBits];
    for (int b = 0; b < m; ++b)
        if (in_tile[b]) st_out[lds_of[b]] = b;
    if (nb != tb || tb > kMaxTileBits) return MOA_ERR_ARG;  // cannot happen: tb <= 12
    const int lt = a.lg_threads;
    for (int j = 0; j < lt; ++j) {
        a.ld_in_lo[j] = int8_t(ld_in[j]);
        a.ld_lds_lo[j] = int8_t(ld_lds[j]);
        a.st_out_lo[j] = int8_t(st_out[j]);
    }
    for (int r = 0; r < (1 << (tb - lt)); ++r) {
        int64_t di = 0, dout = 0;
        int32_t dl = 0;
        for (int j = lt; j < tb; ++j)
            if ((r >> (j - lt)) & 1) {
                di |= int64_t(1) << ld_in[j];
                dl |= int32_t(1) << ld_lds[j];
                dout |= int64_t(1) << st_out[j];
            }
        a.ld_in_hi[r] = di;
        a.ld_lds_hi[r] = dl;
        a.st_out_hi[r] = dout;
    }
    L.tiles = int64_t(1) << nt;
    L.threads = 1 << lt;
    L.lds_bytes = pad_slot(1 << tb) * elem_bytes;
    return MOA_OK;
}

// Validate a gate and fill its kernel arguments and launch shape.
inline moa_status_t plan_gate(int32_t n_qubits, int32_t q, const int32_t* gated_bits, const void* gate,
                              moa_fft_dtype_t dtype, void* rho, GateArgs& a, Launch& L)
{
    if (!gated_bits || !gate || !rho) return MOA_ERR_NULL;
    if (n_qubits < 1 || n_qubits > 15 || q < 1 || q > 4 || q > n_qubits) return MOA_ERR_SIZE;
    if (dtype != MOA_C64 && dtype != MOA_C128) return MOA_ERR_DTYPE;
    const int n = n_qubits;
    bool gated[15] = {false};
    for (int i = 0; i < q; ++i) {
        if (gated_bits[i] < 0 || gated_bits[i] >= n || gated[gated_bits[i]]) return MOA_ERR_ARG;
        gated[gated_bits[i]] = true;
    }
    if (reinterpret_cast<uintptr_t>(rho) & 15u) return MOA_ERR_ARG;
    const bool c128 = dtype == MOA_C128;
    const int eb = c128 ? 16 : 8;
    // Offset bits of rho: column bit b = offset bit b, row bit b = n + b.
    // Tile: the low K column bits (runs of 2^K elements), the gated column
    // bits, the gated row bits, then the lowest free row bits up to the
    // tile size (2^12 elements complex64, 2^11 complex128), all within 2n.
    const int cap = std::min(2 * n, c128 ? 11 : 12);
    const int m = 2 * n;
    bool in_tile[30] = {false};
    int K = std::min(n, c128 ? 6 : 7);
    auto count = [&](int k) {
        int c = k;
        for (int b = 0; b < n; ++b)
            if (gated[b]) c += (b >= k) + 1;
        return c;
    };
    while (K > 0 && count(K) > cap) --K;
    int tb = 0;
    int lds_of[30];
    for (int b = 0; b < K; ++b) {
        in_tile[b] = true;
        lds_of[b] = tb++;
    }
    for (int b = K; b < n; ++b)
        if (gated[b]) {
            in_tile[b] = true;
            lds_of[b] = tb++;
        }
    for (int b = 0; b < n; ++b)
        if (gated[b]) {
            in_tile[n + b] = true;
            lds_of[n + b] = tb++;
        }
    for (int b = 0; b < n && tb < cap; ++b)
        if (!gated[b]) {
            in_tile[n + b] = true;
            lds_of[n + b] = tb++;
        }
    if (tb > kMaxTileBits) return MOA_ERR_ARG;  // cannot happen: cap <= 12
    memset(&a, 0, sizeof(a));
    a.rho = rho;
    a.gate = gate;
    a.tile_bits = tb;
    a.lg_threads = std::min(tb, kLgThreads);
    int nt = 0;
    for (int b = 0; b < m; ++b)
        if (!in_tile[b]) a.nt_addr[nt++] = int8_t(b);
    a.nt_bits = nt;
    int addr_of_lds[kMaxTileBits];
    for (int b = 0; b < m; ++b)
        if (in_tile[b]) addr_of_lds[lds_of[b]] = b;
    for (int j = 0; j < a.lg_threads; ++j) a.lo_addr[j] = int8_t(addr_of_lds[j]);
    for (int r = 0; r < (1 << (tb - a.lg_threads)); ++r) {
        int64_t d = 0;
        for (int j = a.lg_threads; j < tb; ++j)
            if ((r >> (j - a.lg_threads)) & 1) d |= int64_t(1) << addr_of_lds[j];
        a.hi_addr[r] = d;
    }
    // U's index bit r = the r-th lowest gated bit.
    int r = 0;
    for (int b = 0; b < n; ++b)
        if (gated[b]) {
            a.row_lds[r] = int8_t(lds_of[n + b]);
            a.col_lds[r] = int8_t(lds_of[b]);
            ++r;
        }
    int nb = 0;
    for (int j = 0; j < tb; ++j) {
        const int b = addr_of_lds[j];
        const bool g = b < n ? gated[b] : gated[b - n];
        if (!g) a.blk_lds[nb++] = int8_t(j);
    }
    a.blk_bits = nb;
    L.tiles = int64_t(1) << nt;
    L.threads = 1 << a.lg_threads;
    L.lds_bytes = (pad_slot(1 << tb) + (1 << (2 * q))) * eb;
    return MOA_OK;
}

}  // namespace moa_hc
