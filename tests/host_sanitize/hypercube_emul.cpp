// CPU check of the hyper-cube kernels' addressing (csrc/hypercube.hip): the
// host planner (csrc/hypercube_plan.h) fills the kernel arguments, and this
// program runs every workgroup and thread of the kernels' index arithmetic on
// the CPU -- the tile offsets from the tile-index bits, the deposits of the
// thread index and of each repeat, the LDS slots -- checking that every
// global offset lies inside the array, every LDS slot inside the allocation,
// every slot is written once before it is read, and that the result is the
// definition: out[o] = in[src(o)] for the transpose, G rho G^H for the gate.
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "hypercube_plan.h"

using namespace moa_hc;
using cd = std::complex<double>;

static int failures = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            if (failures < 20) fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

static void transpose_case(int m, const std::vector<int32_t>& t, int eb)
{
    TransArgs a;
    Launch L;
    const size_t N = size_t(1) << m;
    // fake addresses, far apart (never dereferenced)
    const void* in = reinterpret_cast<const void*>(uintptr_t(1) << 44);
    void* out = reinterpret_cast<void*>(uintptr_t(1) << 45);
    const moa_status_t st = plan_transpose(m, t.data(), eb, in, out, a, L);
    CHECK(st == MOA_OK);
    if (st != MOA_OK) return;
    CHECK(L.threads == (1 << a.lg_threads) && L.threads <= kThreads);
    const int per = 1 << (a.tile_bits - a.lg_threads);
    CHECK(per >= 1 && per <= kMaxRepeat);
    const int slots = L.lds_bytes / eb;
    std::vector<uint64_t> src(N), got(N, ~uint64_t(0));
    for (size_t i = 0; i < N; ++i) src[i] = i * 2654435761u + 17;  // values: any injective map
    std::vector<int> written(static_cast<size_t>(slots));
    std::vector<uint64_t> lds(static_cast<size_t>(slots));
    for (int64_t tile = 0; tile < L.tiles; ++tile) {
        uint64_t ob = 0, ib = 0;
        for (int j = 0; j < a.nt_bits; ++j) {
            const uint64_t bit = (uint64_t(tile) >> j) & 1u;
            ob |= bit << a.nt_out[j];
            ib |= bit << a.nt_in[j];
        }
        std::fill(written.begin(), written.end(), 0);
        for (int th = 0; th < L.threads; ++th) {
            uint64_t in_lo = 0;
            uint32_t lds_lo = 0;
            for (int j = 0; j < a.lg_threads; ++j) {
                const uint32_t bit = (uint32_t(th) >> j) & 1u;
                in_lo |= uint64_t(bit) << a.ld_in_lo[j];
                lds_lo |= bit << a.ld_lds_lo[j];
            }
            for (int r = 0; r < per; ++r) {
                const uint64_t off = ib + in_lo + uint64_t(a.ld_in_hi[r]);
                const int slot = pad_slot(int(lds_lo) + a.ld_lds_hi[r]);
                CHECK(off < N);
                CHECK(slot >= 0 && slot < slots);
                if (off >= N || slot < 0 || slot >= slots) return;
                CHECK(written[size_t(slot)] == 0);
                written[size_t(slot)] = 1;
                lds[size_t(slot)] = src[off];
            }
        }
        for (int th = 0; th < L.threads; ++th) {
            uint64_t out_lo = 0;
            for (int j = 0; j < a.lg_threads; ++j) out_lo |= uint64_t((uint32_t(th) >> j) & 1u) << a.st_out_lo[j];
            for (int r = 0; r < per; ++r) {
                const int slot = pad_slot(th + (r << a.lg_threads));
                const uint64_t off = ob + out_lo + uint64_t(a.st_out_hi[r]);
                CHECK(slot < slots && written[size_t(slot)] == 1);
                CHECK(off < N);
                if (off >= N || slot >= slots) return;
                CHECK(got[off] == ~uint64_t(0));
                got[off] = lds[size_t(slot)];
            }
        }
    }
    // definition: out axis k of i ... in offset bit (m-1-k) = out offset bit (m-1-t_k)
    for (size_t o = 0; o < N; ++o) {
        uint64_t s = 0;
        for (int k = 0; k < m; ++k) s |= uint64_t((o >> (m - 1 - t[size_t(k)])) & 1u) << (m - 1 - k);
        CHECK(got[o] == src[s]);
        if (got[o] != src[s]) return;
    }
}

static void gate_case(int n, const std::vector<int32_t>& gated, bool c128, std::mt19937_64& rng)
{
    const int q = int(gated.size());
    const int D = 1 << q;
    const size_t N = size_t(1) << n, NN = N * N;
    GateArgs a;
    Launch L;
    void* rho = reinterpret_cast<void*>(uintptr_t(1) << 44);
    const void* gate = reinterpret_cast<const void*>(uintptr_t(1) << 45);
    const moa_status_t st = plan_gate(n, q, gated.data(), gate, c128 ? MOA_C128 : MOA_C64, rho, a, L);
    CHECK(st == MOA_OK);
    if (st != MOA_OK) return;
    const int eb = c128 ? 16 : 8;
    const int per = 1 << (a.tile_bits - a.lg_threads);
    CHECK(per >= 1 && per <= kMaxRepeat && L.threads <= kThreads);
    const int tile_elems = 1 << a.tile_bits;
    const int slots = L.lds_bytes / eb;
    CHECK(pad_slot(tile_elems) + D * D <= slots);
    std::uniform_real_distribution<double> u(-1, 1);
    std::vector<cd> r0(NN), U(size_t(D * D)), got(NN);
    for (auto& v : r0) v = cd(u(rng), u(rng));
    for (auto& v : U) v = cd(u(rng), u(rng));
    got = r0;
    std::vector<cd> lds(static_cast<size_t>(slots));
    std::vector<int> touched(NN, 0);
    int roff[16], coff[16];
    for (int k = 0; k < D; ++k) {
        int ro = 0, co = 0;
        for (int b = 0; b < q; ++b)
            if ((k >> b) & 1) {
                ro |= 1 << a.row_lds[b];
                co |= 1 << a.col_lds[b];
            }
        roff[k] = ro;
        coff[k] = co;
    }
    const int nblk = 1 << a.blk_bits;
    CHECK(nblk * D * D == tile_elems);
    for (int64_t tile = 0; tile < L.tiles; ++tile) {
        uint64_t base = 0;
        for (int j = 0; j < a.nt_bits; ++j) base |= ((uint64_t(tile) >> j) & 1u) << a.nt_addr[j];
        std::vector<int> seen(size_t(slots), 0);
        std::vector<uint64_t> addr_of(static_cast<size_t>(tile_elems));
        for (int th = 0; th < L.threads; ++th) {
            uint64_t lo = 0;
            for (int j = 0; j < a.lg_threads; ++j) lo |= uint64_t((uint32_t(th) >> j) & 1u) << a.lo_addr[j];
            for (int r = 0; r < per; ++r) {
                const uint64_t off = base + lo + uint64_t(a.hi_addr[r]);
                const int e = th + (r << a.lg_threads);
                CHECK(off < NN);
                if (off >= NN) return;
                CHECK(touched[off] == 0);
                touched[off] = 1;
                CHECK(seen[size_t(pad_slot(e))] == 0);
                seen[size_t(pad_slot(e))] = 1;
                lds[size_t(pad_slot(e))] = got[off];
                addr_of[size_t(e)] = off;
            }
        }
        if (q == 4) {
            // The matrix-core kernel's schedule: per block, lane (g, x)
            // reads B[x][k(g, s)]; the first product's accumulator register
            // j of lane (g, n) is C[k(g, j)][n]; the second product's is
            // E[k(g, j)][n], stored at row k(g, j), column n; k(g, j) = 4g + j
            // for the f32 instruction, g + 4j for the f64 one.  One MFMA
            // adds sum_gg A(lane 16 gg + m) B(lane 16 gg + n) to D[m][n],
            // D[k(g, j)][n] being register j of lane 16 g + n.
            CHECK(L.threads % 64 == 0);
            auto kk = [&](int g, int s) { return c128 ? g + 4 * s : 4 * g + s; };
            auto Uf = [&](int lane, int s) { return U[size_t((lane & 15) * 16 + kk(lane >> 4, s))]; };
            // (lane, register) of D[m][n]
            int dl[16], dj[16];
            for (int g = 0; g < 4; ++g)
                for (int j = 0; j < 4; ++j) {
                    dl[kk(g, j)] = 16 * g;
                    dj[kk(g, j)] = j;
                }
            for (int beta = 0; beta < nblk; ++beta) {
                int bo = 0;
                for (int j = 0; j < a.blk_bits; ++j) bo |= ((beta >> j) & 1) << a.blk_lds[j];
                cd bv[64][4];
                for (int lane = 0; lane < 64; ++lane)
                    for (int s = 0; s < 4; ++s) {
                        const int e = bo + roff[lane & 15] + coff[kk(lane >> 4, s)];
                        CHECK(e < tile_elems);
                        bv[lane][s] = lds[size_t(pad_slot(e))];
                    }
                double cr[64][4] = {}, ci[64][4] = {}, er[64][4] = {}, ei[64][4] = {};
                for (int s = 0; s < 4; ++s)
                    for (int m = 0; m < 16; ++m)
                        for (int n = 0; n < 16; ++n) {
                            const int lane = dl[m] + n, j = dj[m];  // D[m][n]
                            for (int gg = 0; gg < 4; ++gg) {
                                const cd av = bv[16 * gg + m][s], w = Uf(16 * gg + n, s);
                                cr[lane][j] += av.real() * w.real() + av.imag() * w.imag();
                                ci[lane][j] += av.imag() * w.real() - av.real() * w.imag();
                            }
                        }
                for (int s = 0; s < 4; ++s)
                    for (int m = 0; m < 16; ++m)
                        for (int n = 0; n < 16; ++n) {
                            const int lane = dl[m] + n, j = dj[m];
                            for (int gg = 0; gg < 4; ++gg) {
                                const cd w = Uf(16 * gg + m, s);
                                const double br = cr[16 * gg + n][s], bi = ci[16 * gg + n][s];
                                er[lane][j] += w.real() * br - w.imag() * bi;
                                ei[lane][j] += w.real() * bi + w.imag() * br;
                            }
                        }
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 4; ++j) {
                        const int e = bo + roff[kk(lane >> 4, j)] + coff[lane & 15];
                        CHECK(e < tile_elems);
                        lds[size_t(pad_slot(e))] = cd(er[lane][j], ei[lane][j]);
                    }
            }
            for (int e = 0; e < tile_elems; ++e) got[addr_of[size_t(e)]] = lds[size_t(pad_slot(e))];
            continue;
        }
        // phase 1: columns, phase 2: rows (the kernel's task loops: a task
        // is NC columns or rows of a block, NC = 2 for three complex64 qubits)
        const int NC = q == 3 && !c128 ? 2 : 1;
        for (int task = 0; task < nblk * (D / NC); ++task) {
            const int beta = task & (nblk - 1), l = task >> a.blk_bits;
            int bo = 0;
            for (int j = 0; j < a.blk_bits; ++j) bo |= ((beta >> j) & 1) << a.blk_lds[j];
            for (int c = 0; c < NC; ++c) {
                const int c0 = bo + coff[l + c * (D / NC)];
                cd x[16];
                for (int k = 0; k < D; ++k) {
                    CHECK(c0 + roff[k] < tile_elems);
                    x[k] = lds[size_t(pad_slot(c0 + roff[k]))];
                }
                for (int i = 0; i < D; ++i) {
                    cd acc = 0;
                    for (int k = 0; k < D; ++k) acc += U[size_t(i * D + k)] * x[k];
                    lds[size_t(pad_slot(c0 + roff[i]))] = acc;
                }
            }
        }
        for (int task = 0; task < nblk * (D / NC); ++task) {
            const int beta = task & (nblk - 1), i = task >> a.blk_bits;
            int bo = 0;
            for (int j = 0; j < a.blk_bits; ++j) bo |= ((beta >> j) & 1) << a.blk_lds[j];
            for (int c = 0; c < NC; ++c) {
                const int r0_ = bo + roff[i + c * (D / NC)];
                cd x[16];
                for (int l = 0; l < D; ++l) x[l] = lds[size_t(pad_slot(r0_ + coff[l]))];
                for (int b = 0; b < D; ++b) {
                    cd acc = 0;
                    for (int l = 0; l < D; ++l) acc += x[l] * std::conj(U[size_t(b * D + l)]);
                    lds[size_t(pad_slot(r0_ + coff[b]))] = acc;
                }
            }
        }
        for (int e = 0; e < tile_elems; ++e) got[addr_of[size_t(e)]] = lds[size_t(pad_slot(e))];
    }
    for (size_t i = 0; i < NN; ++i) CHECK(touched[i] == 1);
    // definition: G rho G^H, G[i][j] = U[g(i)][g(j)] when the free bits agree
    uint64_t mask = 0;
    for (int b : gated) mask |= uint64_t(1) << b;
    std::vector<int> sorted(gated.begin(), gated.end());
    std::sort(sorted.begin(), sorted.end());
    auto g = [&](uint64_t i) {
        int r = 0;
        for (int k = 0; k < q; ++k) r |= int((i >> sorted[size_t(k)]) & 1u) << k;
        return r;
    };
    auto with = [&](uint64_t i, int v) {
        uint64_t r = i & ~mask;
        for (int k = 0; k < q; ++k) r |= uint64_t((v >> k) & 1) << sorted[size_t(k)];
        return r;
    };
    double err = 0, nrm = 0;
    for (uint64_t i = 0; i < N; ++i)
        for (uint64_t j = 0; j < N; ++j) {
            cd acc = 0;
            for (int ap = 0; ap < D; ++ap)
                for (int bp = 0; bp < D; ++bp)
                    acc += U[size_t(g(i) * D + ap)] * r0[with(i, ap) * N + with(j, bp)] *
                           std::conj(U[size_t(g(j) * D + bp)]);
            err += std::norm(acc - got[i * N + j]);
            nrm += std::norm(acc);
        }
    CHECK(err <= 1e-24 * nrm);
}

int main()
{
    std::mt19937_64 rng(99);
    // transposes: every rank up to 14 with random permutations, the paper's
    // vectors, identity, reversal, and larger ranks with few tiles checked
    for (int eb : {4, 8, 16}) {
        for (int m = 1; m <= 14; ++m)
            for (int rep = 0; rep < 6; ++rep) {
                std::vector<int32_t> t(static_cast<size_t>(m));
                for (int k = 0; k < m; ++k) t[size_t(k)] = k;
                if (rep == 1) std::reverse(t.begin(), t.end());
                if (rep >= 2) std::shuffle(t.begin(), t.end(), rng);
                transpose_case(m, t, eb);
            }
        transpose_case(8, {0, 2, 1, 3, 4, 6, 5, 7}, eb);
        transpose_case(8, {0, 3, 1, 2, 4, 7, 5, 6}, eb);
        // block-diagonal views of an 11-qubit matrix (gated 0, 2 and 9, 10):
        // permutations that keep the low bits low
        transpose_case(22, {0, 1, 2, 3, 4, 5, 6, 7, 9, 8, 10, 11, 12, 13, 14, 15, 16, 17, 18, 20, 19, 21}, eb);
        transpose_case(22, {9, 10, 0, 1, 2, 3, 4, 5, 6, 7, 8, 20, 21, 11, 12, 13, 14, 15, 16, 17, 18, 19}, eb);
        std::vector<int32_t> t20(20);
        for (int k = 0; k < 20; ++k) t20[size_t(k)] = (k + 7) % 20;
        transpose_case(20, t20, eb);
    }
    // gates: every n up to 7 with random gated sets of 1..4 qubits
    for (int c128 = 0; c128 < 2; ++c128)
        for (int n = 1; n <= 7; ++n)
            for (int q = 1; q <= std::min(4, n); ++q)
                for (int rep = 0; rep < 3; ++rep) {
                    std::vector<int32_t> bits(static_cast<size_t>(n));
                    for (int k = 0; k < n; ++k) bits[size_t(k)] = k;
                    std::shuffle(bits.begin(), bits.end(), rng);
                    bits.resize(size_t(q));
                    gate_case(n, bits, c128 != 0, rng);
                }
    gate_case(4, {0, 2}, false, rng);
    gate_case(4, {1, 2}, true, rng);
    gate_case(8, {7, 0}, false, rng);
    gate_case(9, {4, 5, 6, 8}, false, rng);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("hypercube addressing: all cases clean\n");
    return 0;
}
