// psi-calculus lowering layer (host side).
//
// The planner describes every array it touches by a shape vector and a
// row-major layout (Ch. 2, "Indexing and Shapes"); the operations it needs
// are the ones the paper uses to derive the normal forms of the
// cache-optimized FFT:
//   gamma / gamma'   index <-> offset (Def. gammadef and its inverse),
//   take / drop      on shape vectors,
//   pct              the psi Correspondence Theorem (Ch. 4, Def. psi_corr):
//                    the sub-array selected by a partial index is one
//                    contiguous run of the ravel, start gamma(j; tau j take s)
//                    * pi(tau j drop s), length pi(tau j drop s),
//   axis_strides     the stride of each axis, i.e. the PCT run length of the
//                    partial index that stops just before it,
//   transpose_view   the strides of t transpose A for a permutation vector t
//                    (i psi (t transpose A) = i[t] psi A).
// The planner lowers a lift to pass descriptors with these: each level's DFT
// axis, batch axes and output layout are read off the strides of the digit
// view of the vector (the operational normal form: starts, stops, strides).
#pragma once

#include <stdint.h>

#include <numeric>
#include <stdexcept>
#include <vector>

namespace moa {
namespace psi {

using Vec = std::vector<int64_t>;

inline int64_t pi(const Vec& v)
{
    int64_t p = 1;
    for (int64_t x : v) p *= x;
    return p;
}

inline Vec take(int64_t k, const Vec& v)
{
    const int64_t n = int64_t(v.size());
    if (k >= 0) return Vec(v.begin(), v.begin() + (k < n ? k : n));
    const int64_t m = -k < n ? -k : n;
    return Vec(v.end() - m, v.end());
}

inline Vec drop(int64_t k, const Vec& v)
{
    const int64_t n = int64_t(v.size());
    if (k >= 0) return Vec(v.begin() + (k < n ? k : n), v.end());
    const int64_t m = -k < n ? -k : n;
    return Vec(v.begin(), v.end() - m);
}

inline Vec reverse(const Vec& v) { return Vec(v.rbegin(), v.rend()); }

// Row-major offset of index p in an array of shape s (the recurrence
// x_0 = p_0, x_j = x_{j-1} s_j + p_j).
inline int64_t gamma(const Vec& s, const Vec& p)
{
    if (p.empty()) return 0;
    int64_t x = p[0];
    for (size_t j = 1; j < p.size(); ++j) x = x * s[j] + p[j];
    return x;
}

inline Vec gamma_inv(const Vec& s, int64_t off)
{
    Vec p(s.size(), 0);
    for (int64_t j = int64_t(s.size()) - 1; j >= 0; --j) {
        p[size_t(j)] = off % s[size_t(j)];
        off /= s[size_t(j)];
    }
    return p;
}

struct Run {
    int64_t start, length;
};

// psi Correspondence Theorem: rav(j psi xi) = (rav xi)[start + iota length].
inline Run pct(const Vec& s, const Vec& j)
{
    const int64_t k = int64_t(j.size());
    const int64_t len = pi(drop(k, s));
    return Run{gamma(take(k, s), j) * len, len};
}

// Stride of each axis of a row-major array: the PCT run length of a partial
// index of length i + 1.
inline Vec axis_strides(const Vec& s)
{
    Vec st(s.size());
    for (size_t i = 0; i < s.size(); ++i) st[i] = pct(s, Vec(i + 1, 0)).length;
    return st;
}

// Strides (in the ravel of A) of the axes of t transpose A: axis t[k] of the
// result is axis k of A, so its stride is A's stride of axis k.
inline Vec transpose_view(const Vec& strides_of_A, const Vec& t)
{
    Vec out(t.size());
    for (size_t k = 0; k < t.size(); ++k) out[size_t(t[k])] = strides_of_A[k];
    return out;
}

inline Vec iota(int64_t n)
{
    Vec v(static_cast<size_t>(n));
    std::iota(v.begin(), v.end(), int64_t(0));
    return v;
}

}  // namespace psi
}  // namespace moa
