"""Index-algebra oracle: A Mathematics of Arrays (MoA) and the psi-calculus.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain, slow Python that
states the definitions of Ch. 2 ("Indexing and Shapes", the operator summary
figure) and the psi Correspondence Theorem (Ch. 4, Def. psi_corr) directly,
so that the printed worked examples of the paper and the product's lowering
layer can be checked against them.  Arrays are ``MArray(shape, ravel)`` --
the first of the two equivalent descriptions of an array in Ch. 2 -- with a
row-major layout.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple


def pi(v: Sequence[int]) -> int:
    """Product of the items of a vector; pi of the empty vector is 1."""
    out = 1
    for x in v:
        out *= int(x)
    return out


def iota(n: int) -> List[int]:
    return list(range(int(n)))


def take(k: int, v: Sequence[int]) -> List[int]:
    """k >= 0: first k items; k < 0: last |k| items."""
    v = list(v)
    return v[:k] if k >= 0 else v[len(v) + k:]


def drop(k: int, v: Sequence[int]) -> List[int]:
    """k >= 0: all but the first k items; k < 0: all but the last |k| items."""
    v = list(v)
    return v[k:] if k >= 0 else v[:len(v) + k]


def rotate(k: int, v: Sequence[int]) -> List[int]:
    """k theta v: (k drop v) cat (k take v) for k >= 0, else (k take v) cat (k drop v)."""
    if k >= 0:
        return drop(k, v) + take(k, v)
    return take(k, v) + drop(k, v)


def gamma(shape: Sequence[int], idx: Sequence[int]) -> int:
    """Row-major offset by the recurrence x_0 = p_0, x_j = x_{j-1} s_j + p_j (Def. gammadef)."""
    if len(idx) == 0:
        return 0
    x = int(idx[0])
    for j in range(1, len(idx)):
        x = x * int(shape[j]) + int(idx[j])
    return x


def gamma_col(shape: Sequence[int], idx: Sequence[int]) -> int:
    """Column-major offset: gamma on the reversed shape and index."""
    return gamma(list(reversed(shape)), list(reversed(idx)))


def gamma_inv(shape: Sequence[int], off: int) -> List[int]:
    """gamma' : offset -> row-major index of an array of the given shape."""
    idx = [0] * len(shape)
    for j in range(len(shape) - 1, -1, -1):
        s = int(shape[j])
        idx[j] = off % s
        off //= s
    return idx


def indices(shape: Sequence[int]):
    """All full indices of an array of this shape, in lexical order."""
    for off in range(pi(shape)):
        yield gamma_inv(shape, off)


@dataclass
class MArray:
    shape: List[int]
    ravel: List

    def __post_init__(self):
        self.shape = [int(s) for s in self.shape]
        self.ravel = list(self.ravel)
        if len(self.ravel) != pi(self.shape):
            raise ValueError("ravel length does not match the shape")

    @property
    def dim(self) -> int:
        return len(self.shape)


def psi(p: Sequence[int], A: MArray):
    """p psi A.  Full index -> the item; partial index of length k -> the
    sub-array of shape (k drop shape) whose items are (p cat q) psi A."""
    p = list(p)
    if len(p) > A.dim:
        raise IndexError("index longer than the dimensionality")
    for pj, sj in zip(p, A.shape):
        if not 0 <= pj < sj:
            raise IndexError("index out of range")
    if len(p) == A.dim:
        return A.ravel[gamma(A.shape, p)]
    sub = drop(len(p), A.shape)
    return MArray(sub, [A.ravel[gamma(A.shape, p + q)] for q in indices(sub)])


def reshape(shape: Sequence[int], A: MArray) -> MArray:
    """shape rho^ A: fill the new shape from the ravel in order, wrapping to the
    start of the ravel when the new array is larger (Ch. 5, "The Importance of
    the Array's Shape")."""
    n = pi(shape)
    src = A.ravel
    if n and not src:
        raise ValueError("cannot reshape an empty array into a non-empty one")
    return MArray(list(shape), [src[i % len(src)] for i in range(n)])


def transpose(A: MArray, perm: Sequence[int] | None = None) -> MArray:
    """Generalized transpose: i psi (t transpose A) = i[t] psi A.  The shape of
    the result satisfies shape[t[k]] = shape_A[k].  perm=None reverses the axes
    (the ordinary 2-D transpose)."""
    t = list(range(A.dim))[::-1] if perm is None else [int(v) for v in perm]
    if sorted(t) != list(range(A.dim)):
        raise ValueError("not a permutation")
    shape = [0] * A.dim
    for k in range(A.dim):
        shape[t[k]] = A.shape[k]
    out = []
    for i in indices(shape):
        out.append(psi([i[t[k]] for k in range(A.dim)], A))
    return MArray(shape, out)


def reverse(A: MArray) -> MArray:
    """Phi A: reversal along axis 0 (Ch. 2, Def. reverse: the shape is kept
    and <i> psi (Phi A) = <s_0 - i - 1> psi A)."""
    s0 = A.shape[0]
    sub = pi(A.shape[1:])
    out = []
    for i in range(s0):
        base = (s0 - 1 - i) * sub
        out.extend(A.ravel[base:base + sub])
    return MArray(A.shape, out)


def take_array(k: int, A: MArray) -> MArray:
    """k take A along axis 0 (0 <= k <= s_0)."""
    sub = pi(A.shape[1:])
    return MArray([k] + A.shape[1:], A.ravel[:k * sub])


def pct(shape: Sequence[int], j: Sequence[int]) -> Tuple[int, int]:
    """psi Correspondence Theorem (Def. psi_corr): the ravel of j psi xi is the
    contiguous run starting at gamma(j; (tau j) take shape) * pi((tau j) drop
    shape) of length pi((tau j) drop shape).  Returns (start, length)."""
    k = len(j)
    length = pi(drop(k, shape))
    return gamma(take(k, shape), j) * length, length


def hyper(A: MArray) -> MArray:
    """The hyper-cube view <2 2 ... 2> rho^ A of an array with 2^d items."""
    n = len(A.ravel)
    d = n.bit_length() - 1
    if 1 << d != n:
        raise ValueError("not a power of two")
    return reshape([2] * d, A)


def reshape_transpose(A: MArray, r: int, c: int) -> MArray:
    """<r c> rho^ (transpose (<r c> rho^ A))  (Ch. 3, Eq. abstract)."""
    return reshape([r, c], transpose(reshape([r, c], A)))


def gate_transpose_vector(n: int, gated_bits: Sequence[int]) -> List[int]:
    """Transpose vector t of Ch. 6 ("The Algorithm", "From qubits to
    permutation vector") for an n-qubit density matrix viewed as the
    hyper-cube D_h of 2n axes (the n row bits, then the n column bits, each
    most significant first; bits are numbered from the right, axes from the
    left, so bit b of a row index is axis n - 1 - b).  t lists, for the row
    half and then (offset by n) the column half, the axes of the bits that
    are not gated followed by the axes of the gated bits, each group in
    increasing axis order -- the arrangement the paper reaches by its swaps.
    Entry k names the axis of D_h that becomes axis k of the block-diagonal
    view (reading: the swaps build the list of source axes in their new
    order), so the view is (inverse t) transpose D_h in the transpose of
    Ch. 2; the gated bits are then the low bits of both indices and the
    2^q x 2^q blocks on the diagonal hold the gated sub-matrices.  For the
    involutive vector of the xaxb example the two readings coincide."""
    n = int(n)
    gated = sorted({int(b) for b in gated_bits})
    if len(gated) != len(list(gated_bits)) or any(not 0 <= b < n for b in gated):
        raise ValueError("gated bits must be distinct positions in [0, n)")
    gated_axes = [n - 1 - b for b in gated]
    free = [ax for ax in range(n) if ax not in gated_axes]
    half = free + sorted(gated_axes)
    return half + [ax + n for ax in half]


def hypercube_transpose(values: Sequence, t: Sequence[int]) -> List:
    """t transpose (<2 ... 2> rho^ values), ravelled (Ch. 6, "Final Expression
    and Normal Form": i psi (t transpose D_h) = i[t] psi D_h)."""
    A = hyper(MArray([len(values)], list(values)))
    return transpose(A, t).ravel


def hypercube_source_offsets(m: int, t: Sequence[int]) -> List[int]:
    """The generic normal form of Ch. 6: for every index i of t transpose D_h
    (in lexical order), the offset gamma(i[t]; s) of the element it names in
    D_h, s = <2 ... 2> of m axes."""
    s = [2] * int(m)
    out = []
    for i in indices(s):
        out.append(gamma(s, [i[int(t[k])] for k in range(int(m))]))
    return out


def inverse_permutation(t: Sequence[int]) -> List[int]:
    """s with s[t[k]] = k."""
    s = [0] * len(t)
    for k, v in enumerate(t):
        s[int(v)] = k
    return s


def block_diagonal_view(values: Sequence, n: int, gated_bits: Sequence[int]) -> List:
    """The block-diagonal arrangement of Ch. 6 of a 2^n x 2^n matrix given by
    its ravel: (inverse t) transpose D_h, t = gate_transpose_vector."""
    return hypercube_transpose(values, inverse_permutation(gate_transpose_vector(n, gated_bits)))
