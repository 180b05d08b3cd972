"""Density-matrix gating oracle (Ch. 6, "Quantum Evolution: the Density
Matrix", "The Algorithm").

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in
complex128.

A gate of q qubits acts on an n-qubit density matrix rho (2^n x 2^n) as the
unitary transformation rho -> G rho G^H, where G is the gate matrix U
(2^q x 2^q) on the gated qubits and the identity on the others:
    G[i, j] = U[g(i), g(j)] if i and j agree on every bit that is not gated,
              0 otherwise,
g(i) packing the gated bits of i, the highest gated bit as the most
significant bit of U's index (the order in which the gated bits sit inside
the diagonal blocks of the paper's block-diagonal arrangement).  Reading:
the paper multiplies "on the right and left by a unitary matrix and its
inverse"; the library applies G rho G^H, the usual evolution, which is that
statement for the gate U^H.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import moa


def gated_index(i: int, gated_bits: Sequence[int]) -> int:
    """g(i): the gated bits of i packed, highest gated bit first."""
    out = 0
    for b in sorted(gated_bits, reverse=True):
        out = (out << 1) | ((int(i) >> int(b)) & 1)
    return out


def gate_matrix(n: int, U, gated_bits: Sequence[int]) -> np.ndarray:
    """The 2^n x 2^n matrix G of the definition above, element by element."""
    N = 1 << int(n)
    U = np.asarray(U, np.complex128)
    mask = 0
    for b in gated_bits:
        mask |= 1 << int(b)
    G = np.zeros((N, N), np.complex128)
    for i in range(N):
        for j in range(N):
            if (i & ~mask) == (j & ~mask):
                G[i, j] = U[gated_index(i, gated_bits), gated_index(j, gated_bits)]
    return G


def apply_gate(rho, U, gated_bits: Sequence[int]) -> np.ndarray:
    """rho -> G rho G^H with G from gate_matrix (n <= 9: a dense product)."""
    rho = np.asarray(rho, np.complex128)
    n = int(rho.shape[-1]).bit_length() - 1
    G = gate_matrix(n, U, gated_bits)
    return G @ rho @ G.conj().T


def apply_gate_blocks(rho, U, gated_bits: Sequence[int]) -> np.ndarray:
    """The same transformation by the route of Ch. 6: view rho through the
    block-diagonal arrangement (moa.block_diagonal_view: the gated bits become
    the low bits of both indices), transform every 2^q x 2^q block B of that
    view as U B U^H, and put the elements back where they came from.  Used
    to pin apply_gate and as the reference for large n (numpy's fancy
    indexing with the offsets of the normal form, no dense G)."""
    rho = np.asarray(rho, np.complex128)
    N = rho.shape[-1]
    n = N.bit_length() - 1
    q = len(gated_bits)
    t = moa.inverse_permutation(moa.gate_transpose_vector(n, gated_bits))
    src = np.asarray(moa_source_offsets_fast(2 * n, t))
    view = rho.reshape(-1)[src].reshape(N >> q, 1 << q, N >> q, 1 << q)
    U = np.asarray(U, np.complex128)
    out_view = np.einsum("ak,rksl,bl->rasb", U, view, U.conj(), optimize=True)
    out = np.empty(N * N, np.complex128)
    out[src] = out_view.reshape(-1)
    return out.reshape(N, N)


def moa_source_offsets_fast(m: int, t: Sequence[int]) -> np.ndarray:
    """gamma(i[t]; <2 ... 2>) for every index i of t transpose D_h in lexical
    order, vectorised: axis k of D_h (bit m-1-k of its offset) takes the value
    of axis t_k of the result (bit m-1-t_k of the result's offset).  Pinned
    against moa.hypercube_source_offsets, the definition written out."""
    m = int(m)
    i = np.arange(1 << m, dtype=np.int64)
    src = np.zeros_like(i)
    for k in range(m):
        bit = (i >> (m - 1 - int(t[k]))) & 1
        src |= bit << (m - 1 - k)
    return src


def hypercube_source_of(m: int, t, offsets) -> np.ndarray:
    """gamma(i[t]; <2 ... 2>) for the result offsets given (any subset of the
    2^m), by the same bit rule as moa_source_offsets_fast: for large arrays
    whose full offset table would not fit the host."""
    m = int(m)
    i = np.asarray(offsets, dtype=np.int64)
    src = np.zeros_like(i)
    for k in range(m):
        src |= ((i >> (m - 1 - int(t[k]))) & 1) << (m - 1 - k)
    return src
