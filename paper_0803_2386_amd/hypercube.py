"""PyTorch front end of the hyper-cube kernels (include/moa_hypercube.h).

PyTorch supplies device memory and the stream; the data movement and the
gate arithmetic run in the HIP kernels of libmoa_fft.so (no fallback).

* :func:`hypercube_transpose` -- t transpose of a 2^m-element tensor viewed
  as a hyper-cube of 2-element axes (Ch. 2 / Ch. 6).
* :func:`block_diagonal_transpose_vector` -- the transpose vector that moves
  the gated qubits of an n-qubit density matrix to its diagonal blocks
  (Ch. 6, "The Algorithm").
* :func:`density_gate` -- rho <- G rho G^H in place, by direct indexing.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import capi

_ELEM = {torch.float32: 4, torch.int32: 4, torch.complex64: 8, torch.float64: 8, torch.int64: 8,
         torch.complex128: 16}


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def hypercube_transpose(x: torch.Tensor, t: Sequence[int], out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out[gamma(i)] = x[gamma(i[t])] over the 2^len(t) elements of x
    (contiguous, on the GPU; 4-, 8- or 16-byte elements)."""
    if x.device.type != "cuda" or not x.is_contiguous():
        raise ValueError("x must be a contiguous GPU tensor")
    if x.dtype not in _ELEM:
        raise TypeError(f"unsupported dtype {x.dtype}")
    if x.numel() != 1 << len(t):
        raise ValueError(f"x has {x.numel()} elements, the hyper-cube of {len(t)} axes {1 << len(t)}")
    if out is None:
        out = torch.empty_like(x)
    capi.moa_hypercube_transpose(list(t), _ELEM[x.dtype], x.data_ptr(), out.data_ptr(), _stream(x.device))
    return out


def block_diagonal_transpose_vector(n_qubits: int, gated_bits: Sequence[int]) -> list:
    """The transpose vector (in the sense of hypercube_transpose) that takes
    an n-qubit density matrix to its block-diagonal view: the axes of the
    free bits first, then those of the gated bits, in both halves; the
    paper's printed vector lists, for each axis of the view, the axis of the
    matrix it takes, which is the inverse of this permutation."""
    n = int(n_qubits)
    g = sorted({int(b) for b in gated_bits})
    if len(g) != len(list(gated_bits)) or any(not 0 <= b < n for b in g):
        raise ValueError("gated bits must be distinct positions in [0, n)")
    axes = [n - 1 - b for b in g]
    half = [a for a in range(n) if a not in axes] + sorted(axes)
    printed = half + [a + n for a in half]
    inv = [0] * (2 * n)
    for k, v in enumerate(printed):
        inv[v] = k
    return inv


def density_gate(rho: torch.Tensor, U: torch.Tensor, gated_bits: Sequence[int]) -> torch.Tensor:
    """rho <- G rho G^H in place (rho: 2^n x 2^n complex, U: 2^q x 2^q of the
    same dtype, both on the GPU); returns rho."""
    if rho.device.type != "cuda" or U.device != rho.device:
        raise ValueError("rho and U must be on the same GPU")
    if rho.dtype not in (torch.complex64, torch.complex128) or U.dtype != rho.dtype:
        raise TypeError("rho and U must both be complex64 or complex128")
    N = rho.shape[-1]
    n = N.bit_length() - 1
    if rho.dim() != 2 or rho.shape[0] != N or (1 << n) != N or not rho.is_contiguous():
        raise ValueError("rho must be a contiguous 2^n x 2^n matrix")
    q = len(gated_bits)
    if tuple(U.shape) != (1 << q, 1 << q):
        raise ValueError(f"U must be {1 << q} x {1 << q}")
    Uc = U.contiguous()
    dt = capi.MOA_C128 if rho.dtype == torch.complex128 else capi.MOA_C64
    capi.moa_density_gate(n, list(gated_bits), Uc.data_ptr(), dt, rho.data_ptr(), _stream(rho.device))
    return rho
