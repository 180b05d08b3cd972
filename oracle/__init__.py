"""FP64 CPU oracle for the MoA dimension-lifted radix-2 FFT.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
path (``paper_0803_2386_amd``) never imports, links or calls it, and this
package never imports the product path: the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc, no fast-math);
this module is argument marshalling over ctypes.  ``moa.py`` holds the
index-algebra oracle (psi, gamma, reshape, transpose, PCT) in plain Python.

Functions (all on numpy ``complex128`` arrays, sign -1 = forward):

* :func:`fft` -- the result oracle: the DFT by the recursive even/odd split of
  its definition (Ch. 3, "Traditional FFT Algorithm", problem statement).
* :func:`dft_brute` -- O(n^2) definition, long double (pins :func:`fft`).
* :func:`fft_lifted` -- the cache-optimized method with reshape-transposes,
  transformed weights and the final transpose (Ch. 3).
* :func:`trans_rshp`, :func:`final_trans`, :func:`bitrev` -- its index moves.
* :func:`lifted_exponents` -- the transformed-weight exponents
  sigma + j c^l ("General Weight Sub-Matrices").
* :func:`fft_batch`, :func:`fft_packed` -- contiguous and uneven batches.
* :func:`fftn` -- the multi-dimensional DFT, the 1-D oracle along each axis.
* :func:`weighted_power_loss` -- L = sum_k w_k |F x|_k^2 and its gradient.

``density.py`` holds the density-matrix gating oracle of Ch. 6 (numpy,
complex128): the gate by its definition G rho G^H and by the block-diagonal
route through the hyper-cube transpose of ``moa.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        lib.moa_or_root.argtypes = [I64, I64, I, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        lib.moa_or_root.restype = None
        lib.moa_or_bitrev.argtypes = [P, I64]
        lib.moa_or_bitrev.restype = None
        lib.moa_or_fft.argtypes = [P, I64, I]
        lib.moa_or_fft.restype = I
        lib.moa_or_fft_batch.argtypes = [P, I64, I64, I, I]
        lib.moa_or_fft_batch.restype = I
        lib.moa_or_fft_packed.argtypes = [P, P, I64, I, I]
        lib.moa_or_fft_packed.restype = I
        lib.moa_or_dft_brute.argtypes = [P, P, I64, I]
        lib.moa_or_dft_brute.restype = I
        lib.moa_or_lift_levels.argtypes = [I64, I64, ctypes.POINTER(I), ctypes.POINTER(I)]
        lib.moa_or_lift_levels.restype = None
        lib.moa_or_trans_rshp.argtypes = [P, P, I64, I64]
        lib.moa_or_trans_rshp.restype = I
        lib.moa_or_final_trans.argtypes = [P, P, I64, I, I64]
        lib.moa_or_final_trans.restype = I
        lib.moa_or_lifted_exponents.argtypes = [I64, I64, I, I, P, ctypes.POINTER(I64)]
        lib.moa_or_lifted_exponents.restype = I
        lib.moa_or_fft_lifted.argtypes = [P, I64, I64, I, I]
        lib.moa_or_fft_lifted.restype = I
        lib.moa_or_weighted_power_loss.argtypes = [P, P, I64, I64, P, I]
        lib.moa_or_weighted_power_loss.restype = ctypes.c_double
        lib.moa_or_max_threads.argtypes = []
        lib.moa_or_max_threads.restype = I
        _lib = lib
    return _lib


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid arguments (rc={rc})")


def max_threads() -> int:
    return int(_load().moa_or_max_threads())


def root(e: int, L: int, sign: int = -1) -> complex:
    """omega_L^e = exp(sign 2 pi i e / L) from the exact integer exponent."""
    re, im = ctypes.c_double(), ctypes.c_double()
    _load().moa_or_root(int(e), int(L), int(sign), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def bitrev(x) -> np.ndarray:
    a = _c128(x).copy()
    _load().moa_or_bitrev(_ptr(a), a.size)
    return a


def fft(x, sign: int = -1) -> np.ndarray:
    """Result oracle on the last axis (any leading batch shape)."""
    a = _c128(x).copy()
    n = a.shape[-1]
    batch = a.size // n if n else 0
    _check(_load().moa_or_fft_batch(_ptr(a), n, batch, int(sign), 1), "fft")
    return a


def fft_batch(x, sign: int = -1, threads: int = 1) -> np.ndarray:
    a = _c128(x).copy()
    n = a.shape[-1]
    _check(_load().moa_or_fft_batch(_ptr(a), n, a.size // n, int(sign), int(threads)), "fft_batch")
    return a


def fft_packed(x, sizes, sign: int = -1, threads: int = 1) -> np.ndarray:
    a = _c128(x).copy()
    s = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
    if int(s.sum()) != a.size:
        raise ValueError("sizes do not sum to the buffer length")
    _check(_load().moa_or_fft_packed(_ptr(a), _ptr(s), s.size, int(sign), int(threads)), "fft_packed")
    return a


def fft_packed_inplace(a: np.ndarray, sizes, sign: int = -1, threads: int = 1) -> np.ndarray:
    """fft_packed on a caller's complex128 C-contiguous buffer, overwritten
    with the result (no copy: for timing the arithmetic alone)."""
    if a.dtype != np.complex128 or not a.flags.c_contiguous or not a.flags.writeable:
        raise ValueError("fft_packed_inplace needs a writeable C-contiguous complex128 array")
    s = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
    if int(s.sum()) != a.size:
        raise ValueError("sizes do not sum to the buffer length")
    _check(_load().moa_or_fft_packed(_ptr(a), _ptr(s), s.size, int(sign), int(threads)), "fft_packed")
    return a


def fftn(x, rank: int, sign: int = -1) -> np.ndarray:
    """DFT over the last `rank` axes: X[k] = sum_j x[j] exp(sign 2 pi i sum_a
    j_a k_a / n_a).  The exponential factorises over the axes, so the
    transform is the 1-D result oracle along each axis in turn -- the
    multi-dimensional FFT built from the one-dimensional one (Ch. 1,
    "Conclusions for the General Radix Approach", footnote)."""
    a = _c128(x).copy()
    if rank < 1 or rank > a.ndim:
        raise ValueError("rank must be between 1 and x.ndim")
    for ax in range(a.ndim - rank, a.ndim):
        moved = np.ascontiguousarray(np.moveaxis(a, ax, -1))
        a = np.moveaxis(fft(moved, sign), -1, ax)
    return np.ascontiguousarray(a)


def dft_brute(x, sign: int = -1) -> np.ndarray:
    a = _c128(x)
    y = np.empty_like(a)
    _check(_load().moa_or_dft_brute(_ptr(a), _ptr(y), a.size, int(sign)), "dft_brute")
    return y


def lift_levels(n: int, c: int) -> tuple[int, int]:
    lm, pm = ctypes.c_int(), ctypes.c_int()
    _load().moa_or_lift_levels(int(n), int(c), ctypes.byref(lm), ctypes.byref(pm))
    return lm.value, pm.value


def trans_rshp(x, c: int) -> np.ndarray:
    a = _c128(x).copy()
    t = np.empty_like(a)
    _check(_load().moa_or_trans_rshp(_ptr(a), _ptr(t), a.size, int(c)), "trans_rshp")
    return a


def final_trans(x, l_max: int, c: int) -> np.ndarray:
    a = _c128(x).copy()
    t = np.empty_like(a)
    _check(_load().moa_or_final_trans(_ptr(a), _ptr(t), a.size, int(l_max), int(c)), "final_trans")
    return a


def lifted_exponents(n: int, c: int, l: int, p: int) -> tuple[np.ndarray, int]:
    e = np.empty(n // 2, dtype=np.int64)
    L = ctypes.c_int64()
    _check(_load().moa_or_lifted_exponents(int(n), int(c), int(l), int(p), _ptr(e), ctypes.byref(L)),
           "lifted_exponents")
    return e, L.value


def fft_lifted(x, c: int, sign: int = -1, stop_level: int = -1) -> np.ndarray:
    a = _c128(x).copy()
    _check(_load().moa_or_fft_lifted(_ptr(a), a.size, int(c), int(sign), int(stop_level)), "fft_lifted")
    return a


def weighted_power_loss(x, w, threads: int = 1, want_grad: bool = True):
    """Return (L, grad) for L = sum_b sum_k w_k |(F x_b)_k|^2; grad = 2 F^H(w . F x)."""
    a = _c128(x)
    n = a.shape[-1]
    wv = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    if wv.size != n:
        raise ValueError("w must have the transform length")
    g = np.empty_like(a) if want_grad else None
    loss = _load().moa_or_weighted_power_loss(_ptr(a), _ptr(wv), n, a.size // n,
                                              _ptr(g) if g is not None else None, int(threads))
    return float(loss), g
