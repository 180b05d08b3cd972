"""PyTorch front end of the gfx950 dimension-lifted FFT.

PyTorch supplies device memory, streams and autograd only; every transform
runs in the HIP kernels of libmoa_fft.so through the C ABI (``capi``).  If
the library is missing or the tensor is not on a GPU, the calls raise --
there is no CPU or library fallback.

* :class:`Plan` -- ``batch`` contiguous transforms of length n with a lift.
* :class:`BatchedPlan` -- an uneven batch of power-of-two lengths, packed.
* :class:`NDPlan` -- ``batch`` contiguous multi-dimensional transforms.
* :func:`fft` / :func:`adjoint` -- cached-plan convenience calls on the last
  axis (unnormalised; ``adjoint(fft(x)) == n * x``).
* :class:`FFTFunction` -- autograd: backward of the forward transform is the
  adjoint transform of the incoming gradient.
"""
from __future__ import annotations

import json
import threading
from typing import Optional, Sequence

import torch

from . import capi

_PREC = {"native": capi.MOA_FFT_PREC_NATIVE, "split_bf16": capi.MOA_FFT_PREC_SPLIT_BF16,
         "split_fp16": capi.MOA_FFT_PREC_SPLIT_FP16}


def _dtype_code(dtype: torch.dtype) -> int:
    if dtype == torch.complex64:
        return capi.MOA_C64
    if dtype == torch.complex128:
        return capi.MOA_C128
    raise TypeError(f"unsupported dtype {dtype}: complex64 or complex128 required")


def _check_tensor(t: torch.Tensor, dtype: torch.dtype, numel: int, device: torch.device, what: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{what} must be on the GPU (got {t.device})")
    if t.device != device:
        raise ValueError(f"{what} is on {t.device}, the plan on {device}")
    if t.dtype != dtype:
        raise TypeError(f"{what} has dtype {t.dtype}, the plan {dtype}")
    if t.numel() != numel:
        raise ValueError(f"{what} has {t.numel()} elements, the plan needs {numel}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


class _PlanBase:
    numel: int
    dtype: torch.dtype
    device: torch.device

    def __init__(self):
        self._h = None

    def _exec(self, direction: int, x: torch.Tensor, out: Optional[torch.Tensor]) -> torch.Tensor:
        if self._h is None:
            raise RuntimeError("plan is closed")
        _check_tensor(x, self.dtype, self.numel, self.device, "input")
        if out is None:
            out = torch.empty_like(x)
        else:
            _check_tensor(out, self.dtype, self.numel, self.device, "output")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        capi.moa_fft_exec(self._h, direction, x.data_ptr(), out.data_ptr(), stream)
        return out

    def forward(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """X_k = sum_j x_j exp(-2 pi i jk/n), unnormalised; in == out allowed."""
        return self._exec(capi.MOA_FFT_FORWARD, x, out)

    def adjoint(self, y: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Conjugate transform Y_j = sum_k y_k exp(+2 pi i jk/n), unnormalised."""
        return self._exec(capi.MOA_FFT_ADJOINT, y, out)

    def run_level(self, level: int, x: torch.Tensor, out: torch.Tensor, direction: int = 0) -> None:
        """Launch only level `level` of the lift (see moa_fft_exec_level)."""
        _check_tensor(x, self.dtype, self.numel, self.device, "input")
        _check_tensor(out, self.dtype, self.numel, self.device, "output")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        capi.moa_fft_exec_level(self._h, direction, level, x.data_ptr(), out.data_ptr(), stream)

    @property
    def num_levels(self) -> int:
        return capi.moa_fft_num_levels(self._h)

    def describe(self) -> dict:
        return json.loads(capi.moa_fft_describe(self._h))

    @property
    def workspace_bytes(self) -> int:
        return capi.moa_fft_workspace_size(self._h)

    def close(self) -> None:
        if self._h is not None:
            capi.moa_fft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan(_PlanBase):
    """``batch`` contiguous transforms of length n through the lift ``lift``
    (outermost factor first, innermost block c last; None = default)."""

    def __init__(self, n: int, batch: int = 1, lift: Optional[Sequence[int]] = None,
                 dtype: torch.dtype = torch.complex64, prec: str = "native", graph: bool = False,
                 tuning: Optional[dict] = None, device: Optional[torch.device] = None,
                 host_only: bool = False):
        super().__init__()
        if prec not in _PREC:
            raise ValueError(f"prec must be one of {sorted(_PREC)}")
        self.n, self.batch, self.dtype, self.prec = int(n), int(batch), dtype, prec
        self.numel = self.n * self.batch
        if host_only:
            self.device = torch.device("cpu")
        else:
            self.device = torch.device(device) if device is not None else torch.device(
                "cuda", torch.cuda.current_device())
        flags = (capi.MOA_FFT_FLAG_GRAPH if graph else 0) | (capi.MOA_FFT_FLAG_HOST_ONLY if host_only else 0)
        with torch.cuda.device(self.device) if not host_only else _nullctx():
            self._h = capi.moa_fft_plan(self.n, self.batch, lift, _dtype_code(dtype), _PREC[prec], flags, tuning)


class BatchedPlan(_PlanBase):
    """Uneven batch: transform i has length sizes[i] (a power of two) and the
    transforms are packed one after the other.  ``per_size`` runs one plain
    launch per distinct size instead of the single fused launch."""

    def __init__(self, sizes: Sequence[int], dtype: torch.dtype = torch.complex64, per_size: bool = False,
                 graph: bool = False, tuning: Optional[dict] = None, device: Optional[torch.device] = None,
                 host_only: bool = False):
        super().__init__()
        self.sizes = [int(s) for s in sizes]
        self.dtype = dtype
        self.numel = sum(self.sizes)
        if host_only:
            self.device = torch.device("cpu")
        else:
            self.device = torch.device(device) if device is not None else torch.device(
                "cuda", torch.cuda.current_device())
        flags = ((capi.MOA_FFT_FLAG_PER_SIZE if per_size else 0) | (capi.MOA_FFT_FLAG_GRAPH if graph else 0)
                 | (capi.MOA_FFT_FLAG_HOST_ONLY if host_only else 0))
        with torch.cuda.device(self.device) if not host_only else _nullctx():
            self._h = capi.moa_fft_plan_batched(self.sizes, _dtype_code(dtype), flags, tuning)


class NDPlan(_PlanBase):
    """``batch`` contiguous multi-dimensional transforms of shape ``dims``
    (row-major, the last axis contiguous): one launch per axis of extent
    > 1, in -> out first, then in place in out."""

    def __init__(self, dims: Sequence[int], batch: int = 1, dtype: torch.dtype = torch.complex64,
                 prec: str = "native", graph: bool = False, tuning: Optional[dict] = None,
                 device: Optional[torch.device] = None, host_only: bool = False):
        super().__init__()
        if prec not in _PREC:
            raise ValueError(f"prec must be one of {sorted(_PREC)}")
        self.dims = [int(d) for d in dims]
        self.batch, self.dtype, self.prec = int(batch), dtype, prec
        n = 1
        for d in self.dims:
            n *= d
        self.n = n
        self.numel = n * self.batch
        if host_only:
            self.device = torch.device("cpu")
        else:
            self.device = torch.device(device) if device is not None else torch.device(
                "cuda", torch.cuda.current_device())
        flags = (capi.MOA_FFT_FLAG_GRAPH if graph else 0) | (capi.MOA_FFT_FLAG_HOST_ONLY if host_only else 0)
        with torch.cuda.device(self.device) if not host_only else _nullctx():
            self._h = capi.moa_fft_plan_nd(self.dims, self.batch, _dtype_code(dtype), _PREC[prec], flags, tuning)


class _nullctx:
    def __enter__(self):
        return None

    def __exit__(self, *a):
        return False


# Plans of the convenience calls, one per (shape, dtype, precision, device,
# stream): a multi-level plan's workspace is shared by its executions, which
# the library requires to be serialised on one stream, so calls from
# different streams get different plans.  An evicted plan is only dropped
# from the cache (its memory goes when the last reference does); a plan used
# while its stream is being captured into a graph is kept for the life of
# the process, since the graph keeps its workspace and tables.
_cache: dict = {}
_pinned: list = []
_cache_lock = threading.Lock()


def _cached(key, make):
    stream = torch.cuda.current_stream(key[-1])
    key = key + (stream.cuda_stream,)
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            if len(_cache) >= 32:
                _cache.pop(next(iter(_cache)))
            p = make()
            _cache[key] = p
        if torch.cuda.is_current_stream_capturing() and not any(q is p for q in _pinned):
            _pinned.append(p)
        return p


def _cached_plan(n: int, batch: int, lift, dtype, prec, device) -> Plan:
    return _cached(("1d", n, batch, tuple(lift) if lift else None, dtype, prec, device),
                   lambda: Plan(n, batch, lift, dtype, prec, device=device))


def _apply(x: torch.Tensor, direction: int, lift, prec) -> torch.Tensor:
    if x.dim() == 0:
        raise ValueError("need at least one dimension")
    n = x.shape[-1]
    xc = x.contiguous()
    batch = xc.numel() // n if n else 0
    p = _cached_plan(n, batch, lift, xc.dtype, prec, xc.device)
    return p._exec(direction, xc, None)


def _apply_nd(x: torch.Tensor, direction: int, ndim: int, prec) -> torch.Tensor:
    if ndim < 1 or ndim > x.dim():
        raise ValueError("ndim must be between 1 and x.dim()")
    dims = [int(d) for d in x.shape[x.dim() - ndim:]]
    xc = x.contiguous()
    n = 1
    for d in dims:
        n *= d
    batch = xc.numel() // n if n else 0
    p = _cached(("nd", tuple(dims), batch, xc.dtype, prec, xc.device),
                lambda: NDPlan(dims, batch, xc.dtype, prec, device=xc.device))
    return p._exec(direction, xc, None)


def fftn(x: torch.Tensor, ndim: int, prec: str = "native") -> torch.Tensor:
    """Forward transform over the last ``ndim`` axes (unnormalised)."""
    return _apply_nd(x, capi.MOA_FFT_FORWARD, ndim, prec)


def adjointn(y: torch.Tensor, ndim: int, prec: str = "native") -> torch.Tensor:
    """Adjoint (conjugate, unnormalised) transform over the last ``ndim`` axes."""
    return _apply_nd(y, capi.MOA_FFT_ADJOINT, ndim, prec)


def fft(x: torch.Tensor, lift: Optional[Sequence[int]] = None, prec: str = "native") -> torch.Tensor:
    """Forward transform along the last axis (unnormalised)."""
    return _apply(x, capi.MOA_FFT_FORWARD, lift, prec)


def adjoint(y: torch.Tensor, lift: Optional[Sequence[int]] = None, prec: str = "native") -> torch.Tensor:
    """Adjoint (conjugate, unnormalised) transform along the last axis."""
    return _apply(y, capi.MOA_FFT_ADJOINT, lift, prec)


class FFTFunction(torch.autograd.Function):
    """y = F x on the last axis; for a real loss L, torch's gradient
    convention gives dL/dx = F^H (dL/dy), computed by the adjoint kernel."""

    @staticmethod
    def forward(ctx, x, lift=None, prec="native"):
        ctx.lift, ctx.prec = lift, prec
        return fft(x, lift, prec)

    @staticmethod
    def backward(ctx, g):
        return adjoint(g.contiguous(), ctx.lift, ctx.prec), None, None


def fft_autograd(x: torch.Tensor, lift=None, prec: str = "native") -> torch.Tensor:
    return FFTFunction.apply(x, lift, prec)


class FFTNFunction(torch.autograd.Function):
    """y = F x over the last ``ndim`` axes; backward is the adjoint transform
    of the incoming gradient over the same axes."""

    @staticmethod
    def forward(ctx, x, ndim, prec="native"):
        ctx.ndim, ctx.prec = ndim, prec
        return fftn(x, ndim, prec)

    @staticmethod
    def backward(ctx, g):
        return adjointn(g.contiguous(), ctx.ndim, ctx.prec), None, None
