"""MI355X (gfx950) dimension-lifted radix-2 FFT after Mullin & Raynolds'
Conformal Computing monograph (MoA / psi-calculus, Ch. 3-5).

The product is the C-ABI library ``libmoa_fft.so`` (include/moa_fft.h) with
hand-written HIP kernels; ``capi`` binds it with ctypes and ``fft`` adds the
PyTorch front end (plans, autograd).  Importing this package does not load
the library; the first call that needs it does, and fails loudly if it is
not built.
"""
from . import capi  # noqa: F401

__all__ = ["capi", "fft", "inputs", "tune"]


def __getattr__(name):
    if name in ("fft", "inputs", "tune"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
