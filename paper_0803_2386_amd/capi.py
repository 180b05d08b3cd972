"""ctypes binding of the C ABI declared in include/moa_fft.h.

Argument marshalling only: every function here forwards to the function of
the same name in libmoa_fft.so.  The library must have been built
(``paper_0803_2386_amd.build.build()``); if it is missing, loading raises --
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmoa_fft.so")

MOA_FFT_FORWARD = 0
MOA_FFT_ADJOINT = 1
MOA_C64 = 0
MOA_C128 = 1
MOA_FFT_PREC_NATIVE = 0
MOA_FFT_PREC_SPLIT_BF16 = 1
MOA_FFT_PREC_SPLIT_FP16 = 2

MOA_OK = 0
MOA_ERR_NULL = 1
MOA_ERR_SIZE = 2
MOA_ERR_LIFT = 3
MOA_ERR_BATCH = 4
MOA_ERR_DTYPE = 5
MOA_ERR_ALLOC = 6
MOA_ERR_HIP = 7
MOA_ERR_STATE = 8
MOA_ERR_ARG = 9
MOA_ERR_TUNING = 10
MOA_ERR_SCRATCH = 11

MOA_FFT_FLAG_HOST_ONLY = 0x1
MOA_FFT_FLAG_PER_SIZE = 0x2
MOA_FFT_FLAG_GRAPH = 0x4
MOA_FFT_FLAG_NO_WORKSPACE = 0x8

MOA_FFT_SCRATCH_BYTES = 64 << 20

EXPORTED = [
    "moa_fft_plan", "moa_fft_plan_tuned", "moa_fft_plan_nd", "moa_fft_plan_nd_tuned",
    "moa_fft_plan_batched", "moa_fft_plan_batched_tuned",
    "moa_fft_exec", "moa_fft_exec_noalloc", "moa_fft_exec_level", "moa_fft_num_levels", "moa_fft_workspace_size", "moa_fft_describe", "moa_fft_describe_size",
    "moa_fft_destroy", "moa_fft_status_string", "moa_fft_max_block",
    "moa_hypercube_transpose", "moa_density_gate",
]


class moa_fft_tuning_t(ctypes.Structure):
    _fields_ = [("cols_per_block", ctypes.c_int32 * 8),
                ("persistent_blocks", ctypes.c_int32),
                ("stream", ctypes.c_int32),
                ("lg_radix", ctypes.c_uint32),
                ("batch_task_lg", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class MoaError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {moa_fft_status_string(status)}")


_lib = None


def load() -> ctypes.CDLL:
    """Load libmoa_fft.so (raises FileNotFoundError if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import paper_0803_2386_amd.build as b; b.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    I64 = ctypes.c_int64
    I32 = ctypes.c_int32
    U32 = ctypes.c_uint32
    E = ctypes.c_int
    TP = ctypes.POINTER(moa_fft_tuning_t)
    I64P = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "moa_fft_plan": ([PP, I64, I64, I64P, I32, E, E, U32], E),
        "moa_fft_plan_tuned": ([PP, I64, I64, I64P, I32, E, E, U32, TP], E),
        "moa_fft_plan_nd": ([PP, I32, I64P, I64, E, E, U32], E),
        "moa_fft_plan_nd_tuned": ([PP, I32, I64P, I64, E, E, U32, TP], E),
        "moa_fft_plan_batched": ([PP, I64P, I64, E, U32], E),
        "moa_fft_plan_batched_tuned": ([PP, I64P, I64, E, U32, TP], E),
        "moa_fft_exec": ([P, E, P, P, P], E),
        "moa_fft_exec_noalloc": ([P, E, P, P, P], E),
        "moa_fft_exec_level": ([P, E, I32, P, P, P], E),
        "moa_fft_num_levels": ([P, ctypes.POINTER(I32)], E),
        "moa_fft_workspace_size": ([P, ctypes.POINTER(ctypes.c_size_t)], E),
        "moa_fft_describe": ([P, ctypes.c_char_p, ctypes.c_size_t], E),
        "moa_fft_describe_size": ([P, ctypes.POINTER(ctypes.c_size_t)], E),
        "moa_fft_destroy": ([P], E),
        "moa_fft_status_string": ([E], ctypes.c_char_p),
        "moa_fft_max_block": ([E], I64),
        "moa_hypercube_transpose": ([I32, ctypes.POINTER(I32), I32, P, P, P], E),
        "moa_density_gate": ([I32, I32, ctypes.POINTER(I32), P, E, P, P], E),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _i64_array(vals):
    if vals is None:
        return None, 0
    vals = [int(v) for v in vals]
    arr = (ctypes.c_int64 * len(vals))(*vals)
    return arr, len(vals)


def _tuning(tuning):
    if tuning is None:
        return None
    t = moa_fft_tuning_t()
    for i, v in enumerate(tuning.get("cols_per_block", [])[:8]):
        t.cols_per_block[i] = int(v)
    t.persistent_blocks = int(tuning.get("persistent_blocks", 0))
    t.stream = int(tuning.get("stream", 0))
    # lg_radix: a list, one log2 radix per level (0 = default), packed 4 bits a level
    packed = 0
    for i, v in enumerate(tuning.get("lg_radix", [])[:8]):
        packed |= (int(v) & 0xF) << (4 * i)
    t.lg_radix = packed
    t.batch_task_lg = int(tuning.get("batch_task_lg", 0))
    return ctypes.pointer(t)


def moa_fft_status_string(status: int) -> str:
    return load().moa_fft_status_string(int(status)).decode()


def moa_fft_max_block(dtype: int) -> int:
    return int(load().moa_fft_max_block(int(dtype)))


def moa_fft_plan(n, batch=1, lift_shape=None, dtype=MOA_C64, prec=MOA_FFT_PREC_NATIVE, flags=0,
                 tuning=None) -> ctypes.c_void_p:
    """Returns the plan handle; raises MoaError with the status on failure."""
    lib = load()
    h = ctypes.c_void_p()
    arr, rank = _i64_array(lift_shape)
    if tuning is None:
        st = lib.moa_fft_plan(ctypes.byref(h), int(n), int(batch), arr, rank, int(dtype), int(prec), int(flags))
    else:
        st = lib.moa_fft_plan_tuned(ctypes.byref(h), int(n), int(batch), arr, rank, int(dtype), int(prec),
                                    int(flags), _tuning(tuning))
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_plan")
    return h


def moa_fft_plan_nd(dims, batch=1, dtype=MOA_C64, prec=MOA_FFT_PREC_NATIVE, flags=0,
                    tuning=None) -> ctypes.c_void_p:
    """Multi-dimensional plan of shape dims (row-major); raises MoaError."""
    lib = load()
    h = ctypes.c_void_p()
    arr, rank = _i64_array(dims)
    if tuning is None:
        st = lib.moa_fft_plan_nd(ctypes.byref(h), rank, arr, int(batch), int(dtype), int(prec), int(flags))
    else:
        st = lib.moa_fft_plan_nd_tuned(ctypes.byref(h), rank, arr, int(batch), int(dtype), int(prec),
                                       int(flags), _tuning(tuning))
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_plan_nd")
    return h


def moa_fft_plan_batched(sizes, dtype=MOA_C64, flags=0, tuning=None) -> ctypes.c_void_p:
    lib = load()
    h = ctypes.c_void_p()
    arr, count = _i64_array(sizes)
    if tuning is None:
        st = lib.moa_fft_plan_batched(ctypes.byref(h), arr, count, int(dtype), int(flags))
    else:
        st = lib.moa_fft_plan_batched_tuned(ctypes.byref(h), arr, count, int(dtype), int(flags), _tuning(tuning))
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_plan_batched")
    return h


def moa_fft_exec(plan, direction, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    st = load().moa_fft_exec(plan, int(direction), ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                             ctypes.c_void_p(stream))
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_exec")


def moa_fft_exec_noalloc(plan, direction, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    st = load().moa_fft_exec_noalloc(plan, int(direction), ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                                     ctypes.c_void_p(stream))
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_exec_noalloc")


def moa_fft_exec_level(plan, direction, level: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    st = load().moa_fft_exec_level(plan, int(direction), int(level), ctypes.c_void_p(in_ptr),
                                   ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream))
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_exec_level")


def moa_fft_num_levels(plan) -> int:
    v = ctypes.c_int32()
    st = load().moa_fft_num_levels(plan, ctypes.byref(v))
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_num_levels")
    return int(v.value)


def moa_fft_workspace_size(plan) -> int:
    v = ctypes.c_size_t()
    st = load().moa_fft_workspace_size(plan, ctypes.byref(v))
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_workspace_size")
    return int(v.value)


def moa_fft_describe(plan) -> str:
    lib = load()
    size = ctypes.c_size_t()
    st = lib.moa_fft_describe_size(plan, ctypes.byref(size))
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_describe_size")
    buf = ctypes.create_string_buffer(int(size.value))
    st = lib.moa_fft_describe(plan, buf, size.value)
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_describe")
    return buf.value.decode()


def moa_fft_destroy(plan) -> None:
    st = load().moa_fft_destroy(plan)
    if st != MOA_OK:
        raise MoaError(st, "moa_fft_destroy")


def _i32_array(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int32 * max(1, len(vals)))(*vals), len(vals)


def moa_hypercube_transpose(t, elem_bytes: int, in_ptr: int, out_ptr: int, stream: int = 0, rank=None) -> None:
    """out = t transpose (<2 ... 2> reshape in) on 2^len(t) elements (see
    include/moa_hypercube.h); rank defaults to len(t)."""
    arr, m = _i32_array(t)
    st = load().moa_hypercube_transpose(int(m if rank is None else rank), arr, int(elem_bytes),
                                        ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream))
    if st != MOA_OK:
        raise MoaError(st, "moa_hypercube_transpose")


def moa_density_gate(n_qubits: int, gated_bits, gate_ptr: int, dtype: int, rho_ptr: int, stream: int = 0,
                     q=None) -> None:
    """rho <- G rho G^H in place for the gate U (device, 2^q x 2^q) on the
    qubits gated_bits (see include/moa_hypercube.h); q defaults to
    len(gated_bits)."""
    arr, k = _i32_array(gated_bits)
    st = load().moa_density_gate(int(n_qubits), int(k if q is None else q), arr, ctypes.c_void_p(gate_ptr),
                                 int(dtype), ctypes.c_void_p(rho_ptr), ctypes.c_void_p(stream))
    if st != MOA_OK:
        raise MoaError(st, "moa_density_gate")
