"""ctypes binding of include/mppi_ceilings.h (libmppi_ceilings.so): measured
VALU issue rates, the one-wave rollout-chain latency and the graph launch
floor that the benchmark reports beside the datasheet peaks.  Measurement
only; not part of the MPPI path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmppi_ceilings.so")

EXPORTS = {
    "mppi_ceiling_valu": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mppi_ceiling_chain": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(C.c_double)]),
    "mppi_ceiling_graph": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                     C.POINTER(C.c_double)]),
    "mppi_ceiling_last_error": (C.c_char_p, []),
}
VALU_MODES = {"fma": 0, "fma+exp": 1, "exp": 2, "mad_u64": 3, "int_xor_add": 4}

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2409_07563_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise RuntimeError(lib().mppi_ceiling_last_error().decode())


def valu(mode: str, blocks: int = 8192, iters: int = 4096, reps: int = 5, stream=None):
    """(lane-instructions per second, us per launch) of an independent-chain
    loop of one VALU instruction kind (VALU_MODES)."""
    import torch
    s = stream or torch.cuda.current_stream()
    sink = torch.empty(blocks * 256, device="cuda")
    us, ops = C.c_double(), C.c_double()
    _check(lib().mppi_ceiling_valu(VALU_MODES[mode], blocks, iters, reps, sink.data_ptr(),
                                   s.cuda_stream, C.byref(us), C.byref(ops)))
    return ops.value / (us.value * 1e-6), us.value


def chain(T: int, reps: int = 50, stream=None) -> float:
    """us per launch of one wave's dependent T-step double-integrator chain."""
    import torch
    s = stream or torch.cuda.current_stream()
    eps = torch.randn(128 * T, device="cuda") * 0.5
    out = torch.empty(64, device="cuda")
    us = C.c_double()
    _check(lib().mppi_ceiling_chain(T, reps, eps.data_ptr(), out.data_ptr(), s.cuda_stream,
                                    C.byref(us)))
    return us.value


def graph(kernels: int = 3, iterations: int = 1, reps: int = 200, stream=None) -> float:
    """us per replay of a graph of `iterations` x `kernels` empty kernels."""
    import torch
    s = stream or torch.cuda.Stream()
    us = C.c_double()
    _check(lib().mppi_ceiling_graph(kernels, iterations, reps, s.cuda_stream, C.byref(us)))
    return us.value
