"""ctypes declarations of include/mppi.h and the loader of libmppi.so.

Argument marshalling only: every step of the MPPI iteration runs in the HIP
kernels of libmppi.so.  The library is built in-tree (see build.py); when it
is missing the import fails loudly — there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmppi.so")

ABI_VERSION = 4
MAX_CONTROL = 8

MPPI_OK, MPPI_EINVAL, MPPI_ENOMEM, MPPI_EDEVICE, MPPI_ESTATE, MPPI_EUNSUPPORTED, \
    MPPI_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "MPPI_OK", -1: "MPPI_EINVAL", -2: "MPPI_ENOMEM", -3: "MPPI_EDEVICE",
                -4: "MPPI_ESTATE", -5: "MPPI_EUNSUPPORTED", -6: "MPPI_ENUMERIC"}

DYNAMICS = {"double_integrator": 0, "bicycle": 1, "quadrotor": 2, "bicycle_mlp": 3}
INTEGRATORS = {"euler": 0, "rk4": 1}
COSTS = {"quadratic": 0, "path_circles": 1, "path_costmap": 2, "hover": 3, "track": 4,
         "goal_circles": 5}
F_DEBUG = 1
F_ACCURATE_TRIG = 2
F_ROLLOUT_LANE = 4
F_ROLLOUT_QUAD = 8
F_REQUIRES_GRAD = 16
F_IMPORTANCE_SAMPLING = 32
F_STEP_SIZE = 64
F_MEAN_SAMPLE = 128
F_BF16_MLP = 256
ROLLOUT_FUSED, ROLLOUT_SPLIT, ROLLOUT_SCAN = 0, 1, 2
UPDATE_TWO_PASS, UPDATE_ONE_PASS, UPDATE_CHUNKED = 0, 1, 2
BATCH_PHASES, BATCH_ONE_LAUNCH = 0, 1
SHIFT_HOLD, SHIFT_ZERO = 0, 1
DEBUG_NOISE, DEBUG_COSTS, DEBUG_WEIGHTS, DEBUG_STATS, DEBUG_CRASHES = 0, 1, 2, 3, 4
PACKED_STATE, PACKED_CONTROLS, PACKED_SAMPLES, PACKED_NOISE = 0, 1, 2, 3

_fp = C.POINTER(C.c_float)


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("dynamics", C.c_uint32),
                ("integrator", C.c_uint32), ("cost", C.c_uint32),
                ("num_samples", C.c_int32), ("horizon", C.c_int32),
                ("state_dim", C.c_int32), ("control_dim", C.c_int32),
                ("dt", C.c_float), ("lam", C.c_float), ("sigma", C.c_float * MAX_CONTROL),
                ("seed", C.c_uint64), ("instance", C.c_uint32), ("flags", C.c_uint32),
                ("step_size", C.c_float), ("zero_mean_fraction", C.c_float)]


class Params(C.Structure):
    _fields_ = [("wheelbase", C.c_float), ("mass", C.c_float), ("inertia", C.c_float * 3),
                ("gravity", C.c_float), ("mlp_hidden", C.c_int32), ("mlp", _fp),
                ("w", C.c_float * 32), ("ref", _fp), ("ref_len", C.c_int32),
                ("num_segments", C.c_int32), ("knots", _fp), ("coef", _fp),
                ("num_circles", C.c_int32), ("cx", _fp), ("cy", _fp), ("r2", _fp),
                ("map_w", C.c_int32), ("map_h", C.c_int32), ("map_x0", C.c_float),
                ("map_y0", C.c_float), ("map_res", C.c_float), ("costmap", _fp),
                ("checkpoint_every", C.c_int32), ("tape_len", C.c_int32),
                ("sigma_t", _fp), ("cost_cosines", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("lanes_per_sample", C.c_int32), ("rollout_block", C.c_int32),
                ("batch_tile", C.c_int32), ("noise_calls", C.c_int32),
                ("rollout_form", C.c_int32), ("cost_waves", C.c_int32),
                ("update_form", C.c_int32), ("batch_form", C.c_int32),
                ("adjoint_tiles", C.c_int32)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


EXPORTS = {
    "mppi_workspace_bytes": (C.c_size_t, [C.POINTER(Config), C.POINTER(Params)]),
    "mppi_create": (C.c_int, [C.POINTER(Config), C.POINTER(Params), C.c_void_p, C.c_size_t,
                              C.c_void_p, C.POINTER(C.c_void_p)]),
    "mppi_create_static": (C.c_int, [C.POINTER(Config), C.POINTER(Params), C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    "mppi_set_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mppi_set_controls": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mppi_set_iteration": (C.c_int, [C.c_void_p, C.c_uint32]),
    "mppi_shift": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "mppi_sample": (C.c_int, [C.c_void_p]),
    "mppi_rollout": (C.c_int, [C.c_void_p]),
    "mppi_set_costs": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mppi_update": (C.c_int, [C.c_void_p]),
    "mppi_iterate": (C.c_int, [C.c_void_p, C.c_int32]),
    "mppi_get_controls": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mppi_get_debug": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "mppi_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mppi_backward_iters": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mppi_theta_len": (C.c_int32, [C.c_void_p]),
    "mppi_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(Tuning)]),
    "mppi_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(Tuning)]),
    "mppi_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_char_p, C.c_size_t]),
    "mppi_set_theta": (C.c_int, [C.c_void_p, _fp]),
    "mppi_destroy": (None, [C.c_void_p]),
    "mppi_last_error": (C.c_char_p, []),
    "mppi_noise": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32, C.c_int32,
                             C.c_int32, _fp, C.c_void_p, C.c_int64, C.c_void_p]),
    "mppi_noise_tables": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mppi_batch_workspace_bytes": (C.c_size_t, [C.POINTER(Config), C.POINTER(Params), C.c_int32]),
    "mppi_create_batch": (C.c_int, [C.POINTER(Config), C.POINTER(Params), C.c_int32, C.c_void_p,
                                    C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "mppi_num_instances": (C.c_int32, [C.c_void_p]),
    "mppi_offsets": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]),
}

_lib = None


class MPPIError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def lib() -> C.CDLL:
    """The loaded libmppi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2409_07563_amd.build` (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> int:
    if status != MPPI_OK:
        raise MPPIError(status, lib().mppi_last_error().decode())
    return status
