"""ctypes binding of libdbasmppi.so (the C ABI in include/dbas_mppi.h).

Argument marshalling only: every step of the controller runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdbasmppi.so")

ABI_VERSION = 2
M, NMAX, PMAX = 2, 6, 16
OK, E_INVALID, E_NOMEM, E_DEVICE, E_NUMERIC, E_BUSY = range(6)
MODELS = {"quad6": 0, "quad5": 1, "car": 2}
STATE_DIM = {"quad6": 6, "quad5": 5, "car": 4}
NORMALISER = {"auto": 0, "on": 1, "off": 2}
INIT_MODE = {"repeat": 0, "zero": 1}
SAMPLING = {"nln": 0, "normal": 1}
COST_MODE = {"dbas": 0, "indicator": 1}
MEM_HOST, MEM_DEVICE = 0, 1

# Every entry point include/dbas_mppi.h declares.
EXPORTS = [
    "mppi_config_default", "mppi_create", "mppi_destroy", "mppi_set_obstacles", "mppi_set_costmap",
    "mppi_set_reference", "mppi_set_exploration", "mppi_set_controls", "mppi_step", "mppi_step_async",
    "mppi_synchronize", "mppi_get_controls", "mppi_get_last_optimal", "mppi_get_costs", "mppi_get_weights",
    "mppi_get_noise", "mppi_get_step_info", "mppi_get_philox_words", "mppi_get_state", "mppi_set_state",
    "mppi_last_error", "mppi_status_string", "mppi_stream", "mppi_profile_enable", "mppi_profile_read",
    "mppi_batch_create", "mppi_batch_destroy", "mppi_batch_step", "mppi_batch_last_error",
    "mppi_server_create", "mppi_server_destroy", "mppi_server_add_robot", "mppi_server_submit",
    "mppi_server_poll", "mppi_server_wait", "mppi_server_now", "mppi_server_get_stats",
    "mppi_server_get_robot", "mppi_server_last_error", "mppi_step_noalloc",
]

NOALLOC_SCRATCH_BYTES = 8 << 20


class MppiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32), ("model", ctypes.c_int32), ("K", ctypes.c_int32), ("T", ctypes.c_int32),
        ("dt", ctypes.c_float), ("mass", ctypes.c_float), ("gravity", ctypes.c_float), ("arm", ctypes.c_float),
        ("inertia", ctypes.c_float), ("wheelbase", ctypes.c_float),
        ("u_min", ctypes.c_float * M), ("u_max", ctypes.c_float * M), ("sigma", ctypes.c_float * M),
        ("mu_ln", ctypes.c_float), ("sigma_ln", ctypes.c_float), ("lam", ctypes.c_float), ("gamma_u", ctypes.c_float),
        ("gamma_b", ctypes.c_float), ("r_b", ctypes.c_float), ("h_eps", ctypes.c_float),
        ("Q", ctypes.c_float * NMAX), ("Qf", ctypes.c_float * NMAX),
        ("P", ctypes.c_int32), ("shape", (ctypes.c_float * 2) * PMAX),
        ("seed", ctypes.c_uint64), ("normaliser", ctypes.c_int32), ("init_mode", ctypes.c_int32),
        ("tile_samples", ctypes.c_int32), ("export_noise", ctypes.c_int32),
        ("adaptive_explore", ctypes.c_int32), ("explore_mu", ctypes.c_float),
        ("sgf_half_window", ctypes.c_int32), ("sgf_order", ctypes.c_int32),
        ("sampling", ctypes.c_int32), ("cost_mode", ctypes.c_int32), ("collision_weight", ctypes.c_float),
        ("reserved", ctypes.c_int32 * 2),
    ]


class Device(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class State(ctypes.Structure):
    _fields_ = [("counter", ctypes.c_uint64), ("S_e", ctypes.c_float), ("T", ctypes.c_int32),
                ("U", ctypes.POINTER(ctypes.c_float))]


class StepInfo(ctypes.Structure):
    _fields_ = [("counter", ctypes.c_uint64), ("status", ctypes.c_int32), ("fp64_tiles", ctypes.c_int32),
                ("rho", ctypes.c_double), ("eta", ctypes.c_double), ("beta0", ctypes.c_float),
                ("beta_d", ctypes.c_float), ("tile_samples", ctypes.c_int32), ("tiles", ctypes.c_int32),
                ("S_e", ctypes.c_float), ("cost_b", ctypes.c_float), ("barrier_form", ctypes.c_int32),
                ("noise_kept", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("dropped", ctypes.c_int64), ("rollout_ms", ctypes.c_double),
                ("update_ms", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("J", ctypes.c_int32), ("obs", ctypes.c_void_p), ("map_w", ctypes.c_int32),
                ("map_h", ctypes.c_int32), ("map_x0", ctypes.c_float), ("map_y0", ctypes.c_float),
                ("map_res", ctypes.c_float), ("sdf", ctypes.c_void_p), ("x_ref", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("device", ctypes.c_int32), ("budget_bytes", ctypes.c_int64),
                ("max_slots", ctypes.c_int32), ("streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 7)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("deferred_budget", ctypes.c_int64), ("deferred_slots", ctypes.c_int64),
                ("peak_bytes_in_flight", ctypes.c_int64), ("mean_batch", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdbasmppi.so not built at {path}: run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    vp, fp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "mppi_config_default": (i32, [i32, i32, i32, ctypes.POINTER(Config)]),
        "mppi_create": (i32, [ctypes.POINTER(Config), ctypes.POINTER(Device), ctypes.POINTER(vp)]),
        "mppi_destroy": (None, [vp]),
        "mppi_set_obstacles": (i32, [vp, i32, vp, i32]),
        "mppi_set_costmap": (i32, [vp, i32, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp, i32]),
        "mppi_set_reference": (i32, [vp, vp, i32]),
        "mppi_set_exploration": (i32, [vp, ctypes.c_float]),
        "mppi_set_controls": (i32, [vp, vp, i32]),
        "mppi_step": (i32, [vp, fp, fp]),
        "mppi_step_async": (i32, [vp, vp, vp]),
        "mppi_synchronize": (i32, [vp]),
        "mppi_get_controls": (i32, [vp, fp]),
        "mppi_get_last_optimal": (i32, [vp, fp]),
        "mppi_get_costs": (i32, [vp, dp]),
        "mppi_get_weights": (i32, [vp, dp]),
        "mppi_get_noise": (i32, [vp, fp]),
        "mppi_get_step_info": (i32, [vp, ctypes.POINTER(StepInfo)]),
        "mppi_get_philox_words": (i32, [vp, u64, ctypes.POINTER(ctypes.c_uint32)]),
        "mppi_get_state": (i32, [vp, ctypes.POINTER(State)]),
        "mppi_set_state": (i32, [vp, ctypes.POINTER(State)]),
        "mppi_last_error": (ctypes.c_char_p, [vp]),
        "mppi_status_string": (ctypes.c_char_p, [i32]),
        "mppi_stream": (vp, [vp]),
        "mppi_profile_enable": (i32, [vp, i32]),
        "mppi_profile_read": (i32, [vp, ctypes.POINTER(Profile)]),
        "mppi_batch_create": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(Device), ctypes.POINTER(vp)]),
        "mppi_batch_destroy": (None, [vp]),
        "mppi_batch_step": (i32, [vp, fp, fp, ctypes.POINTER(i32)]),
        "mppi_batch_last_error": (ctypes.c_char_p, [vp]),
        "mppi_server_create": (i32, [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
        "mppi_server_destroy": (None, [vp]),
        "mppi_server_add_robot": (i32, [vp, ctypes.POINTER(Config), i32, vp, ctypes.POINTER(i32)]),
        "mppi_server_submit": (i32, [vp, i32, fp, fp, ctypes.c_double, ctypes.POINTER(i64)]),
        "mppi_server_poll": (i32, [vp, i64, fp, dp, ctypes.POINTER(i32)]),
        "mppi_server_wait": (i32, [vp, i64, fp, dp, ctypes.POINTER(i32)]),
        "mppi_server_now": (ctypes.c_double, [vp]),
        "mppi_server_get_stats": (i32, [vp, ctypes.POINTER(ServerStats)]),
        "mppi_server_get_robot": (i32, [vp, i32, fp, ctypes.POINTER(u64)]),
        "mppi_server_last_error": (ctypes.c_char_p, [vp]),
        "mppi_step_noalloc": (i32, [ctypes.POINTER(Config), ctypes.POINTER(Problem), i32, vp, vp, vp, u64,
                                    ctypes.c_float, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L
