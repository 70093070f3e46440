"""ctypes loader for libmdhp.so (the HIP library's C ABI, include/mdhp.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels.  Importing this module does not need a GPU; loading the library
does not either (symbols resolve against the HIP runtime), but every compute
call does.  A missing library is an error, never a fallback.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdhp.so")

# Every symbol include/mdhp.h declares.
EXPORTS = (
    "mdhp_plan_create", "mdhp_plan_destroy", "mdhp_plan_windows", "mdhp_plan_events",
    "mdhp_plan_dims", "mdhp_loglik", "mdhp_grad", "mdhp_fit_batch", "mdhp_check_params",
    "mdhp_status_string", "mdhp_last_error", "mdhp_features", "mdhp_surrogate_create",
    "mdhp_surrogate_destroy", "mdhp_surrogate_num_params", "mdhp_surrogate_get_weights",
    "mdhp_surrogate_set_weights", "mdhp_surrogate_forward", "mdhp_surrogate_get_hidden",
    "mdhp_surrogate_backward", "mdhp_surrogate_get_gradients", "mdhp_surrogate_adam",
    "mdhp_surrogate_train_step", "mdhp_warm_start", "mdhp_cold_start", "mdhp_plan_autotune",
    "mdhp_plan_set_schedule", "mdhp_plan_schedule", "mdhp_plan_create_scheduled",
    "mdhp_surrogate_save", "mdhp_surrogate_load", "mdhp_grad_static", "mdhp_simulate",
    "mdhp_attack_times", "mdhp_lstm_sizes", "mdhp_lstm_forward", "mdhp_lstm_backward",
    "mdhp_lstm_timing", "mdhp_lstm_phase_ms", "mdhp_plan_dim_counts",
)

MDHP_OK = 0
STATUS_NAMES = {0: "MDHP_OK", -1: "MDHP_E_INVAL", -2: "MDHP_E_UNSORTED", -3: "MDHP_E_DOMAIN",
                -4: "MDHP_E_PARAM", -5: "MDHP_E_NOMEM", -6: "MDHP_E_HIP", -7: "MDHP_E_IO"}
BETA_SHARED, BETA_PAIR = 0, 1
OPT_PGD, OPT_PADAM, OPT_LBFGS, OPT_EM = 0, 1, 2, 3
SCATTER_MFMA = 1  # the M > 32 schedule with the intensity sums on the matrix cores
SIM_UNTIL_T, SIM_COUNT = 0, 1
ATTACK_PLA, ATTACK_DEA, ATTACK_ASA, ATTACK_DAM = 0, 1, 2, 3
SAMPLER_NPP, SAMPLER_ND, SAMPLER_DRP = 0, 1, 2
LSTM_FWD_PHASES, LSTM_BWD_PHASES = 4, 6
FIT_CONVERGED, FIT_MAX_STEPS, FIT_NONFINITE, FIT_STALLED = 0, 1, 2, 3
MAX_M = 64
TUNE_MAX = 8
TEAM_NEVER = 2147483647


class MdhpBatch(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int64), ("n_events", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("dim", ctypes.c_void_p), ("T", ctypes.c_void_p)]


class MdhpFitOpts(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_int32), ("optimizer", ctypes.c_int32),
                ("fix_beta", ctypes.c_int32), ("history", ctypes.c_int32),
                ("lr", ctypes.c_double), ("ll_tol", ctypes.c_double),
                ("mu_floor_rel", ctypes.c_double), ("beta_floor_rel", ctypes.c_double),
                ("adam_b1", ctypes.c_double), ("adam_b2", ctypes.c_double),
                ("adam_eps", ctypes.c_double), ("check_params", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class MdhpLstmDims(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int32), ("L", ctypes.c_int32), ("D", ctypes.c_int32),
                ("H", ctypes.c_int32), ("M", ctypes.c_int32), ("beta_mode", ctypes.c_int32)]


class MdhpTuneResult(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("chosen", ctypes.c_int32),
                ("value", ctypes.c_int32 * TUNE_MAX), ("ms", ctypes.c_float * TUNE_MAX)]


class MdhpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Loads the in-tree libmdhp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2411_10258_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.mdhp_plan_create.argtypes = [ctypes.POINTER(MdhpBatch), I32, I32, P, ctypes.POINTER(P)]
    lib.mdhp_plan_destroy.argtypes = [P]
    lib.mdhp_plan_destroy.restype = None
    for name in ("mdhp_plan_windows", "mdhp_plan_events"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = I64
    lib.mdhp_plan_dims.argtypes = [P]
    lib.mdhp_plan_dims.restype = I32
    lib.mdhp_loglik.argtypes = [P, P, P, P, P, P]
    lib.mdhp_grad.argtypes = [P, P, P, P, P, P, P, P, P]
    lib.mdhp_fit_batch.argtypes = [P, ctypes.POINTER(MdhpFitOpts), P, P, P, P, P, P, P, P]
    lib.mdhp_check_params.argtypes = [P, P, P, P, P]
    lib.mdhp_cold_start.argtypes = [P, P, P, P, P]
    lib.mdhp_plan_autotune.argtypes = [P, ctypes.POINTER(MdhpBatch), ctypes.POINTER(MdhpFitOpts),
                                       I32, ctypes.POINTER(MdhpTuneResult), P]
    lib.mdhp_plan_set_schedule.argtypes = [P, ctypes.POINTER(MdhpBatch), I32, P]
    lib.mdhp_plan_create_scheduled.argtypes = [ctypes.POINTER(MdhpBatch), I32, I32, I32, P,
                                               ctypes.POINTER(P)]
    lib.mdhp_plan_create_scheduled.restype = I32
    lib.mdhp_plan_dim_counts.argtypes = [P, P, P]
    lib.mdhp_plan_schedule.argtypes = [P]
    lib.mdhp_plan_schedule.restype = I32
    lib.mdhp_features.argtypes = [ctypes.POINTER(MdhpBatch), I32, I32, P, P]
    lib.mdhp_surrogate_create.argtypes = [I32, I32, I32, I32, ctypes.c_uint64, ctypes.POINTER(P)]
    lib.mdhp_surrogate_destroy.argtypes = [P]
    lib.mdhp_surrogate_destroy.restype = None
    lib.mdhp_surrogate_num_params.argtypes = [P]
    lib.mdhp_surrogate_num_params.restype = I64
    lib.mdhp_surrogate_get_weights.argtypes = [P, P, P]
    lib.mdhp_surrogate_set_weights.argtypes = [P, P, P]
    lib.mdhp_surrogate_get_gradients.argtypes = [P, P, P]
    lib.mdhp_surrogate_forward.argtypes = [P, P, I32, P, P]
    lib.mdhp_surrogate_get_hidden.argtypes = [P, I32, P, P, P]
    lib.mdhp_surrogate_backward.argtypes = [P, P, I32, P, P, P]
    lib.mdhp_surrogate_adam.argtypes = [P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, P]
    lib.mdhp_surrogate_train_step.argtypes = [P, P, I32, P, ctypes.c_float, P, P]
    lib.mdhp_warm_start.argtypes = [P, P, P, P, ctypes.POINTER(MdhpFitOpts), P, P, P, P, P, P,
                                    P, P]
    lib.mdhp_surrogate_save.argtypes = [P, ctypes.c_char_p, P, I64, P]
    lib.mdhp_surrogate_load.argtypes = [P, ctypes.c_char_p, P, I64, ctypes.POINTER(I64), P]
    lib.mdhp_grad_static.argtypes = [ctypes.POINTER(MdhpBatch), I32, P, P, P, P, P, P, P, P]
    lib.mdhp_simulate.argtypes = [I64, I32, I32, P, P, P, I32, P, P, ctypes.c_uint64, I64, P, P,
                                  P, P, P]
    lib.mdhp_attack_times.argtypes = [I64, P, P, P, P, P, ctypes.c_uint64, I64, P, P, P]
    LD = ctypes.POINTER(MdhpLstmDims)
    lib.mdhp_lstm_sizes.argtypes = [LD, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    lib.mdhp_lstm_forward.argtypes = [LD, P, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.mdhp_lstm_backward.argtypes = [LD, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.mdhp_lstm_timing.argtypes = [I32]
    lib.mdhp_lstm_phase_ms.argtypes = [P, P]
    lib.mdhp_status_string.argtypes = [I32]
    lib.mdhp_status_string.restype = ctypes.c_char_p
    lib.mdhp_last_error.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    for name in ("mdhp_plan_create", "mdhp_loglik", "mdhp_grad", "mdhp_fit_batch",
                 "mdhp_check_params", "mdhp_last_error", "mdhp_features", "mdhp_surrogate_create",
                 "mdhp_surrogate_get_weights", "mdhp_surrogate_set_weights",
                 "mdhp_surrogate_get_gradients", "mdhp_surrogate_forward",
                 "mdhp_surrogate_get_hidden", "mdhp_surrogate_backward", "mdhp_surrogate_adam",
                 "mdhp_surrogate_train_step", "mdhp_warm_start", "mdhp_cold_start",
                 "mdhp_plan_autotune", "mdhp_plan_set_schedule", "mdhp_surrogate_save",
                 "mdhp_surrogate_load", "mdhp_grad_static", "mdhp_simulate",
                 "mdhp_attack_times", "mdhp_lstm_sizes", "mdhp_lstm_forward",
                 "mdhp_lstm_backward", "mdhp_lstm_timing", "mdhp_lstm_phase_ms",
                 "mdhp_plan_dim_counts"):
        getattr(lib, name).restype = I32
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != MDHP_OK:
        lib = load()
        buf = ctypes.create_string_buffer(512)
        lib.mdhp_last_error(buf, len(buf))
        raise MdhpError(status, buf.value.decode(errors="replace"))
