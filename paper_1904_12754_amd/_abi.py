"""ctypes declarations of the C-ABI in include/mlmc_expv.h (argument marshalling only).

The library is loaded from this package directory; if it is missing the import of the
binding raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlmc_expv.so")

MLMC_OK = 0
MLMC_ERR_INVALID_ARG = 1
MLMC_ERR_INVALID_MATRIX = 2
MLMC_ERR_OUT_OF_MEMORY = 3
MLMC_ERR_HIP = 4
MLMC_ERR_NONFINITE = 5
MLMC_ERR_NOT_CONVERGED = 6
MLMC_ERR_UNSUPPORTED = 7
MLMC_ERR_RNG_OVERFLOW = 8

MLMC_MEMORY_HOST = 0
MLMC_MEMORY_DEVICE = 1

MLMC_DTYPE_F32 = 0
MLMC_DTYPE_F64 = 1
MLMC_PRECISION_FP64 = 0
MLMC_PRECISION_FP32 = 1
MLMC_MAX_LEVELS = 40

# every symbol the header declares
EXPORTS = ("mlmc_expv_plan", "mlmc_expv_plan_info", "mlmc_expv_run", "mlmc_expv_level_sums",
           "mlmc_expv_level_sums_noalloc",
           "mlmc_expv_run_source", "mlmc_expv_level_sums_source", "mlmc_expv_functional",
           "mlmc_expv_functional_level_sums", "mlmc_expv_forward", "mlmc_expv_forward_level_sums",
           "mlmc_expv_trace", "mlmc_expv_destroy", "mlmc_expv_batch_create",
           "mlmc_expv_batch_launch", "mlmc_expv_batch_stats", "mlmc_expv_batch_info",
           "mlmc_expv_batch_destroy", "mlmc_expv_proposal_set", "mlmc_expv_proposal_enable",
           "mlmc_expv_proposal_tables", "mlmc_expv_proposal_loss_grad",
           "mlmc_expv_proposal_train", "mlmc_expv_run_learned", "mlmc_status_string",
           "mlmc_last_error",
           "mlmc_probe_gather", "mlmc_probe_gather_mode", "mlmc_probe_valu")

MLMC_PROPOSAL_PARAMS = 5703
MLMC_PROBE_LDS = 1
MLMC_PROBE_DEPENDENT = 2
MLMC_BATCH_TUNE_MAX = 12


class CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
                ("col_idx", ctypes.POINTER(ctypes.c_int32)),
                ("values", ctypes.c_void_p),
                ("values_dtype", ctypes.c_int32),
                ("memory", ctypes.c_int32)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double),
                ("precision", ctypes.c_int32),
                ("l0", ctypes.c_int32),
                ("rows", ctypes.POINTER(ctypes.c_int64)),
                ("n_rows", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_rows", ctypes.c_int64), ("n_slots", ctypes.c_int64),
                ("l0", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("beta", ctypes.c_double), ("r_max", ctypes.c_double),
                ("d_min", ctypes.c_double), ("d_max", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("jump_probability", ctypes.c_double),
                ("screened", ctypes.c_int32), ("pad", ctypes.c_int32)]


class RunOpts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64),
                ("instance", ctypes.c_int32),
                ("num_levels", ctypes.c_int32),
                ("walks", ctypes.POINTER(ctypes.c_int64)),
                ("eps", ctypes.c_double),
                ("pilot_walks", ctypes.c_int64),
                ("max_levels", ctypes.c_int32),
                ("max_walks", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("l0", ctypes.c_int32), ("num_levels", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("driver_iterations", ctypes.c_int32),
                ("walks", ctypes.c_int64 * MLMC_MAX_LEVELS),
                ("jumps", ctypes.c_int64 * MLMC_MAX_LEVELS),
                ("level_mean_rms", ctypes.c_double * MLMC_MAX_LEVELS),
                ("level_var", ctypes.c_double * MLMC_MAX_LEVELS),
                ("level_cost", ctypes.c_double * MLMC_MAX_LEVELS),
                ("steps", ctypes.c_int64), ("total_jumps", ctypes.c_int64),
                ("nonfinite", ctypes.c_int64),
                ("est_variance", ctypes.c_double), ("est_bias", ctypes.c_double),
                ("kernel_ms", ctypes.c_double),
                ("walk_kernel_ms", ctypes.c_double),
                ("walk_launches", ctypes.c_int64)]

    def to_dict(self) -> dict:
        L = self.num_levels
        return {
            "l0": self.l0, "num_levels": L, "converged": bool(self.converged),
            "driver_iterations": self.driver_iterations,
            "walks": list(self.walks[:L]), "jumps": list(self.jumps[:L]),
            "level_mean_rms": list(self.level_mean_rms[:L]),
            "level_var": list(self.level_var[:L]), "level_cost": list(self.level_cost[:L]),
            "steps": self.steps, "total_jumps": self.total_jumps, "nonfinite": self.nonfinite,
            "est_variance": self.est_variance, "est_bias": self.est_bias,
            "kernel_ms": self.kernel_ms,
            "walk_kernel_ms": self.walk_kernel_ms, "walk_launches": self.walk_launches,
        }


class BatchDesc(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32),
                ("plans", ctypes.POINTER(ctypes.c_void_p)),
                ("u", ctypes.POINTER(ctypes.c_void_p)),
                ("nrhs", ctypes.POINTER(ctypes.c_int32)),
                ("u_dtype", ctypes.c_int32),
                ("x", ctypes.POINTER(ctypes.c_void_p)),
                ("num_levels", ctypes.c_int32),
                ("walks", ctypes.POINTER(ctypes.c_int64)),
                ("autotune", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("walks_per_item", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("graph_nodes", ctypes.c_int32), ("phases", ctypes.c_int32),
                ("items", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("tune_count", ctypes.c_int32),
                ("tune_walks_per_item", ctypes.c_int32 * MLMC_BATCH_TUNE_MAX),
                ("tune_waves_per_cu", ctypes.c_int32 * MLMC_BATCH_TUNE_MAX),
                ("pad", ctypes.c_int32),
                ("tune_ms", ctypes.c_double * MLMC_BATCH_TUNE_MAX)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("init_params", ctypes.POINTER(ctypes.c_float)),
                ("pilot_walks", ctypes.c_int64), ("capture_walks", ctypes.c_int32),
                ("sample_stride", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("shrink", ctypes.c_double), ("num_levels", ctypes.c_int32),
                ("judge_walks", ctypes.c_int32)]


class TrainStats(ctypes.Structure):
    _fields_ = [("transitions", ctypes.c_int64), ("held_out", ctypes.c_int64),
                ("steps", ctypes.c_int32), ("n_losses", ctypes.c_int32),
                ("best_step", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("train_ms", ctypes.c_double),
                ("first_loss", ctypes.c_double), ("last_loss", ctypes.c_double),
                ("first_val_loss", ctypes.c_double), ("best_val_loss", ctypes.c_double),
                ("judge_var_plain", ctypes.c_double), ("judge_var_learned", ctypes.c_double),
                ("accepted", ctypes.c_int32), ("pad2", ctypes.c_int32),
                ("losses", ctypes.c_double * 64)]

    def to_dict(self) -> dict:
        return {"transitions": self.transitions, "held_out": self.held_out,
                "steps": self.steps, "best_step": self.best_step, "train_ms": self.train_ms,
                "first_loss": self.first_loss, "last_loss": self.last_loss,
                "first_val_loss": self.first_val_loss, "best_val_loss": self.best_val_loss,
                "judge_var_plain": self.judge_var_plain,
                "judge_var_learned": self.judge_var_learned, "accepted": bool(self.accepted),
                "losses": list(self.losses[:self.n_losses])}


_lib = None


def load() -> ctypes.CDLL:
    """Load libmlmc_expv.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1904_12754_amd.build` (there is no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32, i64, u32, u64, f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                               ctypes.c_double)
    L.mlmc_expv_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(CSR),
                                 ctypes.POINTER(PlanOpts), vp]
    L.mlmc_expv_plan.restype = ctypes.c_int
    L.mlmc_expv_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.mlmc_expv_plan_info.restype = ctypes.c_int
    L.mlmc_expv_run.argtypes = [vp, vp, i32, i32, ctypes.POINTER(RunOpts), vp,
                                ctypes.POINTER(Stats), vp]
    L.mlmc_expv_run.restype = ctypes.c_int
    L.mlmc_expv_level_sums.argtypes = [vp, vp, i32, i32, u64, i32, i32, u32, u32, vp, vp,
                                       ctypes.POINTER(i64), vp, vp]
    L.mlmc_expv_level_sums.restype = ctypes.c_int
    L.mlmc_expv_level_sums_noalloc.argtypes = L.mlmc_expv_level_sums.argtypes
    L.mlmc_expv_level_sums_noalloc.restype = ctypes.c_int
    L.mlmc_expv_run_source.argtypes = [vp, vp, vp, i32, ctypes.POINTER(RunOpts), vp,
                                        ctypes.POINTER(Stats), vp]
    L.mlmc_expv_run_source.restype = ctypes.c_int
    L.mlmc_expv_level_sums_source.argtypes = [vp, vp, vp, i32, u64, i32, i32, u32, u32, vp, vp,
                                              ctypes.POINTER(i64), vp, vp]
    L.mlmc_expv_level_sums_source.restype = ctypes.c_int
    L.mlmc_expv_functional.argtypes = [vp, vp, vp, i32, ctypes.POINTER(RunOpts),
                                        ctypes.POINTER(f64), ctypes.POINTER(f64),
                                        ctypes.POINTER(Stats), vp]
    L.mlmc_expv_functional.restype = ctypes.c_int
    L.mlmc_expv_functional_level_sums.argtypes = [vp, vp, vp, i32, u64, i32, i32, u32, u32,
                                                   ctypes.POINTER(f64), ctypes.POINTER(f64),
                                                   ctypes.POINTER(i64), ctypes.POINTER(u64),
                                                   ctypes.POINTER(f64), vp]
    L.mlmc_expv_functional_level_sums.restype = ctypes.c_int
    L.mlmc_expv_forward.argtypes = [vp, vp, i32, ctypes.POINTER(RunOpts), vp, vp,
                                    ctypes.POINTER(Stats), vp]
    L.mlmc_expv_forward.restype = ctypes.c_int
    L.mlmc_expv_forward_level_sums.argtypes = [vp, vp, i32, u64, i32, i32, u32, u32, vp, vp,
                                               ctypes.POINTER(i64), ctypes.POINTER(u64),
                                               ctypes.POINTER(f64), vp]
    L.mlmc_expv_forward_level_sums.restype = ctypes.c_int
    L.mlmc_expv_trace.argtypes = [vp, u64, i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.mlmc_expv_trace.restype = ctypes.c_int
    L.mlmc_expv_destroy.argtypes = [vp]
    L.mlmc_expv_destroy.restype = None
    L.mlmc_expv_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(BatchDesc), vp]
    L.mlmc_expv_batch_create.restype = ctypes.c_int
    L.mlmc_expv_batch_launch.argtypes = [vp, u64, vp]
    L.mlmc_expv_batch_launch.restype = ctypes.c_int
    L.mlmc_expv_batch_stats.argtypes = [vp, ctypes.POINTER(Stats), vp]
    L.mlmc_expv_batch_stats.restype = ctypes.c_int
    L.mlmc_expv_batch_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    L.mlmc_expv_batch_info.restype = ctypes.c_int
    L.mlmc_expv_batch_destroy.argtypes = [vp]
    L.mlmc_expv_batch_destroy.restype = None
    fp = ctypes.POINTER(ctypes.c_float)
    L.mlmc_expv_proposal_set.argtypes = [vp, fp, vp, i32, vp]
    L.mlmc_expv_proposal_set.restype = ctypes.c_int
    L.mlmc_expv_proposal_enable.argtypes = [vp, i32]
    L.mlmc_expv_proposal_enable.restype = ctypes.c_int
    L.mlmc_expv_proposal_tables.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.mlmc_expv_proposal_tables.restype = ctypes.c_int
    L.mlmc_expv_proposal_loss_grad.argtypes = [vp, fp, vp, i32, i32, ctypes.POINTER(i64),
                                               ctypes.POINTER(i32), fp, f64, fp,
                                               ctypes.POINTER(f64), vp]
    L.mlmc_expv_proposal_loss_grad.restype = ctypes.c_int
    L.mlmc_expv_proposal_train.argtypes = [vp, vp, i32, ctypes.POINTER(TrainOpts), fp,
                                           ctypes.POINTER(TrainStats), vp]
    L.mlmc_expv_proposal_train.restype = ctypes.c_int
    L.mlmc_expv_run_learned.argtypes = [vp, vp, i32, ctypes.POINTER(RunOpts),
                                        ctypes.POINTER(TrainOpts), fp, vp, ctypes.POINTER(Stats),
                                        ctypes.POINTER(TrainStats), vp]
    L.mlmc_expv_run_learned.restype = ctypes.c_int
    L.mlmc_probe_gather.argtypes = [vp, i32, i32, i32, ctypes.POINTER(u64), ctypes.POINTER(f64), vp]
    L.mlmc_probe_gather.restype = ctypes.c_int
    L.mlmc_probe_gather_mode.argtypes = [vp, i32, i32, i32, i32, ctypes.POINTER(u64),
                                         ctypes.POINTER(f64), vp]
    L.mlmc_probe_gather_mode.restype = ctypes.c_int
    L.mlmc_probe_valu.argtypes = [i32, i32, ctypes.POINTER(u64), ctypes.POINTER(f64), vp]
    L.mlmc_probe_valu.restype = ctypes.c_int
    L.mlmc_status_string.argtypes = [ctypes.c_int]
    L.mlmc_status_string.restype = ctypes.c_char_p
    L.mlmc_last_error.argtypes = []
    L.mlmc_last_error.restype = ctypes.c_char_p
    del f64
    _lib = L
    return L


class MLMCError(RuntimeError):
    def __init__(self, code: int, detail: str):
        self.code = code
        super().__init__(f"mlmc status {code}: {detail}")


def check(code: int, allow=()) -> int:
    if code != MLMC_OK and code not in allow:
        L = load()
        raise MLMCError(code, f"{L.mlmc_status_string(code).decode()}: "
                              f"{L.mlmc_last_error().decode()}")
    return code
