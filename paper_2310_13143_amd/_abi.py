"""ctypes mirror of include/acopf_admm.h and include/acopf_mlp.h, and loader of
the in-tree library."""
from __future__ import annotations

import ctypes
import os
from ctypes import c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libacopf_admm.so")

ACOPF_OK = 0
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "HIP", -3: "NONCONVEX_LINE", -4: "NUMERIC",
                -5: "UNSUPPORTED", -6: "BARRIER"}
HESSIAN_PSD, HESSIAN_RAW, HESSIAN_RAW_LOCAL = 0, 1, 2
SWEEP_PERSISTENT, SWEEP_LAUNCHES, SWEEP_GRAPH = 0, 1, 2
ADMM_CONVERGED, ADMM_MAX_SWEEPS, ADMM_FAILED = 0, 1, 2
START_ZERO, START_PREVIOUS, START_GIVEN = 0, 1, 2
PI_ALWAYS, PI_IF_CONVERGED = 0, 1
LINE_FEATURES, GEN_FEATURES, LINE_OUTPUTS, GEN_OUTPUTS = 25, 11, 16, 4
WARM_LAM_SCALE, WARM_RHO_CLIP = 1e3, 10.0
MLP_HIDDEN = 64

GRID_BUS_FIELDS = ("vmin", "vmax", "pd", "qd", "gsh", "bsh")
GRID_LINE_INT = ("line_from", "line_to")
GRID_LINE_FIELDS = ("gii", "bii", "gij", "bij", "gji", "bji", "gjj", "bjj", "smax_ij", "smax_ji")
GRID_GEN_INT = ("gen_bus",)
GRID_GEN_FIELDS = ("pmin", "pmax", "qmin", "qmax", "cost2", "cost1")
ITERATE_FIELDS = ("pg", "qg", "w", "th", "wR", "wI", "pi")
STATE_FIELDS = ("xg", "xbar_g", "lam_g", "rho_g", "xl", "xbar_f", "lam_l", "rho_l", "dw", "dth", "nu", "mu",
                "sum_r_g", "sum_s_g", "sum_r_l", "sum_s_l")


class Grid(ctypes.Structure):
    _fields_ = ([("n_bus", c_int32), ("n_line", c_int32), ("n_gen", c_int32), ("ref_bus", c_int32),
                 ("n_scen", c_int32), ("reserved", c_int32)]
                + [(n, c_void_p) for n in GRID_BUS_FIELDS + GRID_LINE_INT + GRID_LINE_FIELDS
                   + GRID_GEN_INT + GRID_GEN_FIELDS])


class Iterate(ctypes.Structure):
    _fields_ = [(n, c_void_p) for n in ITERATE_FIELDS]


class AdmmParams(ctypes.Structure):
    _fields_ = [("max_sweeps", c_int32), ("eps_pri", c_double), ("eps_dual", c_double),
                ("sweep_mode", c_int32), ("block_size", c_int32), ("max_blocks", c_int32), ("trace", c_int32),
                ("balance_every", c_int32), ("balance_mu", c_double), ("balance_tau", c_double),
                ("norm_inf", c_int32)]


class AdmmResult(ctypes.Structure):
    _fields_ = [("sweeps", c_int32), ("outcome", c_int32), ("r_norm", c_double), ("s_norm", c_double),
                ("infeasible_lines", c_int32), ("blocks", c_int32), ("status", c_int32),
                ("relaxed_lines", c_int32)]


class AdmmState(ctypes.Structure):
    _fields_ = [(n, c_void_p) for n in STATE_FIELDS]


class SqpParams(ctypes.Structure):
    _fields_ = [("mu", c_double), ("delta_max", c_double), ("grow_ratio", c_double),
                ("hessian_mode", c_int32), ("warm_start", c_int32), ("admm", AdmmParams),
                ("lam_g0", c_void_p), ("lam_l0", c_void_p), ("pi_update", c_int32), ("soc", c_int32),
                ("stop", c_int32), ("restore", c_int32), ("tol_primal", c_double), ("tol_dual", c_double),
                ("tol_step", c_double), ("delta_min", c_double)]


class SqpState(ctypes.Structure):
    _fields_ = [("delta", c_double), ("accepted", c_int32), ("admm_sweeps", c_int32), ("ared", c_double),
                ("pred", c_double), ("step_inf", c_double), ("objective", c_double), ("merit", c_double),
                ("admm_r", c_double), ("admm_s", c_double), ("admm_ms", c_double), ("status", c_int32),
                ("soc_sweeps", c_int32)]


class SqpOutcome(ctypes.Structure):
    _fields_ = [("done", c_int32), ("reason", c_int32), ("iterations", c_int32), ("reserved", c_int32),
                ("seconds", c_double)]


class ResidualsReport(ctypes.Structure):
    _fields_ = [(n, c_double) for n in ("primal", "balance", "c11", "c12", "limit", "bounds", "dual")]


EXPORTS = ("acopf_last_error", "acopf_workspace_bytes", "acopf_setup", "acopf_setup_batch", "acopf_set_delta",
           "acopf_qp_build", "acopf_admm_init", "acopf_admm_solve", "acopf_admm_result_batch",
           "acopf_admm_result_get", "acopf_admm_state_get", "acopf_step", "acopf_sqp_step",
           "acopf_sqp_step_batch", "acopf_sqp_outcome_batch", "acopf_linfeas", "acopf_residuals",
           "acopf_residuals_batch", "acopf_features",
           "acopf_warm_targets", "acopf_warm_decode", "acopf_mlp_param_count", "acopf_mlp_scratch_bytes",
           "acopf_mlp_forward", "acopf_mlp_gradient", "acopf_mlp_gradient_noalloc", "acopf_mlp_adam", "acopf_mlp_feature_stats",
           "acopf_mlp_standardize", "acopf_mlp_fold")
SIZE_RETURNING = ("acopf_workspace_bytes", "acopf_mlp_param_count", "acopf_mlp_scratch_bytes")


class AcopfError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built (there is no
    other implementation to fall back to)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run paper_2310_13143_amd/build.py)")
    lib = ctypes.CDLL(path)
    lib.acopf_last_error.restype = ctypes.c_char_p
    lib.acopf_workspace_bytes.restype = c_size_t
    lib.acopf_workspace_bytes.argtypes = [c_int32, c_int32, c_int32, c_int32]
    P = ctypes.POINTER
    lib.acopf_setup.argtypes = [P(Grid), c_void_p, c_size_t, c_void_p]
    lib.acopf_setup_batch.argtypes = [P(Grid), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                      c_void_p]
    lib.acopf_set_delta.argtypes = [P(Grid), c_void_p, c_void_p, c_void_p]
    lib.acopf_admm_result_batch.argtypes = [P(Grid), c_void_p, c_void_p, c_void_p]
    lib.acopf_sqp_step_batch.argtypes = [P(Grid), P(Iterate), P(Iterate), c_void_p, c_void_p, P(SqpParams),
                                         c_void_p, c_void_p, c_void_p]
    lib.acopf_residuals_batch.argtypes = [P(Grid), P(Iterate), c_void_p, c_void_p, c_void_p]
    lib.acopf_sqp_outcome_batch.argtypes = [P(Grid), c_void_p, c_void_p, c_void_p]
    lib.acopf_qp_build.argtypes = [P(Grid), P(Iterate), c_double, c_int32, c_void_p, c_void_p]
    lib.acopf_admm_init.argtypes = [P(Grid), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.acopf_admm_solve.argtypes = [P(Grid), P(AdmmParams), c_void_p, c_void_p, P(AdmmResult)]
    lib.acopf_admm_result_get.argtypes = [P(Grid), c_void_p, c_void_p, P(AdmmResult)]
    lib.acopf_admm_state_get.argtypes = [P(Grid), c_void_p, P(AdmmState), c_void_p]
    lib.acopf_step.argtypes = [P(Grid), P(Iterate), c_void_p, P(Iterate), c_void_p]
    lib.acopf_sqp_step.argtypes = [P(Grid), P(Iterate), P(Iterate), c_void_p, c_void_p, P(SqpParams), c_void_p,
                                   c_void_p, P(SqpState)]
    lib.acopf_residuals.argtypes = [P(Grid), P(Iterate), c_void_p, c_void_p, P(ResidualsReport)]
    lib.acopf_linfeas.argtypes = [P(Grid), P(Iterate), c_double, P(AdmmParams), c_void_p, c_void_p, c_void_p]
    lib.acopf_features.argtypes = [P(Grid), P(Iterate), c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_int64,
                                   c_void_p]
    lib.acopf_warm_targets.argtypes = [P(Grid), c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p]
    lib.acopf_warm_decode.argtypes = [P(Grid), c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_double, c_double,
                                      c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.acopf_mlp_param_count.restype = c_size_t
    lib.acopf_mlp_param_count.argtypes = [c_int32, c_int32]
    lib.acopf_mlp_scratch_bytes.restype = c_size_t
    lib.acopf_mlp_scratch_bytes.argtypes = [c_int32, c_int32, c_int64]
    lib.acopf_mlp_forward.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_int64, c_int64, c_void_p, c_int64,
                                      c_void_p]
    lib.acopf_mlp_gradient.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_int64, c_void_p, c_int64, c_int64,
                                       c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.acopf_mlp_gradient_noalloc.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_int64, c_void_p, c_int64,
                                               c_int64, c_void_p, c_void_p, c_void_p]
    lib.acopf_mlp_adam.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_float, c_float,
                                   c_float, c_float, c_void_p]
    lib.acopf_mlp_feature_stats.argtypes = [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_void_p, c_void_p]
    lib.acopf_mlp_standardize.argtypes = [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_void_p, c_double,
                                          c_void_p]
    lib.acopf_mlp_fold.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    for name in EXPORTS[1:]:
        if name not in SIZE_RETURNING:
            getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def check(code: int):
    if code != ACOPF_OK:
        raise AcopfError(code, load().acopf_last_error().decode())
