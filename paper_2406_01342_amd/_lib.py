"""ctypes declarations of libpolyclean.so (see include/polyclean.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any operator.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpolyclean.so")

PC_OK = 0
PC_WARN_NOT_CONVERGED = 1
PC_ERR_INVALID_ARG = -1
PC_ERR_OUT_OF_MEMORY = -2
PC_ERR_DEVICE = -3
PC_ERR_CAPACITY = -4
PC_ERR_UNSUPPORTED = -5
STATUS_NAMES = {0: "PC_OK", 1: "PC_WARN_NOT_CONVERGED", -1: "PC_ERR_INVALID_ARG",
                -2: "PC_ERR_OUT_OF_MEMORY", -3: "PC_ERR_DEVICE", -4: "PC_ERR_CAPACITY",
                -5: "PC_ERR_UNSUPPORTED"}

PC_UV_WAVELENGTHS, PC_UV_METRES = 0, 1
PC_PREC_FP32, PC_PREC_FP64 = 0, 1


class PcGeometry(C.Structure):
    _fields_ = [("nvis", C.c_int64), ("u", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double)), ("uv_units", C.c_int32), ("freq_hz", C.c_double),
                ("npix", C.c_int32), ("fov_rad", C.c_double), ("nufft_eps", C.c_double),
                ("upsamp", C.c_double), ("precision", C.c_int32)]


class PcPlanInfo(C.Structure):
    _fields_ = [("nvis", C.c_int64), ("npix", C.c_int32), ("fine", C.c_int32),
                ("kernel_width", C.c_int32), ("kernel_beta", C.c_double),
                ("band_u0", C.c_int32), ("band_nu", C.c_int32), ("band_v0", C.c_int32),
                ("band_nv", C.c_int32), ("wraps", C.c_int32), ("tile", C.c_int32),
                ("n_tiles", C.c_int64), ("n_chunks", C.c_int64), ("n_partials", C.c_int64),
                ("footprint", C.c_size_t), ("precision", C.c_int32), ("w_planes", C.c_int32),
                ("w_first", C.c_double), ("w_step", C.c_double)]


class PcSolveParams(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("alpha", C.c_double), ("delta", C.c_double),
                ("max_iter", C.c_int32), ("rel_obj_tol", C.c_double), ("rel_gap_tol", C.c_double),
                ("inner_tol0", C.c_double), ("inner_tol_min", C.c_double),
                ("inner_max_iter", C.c_int32), ("positivity", C.c_int32),
                ("want_certificate", C.c_int32), ("log_every", C.c_int32),
                ("grid_atoms", C.c_int32), ("gram_atoms", C.c_int32),
                ("n_scales", C.c_int32), ("scale_sigma", C.c_double * 8),
                ("scale_gamma", C.c_double * 8), ("x0_pix", C.POINTER(C.c_int32)),
                ("x0_w", C.POINTER(C.c_double)), ("x0_n", C.c_int64)]


class PcSolveResult(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("pix", C.POINTER(C.c_int32)),
                ("weight", C.POINTER(C.c_double)), ("cert", C.c_void_p), ("natoms", C.c_int64),
                ("objective", C.c_double), ("rel_gap", C.c_double), ("lambda_", C.c_double),
                ("lambda_max", C.c_double), ("cert_max", C.c_double), ("cert_argmax", C.c_int64),
                ("iters", C.c_int32), ("inner_iters", C.c_int32), ("converged", C.c_int32),
                ("seconds", C.c_double), ("adjoint_seconds", C.c_double),
                ("adjoint_calls", C.c_int32)]


class PcKernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("ms", C.c_double),
                ("bytes", C.c_double), ("work", C.c_double)]


class PcBatcherStats(C.Structure):
    _fields_ = [("batches", C.c_int64), ("requests", C.c_int64), ("visibilities", C.c_int64),
                ("max_batch", C.c_int32), ("pad", C.c_int32), ("seconds", C.c_double),
                ("forwards", C.c_int64), ("restricted_adjoints", C.c_int64)]


_P = C.c_void_p
_I64 = C.c_int64
_PD = C.POINTER(C.c_double)
_PI64 = C.POINTER(C.c_int64)

# name -> (restype, argtypes); every symbol include/polyclean.h declares.
SIGNATURES = {
    "pc_plan_footprint": (C.c_int, [C.POINTER(PcGeometry), C.POINTER(C.c_size_t)]),
    "pc_plan_create": (C.c_int, [C.POINTER(PcGeometry), _P, C.POINTER(_P)]),
    "pc_plan_destroy": (None, [_P]),
    "pc_device_pool_trim": (C.c_int, [C.c_int32, C.POINTER(C.c_size_t)]),
    "pc_plan_get_info": (C.c_int, [_P, C.POINTER(PcPlanInfo)]),
    "pc_last_error": (C.c_char_p, []),
    "pc_adjoint_grid": (C.c_int, [_P, _P, _P, _PD, _PI64, _P]),
    "pc_forward_sparse": (C.c_int, [_P, _I64, _P, _P, _P, _P]),
    "pc_forward_grid": (C.c_int, [_P, _P, _P, _P]),
    "pc_forward_grid_rows": (C.c_int, [_P, _P, _P, _P, _P]),
    "pc_adjoint_grid_rows": (C.c_int, [_P, _P, _P, _P, _P]),
    "pc_adjoint_sparse": (C.c_int, [_P, _P, _I64, _P, _P, _P]),
    "pc_dual_certificate": (C.c_int, [_P, _P, _I64, _P, _P, C.c_double, _P, _PD, _PI64, _P]),
    "pc_restricted_gradient": (C.c_int, [_P, _P, _I64, _P, _P, _P, _P, _P]),
    "pc_restricted_gradient_grid": (C.c_int, [_P, _P, _I64, _P, _P, _P, _P, _P]),
    "pc_restricted_gradient_noalloc": (C.c_int, [_P, _P, _I64, _P, _P, _P, _P, _P]),
    "pc_adjoint_grid_f64": (C.c_int, [_P, _P, _P, _PD, _PI64, _P]),
    "pc_adjoint_grid_ms": (C.c_int, [_P, _P, C.c_int32, _PD, _PD, _P, _PD, _PI64, _P]),
    "pc_forward_sparse_f64": (C.c_int, [_P, _I64, _P, _P, _P, _P]),
    "pc_adjoint_sparse_f64": (C.c_int, [_P, _P, _I64, _P, _P, _P]),
    "pc_dual_certificate_f64": (C.c_int, [_P, _P, _I64, _P, _P, C.c_double, _P, _PD, _PI64, _P]),
    "pc_adjoint_grid_batch": (C.c_int, [C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.c_int32,
                                        _PD, _PI64, _P]),
    "pc_solve_params_default": (None, [C.POINTER(PcSolveParams)]),
    "pc_polyclean_solve": (C.c_int, [_P, _P, C.POINTER(PcSolveParams),
                                     C.POINTER(PcSolveResult), _P]),
    "pc_solver_create": (C.c_int, [_P, _P, C.POINTER(PcSolveParams), _P, C.POINTER(_P)]),
    "pc_solver_step": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "pc_solver_result": (C.c_int, [_P, C.POINTER(PcSolveResult)]),
    "pc_solver_destroy": (None, [_P]),
    "pc_batcher_create": (C.c_int, [C.c_int32, C.POINTER(_P)]),
    "pc_batcher_get_stats": (C.c_int, [_P, C.POINTER(PcBatcherStats)]),
    "pc_batcher_destroy": (None, [_P]),
    "pc_solver_create_batched": (C.c_int, [_P, _P, C.POINTER(PcSolveParams), _P, _P,
                                           C.POINTER(_P)]),
    "pc_plan_profile": (C.c_int, [_P, C.c_int32]),
    "pc_plan_kernel_stat_count": (C.c_int32, [_P]),
    "pc_plan_kernel_stat": (C.c_int, [_P, C.c_int32, C.POINTER(PcKernelStat)]),
}

_lib = None


def load() -> C.CDLL:
    """Load libpolyclean.so and declare its functions; raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
            "(there is no fallback implementation)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PolycleanError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, fn: str) -> int:
    if status < 0:
        raise PolycleanError(status, fn, load().pc_last_error().decode())
    return status
