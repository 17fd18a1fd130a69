"""ctypes binding of the C ABI in include/amp_pcg.h (argument marshalling only).

Every numerical step runs in the HIP library; this module only passes
device pointers, sizes and the current torch stream across the boundary.
It fails loudly when the library cannot be loaded: there is no CPU path.
"""

from __future__ import annotations

import ctypes
import os
import threading

from . import build as _build

AMP_OK, AMP_ERR_ARG, AMP_ERR_NOT_CONVERGED, AMP_ERR_BREAKDOWN, AMP_ERR_HIP, AMP_ERR_OOM = range(6)
PC_IDENTITY, PC_JACOBI, PC_CHEBYSHEV = 0, 1, 2
ETA_MODES = {"delay": 0, "linear": 1, "fixed64": 2, "fixed32": 3}
SCALINGS = {"pow2": 0, "paper": 1, "none": 2}
PRESETS = {"pcg64": 0, "amp64": 1, "amp16": 2, "amp_ur": 3}

EXPORTED = [
    "amp_version", "amp_status_string", "amp_last_error", "amp_options_default",
    "amp_options_preset", "amp_matrix_create", "amp_matrix_create_ex", "amp_matrix_destroy", "amp_matrix_info",
    "amp_precond_create", "amp_precond_destroy", "amp_pcg_solve", "amp_spmv", "amp_spmv_step",
    "amp_precond_apply", "amp_selector_replay", "amp_paper_kernel_bytes",
    "amp_matrix_update_values", "amp_precond_update", "amp_fv_nnz", "amp_fv_csr", "amp_fv_grad_theta",
    "amp_pcg_solve_batched", "amp_tune_group_rows", "amp_pcg_solve_noalloc", "amp_stream_probe",
    "amp_set_allocator", "amp_precond_bounds", "amp_matrix_tuning_default", "amp_tune_lanes",
    "amp_hexop_create", "amp_hexop_destroy", "amp_hexop_info", "amp_hexop_apply", "amp_hexop_diagonal",
    "amp_matrix_from_hexop", "amp_pmg_params_default", "amp_precond_create_pmg", "amp_pmg_info", "amp_pmg_apply",
]

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("u0", ctypes.c_int), ("tau_zs", ctypes.c_double), ("tau_zh", ctypes.c_double),
                ("eta_mode", ctypes.c_int), ("d", ctypes.c_int), ("C", ctypes.c_double),
                ("ell", ctypes.c_int), ("scaling", ctypes.c_int), ("T_z", ctypes.c_int),
                ("T_p", ctypes.c_int), ("spmv32_diff", ctypes.c_int), ("verify", ctypes.c_int),
                ("max_replacements", ctypes.c_int), ("rr_period", ctypes.c_int),
                ("batch", ctypes.c_int), ("group_rows", ctypes.c_int), ("graph", ctypes.c_int),
                ("solo_rows", ctypes.c_int), ("spmv_timing", ctypes.c_int), ("defer_x", ctypes.c_int),
                ("delta_history", ctypes.c_void_p),
                ("prec_history", ctypes.c_void_p), ("scalar_history", ctypes.c_void_p),
                ("rr_switch", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_res_updated", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("k_z32", ctypes.c_int), ("k_z16", ctypes.c_int),
                ("k_r32", ctypes.c_int), ("n_replacements", ctypes.c_int),
                ("t_solve_ms", ctypes.c_double), ("spmv_ms", ctypes.c_double), ("spmv_launches", ctypes.c_int),
                ("cheb_ms", ctypes.c_double), ("cheb_launches", ctypes.c_int)]


class MatrixStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("n", "nnz", "slots", "bytes", "nslices", "offset_slices", "meta_bytes", "lanes_per_row")]


class HexStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("elements", ctypes.c_int64), ("local", ctypes.c_int64),
                ("order", ctypes.c_int), ("lambda_", ctypes.c_double), ("flops_per_element", ctypes.c_double)]


class MatrixTuning(ctypes.Structure):
    _fields_ = [("lanes_per_row", ctypes.c_int), ("offset_mode", ctypes.c_int)]


class PmgParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("orders", ctypes.c_int * 4), ("degree", ctypes.c_int),
                ("coarse_degree", ctypes.c_int), ("lo_ratio", ctypes.c_double), ("hi_margin", ctypes.c_double),
                ("coarse_lo_ratio", ctypes.c_double), ("rho", ctypes.c_double * 4), ("power_iters", ctypes.c_int)]


class PmgStats(ctypes.Structure):
    _fields_ = [("params", PmgParams), ("gain", ctypes.c_double), ("n", ctypes.c_int64 * 4),
                ("bytes", ctypes.c_int64)]


_lib = None
_lock = threading.Lock()


class AmpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


def library_path() -> str:
    return _build.LIB


def load(build_if_missing: bool = True):
    """Load libamppcg.so (building it once if nothing is built yet)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = _build.LIB
        if not os.path.exists(path):
            if not build_if_missing:
                raise RuntimeError(f"HIP library not built: {path}")
            _build.build()
        L = ctypes.CDLL(path)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.amp_version.restype = i32
        L.amp_status_string.argtypes = [i32]
        L.amp_status_string.restype = ctypes.c_char_p
        L.amp_last_error.restype = ctypes.c_char_p
        L.amp_options_default.argtypes = [ctypes.POINTER(Options)]
        L.amp_options_default.restype = None
        L.amp_options_preset.argtypes = [ctypes.POINTER(Options), i32]
        L.amp_matrix_create.argtypes = [ctypes.POINTER(Csr), ctypes.POINTER(MatrixTuning), vp, ctypes.POINTER(vp)]
        L.amp_hexop_create.argtypes = [i32, i32, i32, i32, vp, dbl, vp, ctypes.POINTER(vp)]
        L.amp_hexop_destroy.argtypes = [vp]
        L.amp_hexop_destroy.restype = None
        L.amp_hexop_info.argtypes = [vp, ctypes.POINTER(HexStats)]
        L.amp_hexop_apply.argtypes = [vp, i32, i32, vp, vp, vp, vp]
        L.amp_hexop_diagonal.argtypes = [vp, vp, vp]
        L.amp_matrix_from_hexop.argtypes = [vp, vp, ctypes.POINTER(vp)]
        L.amp_pmg_params_default.argtypes = [ctypes.POINTER(PmgParams)]
        L.amp_pmg_params_default.restype = None
        L.amp_precond_create_pmg.argtypes = [vp, ctypes.POINTER(PmgParams), vp, ctypes.POINTER(vp)]
        L.amp_pmg_info.argtypes = [vp, ctypes.POINTER(PmgStats)]
        L.amp_pmg_apply.argtypes = [vp, vp, vp, i32, vp]
        L.amp_matrix_tuning_default.argtypes = [ctypes.POINTER(MatrixTuning)]
        L.amp_matrix_tuning_default.restype = None
        L.amp_tune_lanes.argtypes = [ctypes.POINTER(Csr), ctypes.POINTER(i32), i32, i32, ctypes.POINTER(i32),
                                     ctypes.POINTER(dbl), vp]
        L.amp_matrix_create_ex.argtypes = [ctypes.POINTER(Csr), i32, vp, ctypes.POINTER(vp)]
        L.amp_matrix_destroy.argtypes = [vp]
        L.amp_matrix_destroy.restype = None
        L.amp_matrix_info.argtypes = [vp, ctypes.POINTER(MatrixStats)]
        L.amp_precond_create.argtypes = [vp, i32, i32, dbl, dbl, vp, ctypes.POINTER(vp)]
        L.amp_precond_destroy.argtypes = [vp]
        L.amp_precond_destroy.restype = None
        L.amp_pcg_solve.argtypes = [vp, vp, vp, vp, dbl, i32, ctypes.POINTER(Options),
                                    ctypes.POINTER(Result), vp]
        L.amp_stream_probe.argtypes = [i32, vp, vp, i64, vp]
        L.amp_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
        L.amp_precond_bounds.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                         ctypes.POINTER(dbl)]
        L.amp_pcg_solve_noalloc.argtypes = [vp, vp, vp, vp, dbl, i32, ctypes.POINTER(Options),
                                            ctypes.POINTER(Result), vp]
        L.amp_pcg_solve_batched.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                            ctypes.POINTER(vp), ctypes.POINTER(dbl), i32,
                                            ctypes.POINTER(Options), ctypes.POINTER(Result), vp]
        L.amp_tune_group_rows.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                          ctypes.POINTER(vp), ctypes.POINTER(dbl), i32, ctypes.POINTER(i32), i32,
                                          ctypes.POINTER(Options), ctypes.POINTER(i32), ctypes.POINTER(dbl), vp]
        L.amp_spmv.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
        L.amp_spmv_step.argtypes = [vp, i32, i32, i32, dbl, vp]
        L.amp_precond_apply.argtypes = [vp, i32, i32, vp, dbl, vp, vp, vp]
        L.amp_selector_replay.argtypes = [ctypes.POINTER(dbl), i32, dbl, dbl, ctypes.POINTER(Options),
                                          ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.amp_paper_kernel_bytes.argtypes = [i32, i32, ctypes.POINTER(dbl)]
        L.amp_matrix_update_values.argtypes = [vp, ctypes.POINTER(Csr), vp]
        L.amp_precond_update.argtypes = [vp, vp]
        L.amp_fv_nnz.argtypes = [i32, i32, i32, i32, ctypes.POINTER(i64)]
        L.amp_fv_csr.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp]
        L.amp_fv_grad_theta.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp]
        for name in EXPORTED:
            if not hasattr(L, name):
                raise RuntimeError(f"{path} does not export {name}")
        _lib = L
        return L


def status_name(s: int) -> str:
    L = _lib
    if L is None:
        return str(s)
    return L.amp_status_string(int(s)).decode()


def last_error() -> str:
    return load().amp_last_error().decode()


def check(status: int, what: str = ""):
    if status != AMP_OK:
        raise AmpError(status, f"{what}: {last_error()}")


def make_options(preset: str = "amp64", **kw) -> Options:
    L = load()
    o = Options()
    check(L.amp_options_preset(ctypes.byref(o), PRESETS[preset]), "amp_options_preset")
    for k, v in kw.items():
        if k == "eta":
            o.eta_mode = ETA_MODES[v]
        elif k == "scaling":
            o.scaling = SCALINGS[v]
        elif k == "spmv32":
            o.spmv32_diff = 1 if v == "diff" else 0
        elif k == "tau_zs" or k == "tau_zh" or k == "C":
            setattr(o, k, float(v))
        elif hasattr(o, k) and k not in ("delta_history", "prec_history", "scalar_history"):
            setattr(o, k, int(v))
        else:
            raise KeyError(f"unknown option {k}")
    return o
