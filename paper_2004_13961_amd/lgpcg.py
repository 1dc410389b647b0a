"""ctypes binding of liblgpcg (include/lgpcg.h): argument marshalling only.

Every computation happens in the HIP library. PyTorch supplies device memory
(uint8 buffers sized by the library's size queries) and the current stream.
If the library has not been built this module raises at first use; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblgpcg.so")

LGP_F64, LGP_F32, LGP_BF16, LGP_F32_ONLY = 0, 1, 2, 3
DTYPES = {"f64": LGP_F64, "f32": LGP_F32, "bf16": LGP_BF16, "f32only": LGP_F32_ONLY}

STATUS = {
    0: "LGP_OK", 1: "LGP_E_ARG", 2: "LGP_E_NOMEM", 3: "LGP_E_COEF", 4: "LGP_E_ILU_PIVOT",
    5: "LGP_E_NOCONV", 6: "LGP_E_BREAKDOWN", 7: "LGP_E_HIP", 8: "LGP_E_UNSUPPORTED",
}

EXPORTS = [
    "lgp_version", "lgp_status_str", "lgp_last_hip_error", "lgp_gauss_legendre",
    "lgp_problem_bytes", "lgp_build_problem", "lgp_build_problem_diag", "lgp_destroy_problem", "lgp_load_vector",
    "lgp_matvec", "lgp_factor_bytes", "lgp_factor_M", "lgp_factor_bytes_dir", "lgp_factor_M_dir",
    "lgp_destroy_factor",
    "lgp_precond_apply", "lgp_ilu_forward", "lgp_ilu_backward", "lgp_factor_describe",
    "lgp_solve_workspace_bytes", "lgp_pcg_solve", "lgp_factor_const_bytes", "lgp_factor_const",
    "lgp_pcg_solve_noalloc_max_bytes", "lgp_pcg_solve_noalloc", "lgp_ilu_forward_f32", "lgp_ilu_backward_f32",
    "lgp_batch_workspace_bytes", "lgp_batch_create", "lgp_batch_add", "lgp_batch_step", "lgp_batch_info",
    "lgp_batch_remove", "lgp_batch_destroy", "lgp_pcg_solve_batched",
    "lgp_dlt_bytes", "lgp_dlt_create", "lgp_dlt_lines", "lgp_matvec_fast", "lgp_dlt_blocks", "lgp_dlt_destroy",
]


class LgpError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s" % (where, STATUS.get(status, status)))


class FactorDesc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("N", ctypes.c_int), ("n1", ctypes.c_int),
                ("Ta", ctypes.c_int), ("Tb", ctypes.c_int), ("n", ctypes.c_int64),
                ("noff", ctypes.c_int), ("n_lower", ctypes.c_int),
                ("offsets", ctypes.POINTER(ctypes.c_int)), ("L", ctypes.c_void_p),
                ("D", ctypes.c_void_p), ("levels", ctypes.c_int), ("ld", ctypes.c_int),
                ("factor_kernel_ms", ctypes.c_double), ("factor_kernel", ctypes.c_int),
                ("layout", ctypes.c_int), ("invD", ctypes.c_void_p),
                ("factor_launches", ctypes.c_int), ("factor_waits", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int), ("inner", ctypes.c_int),
                ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("check_every", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("relres_true", ctypes.c_double),
                ("relres_recursive", ctypes.c_double), ("status", ctypes.c_int)]


_lib = None


def lib():
    """Load the in-tree library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblgpcg.so is not built (run `python -m paper_2004_13961_amd.build`)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double)
    sig = {
        "lgp_version": (i32, []),
        "lgp_status_str": (ctypes.c_char_p, [i32]),
        "lgp_last_hip_error": (i32, []),
        "lgp_gauss_legendre": (i32, [i32, dp, dp]),
        "lgp_problem_bytes": (sz, [i32, i32]),
        "lgp_build_problem": (i32, [i32, i32, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]),
        "lgp_build_problem_diag": (i32, [i32, i32, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]),
        "lgp_destroy_problem": (None, [vp]),
        "lgp_load_vector": (i32, [vp, vp, vp, vp]),
        "lgp_matvec": (i32, [vp, vp, vp, i32, vp]),
        "lgp_factor_bytes": (sz, [vp, i32, i32, i32]),
        "lgp_factor_M": (i32, [vp, i32, i32, i32, vp, sz, vp, ctypes.POINTER(vp)]),
        "lgp_factor_bytes_dir": (sz, [vp, ctypes.POINTER(i32), i32, i32]),
        "lgp_factor_M_dir": (i32, [vp, ctypes.POINTER(i32), i32, i32, vp, sz, vp, ctypes.POINTER(vp)]),
        "lgp_destroy_factor": (None, [vp]),
        "lgp_factor_const_bytes": (sz, [vp]),
        "lgp_factor_const": (i32, [vp, vp, sz, vp, ctypes.POINTER(vp)]),
        "lgp_precond_apply": (i32, [vp, vp, vp, vp]),
        "lgp_ilu_forward": (i32, [vp, vp, vp, vp]),
        "lgp_ilu_backward": (i32, [vp, vp, vp, vp]),
        "lgp_ilu_forward_f32": (i32, [vp, vp, vp, vp]),
        "lgp_batch_workspace_bytes": (sz, [vp, i32]),
        "lgp_batch_create": (i32, [vp, i32, vp, sz, vp, ctypes.POINTER(vp)]),
        "lgp_batch_add": (i32, [vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(i32)]),
        "lgp_batch_step": (i32, [vp, i32, ctypes.POINTER(i32)]),
        "lgp_batch_info": (i32, [vp, i32, ctypes.POINTER(SolveInfo), ctypes.POINTER(i32)]),
        "lgp_batch_remove": (i32, [vp, i32]),
        "lgp_batch_destroy": (None, [vp]),
        "lgp_pcg_solve_batched": (i32, [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), ctypes.POINTER(SolveOpts), vp, sz, vp,
                                        ctypes.POINTER(SolveInfo)]),
        "lgp_ilu_backward_f32": (i32, [vp, vp, vp, vp]),
        "lgp_factor_describe": (i32, [vp, ctypes.POINTER(FactorDesc)]),
        "lgp_solve_workspace_bytes": (sz, [vp, i32]),
        "lgp_pcg_solve": (i32, [vp, vp, vp, vp, ctypes.POINTER(SolveOpts), vp, sz, vp,
                                ctypes.POINTER(SolveInfo)]),
        "lgp_pcg_solve_noalloc_max_bytes": (sz, []),
        "lgp_dlt_bytes": (sz, [vp]),
        "lgp_dlt_create": (i32, [vp, vp, sz, vp, ctypes.POINTER(vp)]),
        "lgp_dlt_lines": (i32, [vp, i32, i64, vp, vp, vp]),
        "lgp_matvec_fast": (i32, [vp, vp, vp, vp]),
        "lgp_dlt_blocks": (i32, [vp]),
        "lgp_dlt_destroy": (None, [vp]),
        "lgp_pcg_solve_noalloc": (i32, [vp, vp, vp, vp, ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveInfo)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status: int, where: str):
    if status != 0:
        raise LgpError(status, where)


def gauss_legendre(N: int):
    """Library nodes and weights (host computation, no GPU needed)."""
    x = np.zeros(N + 1)
    w = np.zeros(N + 1)
    check(lib().lgp_gauss_legendre(N, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "lgp_gauss_legendre")
    return x, w
