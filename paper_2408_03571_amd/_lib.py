"""ctypes binding of libhelmschwarz (include/helmschwarz.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Device buffers are torch tensors (complex128, CUDA/ROCm device, contiguous);
their data_ptr() and torch's current stream are handed to the C ABI.  If the
library is not built, loading raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhelmschwarz.so")

HS_OK, HS_EINVAL, HS_ENOMEM, HS_ESINGULAR, HS_ENOCONV, HS_ENAN, HS_EHIP = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "HS_OK", -1: "HS_EINVAL", -2: "HS_ENOMEM", -3: "HS_ESINGULAR", -4: "HS_ENOCONV",
                -5: "HS_ENAN", -6: "HS_EHIP"}
HS_BC_DIRICHLET, HS_BC_SOMMERFELD = 0, 1
HS_AS2, HS_RAS2, HS_SHS2 = 0, 1, 2
HS_C128, HS_C64, HS_C64X, HS_C64S = 0, 1, 2, 3
HS_ORTHO_DCGS2, HS_ORTHO_MGS = 0, 1
HS_COARSE_BEZIER, HS_COARSE_P1 = 0, 1

c_void_p = ctypes.c_void_p
c_int = ctypes.c_int
c_double = ctypes.c_double
c_int64 = ctypes.c_int64
c_size_t = ctypes.c_size_t


class GmresStats(ctypes.Structure):
    _fields_ = [("iters", c_int), ("converged", c_int), ("relres_implicit", c_double),
                ("relres_true", c_double), ("ms_solve", c_double), ("steps", c_int), ("host_checks", c_int)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("ortho", c_int), ("graph", c_int), ("check_every", c_int), ("basis_prec", c_int)]


class PrecondInfo(ctypes.Structure):
    _fields_ = [("n_fine", c_int64), ("n_coarse", c_int64), ("coarse_per_dim", c_int),
                ("coarse_reach", c_int), ("nsub_total", c_int), ("local_total", c_int64),
                ("local_factor_bytes", c_int64), ("coarse_factor_bytes", c_int64),
                ("nd_fronts", c_int), ("nd_levels", c_int), ("ms_setup_local", c_double),
                ("ms_setup_coarse", c_double), ("coarse_solve_bytes", c_int64), ("coarse_basis", c_int),
                ("workspace_bytes", c_int64), ("setup_scratch_bytes", c_int64), ("apply_work_bytes", c_int64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "hs_assemble": (c_int, [c_int, c_double, c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    "hs_problem_size": (c_int64, [c_void_p]),
    "hs_spmv": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hs_schwarz_workspace_bytes": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, ctypes.POINTER(c_size_t)]),
    "hs_schwarz_workspace_bytes_ex": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_int, c_int,
                                              ctypes.POINTER(c_size_t)]),
    "hs_setup_schwarz": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_int, c_void_p, c_size_t, c_void_p,
                                 ctypes.POINTER(c_void_p)]),
    "hs_setup_schwarz_ex": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_void_p, c_size_t,
                                    c_void_p, ctypes.POINTER(c_void_p)]),
    "hs_apply_Minv": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hs_apply_Minv_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hs_precond_set_schedule": (c_int, [c_void_p, c_int, c_int]),
    "hs_precond_get_schedule": (c_int, [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "hs_gmres_workspace_bytes": (c_int, [c_void_p, c_int, ctypes.POINTER(c_size_t)]),
    "hs_gmres_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int, c_void_p,
                               c_size_t, c_void_p, c_void_p, ctypes.POINTER(GmresStats)]),
    "hs_gmres_solve_ex": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int,
                                  ctypes.POINTER(GmresOpts), c_void_p, c_size_t, c_void_p, c_void_p,
                                  ctypes.POINTER(GmresStats)]),
    "hs_set_arnoldi_config": (c_int, [c_int64, c_int, c_int]),
    "hs_batch_workspace_bytes": (c_int, [c_int, ctypes.POINTER(c_void_p), ctypes.POINTER(c_size_t)]),
    "hs_batch_create": (c_int, [c_int, ctypes.POINTER(c_void_p), c_void_p, c_size_t, ctypes.POINTER(c_void_p)]),
    "hs_batch_destroy": (None, [c_void_p]),
    "hs_batch_offsets": (c_int, [c_void_p, ctypes.POINTER(c_int64)]),
    "hs_batch_apply_Minv": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hs_batch_set_local_grid": (c_int, [c_void_p, c_int]),
    "hs_batch_set_schedule": (c_int, [c_void_p, c_int, c_int]),
    "hs_batch_time": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int, c_void_p, ctypes.POINTER(c_double)]),
    "hs_batch_gmres_workspace_bytes": (c_int, [c_void_p, c_int, ctypes.POINTER(c_size_t)]),
    "hs_batch_gmres_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, ctypes.POINTER(GmresOpts),
                                     c_void_p, c_size_t, c_void_p, ctypes.POINTER(GmresStats)]),
    "hs_gmres_batch_workspace_bytes": (c_int, [c_int, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_int,
                                               ctypes.POINTER(c_size_t)]),
    "hs_gmres_solve_batch": (c_int, [c_int, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                     ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_double, c_int, c_void_p,
                                     c_size_t, c_void_p, ctypes.POINTER(GmresStats)]),
    "hs_get_arnoldi_config": (c_int, [c_int64, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "hs_time_arnoldi": (c_int, [c_void_p, c_int, c_int, c_void_p, c_size_t, c_void_p, c_int, c_void_p,
                                ctypes.POINTER(c_double)]),
    "hs_time_arnoldi_ex": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_size_t, c_void_p, c_int, c_void_p,
                                   ctypes.POINTER(c_double)]),
    "hs_precond_get_info": (c_int, [c_void_p, ctypes.POINTER(PrecondInfo)]),
    "hs_coarse_restrict": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hs_coarse_prolong": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hs_coarse_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hs_coarse_matrix": (c_int, [c_void_p, c_void_p, c_void_p]),
    "hs_local_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hs_time_step": (c_int, [c_void_p, c_int, c_void_p, c_int, c_void_p, ctypes.POINTER(c_double)]),
    "hs_k2_gradient": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p]),
    "hs_nd_plan_check": (c_int, [c_int, c_int, c_int, c_int, ctypes.POINTER(c_int64)]),
    "hs_nd_level_stats": (c_int, [c_void_p, c_int, ctypes.POINTER(c_int64)]),
    "hs_nd_plan_level_stats": (c_int, [c_int, c_int, c_int, c_int, c_int, ctypes.POINTER(c_int64)]),
    "hs_destroy_problem": (None, [c_void_p]),
    "hs_destroy_precond": (None, [c_void_p]),
    "hs_last_error": (ctypes.c_char_p, []),
}

_lib = None


class HSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libhelmschwarz.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2408_03571_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, allow=()):
    if status != HS_OK and status not in allow:
        raise HSError(status, load().hs_last_error().decode())
    return status
