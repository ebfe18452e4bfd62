"""MI355X-native two-level Schwarz / Bezier coarse-space GMRES solver for the
2-D Helmholtz equation (arXiv 2408.03571), behind the C ABI of
include/helmschwarz.h.

The functions below carry the names of the C entry points and only marshal
arguments: torch tensors supply device memory, torch's current stream is the
HIP stream.  Nothing here computes; if libhelmschwarz.so is missing every call
raises.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (HS_AS2, HS_BC_DIRICHLET, HS_BC_SOMMERFELD, HS_C64, HS_C64S, HS_C64X, HS_C128, HS_COARSE_BEZIER,
                   HS_COARSE_P1, HS_EHIP, HS_EINVAL, HS_ENAN, HS_ENOCONV, HS_ENOMEM,
                   HS_ESINGULAR, HS_OK, HS_ORTHO_DCGS2, HS_ORTHO_MGS, HS_RAS2, HS_SHS2, GmresOpts, GmresStats, HSError,
                   PrecondInfo)

__all__ = [
    "Problem", "Precond", "hs_assemble", "hs_problem_size", "hs_spmv", "hs_setup_schwarz", "hs_setup_schwarz_ex",
    "hs_apply_Minv", "hs_apply_Minv_noalloc", "hs_nd_level_stats", "hs_nd_plan_level_stats", "hs_schwarz_workspace_bytes",
    "hs_batch_workspace_bytes", "hs_batch_gmres_solve", "hs_gmres_batch_workspace_bytes", "hs_precond_set_schedule", "hs_precond_get_schedule",
    "hs_gmres_workspace_bytes", "hs_gmres_solve", "hs_precond_get_info", "hs_coarse_restrict",
    "hs_coarse_prolong", "hs_coarse_solve", "hs_coarse_matrix", "hs_local_solve", "hs_nd_plan_check",
    "Batch", "hs_batch_create", "hs_batch_apply_Minv", "hs_batch_gmres_workspace_bytes", "hs_gmres_solve_batch", "hs_batch_time", "hs_batch_set_local_grid", "hs_batch_set_schedule",
    "hs_time_step", "hs_time_arnoldi", "hs_time_arnoldi_ex", "hs_set_arnoldi_config", "hs_get_arnoldi_config", "hs_k2_gradient", "HelmholtzSolve", "helmholtz_solve",
    "HelmholtzSolveMulti", "helmholtz_solve_multi",
    "HS_BC_DIRICHLET", "HS_BC_SOMMERFELD", "HS_AS2", "HS_RAS2", "HS_SHS2", "HS_C128", "HS_C64", "HS_C64X", "HS_C64S", "HS_ORTHO_DCGS2",
    "HS_ORTHO_MGS", "HS_COARSE_BEZIER", "HS_COARSE_P1", "HSError", "HS_ENAN", "HS_ENOMEM", "HS_EHIP",
]


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype_name="complex128"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"tensor must be {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.is_conj() or t.is_neg():
        # a lazy conjugate / negative view: the memory holds the unresolved values
        raise ValueError("tensor is a lazy conj/neg view; call resolve_conj()/resolve_neg() first")
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """Owning wrapper of an hs_problem handle (keeps the k^2 field alive)."""

    def __init__(self, handle, n, k, bc, k2):
        self.handle = handle
        self.n, self.k, self.bc, self.k2 = n, k, bc, k2
        self.size = _lib.load().hs_problem_size(handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        self.handle = None
        if h and _lib is not None and _lib._lib is not None:
            _lib._lib.hs_destroy_problem(h)


def _workspace(nbytes: int, device):
    """A caller-owned device workspace (torch uint8, 256-byte aligned)."""
    import torch
    ws = torch.empty(max(1, int(nbytes)) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(1, int(nbytes))]


def _device(stream=None):
    import torch
    return torch.device("cuda", torch.cuda.current_device())


class Precond:
    """Owning wrapper of an hs_precond handle and of the workspace it lives in."""

    def __init__(self, handle, problem, ws=None):
        self.handle = handle
        self.problem = problem
        self.ws = ws

    def __del__(self):
        h = getattr(self, "handle", None)
        self.handle = None
        if h and _lib is not None and _lib._lib is not None:
            _lib._lib.hs_destroy_precond(h)
        self.ws = None


class Batch:
    """Handle of hs_batch_create; keeps its preconditioners and workspace alive."""

    def __init__(self, handle, precs, offsets, ws=None):
        self.handle = handle
        self.precs = precs
        self.offsets = offsets
        self.ws = ws

    def __del__(self):
        h = getattr(self, "handle", None)
        self.handle = None
        if h and _lib is not None and _lib._lib is not None:
            _lib._lib.hs_batch_destroy(h)
        self.ws = None


def hs_batch_workspace_bytes(precs) -> int:
    lib = _lib.load()
    arr = (ctypes.c_void_p * len(precs))(*[M.handle for M in precs])
    nb = ctypes.c_size_t()
    _lib.check(lib.hs_batch_workspace_bytes(len(precs), arr, ctypes.byref(nb)))
    return int(nb.value)


def hs_batch_create(precs, ws=None) -> Batch:
    """Group preconditioners into one batch (all share variant and prec); its
    tables live in a workspace of hs_batch_workspace_bytes (allocated here
    when ws is None)."""
    lib = _lib.load()
    arr = (ctypes.c_void_p * len(precs))(*[M.handle for M in precs])
    nbytes = hs_batch_workspace_bytes(precs)
    if ws is None:
        ws = _workspace(nbytes, _device())
    out = ctypes.c_void_p()
    _lib.check(lib.hs_batch_create(len(precs), arr, ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                   ctypes.byref(out)))
    offs = (ctypes.c_int64 * (len(precs) + 1))()
    _lib.check(lib.hs_batch_offsets(out, offs))
    return Batch(out, list(precs), list(offs), ws)


def hs_batch_apply_Minv(B: Batch, r, z, stream=None):
    _lib.check(_lib.load().hs_batch_apply_Minv(B.handle, _ptr(r), _ptr(z), _stream(stream)))


def hs_batch_set_schedule(B: Batch, fork_level: int, local_grid: int = 0):
    """Fork the batched local solves after fork_level forward coarse levels,
    in local_grid persistent workgroups (0 = one per subdomain)."""
    _lib.check(_lib.load().hs_batch_set_schedule(B.handle, int(fork_level), int(local_grid)))


def hs_batch_set_local_grid(B: Batch, grid: int):
    """Workgroups of the persistent batched local-solve launch (0 = one per subdomain)."""
    _lib.check(_lib.load().hs_batch_set_local_grid(B.handle, int(grid)))


def hs_batch_time(B: Batch, which: int, r, reps: int = 10, stream=None, z=None) -> float:
    """Mean ms of one batched step (0 local solves, 1 coarse chain, 2 whole
    application, 3 restriction stages, 4 nested-dissection solves); the
    whole application writes z (a batch vector, allocated here if None)."""
    import torch
    if which == 2 and z is None:
        z = torch.empty_like(r)
    ms = ctypes.c_double()
    _lib.check(_lib.load().hs_batch_time(B.handle, int(which), _ptr(r), _ptr(z) if z is not None else None,
                                         int(reps), _stream(stream), ctypes.byref(ms)))
    return float(ms.value)


def hs_batch_gmres_workspace_bytes(B: Batch, maxit: int) -> int:
    nb = ctypes.c_size_t()
    _lib.check(_lib.load().hs_batch_gmres_workspace_bytes(B.handle, int(maxit), ctypes.byref(nb)))
    return int(nb.value)


def hs_batch_gmres_solve(B: Batch, b, x, tol: float = 1e-6, maxit: int = 200, ws=None, stream=None,
                         graph: bool = True, check_every: int = 0, raise_on_noconv: bool = False,
                         basis_prec: int = HS_C128):
    """Flexible GMRES on every instance of the batch (batch vectors b, x).
    Returns a list of per-instance stats dicts."""
    import torch
    lib = _lib.load()
    nbytes = hs_batch_gmres_workspace_bytes(B, maxit)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    if ws.numel() * ws.element_size() < nbytes:
        raise ValueError("workspace too small")
    count = len(B.precs)
    st = (GmresStats * count)()
    opts = GmresOpts(HS_ORTHO_DCGS2, 1 if graph else 0, int(check_every), int(basis_prec))
    status = lib.hs_batch_gmres_solve(B.handle, _ptr(b), _ptr(x), float(tol), int(maxit), ctypes.byref(opts),
                                      ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(nbytes), _stream(stream), st)
    _lib.check(status, allow=() if raise_on_noconv else (HS_ENOCONV,))
    return [{"iters": s.iters, "converged": bool(s.converged), "relres_implicit": s.relres_implicit,
             "relres_true": s.relres_true, "ms_solve": s.ms_solve, "steps": s.steps,
             "host_checks": s.host_checks, "status": status} for s in st]



def hs_gmres_batch_workspace_bytes(problems, precs, maxit: int) -> int:
    lib = _lib.load()
    n = len(precs)
    Pa = (ctypes.c_void_p * n)(*[P.handle for P in problems])
    Ma = (ctypes.c_void_p * n)(*[M.handle for M in precs])
    nb = ctypes.c_size_t()
    _lib.check(lib.hs_gmres_batch_workspace_bytes(n, Pa, Ma, int(maxit), ctypes.byref(nb)))
    return int(nb.value)


def hs_gmres_solve_batch(problems, precs, bs, xs, tol: float = 1e-6, maxit: int = 200, ws=None, stream=None,
                         raise_on_noconv: bool = False):
    """Flexible GMRES on several instances given as plain lists (one right-
    hand side and one solution tensor per instance), through the one call
    hs_gmres_solve_batch: the batch's tables, its GMRES workspace and the
    concatenated vectors all live in ws.  Returns per-instance stats dicts."""
    lib = _lib.load()
    n = len(precs)
    nbytes = hs_gmres_batch_workspace_bytes(problems, precs, maxit)
    if ws is None:
        ws = _workspace(nbytes, bs[0].device)
    Pa = (ctypes.c_void_p * n)(*[P.handle for P in problems])
    Ma = (ctypes.c_void_p * n)(*[M.handle for M in precs])
    ba = (ctypes.c_void_p * n)(*[_ptr(b).value for b in bs])
    xa = (ctypes.c_void_p * n)(*[_ptr(x).value for x in xs])
    st = (GmresStats * n)()
    status = lib.hs_gmres_solve_batch(n, Pa, Ma, ba, xa, float(tol), int(maxit), ctypes.c_void_p(ws.data_ptr()),
                                      ctypes.c_size_t(ws.numel()), _stream(stream), st)
    _lib.check(status, allow=() if raise_on_noconv else (HS_ENOCONV,))
    return [{"iters": s_.iters, "converged": bool(s_.converged), "relres_implicit": s_.relres_implicit,
             "relres_true": s_.relres_true, "ms_solve": s_.ms_solve, "steps": s_.steps,
             "host_checks": s_.host_checks, "status": status} for s_ in st]

def hs_assemble(n: int, k: float, bc: int, k2=None) -> Problem:
    """Sec. 2: the five-point MP-1 / MP-2 operator (generated on the fly)."""
    lib = _lib.load()
    out = ctypes.c_void_p()
    k2p = _ptr(k2, "float64") if k2 is not None else None
    _lib.check(lib.hs_assemble(int(n), float(k), int(bc), k2p, ctypes.byref(out)))
    return Problem(out, n, k, bc, k2)


def hs_problem_size(P: Problem) -> int:
    return int(_lib.load().hs_problem_size(P.handle))


def hs_spmv(P: Problem, x, y, stream=None):
    _lib.check(_lib.load().hs_spmv(P.handle, _ptr(x), _ptr(y), _stream(stream)))


def _nsub_xy(nsub):
    return (int(nsub), int(nsub)) if isinstance(nsub, int) else (int(nsub[0]), int(nsub[1]))


def hs_schwarz_workspace_bytes(P: Problem, nsub, overlap: int = 2, ratio: int = 2, prec: int = HS_C128,
                               variant: int = None, basis: int = None) -> int:
    """Device bytes a preconditioner needs (nsub: int or (nsub_x, nsub_y)).
    With variant and basis the exact figure (hs_schwarz_workspace_bytes_ex),
    else the largest over them."""
    lib = _lib.load()
    nsx, nsy = _nsub_xy(nsub)
    nb = ctypes.c_size_t()
    if variant is None and basis is None:
        _lib.check(lib.hs_schwarz_workspace_bytes(P.handle, nsx, nsy, int(overlap), int(ratio), int(prec),
                                                  ctypes.byref(nb)))
    else:
        _lib.check(lib.hs_schwarz_workspace_bytes_ex(
            P.handle, nsx, nsy, int(overlap), int(ratio), int(HS_RAS2 if variant is None else variant), int(prec),
            int(HS_COARSE_BEZIER if basis is None else basis), ctypes.byref(nb)))
    return int(nb.value)


def hs_setup_schwarz(P: Problem, nsub, overlap: int = 2, ratio: int = 2, variant: int = HS_RAS2,
                     prec: int = HS_C128, stream=None, basis: int = HS_COARSE_BEZIER, ws=None) -> Precond:
    """Sec. 3-4: the two-level preconditioner (nsub: subdomains per dimension,
    or (nsub_x, nsub_y)).  Its factors and scratch live in a caller-owned
    workspace, a torch uint8 tensor allocated here when ws is None."""
    lib = _lib.load()
    nsx, nsy = _nsub_xy(nsub)
    nbytes = hs_schwarz_workspace_bytes(P, (nsx, nsy), overlap, ratio, prec, variant, basis)
    if ws is None:
        ws = _workspace(nbytes, _device())
    out = ctypes.c_void_p()
    _lib.check(lib.hs_setup_schwarz_ex(P.handle, nsx, nsy, int(overlap), int(ratio), int(variant), int(prec),
                                       int(basis), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                       _stream(stream), ctypes.byref(out)))
    return Precond(out, P, ws)


def hs_setup_schwarz_ex(P: Problem, nsub, overlap: int, ratio: int, variant: int, prec: int, basis: int,
                        stream=None, ws=None) -> Precond:
    return hs_setup_schwarz(P, nsub, overlap, ratio, variant, prec, stream=stream, basis=basis, ws=ws)


def hs_apply_Minv(M: Precond, r, z, stream=None):
    _lib.check(_lib.load().hs_apply_Minv(M.handle, _ptr(r), _ptr(z), _stream(stream)))


def hs_apply_Minv_noalloc(M: Precond, r, z, stream=None):
    """z = M^{-1} r through the library's static scratch array (no allocation)."""
    _lib.check(_lib.load().hs_apply_Minv_noalloc(M.handle, _ptr(r), _ptr(z), _stream(stream)))


def hs_gmres_workspace_bytes(P: Problem, maxit: int) -> int:
    n = ctypes.c_size_t()
    _lib.check(_lib.load().hs_gmres_workspace_bytes(P.handle, int(maxit), ctypes.byref(n)))
    return int(n.value)


def hs_gmres_solve(P: Problem, M: Precond, b, x, tol: float = 1e-6, maxit: int = 200, ws=None,
                   history: bool = True, stream=None, raise_on_noconv: bool = False,
                   ortho: int = HS_ORTHO_DCGS2, graph: bool = True, check_every: int = 0,
                   basis_prec: int = HS_C128):
    """Flexible GMRES (Sec. 5) through hs_gmres_solve_ex.  Returns (stats
    dict, history list).  basis_prec = HS_C64 stores the Krylov basis in
    complex64 (hs_gmres_opts.basis_prec)."""
    import torch
    lib = _lib.load()
    nbytes = hs_gmres_workspace_bytes(P, maxit)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    if ws.numel() * ws.element_size() < nbytes:
        raise ValueError("workspace too small")
    hist = (ctypes.c_double * (maxit + 1))() if history else None
    st = GmresStats()
    opts = GmresOpts(int(ortho), 1 if graph else 0, int(check_every), int(basis_prec))
    status = lib.hs_gmres_solve_ex(P.handle, M.handle, _ptr(b), _ptr(x), float(tol), int(maxit),
                                   ctypes.byref(opts), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(nbytes),
                                   ctypes.cast(hist, ctypes.c_void_p) if hist is not None else None,
                                   _stream(stream), ctypes.byref(st))
    _lib.check(status, allow=() if raise_on_noconv else (HS_ENOCONV,))
    stats = {"iters": st.iters, "converged": bool(st.converged), "relres_implicit": st.relres_implicit,
             "relres_true": st.relres_true, "ms_solve": st.ms_solve, "steps": st.steps,
             "host_checks": st.host_checks, "status": status}
    h = list(hist[: st.iters + 1]) if hist is not None else None
    return stats, h


def hs_set_arnoldi_config(n_unknowns: int, ept: int, rows: int):
    """Launch shape of the DCGS2 passes for problems of n_unknowns unknowns
    (ept in 1, 2, 4, 8; rows in 2, 4; both 0 = built-in)."""
    _lib.check(_lib.load().hs_set_arnoldi_config(int(n_unknowns), int(ept), int(rows)))


def hs_get_arnoldi_config(n_unknowns: int):
    e, r = ctypes.c_int(), ctypes.c_int()
    _lib.check(_lib.load().hs_get_arnoldi_config(int(n_unknowns), ctypes.byref(e), ctypes.byref(r)))
    return e.value, r.value


def hs_time_arnoldi(P: Problem, k: int, which: int, ws, r, reps: int = 10, stream=None,
                    basis_prec: int = HS_C128) -> float:
    """Mean ms per launch of a DCGS2 pass at Arnoldi step k (0 dot pass,
    1 update pass, 2 fold + Hessenberg column + scale) with the basis stored
    as basis_prec; ws sized by hs_gmres_workspace_bytes(P, k + 1) or more."""
    ms = ctypes.c_double()
    lib = _lib.load()
    args = (ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * ws.element_size()), _ptr(r), int(reps),
            _stream(stream), ctypes.byref(ms))
    if basis_prec == HS_C128:
        _lib.check(lib.hs_time_arnoldi(P.handle, int(k), int(which), *args))
    else:
        _lib.check(lib.hs_time_arnoldi_ex(P.handle, int(k), int(which), int(basis_prec), *args))
    return float(ms.value)


def hs_time_arnoldi_ex(P: Problem, k: int, which: int, basis_prec: int, ws, r, reps: int = 10, stream=None) -> float:
    ms = ctypes.c_double()
    _lib.check(_lib.load().hs_time_arnoldi_ex(P.handle, int(k), int(which), int(basis_prec),
                                              ctypes.c_void_p(ws.data_ptr()),
                                              ctypes.c_size_t(ws.numel() * ws.element_size()), _ptr(r), int(reps),
                                              _stream(stream), ctypes.byref(ms)))
    return float(ms.value)


def hs_precond_set_schedule(M: Precond, fork_level: int, local_grid: int = 0):
    _lib.check(_lib.load().hs_precond_set_schedule(M.handle, int(fork_level), int(local_grid)))


def hs_precond_get_schedule(M: Precond):
    f, g = ctypes.c_int(), ctypes.c_int()
    _lib.check(_lib.load().hs_precond_get_schedule(M.handle, ctypes.byref(f), ctypes.byref(g)))
    return f.value, g.value


def hs_nd_level_stats(M: Precond, level: int) -> dict:
    """Per-level figures of the nested-dissection coarse solve (host only)."""
    out = (ctypes.c_int64 * 8)()
    _lib.check(_lib.load().hs_nd_level_stats(M.handle, level, out))
    keys = ("fronts", "g_entries", "v_entries", "fwd_workgroups", "bwd_workgroups", "max_nI", "max_nB",
            "subtree_workgroups")
    return dict(zip(keys, list(out)))


def hs_nd_plan_level_stats(ncx: int, ncy: int, reach: int, leaf: int = 8) -> list:
    """Per-level figures of the nested-dissection plan of a coarse grid (host only)."""
    lib = _lib.load()
    keys = ("fronts", "g_entries", "v_entries", "fwd_workgroups", "bwd_workgroups", "max_nI", "max_nB",
            "subtree_workgroups")
    out, lv = [], 0
    while True:
        buf = (ctypes.c_int64 * 8)()
        if lib.hs_nd_plan_level_stats(int(ncx), int(ncy), int(reach), int(leaf), lv, buf) != HS_OK:
            break
        out.append(dict(zip(keys, list(buf))))
        lv += 1
    if not out:
        _lib.check(HS_EINVAL if ncx < 1 else lib.hs_nd_plan_level_stats(int(ncx), int(ncy), int(reach),
                                                                         int(leaf), 0, (ctypes.c_int64 * 8)()))
    return out


def hs_precond_get_info(M: Precond) -> dict:
    info = PrecondInfo()
    _lib.check(_lib.load().hs_precond_get_info(M.handle, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in PrecondInfo._fields_}


def hs_coarse_restrict(M: Precond, r, r0, stream=None):
    _lib.check(_lib.load().hs_coarse_restrict(M.handle, _ptr(r), _ptr(r0), _stream(stream)))


def hs_coarse_prolong(M: Precond, e0, z, stream=None):
    _lib.check(_lib.load().hs_coarse_prolong(M.handle, _ptr(e0), _ptr(z), _stream(stream)))


def hs_coarse_solve(M: Precond, r0, e0, stream=None):
    _lib.check(_lib.load().hs_coarse_solve(M.handle, _ptr(r0), _ptr(e0), _stream(stream)))


def hs_coarse_matrix(M: Precond, stencil, stream=None):
    _lib.check(_lib.load().hs_coarse_matrix(M.handle, _ptr(stencil), _stream(stream)))


def hs_local_solve(M: Precond, r, zloc, stream=None):
    _lib.check(_lib.load().hs_local_solve(M.handle, _ptr(r), _ptr(zloc), _stream(stream)))


def hs_time_step(M: Precond, which: int, r, reps: int = 10, stream=None) -> float:
    """Mean ms per launch of one step (0 local solves, 1 coarse solve, 2 whole
    M^{-1} apply, 3 SpMV, 4 one MGS projection), timed with HIP events on the
    stream."""
    ms = ctypes.c_double()
    _lib.check(_lib.load().hs_time_step(M.handle, int(which), _ptr(r), int(reps), _stream(stream),
                                        ctypes.byref(ms)))
    return float(ms.value)


def hs_k2_gradient(P: Problem, u, lam, scale: float, grad, stream=None):
    """grad += scale * Re(dA_ll/dk^2 u lam) on the grid nodes of the unknowns."""
    _lib.check(_lib.load().hs_k2_gradient(P.handle, _ptr(u), _ptr(lam), float(scale), _ptr(grad, "float64"),
                                          _stream(stream)))


def hs_nd_plan_check(ncx: int, ncy: int, reach: int, leaf: int) -> dict:
    """Host-only structural check of the nested-dissection plan."""
    stats = (ctypes.c_int64 * 8)()
    _lib.check(_lib.load().hs_nd_plan_check(int(ncx), int(ncy), int(reach), int(leaf), stats))
    keys = ["fronts", "levels", "g_elems", "v_elems", "f_elems", "max_nI", "max_nB", "max_nF"]
    return dict(zip(keys, list(stats)))


from .autograd import HelmholtzSolve, HelmholtzSolveMulti, helmholtz_solve, helmholtz_solve_multi  # noqa: E402
