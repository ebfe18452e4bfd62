"""Differentiable Helmholtz solve: u = A(k^2)^{-1} f through the two-level
Schwarz preconditioned flexible GMRES of the C ABI.

Backward (A is complex symmetric, Sec. 2, so A^{-H} = conj(A^{-1})): torch
hands over g = 2 dL/du* for a real loss L.  With du = -A^{-1} (dA) u, a real
parameter gets dL/dk^2 = Re(conj(g)^T du/dk^2), so one unconjugated adjoint
solve lam = A^{-1} conj(g), reusing the forward preconditioner, gives
  dL/dk^2_l = -Re( dA_ll/dk^2_l u_l lam_l )   (hs_k2_gradient, scale -1)
  grad_f    = A^{-H} g = conj(lam).
Several sources on one field (HelmholtzSolveMulti): one problem and one
preconditioner serve every forward solve and every adjoint solve; the
sources are solved together as one batch that repeats the preconditioner
(each launch of M^{-1} serves every source), and the per-node gradient terms
of all sources accumulate into one field on the device.

Argument marshalling only: both solves and the gradient run in the HIP
library.
"""
from __future__ import annotations

import torch

from . import (HS_BC_SOMMERFELD, HS_C128, HS_RAS2, hs_assemble, hs_batch_create, hs_gmres_solve,
               hs_batch_gmres_solve, hs_k2_gradient, hs_setup_schwarz)


class HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k2, f, n, bc, nsub, overlap, ratio, variant, prec, tol, maxit, adj_tol):
        k2c = k2.detach().reshape(-1).contiguous().to(torch.float64)
        P = hs_assemble(n, 1.0, bc, k2c)
        M = hs_setup_schwarz(P, nsub, overlap, ratio, variant, prec)
        u = torch.zeros(f.shape[-1], dtype=torch.complex128, device=f.device)
        st, _ = hs_gmres_solve(P, M, f.to(torch.complex128).resolve_conj().resolve_neg().contiguous(), u, tol=tol, maxit=maxit, history=False,
                               raise_on_noconv=True)
        ctx.P, ctx.M, ctx.k2c = P, M, k2c
        ctx.maxit, ctx.adj_tol = maxit, adj_tol
        ctx.k2_shape = k2.shape
        ctx.save_for_backward(u)
        ctx.stats = st
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        rhs = grad_u.to(torch.complex128).conj().resolve_conj().contiguous()
        lam = torch.zeros_like(u)
        hs_gmres_solve(ctx.P, ctx.M, rhs, lam, tol=ctx.adj_tol, maxit=ctx.maxit, history=False,
                       raise_on_noconv=True)
        grad_k2 = torch.zeros_like(ctx.k2c)
        hs_k2_gradient(ctx.P, u, lam, -1.0, grad_k2)
        grad_f = torch.conj(lam)
        return (grad_k2.reshape(ctx.k2_shape), grad_f) + (None,) * 10


def _solve_all(B, F, U, tol, maxit, basis_prec):
    """Every row of F through the batch B (one instance per row, rows
    contiguous, so F and U are batch vectors as they stand)."""
    stats = hs_batch_gmres_solve(B, F.reshape(-1), U.reshape(-1), tol=tol, maxit=maxit, raise_on_noconv=True,
                                 basis_prec=basis_prec)
    return stats


class HelmholtzSolveMulti(torch.autograd.Function):
    """U[s] = A(k^2)^{-1} F[s] for the rows s of F, sharing one set-up."""

    @staticmethod
    def forward(ctx, k2, F, n, bc, nsub, overlap, ratio, variant, prec, tol, maxit, adj_tol, basis_prec):
        k2c = k2.detach().reshape(-1).contiguous().to(torch.float64)
        P = hs_assemble(n, 1.0, bc, k2c)
        M = hs_setup_schwarz(P, nsub, overlap, ratio, variant, prec)
        Fc = F.to(torch.complex128).resolve_conj().resolve_neg().contiguous()
        U = torch.zeros_like(Fc)
        B = hs_batch_create([M] * Fc.shape[0])
        stats = _solve_all(B, Fc, U, tol, maxit, basis_prec)
        ctx.P, ctx.M, ctx.B, ctx.k2c = P, M, B, k2c
        ctx.maxit, ctx.adj_tol, ctx.basis_prec = maxit, adj_tol, basis_prec
        ctx.k2_shape = k2.shape
        ctx.save_for_backward(U)
        ctx.stats = stats
        return U

    @staticmethod
    def backward(ctx, grad_U):
        (U,) = ctx.saved_tensors
        rhs = grad_U.to(torch.complex128).conj().resolve_conj().contiguous()
        lam = torch.zeros_like(U)
        grad_k2 = torch.zeros_like(ctx.k2c)
        ctx.adjoint_stats = _solve_all(ctx.B, rhs, lam, ctx.adj_tol, ctx.maxit, ctx.basis_prec)
        for s in range(U.shape[0]):
            hs_k2_gradient(ctx.P, U[s], lam[s], -1.0, grad_k2)
        return (grad_k2.reshape(ctx.k2_shape), torch.conj(lam)) + (None,) * 11


def helmholtz_solve_multi(k2, F, n, bc=HS_BC_SOMMERFELD, nsub=8, overlap=2, ratio=2, variant=HS_RAS2,
                          prec=HS_C128, tol=1e-10, maxit=1000, adj_tol=None, basis_prec=HS_C128):
    """U[s] = A(k2)^{-1} F[s] for every row of F (nsrc x unknowns, complex128),
    one problem and one preconditioner for all forward and adjoint solves;
    gradients to k2 (n x n float64) and F."""
    return HelmholtzSolveMulti.apply(k2, F, n, bc, nsub, overlap, ratio, variant, prec, tol, maxit,
                                     tol if adj_tol is None else adj_tol, basis_prec)


def helmholtz_solve(k2, f, n, bc=HS_BC_SOMMERFELD, nsub=8, overlap=2, ratio=2, variant=HS_RAS2, prec=HS_C128,
                    tol=1e-10, maxit=1000, adj_tol=None):
    """u = A(k2)^{-1} f with gradients to k2 (n x n float64 field on the grid
    nodes) and f (complex128 on the unknowns)."""
    return HelmholtzSolve.apply(k2, f, n, bc, nsub, overlap, ratio, variant, prec, tol, maxit,
                                tol if adj_tol is None else adj_tol)
