"""Gradient of a receiver misfit with respect to a heterogeneous k^2 field
(oracle).

The paper assumes a constant wavenumber (Sec. 2); the differentiation workload
lets k^2 vary per node in the volume term and takes k = sqrt(k^2) in the
Sommerfeld boundary term.  A(k^2) is complex symmetric (Sec. 2, A = A^T), so
the adjoint of a solve is one more solve with the same matrix and the same
preconditioner, applied to a conjugated right-hand side.

Loss over sources s:  L = sum_s 1/2 ||P u_s - d_s||^2,  A u_s = f_s,
P = restriction to the receiver column.
dL = Re((P u - d)^H P du),  du = -A^{-1} (dA) u,  A^{-H} = conj(A^{-1})
=> solve A lambda_s = conj(P^T (P u_s - d_s)) (unconjugated adjoint)
=> dL/d(k^2)_l = sum_s Re(-lambda_{s,l} (dA_ll/dk^2_l) u_{s,l}).
"""
from __future__ import annotations

import numpy as np

from .problem import diag_dk2, unknown_lo_hi


def receiver_indices(n: int, bc: int, col: int) -> np.ndarray:
    lo, hi = unknown_lo_hi(n, bc)
    nu = hi - lo
    return (np.arange(lo, hi) - lo) * nu + (col - lo)


def loss_and_grad(n, bc, k2, sources, data, recv_col, solve):
    """``solve(rhs)`` returns A(k2)^{-1} rhs.  Returns (L, dL/dk2 on the
    unknowns, list of u_s)."""
    from .problem import rhs
    P = receiver_indices(n, bc, recv_col)
    dA = diag_dk2(n, bc, k2=k2)
    L = 0.0
    grad = np.zeros(dA.size)
    us = []
    for s, src in enumerate(sources):
        u = solve(rhs(n, bc, [src]))
        us.append(u)
        res = u[P] - data[s]
        L += 0.5 * np.vdot(res, res).real
        g = np.zeros_like(u)
        g[P] = res
        lam = solve(np.conj(g))
        grad += np.real(-lam * dA * u)
    return L, grad, us
