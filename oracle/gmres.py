"""Unrestarted, right-preconditioned flexible GMRES with modified Gram-Schmidt
(oracle).

Sec. 5 runs GMRES to a relative tolerance with an iteration cap; it does not
state the side of preconditioning, restarts or the orthogonalisation.
Reading: right preconditioning in the flexible form (the preconditioned
directions z_j are stored and x = Z_j y), no restart, modified Gram-Schmidt,
x_0 = 0.  One iteration = one application of M^{-1}.

Step j:  z_j = M^{-1} v_j;  w = A z_j;  for i <= j: h_ij = v_i^H w,
w -= h_ij v_i;  h_{j+1,j} = ||w||;  v_{j+1} = w / h_{j+1,j};  the previous
complex Givens rotations act on column j and a new one annihilates h_{j+1,j};
stop when |g_{j+1}| <= tol * ||b||, then confirm with the true residual
||b - A x|| / ||b|| and keep iterating (no restart) if it is still above tol.

Givens convention: for (a, b) -> (r, 0): c = |a| / sqrt(|a|^2 + |b|^2)
(real), s = (a / |a|) conj(b) / sqrt(|a|^2 + |b|^2); a = 0 gives c = 0,
s = 1.  Rotation: [c, s; -conj(s), c].
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    converged: bool
    history: list            # implicit relative residual after each iteration
    relres_true: float
    V: np.ndarray | None = None
    Z: np.ndarray | None = None
    H: np.ndarray | None = None


def givens(a: complex, b: complex):
    if a == 0:
        return 0.0, 1.0 + 0j
    na = abs(a)
    nrm = np.hypot(na, abs(b))
    c = na / nrm
    s = (a / na) * np.conj(b) / nrm
    return c, s


def fgmres(A_mul, M_apply, b: np.ndarray, tol: float = 1e-6, maxit: int = 200,
           keep_basis: bool = False) -> GmresResult:
    b = np.asarray(b, dtype=np.complex128)
    N = b.size
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return GmresResult(np.zeros_like(b), 0, True, [0.0], 0.0)
    V = np.zeros((maxit + 1, N), dtype=np.complex128)
    Z = np.zeros((maxit, N), dtype=np.complex128)
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    R = np.zeros((maxit + 1, maxit), dtype=np.complex128)   # rotated H
    cs = np.zeros(maxit)
    sn = np.zeros(maxit, dtype=np.complex128)
    g = np.zeros(maxit + 1, dtype=np.complex128)
    g[0] = beta
    V[0] = b / beta
    history = [1.0]
    x = np.zeros_like(b)
    relres_true = 1.0
    converged = False
    j = 0
    for j in range(maxit):
        Z[j] = M_apply(V[j])
        w = A_mul(Z[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        breakdown = H[j + 1, j] == 0.0
        if not breakdown:
            V[j + 1] = w / H[j + 1, j]
        col = H[:j + 2, j].copy()
        for i in range(j):
            t = cs[i] * col[i] + sn[i] * col[i + 1]
            col[i + 1] = -np.conj(sn[i]) * col[i] + cs[i] * col[i + 1]
            col[i] = t
        cs[j], sn[j] = givens(col[j], col[j + 1])
        col[j] = cs[j] * col[j] + sn[j] * col[j + 1]
        col[j + 1] = 0.0
        R[:j + 2, j] = col
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        history.append(abs(g[j + 1]) / beta)
        if history[-1] <= tol or breakdown:
            y = _back_substitute(R[:j + 1, :j + 1], g[:j + 1])
            x = Z[:j + 1].T @ y
            relres_true = np.linalg.norm(b - A_mul(x)) / beta
            if relres_true <= tol or breakdown:
                converged = relres_true <= tol
                break
    else:
        y = _back_substitute(R[:j + 1, :j + 1], g[:j + 1])
        x = Z[:j + 1].T @ y
        relres_true = np.linalg.norm(b - A_mul(x)) / beta
    res = GmresResult(x, j + 1, converged, history, relres_true)
    if keep_basis:
        res.V, res.Z, res.H = V[:j + 2], Z[:j + 1], H[:j + 2, :j + 1]
    return res


def _back_substitute(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    m = g.size
    y = np.zeros(m, dtype=np.complex128)
    for i in range(m - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:m] @ y[i + 1:m]) / R[i, i]
    return y
