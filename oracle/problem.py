"""Model problems and their five-point discretisation (oracle).

Sec. 2 of the paper: -Laplace(u) - k^2 u = delta(x - 1/2, y - 1/2) on the unit
square, with u = 0 on the boundary (MP-1, eq. BVP_MP-1) or the first-order
Sommerfeld condition du/dn - i k u = 0 (MP-2).  A uniform grid with n nodes
per dimension, h = 1/(n-1), and a second-order finite-difference scheme give
A u = f (eq. LS_final); A is symmetric, real for MP-1 and complex symmetric,
non-Hermitian for MP-2.

Readings (the paper gives no boundary scheme and no scaling):
* the operator is the negative Laplacian (the source prints a garbled
  "-nabla u"); rows are unscaled, entries O(1/h^2); the point source is
  e_src / h^2;
* Sommerfeld rows use a centred ghost node, u_ghost = u_mirror + 2 i k h u_b,
  substituted into the interior stencil, and edge / corner rows are scaled by
  1/2 / 1/4 so that A is exactly symmetric;
* with a heterogeneous k^2 field, k = sqrt(k^2) at the boundary node.

Unknown ordering: Sommerfeld uses all n^2 nodes, Dirichlet the (n-2)^2
interior nodes; linear index l = (j - lo) * nu + (i - lo), x fastest.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

DIRICHLET = 0
SOMMERFELD = 1


def unknown_lo_hi(n: int, bc: int) -> tuple[int, int]:
    """Grid indices [lo, hi) that carry unknowns along one dimension."""
    return (0, n) if bc == SOMMERFELD else (1, n - 1)


def n_unknowns(n: int, bc: int) -> int:
    lo, hi = unknown_lo_hi(n, bc)
    return (hi - lo) ** 2


def k2_nodes(n: int, k: float | None, k2: np.ndarray | None) -> np.ndarray:
    """k^2 on all grid nodes as an (n, n) array indexed [j, i]."""
    if k2 is not None:
        k2 = np.asarray(k2, dtype=np.float64)
        assert k2.shape == (n, n)
        return k2
    return np.full((n, n), float(k) ** 2)


def row_scale(n: int, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """Sommerfeld row scaling: 1 inside, 1/2 on an edge, 1/4 at a corner."""
    e = (i == 0).astype(int) + (i == n - 1) + (j == 0) + (j == n - 1)
    return 0.5 ** e


def assemble(n: int, bc: int, k: float | None = None, k2: np.ndarray | None = None):
    """Return the sparse matrix A (CSR, complex128) of eq. (LS_final)."""
    assert n % 2 == 1 and n >= 5
    h = 1.0 / (n - 1)
    lo, hi = unknown_lo_hi(n, bc)
    nu = hi - lo
    K2 = k2_nodes(n, k, k2)
    jj, ii = np.meshgrid(np.arange(lo, hi), np.arange(lo, hi), indexing="ij")
    i = ii.ravel()
    j = jj.ravel()
    row = (j - lo) * nu + (i - lo)
    kk2 = K2[j, i]
    rows, cols, vals = [], [], []
    if bc == DIRICHLET:
        rows.append(row)
        cols.append(row)
        vals.append((4.0 / h ** 2 - kk2).astype(np.complex128))
        for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
            ni, nj = i + di, j + dj
            ok = (ni >= lo) & (ni < hi) & (nj >= lo) & (nj < hi)
            rows.append(row[ok])
            cols.append(((nj - lo) * nu + (ni - lo))[ok])
            vals.append(np.full(ok.sum(), -1.0 / h ** 2, dtype=np.complex128))
    else:
        # number of ghost normals at the node and the symmetric row scale
        e = (i == 0).astype(int) + (i == n - 1) + (j == 0) + (j == n - 1)
        w = 0.5 ** e
        kb = np.sqrt(kk2)
        rows.append(row)
        cols.append(row)
        vals.append(w * (4.0 / h ** 2 - kk2 - 2j * kb * e / h))
        for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
            ni, nj = i + di, j + dj
            ok = (ni >= 0) & (ni < n) & (nj >= 0) & (nj < n)
            # the opposite neighbour is a ghost: its mirror is this neighbour
            mi, mj = i - di, j - dj
            ghost = (mi < 0) | (mi >= n) | (mj < 0) | (mj >= n)
            coef = np.where(ghost, -2.0, -1.0) / h ** 2 * w
            rows.append(row[ok])
            cols.append((nj * n + ni)[ok])
            vals.append(coef[ok].astype(np.complex128))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    A = sp.coo_matrix((v, (r, c)), shape=(nu * nu, nu * nu)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def rhs(n: int, bc: int, sources=None, weights=None) -> np.ndarray:
    """Point sources: f = sum_s w_s e_s / h^2, times the row scale of the
    source node for Sommerfeld edge / corner rows.  Default: unit source at
    the centre node."""
    h = 1.0 / (n - 1)
    lo, hi = unknown_lo_hi(n, bc)
    nu = hi - lo
    if sources is None:
        c = (n - 1) // 2
        sources = [(c, c)]
    if weights is None:
        weights = [1.0] * len(sources)
    f = np.zeros(nu * nu, dtype=np.complex128)
    for (si, sj), ws in zip(sources, weights):
        assert lo <= si < hi and lo <= sj < hi
        scale = 1.0
        if bc == SOMMERFELD:
            scale = float(row_scale(n, np.array(si), np.array(sj)))
        f[(sj - lo) * nu + (si - lo)] += ws * scale / h ** 2
    return f


def diag_dk2(n: int, bc: int, k: float | None = None, k2: np.ndarray | None = None) -> np.ndarray:
    """d A_ll / d(k^2)_l on the unknowns (A depends on k^2 only through its
    diagonal).  Interior: -1.  Sommerfeld edge / corner rows: the scaled
    volume term -w plus the derivative of -w * 2 i e k / h with
    k = sqrt(k^2), i.e. -w * i e / (k h)."""
    h = 1.0 / (n - 1)
    lo, hi = unknown_lo_hi(n, bc)
    K2 = k2_nodes(n, k, k2)
    jj, ii = np.meshgrid(np.arange(lo, hi), np.arange(lo, hi), indexing="ij")
    i = ii.ravel()
    j = jj.ravel()
    kk2 = K2[j, i]
    if bc == DIRICHLET:
        return -np.ones(i.size, dtype=np.complex128)
    e = (i == 0).astype(int) + (i == n - 1) + (j == 0) + (j == n - 1)
    w = 0.5 ** e
    return -w - 1j * w * e / (np.sqrt(kk2) * h)
