"""Bezier coarse restriction R_0 (oracle).

Sec. 4, eq. (GCS:HO_R_0): for H = 2h the coarse value at coarse node i is
(u_{m-2} + 4 u_{m-1} + 6 u_m + 4 u_{m+1} + u_{m+2}) / 8 with m = 2i - 1 in
the paper's 1-based numbering; the prolongation is R_0^T.

Readings:
* 0-based: coarse node c sits on fine node 2c; taps outside [0, n-1] are
  dropped (truncated at the two ends);
* 2-D: R_0 = R_y kron R_x (tensor product), which gives a 25-point coarse
  matrix, consistent with the remark that the Bezier coarse matrix is less
  sparse than the linear one;
* Dirichlet: rows = interior coarse nodes, columns = interior fine nodes
  (taps on boundary nodes drop out, the coarse functions vanish on the
  boundary);
* H = 2^L h: the product of the ratio-2 operators on successively coarser
  grids, each stage taken on that stage's unknowns.

The linear coarse space the paper compares against (P1, Sec. 4) is read as
linear interpolation: the prolongation puts
weight 1 on the coincident fine node and 1/2 on its two neighbours, R_0 is
its transpose, i.e. taps (1/2, 1, 1/2) at stride 2; two stages give the
ratio-4 hat 1 - |o|/4.  The scale of R_0 cancels in R_0^T A_0^{-1} R_0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .problem import DIRICHLET, SOMMERFELD

TAPS = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 8.0
P1_TAPS = np.array([0.0, 0.5, 1.0, 0.5, 0.0])
BEZIER, P1 = "bezier", "p1"


def restriction_1d_full(nf: int, kind: str = BEZIER) -> sp.csr_matrix:
    """Ratio-2 restriction on all nodes: (nc x nf), nc = (nf - 1)/2 + 1."""
    assert nf % 2 == 1
    taps = TAPS if kind == BEZIER else P1_TAPS
    nc = (nf - 1) // 2 + 1
    rows, cols, vals = [], [], []
    for c in range(nc):
        for d in range(-2, 3):
            f = 2 * c + d
            if 0 <= f < nf and taps[d + 2] != 0.0:
                rows.append(c)
                cols.append(f)
                vals.append(taps[d + 2])
    return sp.csr_matrix((vals, (rows, cols)), shape=(nc, nf))


def restriction_1d(nf: int, bc: int, ratio: int = 2, kind: str = BEZIER) -> sp.csr_matrix:
    """1-D restriction for coarse ratio ``ratio`` (a power of two), on the
    unknowns of boundary condition ``bc``."""
    assert ratio >= 2 and ratio & (ratio - 1) == 0
    R = None
    n = nf
    while ratio > 1:
        assert (n - 1) % 2 == 0
        S = restriction_1d_full(n, kind)
        if bc == DIRICHLET:
            S = S[1:-1, 1:-1]
        R = S if R is None else S @ R
        n = (n - 1) // 2 + 1
        ratio //= 2
    return R.tocsr()


def restriction_2d(n: int, bc: int, ratio: int = 2, kind: str = BEZIER) -> sp.csr_matrix:
    """2-D R_0 on the unknowns (x fastest on both grids)."""
    R1 = restriction_1d(n, bc, ratio, kind)
    return sp.kron(R1, R1, format="csr")


def coarse_matrix(A: sp.spmatrix, R0: sp.spmatrix) -> sp.csr_matrix:
    """Galerkin coarse matrix A_0 = R_0 A R_0^T (eqs. DDM:SO_AS / SO_SAS)."""
    A0 = (R0 @ A @ R0.T).tocsr()
    A0.sum_duplicates()
    A0.sort_indices()
    return A0
