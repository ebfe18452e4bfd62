"""Closed-form solution of the discrete MP-1 system (oracle pin).

Sec. 2, MP-1 (eq. BVP_MP-1) with the five-point scheme: the Dirichlet matrix
is diagonalised by the discrete sine modes
  phi_pq(i, j) = sin(p pi i / (n-1)) sin(q pi j / (n-1)),  p, q = 1..n-2,
with eigenvalues lambda_pq = (4/h^2)(sin^2(p pi h / 2) + sin^2(q pi h / 2)) - k^2.
Expanding the point source e_c / h^2 (c the centre node) in these orthogonal
modes, whose squared norm is ((n-1)/2)^2, gives the exact discrete solution
  u(i, j) = sum_pq (2/(n-1))^2 phi_pq(c) phi_pq(i, j) / (h^2 lambda_pq).
Evaluated with separable sums (an O(n^3) contraction).
"""
from __future__ import annotations

import numpy as np


def mp1_discrete_solution(n: int, k: float, src=None) -> np.ndarray:
    """Exact solution of A u = e_src / h^2 on the (n-2)^2 interior unknowns."""
    h = 1.0 / (n - 1)
    m = n - 2
    if src is None:
        c = (n - 1) // 2
        src = (c, c)
    si, sj = src
    p = np.arange(1, m + 1)
    idx = np.arange(1, m + 1)
    S = np.sin(np.pi * np.outer(p, idx) / (n - 1))          # S[p, i]
    lam1 = (4.0 / h ** 2) * np.sin(p * np.pi * h / 2) ** 2
    lam = lam1[:, None] + lam1[None, :] - k * k              # [p, q]
    coef = (2.0 / (n - 1)) ** 2 * np.outer(np.sin(np.pi * p * si / (n - 1)),
                                           np.sin(np.pi * p * sj / (n - 1))) / (h * h * lam)
    # u[j, i] = sum_{p,q} coef[p, q] S[p, i] S[q, j]
    U = S.T @ coef @ S            # [i, j]
    return U.T.ravel().astype(np.complex128)   # x fastest
