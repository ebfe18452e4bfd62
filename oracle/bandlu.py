"""Hand-written blocked band LU with partial pivoting (oracle).

Sec. 3: the local problems R_i A R_i^T and the coarse problem R_0 A R_0^T are
solved exactly ("sparse direct solver").  With x-fastest ordering both are
band matrices (half bandwidth = the grid line length of the subdomain, or
2 * coarse line length + 2 for the 25-point coarse matrix), so the oracle uses
a band LU.

Algorithm (right-looking, blocked, partial pivoting within the band):
for each panel of ``nb`` columns starting at column k
  1. take the dense window of rows [k, k+kb+kl) that can be non-zero in the
     panel columns, and the columns to its right that those rows can reach;
  2. factor the panel columns with partial pivoting (largest modulus, lowest
     row index on ties), swapping whole window rows;
  3. U12 = L11^{-1} A12 and A22 -= L21 U12 (library matmul / triangular solve
     as the BLAS-3 step).
Row swaps of a panel touch only that panel's window, so earlier panels'
multipliers stay where they were stored (product form across panels), and
the solve replays panel by panel: swaps, unit-lower panel solve, update of
the rows below, then blocked back substitution with U.

Storage: column-major band with generous bandwidths (lower kl + nb, upper
kl + ku + nb) viewed as a dense N x N matrix with column stride ldab - 1, so
every window above is an ordinary strided dense block.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from numpy.lib.stride_tricks import as_strided


class BandLU:
    def __init__(self, A: sp.spmatrix, kl: int, ku: int, dtype=np.complex128, nb: int = 32):
        A = sp.csr_matrix(A)
        self.N = N = A.shape[0]
        self.kl, self.ku, self.nb = kl, ku, nb
        self.dtype = np.dtype(dtype)
        self.klp = kl + nb                # stored lower bandwidth
        self.kup = kl + ku + nb           # stored upper bandwidth
        self.ldab = self.klp + self.kup + 1
        self.buf = np.zeros(self.ldab * N + 1, dtype=self.dtype)
        isz = self.buf.itemsize
        self.D = as_strided(self.buf[self.kup:], shape=(N, N),
                            strides=(isz, (self.ldab - 1) * isz), writeable=True)
        coo = A.tocoo()
        off = coo.row - coo.col
        if off.size and (off.max() > kl or -off.min() > ku):
            raise ValueError("matrix exceeds the declared bandwidth")
        # element (r, j) lives at flat index kup + r + j * (ldab - 1)
        self.buf[self.kup + coo.row + coo.col * (self.ldab - 1)] = coo.data.astype(self.dtype)
        self.piv = np.zeros(N, dtype=np.int64)
        self.panels = []
        self.factored = False

    # -- factorisation -------------------------------------------------
    def factor(self):
        N, kl, ku, nb, D = self.N, self.kl, self.ku, self.nb, self.D
        tiny = 0.0
        for k in range(0, N, nb):
            kb = min(nb, N - k)
            r1 = min(N, k + kb + kl)          # rows that can touch the panel
            c1 = min(N, k + kb + kl + ku)     # columns those rows can reach
            W = D[k:r1, k:c1]
            for c in range(kb):
                col = np.abs(W[c:, c])
                p = c + int(np.argmax(col))
                if col[p - c] <= tiny:
                    raise ZeroDivisionError(f"zero pivot in column {k + c}")
                self.piv[k + c] = k + p
                if p != c:
                    tmp = W[c, :].copy()
                    W[c, :] = W[p, :]
                    W[p, :] = tmp
                W[c + 1:, c] /= W[c, c]
                if c + 1 < kb:
                    W[c + 1:, c + 1:kb] -= np.outer(W[c + 1:, c], W[c, c + 1:kb])
            if c1 > k + kb:
                L11 = np.array(W[:kb, :kb])
                A12 = np.array(W[:kb, kb:])
                U12 = sla.solve_triangular(L11, A12, lower=True, unit_diagonal=True)
                W[:kb, kb:] = U12
                if r1 > k + kb:
                    W[kb:, kb:] -= np.array(W[kb:, :kb]) @ U12
            self.panels.append((k, kb, r1, c1))
        self.factored = True
        return self

    # -- solve -----------------------------------------------------------
    def solve(self, b: np.ndarray) -> np.ndarray:
        assert self.factored
        D = self.D
        x = np.array(b, dtype=self.dtype).copy()
        for (k, kb, r1, c1) in self.panels:
            for c in range(kb):
                p = self.piv[k + c]
                if p != k + c:
                    x[k + c], x[p] = x[p], x[k + c]
            L11 = np.array(D[k:k + kb, k:k + kb])
            x[k:k + kb] = sla.solve_triangular(L11, x[k:k + kb], lower=True, unit_diagonal=True)
            if r1 > k + kb:
                x[k + kb:r1] -= np.array(D[k + kb:r1, k:k + kb]) @ x[k:k + kb]
        for (k, kb, r1, c1) in reversed(self.panels):
            y = x[k:k + kb]
            if c1 > k + kb:
                y = y - np.array(D[k:k + kb, k + kb:c1]) @ x[k + kb:c1]
            U11 = np.array(D[k:k + kb, k:k + kb])
            x[k:k + kb] = sla.solve_triangular(U11, y, lower=False)
        return x

    # -- helpers for checks ----------------------------------------------
    def dense_LU(self):
        """Rebuild P, L, U densely (small N only) so that P A = L U, where the
        product-form row swaps are folded into one permutation and L is
        re-ordered accordingly."""
        N = self.N
        U = np.zeros((N, N), dtype=self.dtype)
        for r in range(N):
            j1 = min(N, r + self.kl + self.ku + self.nb + 1)
            U[r, r:j1] = self.D[r, r:j1]
        # replay the elimination on the identity to recover P and L:
        # forward solve maps b -> L^{-1} P b
        Linv_P = np.stack([self._forward(np.eye(N, dtype=self.dtype)[:, j]) for j in range(N)], axis=1)
        return Linv_P, U

    def _forward(self, b):
        D = self.D
        x = b.copy()
        for (k, kb, r1, c1) in self.panels:
            for c in range(kb):
                p = self.piv[k + c]
                if p != k + c:
                    x[k + c], x[p] = x[p], x[k + c]
            L11 = np.array(D[k:k + kb, k:k + kb])
            x[k:k + kb] = sla.solve_triangular(L11, x[k:k + kb], lower=True, unit_diagonal=True)
            if r1 > k + kb:
                x[k + kb:r1] -= np.array(D[k + kb:r1, k:k + kb]) @ x[k:k + kb]
        return x


def bandwidths(A: sp.spmatrix) -> tuple[int, int]:
    coo = sp.coo_matrix(A)
    off = coo.row - coo.col
    return int(max(0, off.max())), int(max(0, -off.min()))
