"""Two-level overlapping Schwarz preconditioners (oracle).

Sec. 3:
* AS2, eq. (DDM:SO_AS):  M^{-1} = R_0^T A_0^{-1} R_0 + sum_i R_i^T A_i^{-1} R_i
* SAS2, eq. (DDM:SO_SAS): M^{-1} = R_0^T A_0^{-1} R_0 + sum_i R_i^T D_i A_i^{-1} R_i
  with diagonal D_i, sum_i R_i^T D_i R_i = I; with Boolean D_i (the owned
  block) this is restricted additive Schwarz, called RAS2 here.
* SHS2, eq. (DDM:SO_SHS): M^{-1} = Q + (sum_i R_i^T D_i A_i^{-1} R_i)(I - A Q)
  with Q = R_0^T A_0^{-1} R_0 and the same D_i: the coarse correction is
  applied first and the local solves act on the deflated residual.
with A_i = R_i A R_i^T, A_0 = R_0 A R_0^T and exact local / coarse solves
(here: the hand-written band LU of ``bandlu``).

The mixed-precision form rounds only the local factorisations and solves to
complex64 (R_i r is cast down, solved in complex64, cast back); the coarse
solve and everything else stay complex128.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .bandlu import BandLU, bandwidths
from .bezier import coarse_matrix, restriction_2d
from .decomp import decompose

AS2 = 0
RAS2 = 1
SHS2 = 2


class Schwarz:
    def __init__(self, A: sp.spmatrix, n: int, bc: int, nsub: int, overlap: int = 2,
                 ratio: int = 2, variant: int = RAS2, local_dtype=np.complex128,
                 coarse: bool = True, nb: int = 32, coarse_space: str = "bezier"):
        self.A = sp.csr_matrix(A)
        self.n, self.bc, self.variant = n, bc, variant
        self.local_dtype = np.dtype(local_dtype)
        # nsub: subdomains per dimension, or (nsub_x, nsub_y)
        nsx, nsy = (nsub, nsub) if np.isscalar(nsub) else (int(nsub[0]), int(nsub[1]))
        self.subs = decompose(n, bc, nsx, nsy, overlap)
        self.local = []
        for s in self.subs:
            Ai = self.A[s.idx][:, s.idx]
            kl, ku = bandwidths(Ai)
            self.local.append(BandLU(Ai, kl, ku, dtype=self.local_dtype, nb=nb).factor())
        self.coarse = coarse
        if coarse:
            self.R0 = restriction_2d(n, bc, ratio, coarse_space)
            self.A0 = coarse_matrix(self.A, self.R0)
            kl, ku = bandwidths(self.A0)
            self.coarse_lu = BandLU(self.A0, kl, ku, dtype=np.complex128, nb=nb).factor()

    def local_solve(self, s: int, r: np.ndarray) -> np.ndarray:
        """A_i^{-1} R_i r in the local precision, returned in complex128."""
        sub = self.subs[s]
        ri = r[sub.idx].astype(self.local_dtype)
        return self.local[s].solve(ri).astype(np.complex128)

    def coarse_solve(self, r: np.ndarray) -> np.ndarray:
        """R_0^T A_0^{-1} R_0 r."""
        r0 = self.R0 @ r
        e0 = self.coarse_lu.solve(r0)
        return self.R0.T @ e0

    def apply(self, r: np.ndarray) -> np.ndarray:
        r = np.asarray(r, dtype=np.complex128)
        z = np.zeros_like(r)
        if self.coarse:
            z += self.coarse_solve(r)
        if self.variant == SHS2:
            # local solves on the deflated residual (I - A Q) r
            t = r - self.A @ z
        else:
            t = r
        for s, sub in enumerate(self.subs):
            zi = self.local_solve(s, t)
            if self.variant in (RAS2, SHS2):
                np.add.at(z, sub.idx[sub.owned], zi[sub.owned])
            else:
                np.add.at(z, sub.idx, zi)
        return z
