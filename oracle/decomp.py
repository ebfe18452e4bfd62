"""Overlapping domain decomposition (oracle).

Sec. 3: a non-overlapping decomposition of the closed domain is extended by
layers of grid nodes to overlapping subdomains Omega_i; R_i is the 0/1
restriction from Omega to Omega_i, and the scaled (restricted) variant uses
diagonal D_i with sum_i R_i^T D_i R_i = I (eq. DDM:SO_SAS).

Readings:
* per dimension, node i (grid index) is owned by block
  min(Ns - 1, floor(i * Ns / (n - 1))); interface nodes go to the upper
  block, the last block also takes i = n - 1;
* each owned block is extended by ``overlap`` node layers on each side and
  clipped to the unknowns;
* D_i is the indicator of the owned (non-overlapping) block (classic
  restricted additive Schwarz).
The 2-D subdomain is the tensor product; local ordering is x fastest.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from .problem import unknown_lo_hi


@dataclasses.dataclass
class Subdomain:
    own: tuple          # owned grid ranges (x0, x1, y0, y1), half open
    ext: tuple          # extended grid ranges (x0, x1, y0, y1), half open
    idx: np.ndarray     # global unknown index of every local node (x fastest)
    owned: np.ndarray   # bool mask of owned local nodes (D_i)

    @property
    def nx(self) -> int:
        return self.ext[1] - self.ext[0]

    @property
    def ny(self) -> int:
        return self.ext[3] - self.ext[2]


def owner_blocks(n: int, bc: int, ns: int) -> list[tuple[int, int]]:
    """Owned grid-index ranges [a, b) per block along one dimension."""
    lo, hi = unknown_lo_hi(n, bc)
    owner = np.minimum(ns - 1, (np.arange(lo, hi) * ns) // (n - 1))
    blocks = []
    for s in range(ns):
        sel = np.nonzero(owner == s)[0]
        if sel.size == 0:
            raise ValueError("empty subdomain block")
        blocks.append((lo + int(sel[0]), lo + int(sel[-1]) + 1))
    return blocks


def decompose(n: int, bc: int, nsx: int, nsy: int, overlap: int) -> list[Subdomain]:
    lo, hi = unknown_lo_hi(n, bc)
    nu = hi - lo
    bx = owner_blocks(n, bc, nsx)
    by = owner_blocks(n, bc, nsy)
    for a, b in bx + by:
        if b - a < overlap + 1:
            raise ValueError("block narrower than overlap + 1")
    subs = []
    for (y0, y1) in by:
        for (x0, x1) in bx:
            ex0, ex1 = max(lo, x0 - overlap), min(hi, x1 + overlap)
            ey0, ey1 = max(lo, y0 - overlap), min(hi, y1 + overlap)
            jj, ii = np.meshgrid(np.arange(ey0, ey1), np.arange(ex0, ex1), indexing="ij")
            idx = ((jj - lo) * nu + (ii - lo)).ravel()
            owned = ((ii >= x0) & (ii < x1) & (jj >= y0) & (jj < y1)).ravel()
            subs.append(Subdomain((x0, x1, y0, y1), (ex0, ex1, ey0, ey1), idx, owned))
    return subs
