"""Seeded synthetic workloads for the Helmholtz / two-level Schwarz path.

This module only describes *inputs*: grid sizes, wavenumbers, decomposition
parameters, seeded random vectors, point-source positions and the
heterogeneous k^2 field.  It holds none of the method's arithmetic (no
assembly, no restriction, no factorisation, no Krylov step), so both the CPU
oracle (``oracle/``) and the HIP path may draw from it without sharing any
computational code.

The five named configurations restate the workloads the method is exercised
on: the two model problems of Sec. 2 (MP-1 Dirichlet, MP-2 Sommerfeld) at the
sizes the solver is measured on, plus the precision / batching /
differentiation variants.  All randomness goes through
``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import numpy as np

DIRICHLET = 0
SOMMERFELD = 1

AS2 = 0
RAS2 = 1

C128 = 0
C64 = 1


@dataclasses.dataclass(frozen=True)
class Config:
    """One solver workload.

    n        nodes per dimension (h = 1/(n-1)), odd
    k        constant wavenumber (ignored when a k^2 field is supplied)
    bc       DIRICHLET (MP-1) or SOMMERFELD (MP-2)
    nsub     subdomains per dimension
    overlap  overlap delta in node layers added on each side of an owned block
    ratio    coarse ratio r = H/h (power of two)
    variant  AS2 or RAS2
    prec     local-solve precision C128 or C64
    tol      GMRES relative-residual tolerance
    maxit    iteration cap
    src      point-source node (i, j); None means the centre node
    """
    name: str
    n: int
    k: float
    bc: int
    nsub: int
    overlap: int = 2
    ratio: int = 2
    variant: int = RAS2
    prec: int = C128
    tol: float = 1e-6
    maxit: int = 200
    src: tuple | None = None

    @property
    def h(self) -> float:
        return 1.0 / (self.n - 1)

    def source(self) -> tuple:
        if self.src is not None:
            return self.src
        c = (self.n - 1) // 2
        return (c, c)


MP1 = Config("MP-1", n=65, k=20.0, bc=DIRICHLET, nsub=4)
MP2 = Config("MP-2", n=257, k=80.0, bc=SOMMERFELD, nsub=8)
PRECISION = Config("Precision", n=1025, k=320.0, bc=SOMMERFELD, nsub=16, prec=C64)
PRECISION_FP64 = dataclasses.replace(PRECISION, name="Precision-fp64", prec=C128)

CONFIGS = {c.name: c for c in (MP1, MP2, PRECISION, PRECISION_FP64)}


def random_vector(nu: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Unit-norm vector with i.i.d. N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(nu) + 1j * rng.standard_normal(nu)
    v /= np.linalg.norm(v)
    return v.astype(dtype)


def random_vectors(count: int, nu: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, nu)) + 1j * rng.standard_normal((count, nu))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def batching_instances(count: int = 48, seed: int = 0):
    """The uneven batch: n drawn from {129,193,257,385,513}, k = 0.3/h, a
    point source at a uniform interior node, nsub = n//64 + 2, overlap 2,
    coarse ratio 4, Sommerfeld boundary."""
    rng = np.random.default_rng(seed)
    sizes = np.array([129, 193, 257, 385, 513])
    out = []
    for b in range(count):
        n = int(rng.choice(sizes))
        k = 0.3 * (n - 1)
        i, j = (int(v) for v in rng.integers(1, n - 1, size=2))
        out.append(Config(f"batch{b}", n=n, k=k, bc=SOMMERFELD, nsub=n // 64 + 2,
                          overlap=2, ratio=4, variant=RAS2, prec=C64, src=(i, j)))
    return out


def gaussian_bump_field(n: int, seed: int, nbumps: int = 8, sigma: float = 0.08) -> np.ndarray:
    """g(x, y) = sum_b a_b exp(-|x - c_b|^2 / (2 sigma^2)), a_b ~ U[-1, 1],
    c_b ~ U[0,1]^2, normalised so that max |g| over the nodes is 1.
    Returned as an (n, n) array indexed [j, i] (y, x)."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(-1.0, 1.0, nbumps)
    cen = rng.uniform(0.0, 1.0, (nbumps, 2))
    x = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    g = np.zeros((n, n))
    for a, (cx, cy) in zip(amp, cen):
        g += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * sigma ** 2))
    return g / np.abs(g).max()


def k2_field(n: int, k0: float, seed: int, strength: float = 0.2) -> np.ndarray:
    """Heterogeneous k^2 = k0^2 (1 + strength * g) on the nodes, [j, i]."""
    return k0 * k0 * (1.0 + strength * gaussian_bump_field(n, seed))


def differentiation_setup(n: int = 513, k0: float = 150.0, nsrc: int = 4, seed: int = 0):
    """Sources at seeded interior nodes with x < 0.8 and the receiver column
    nearest x = 0.9."""
    rng = np.random.default_rng(seed + 100)
    imax = int(0.8 * (n - 1))
    srcs = [(int(rng.integers(1, imax)), int(rng.integers(1, n - 1))) for _ in range(nsrc)]
    recv_col = int(round(0.9 * (n - 1)))
    return srcs, recv_col
