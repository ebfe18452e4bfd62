"""Write tests/golden/gmres_mp2_n513.json from the CPU oracle alone.

The workload is MP-2 (Sec. 2, Sommerfeld) at n = 513, k = 160 (kh = 0.3125,
the benchmark's kh), with the benchmark's decomposition geometry: 8 x 8
subdomains of 64h, overlap 2, the Bezier coarse space at H = 2h (Sec. 4),
RAS2 (eq. DDM:SO_SAS with Boolean D_i), unrestarted right-preconditioned
flexible GMRES to a relative residual of 1e-6 (Sec. 5), x_0 = 0, unit point
source at the centre.

Three oracle solves are recorded:
  fp64       complex128 local factors and solves;
  fp64_pert  the same with M^{-1} z perturbed by seeded relative noise of
             1e-12 (numpy default_rng(1)), which measures how far rounding
             alone moves this Krylov process;
  c64        complex64 local factors and solves (the mixed form: R_i r cast
             down, solved, cast back), everything else complex128.
For each: the iteration count, the implicit residual history, the true
relative residual, ||x||_2 and 1024 solution entries at seeded positions
(numpy default_rng(513), shared by the three runs).

Only oracle/ is imported.  Runtime: tens of minutes on a few host cores.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import gmres, problem, schwarz  # noqa: E402

N, K, NSUB, OVERLAP, RATIO, TOL, MAXIT = 513, 160.0, 8, 2, 2, 1e-6, 400
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gmres_mp2_n513.json")


def record(res, idx):
    return {"iters": int(res.iters), "converged": bool(res.converged),
            "relres_true": float(res.relres_true),
            "history": [float(h) for h in res.history],
            "x_norm": float(np.linalg.norm(res.x)),
            "x_samples_re": [float(v) for v in res.x[idx].real],
            "x_samples_im": [float(v) for v in res.x[idx].imag]}


def main():
    bc = problem.SOMMERFELD
    A = problem.assemble(N, bc, k=K)
    f = problem.rhs(N, bc)
    idx = np.sort(np.random.default_rng(513).choice(A.shape[0], size=1024, replace=False))
    out = {"cite": "Sec. 2 (MP-2), Sec. 3 (RAS2, eq. DDM:SO_SAS), Sec. 4 (eq. GCS:HO_R_0), Sec. 5 (GMRES)",
           "n": N, "k": K, "nsub": NSUB, "overlap": OVERLAP, "ratio": RATIO, "variant": "RAS2", "tol": TOL,
           "maxit": MAXIT, "source": "centre", "sample_idx": [int(i) for i in idx], "runs": {}}
    runs = (("fp64", np.complex128, False), ("fp64_pert", np.complex128, True), ("c64", np.complex64, False))
    for name, dt, pert in runs:
        t0 = time.time()
        S = schwarz.Schwarz(A, N, bc, NSUB, overlap=OVERLAP, ratio=RATIO, variant=schwarz.RAS2, local_dtype=dt)
        apply = S.apply
        if pert:
            rng = np.random.default_rng(1)
            apply = lambda v: S.apply(v) * (1 + 1e-12 * rng.standard_normal(v.size))  # noqa: E731
        res = gmres.fgmres(lambda v: A @ v, apply, f, tol=TOL, maxit=MAXIT)
        out["runs"][name] = record(res, idx)
        print(f"{name}: {res.iters} iterations, true relres {res.relres_true:.3e}, {time.time() - t0:.0f} s",
              flush=True)
        del S
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
