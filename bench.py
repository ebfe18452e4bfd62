"""Benchmark: GMRES time-to-1e-6 and M^{-1} applies/s, mixed vs FP64, on the
MP-2 workload n = 1025 (h = 1/1024), k = 320, 16 x 16 subdomains, overlap 2,
Bezier coarse space H = 2h, two-level RAS, on one MI355X.

A step is one pass of the whole hot path: build the two-level preconditioner
(local factors + Galerkin coarse matrix + coarse factorisation) and run
flexible GMRES to a true relative residual of 1e-6 from x0 = 0.  `value` is
the mixed form's solves per second (1000 / time-to-1e-6 in ms); the line also
carries the FP64 form, the applies/s of both, the roofline of the local-solve
kernel and the CPU oracle on a bounded sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

N_GRID, K_WAVE, NSUB, OVERLAP, RATIO = 1025, 320.0, 16, 2, 2
TOL, MAXIT = 1e-6, 1500


def local_solve_bytes(info_sizes, prec_bytes):
    """Algorithmic bytes of one launch of the batched local solves: every Schur
    inverse G_j (n_x^2 entries per grid line) is read twice, the right-hand
    side is gathered once in complex128 and the local solution written once."""
    total = 0
    for nx, ny in info_sizes:
        total += 2 * ny * nx * nx * prec_bytes + nx * ny * (16 + prec_bytes)
    return total


def subdomain_sizes(n, nsub, overlap):
    from workloads import SOMMERFELD  # noqa: F401  (inputs module: no method arithmetic)
    # owned blocks along one axis: node i -> min(nsub-1, i*nsub // (n-1))
    blocks = {}
    for i in range(n):
        s = min(nsub - 1, (i * nsub) // (n - 1))
        a, b = blocks.get(s, (i, i + 1))
        blocks[s] = (min(a, i), max(b, i + 1))
    ext = [(max(0, a - overlap), min(n, b + overlap)) for a, b in (blocks[s] for s in range(nsub))]
    return [(x1 - x0, y1 - y0) for (y0, y1) in ext for (x0, x1) in ext]


def gpu_run(args):
    import numpy as np
    import torch

    import paper_2408_03571_amd as hs
    from workloads import random_vectors

    dev = "cuda:0"
    torch.cuda.set_device(0)
    n = N_GRID
    nu = n * n
    # point source at the centre: f = e_c / h^2 (Sec. 2, MP-2)
    h = 1.0 / (n - 1)
    c = (n - 1) // 2
    b = torch.zeros(nu, dtype=torch.complex128, device=dev)
    b[c * n + c] = 1.0 / (h * h)
    P = hs.hs_assemble(n, K_WAVE, hs.HS_BC_SOMMERFELD)
    ws = torch.empty(hs.hs_gmres_workspace_bytes(P, MAXIT), dtype=torch.uint8, device=dev)
    x = torch.zeros_like(b)

    def one_step(prec):
        M = hs.hs_setup_schwarz(P, NSUB, OVERLAP, RATIO, hs.HS_RAS2, prec)
        st, _ = hs.hs_gmres_solve(P, M, b, x, tol=TOL, maxit=MAXIT, ws=ws, history=False)
        info = hs.hs_precond_get_info(M)
        del M
        return st, info

    forms = {}
    for name, prec in (("mixed", hs.HS_C64), ("fp64", hs.HS_C128)):
        for _ in range(args.warmup):
            one_step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(args.steps):
            stats.append(one_step(prec))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        st, info = stats[-1]
        forms[name] = {"ms_per_solve": ms, "iters": st["iters"], "relres_true": st["relres_true"],
                       "converged": st["converged"], "ms_setup_local": info["ms_setup_local"],
                       "ms_setup_coarse": info["ms_setup_coarse"], "info": info}
        print(f"[bench] {name}: {ms:.1f} ms/solve, {st['iters']} its, relres {st['relres_true']:.2e}, "
              f"setup local {info['ms_setup_local']:.1f} ms coarse {info['ms_setup_coarse']:.1f} ms", flush=True)

    # applies/s and the roofline of the local-solve kernel
    vecs = torch.from_numpy(random_vectors(2, nu, seed=0)).to(dev)
    z = torch.empty_like(b)
    sizes = subdomain_sizes(n, NSUB, OVERLAP)
    for name, prec in (("mixed", hs.HS_C64), ("fp64", hs.HS_C128)):
        M = hs.hs_setup_schwarz(P, NSUB, OVERLAP, RATIO, hs.HS_RAS2, prec)
        for _ in range(10):
            hs.hs_apply_Minv(M, vecs[0], z)
        ms_apply = hs.hs_time_step(M, 2, vecs[1], reps=100)
        ms_local = hs.hs_time_step(M, 0, vecs[1], reps=50)
        ms_coarse = hs.hs_time_step(M, 1, vecs[1], reps=50)
        forms[name]["applies_per_s"] = 1e3 / ms_apply
        forms[name]["ms_apply"] = ms_apply
        forms[name]["ms_local_solve"] = ms_local
        forms[name]["ms_coarse_solve"] = ms_coarse
        forms[name]["local_solve_bytes"] = local_solve_bytes(sizes, 8 if prec == hs.HS_C64 else 16)
        print(f"[bench] {name}: apply {ms_apply:.3f} ms ({1e3 / ms_apply:.0f}/s), local {ms_local:.3f} ms, "
              f"coarse {ms_coarse:.3f} ms", flush=True)
        del M
    return forms


def cpu_baseline(gpu_iters, seconds_budget=25.0):
    """The oracle on the host cores, on a bounded sample of the same workload:
    four of the 256 local band-LU factor + solves, and the band-LU factor and
    solve of a leading block of A_0 (same bandwidth, 1/32 of its rows); band LU
    costs grow linearly with the rows at fixed bandwidth, so both scale to the
    full workload, and an M^{-1} application to one GMRES solve with the GPU's
    iteration count (the oracle runs the same algorithm)."""
    import numpy as np

    from oracle import bandlu, bezier, decomp, problem
    t_start = time.perf_counter()
    n, bc = N_GRID, problem.SOMMERFELD
    A = problem.assemble(n, bc, k=K_WAVE)
    subs = decomp.decompose(n, bc, NSUB, NSUB, OVERLAP)
    pick = [0, 17, 120, 255]
    t_lf = t_ls = 0.0
    rng = np.random.default_rng(0)
    for s in pick:
        sub = subs[s]
        Ai = A[sub.idx][:, sub.idx]
        kl, ku = bandlu.bandwidths(Ai)
        t0 = time.perf_counter()
        lu = bandlu.BandLU(Ai, kl, ku, dtype=np.complex64).factor()
        t1 = time.perf_counter()
        lu.solve(rng.standard_normal(sub.idx.size).astype(np.complex64))
        t2 = time.perf_counter()
        t_lf += t1 - t0
        t_ls += t2 - t1
    scale_loc = len(subs) / len(pick)
    R0 = bezier.restriction_2d(n, bc, RATIO)
    A0 = bezier.coarse_matrix(A, R0)
    kl, ku = bandlu.bandwidths(A0)
    rows = A0.shape[0] // 32
    A0s = A0[:rows][:, :rows]
    t0 = time.perf_counter()
    lu = bandlu.BandLU(A0s, kl, ku).factor()
    t1 = time.perf_counter()
    lu.solve(rng.standard_normal(rows) + 0j)
    t2 = time.perf_counter()
    scale_c = A0.shape[0] / rows
    setup_s = t_lf * scale_loc + (t1 - t0) * scale_c
    apply_s = t_ls * scale_loc + (t2 - t1) * scale_c
    total_s = setup_s + gpu_iters * apply_s
    cores = os.cpu_count()
    return {"value": 1.0 / total_s, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "est_setup_s": setup_s, "est_apply_s": apply_s, "est_time_to_solution_s": total_s,
            "applies_per_s": 1.0 / apply_s, "wall_s_of_sample": time.perf_counter() - t_start,
            "sample": f"oracle band-LU factor+solve of 4/256 complex64 subdomains (x64) and of the leading "
                      f"{rows}/{A0.shape[0]} rows of A_0 (x{scale_c:.0f}); time-to-solution = setup + "
                      f"{gpu_iters} applies (GPU iteration count); BLAS threads = host cores"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the solver has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    forms = gpu_run(args)
    mx, fp = forms["mixed"], forms["fp64"]
    achieved = mx["local_solve_bytes"] / (mx["ms_local_solve"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "local_solve_kernel<float>", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "bytes_per_launch": mx["local_solve_bytes"], "ms_per_launch": mx["ms_local_solve"]}
    cpu = None if args.no_cpu else cpu_baseline(mx["iters"])
    line = {
        "metric": "GMRES time-to-1e-6 + M^-1 applies/s, mixed vs FP64, MP-2 n=1025 k=320",
        "value": 1e3 / mx["ms_per_solve"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mx["ms_per_solve"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64 local / c128 coarse+Krylov",
        "data": "synthetic",
        "config": {"workload": "MP-2 n=1025 (h=1/1024) k=320, point source at the centre, 16x16 subdomains, "
                               "overlap 2, Bezier H=2h, RAS2, FGMRES tol 1e-6",
                   "unknowns": N_GRID * N_GRID, "coarse_unknowns": mx["info"]["n_coarse"]},
        "time_to_solution_ms": {"mixed": mx["ms_per_solve"], "fp64": fp["ms_per_solve"]},
        "speedup_mixed_vs_fp64": fp["ms_per_solve"] / mx["ms_per_solve"],
        "iterations": {"mixed": mx["iters"], "fp64": fp["iters"]},
        "relres_true": {"mixed": mx["relres_true"], "fp64": fp["relres_true"]},
        "setup_ms": {"mixed": {"local": mx["ms_setup_local"], "coarse": mx["ms_setup_coarse"]},
                     "fp64": {"local": fp["ms_setup_local"], "coarse": fp["ms_setup_coarse"]}},
        "applies_per_s": {"mixed": mx["applies_per_s"], "fp64": fp["applies_per_s"]},
        "apply_ms_breakdown": {f: {"apply": forms[f]["ms_apply"], "local_solve": forms[f]["ms_local_solve"],
                                   "coarse_solve": forms[f]["ms_coarse_solve"]} for f in forms},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
