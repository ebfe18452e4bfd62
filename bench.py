"""Benchmark: GMRES time-to-1e-6 and M^{-1} applies/s, mixed vs FP64, on the
MP-2 workload n = 1025 (h = 1/1024), k = 320, 16 x 16 subdomains, overlap 2,
Bezier coarse space H = 2h, two-level RAS, on one MI355X.

A step is one pass of the whole hot path: build the two-level preconditioner
(local factors + Galerkin coarse matrix + coarse factorisation) and run
flexible GMRES to a true relative residual of 1e-6 from x0 = 0.  `value` is
the mixed form's solves per second (1000 / time-to-1e-6 in ms; local factors
and solves in complex64); the line also carries the form with complex64
factor storage and complex128 solve arithmetic (mixed_s), the FP64 form, the
applies/s of every form, the roofline of the dominant kernel (measured live
with HIP events on its stream) and of the other hot kernels, and the CPU
oracle on a bounded sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--forms mixed,mixed_s,fp64]
  python bench.py --profile-kernels     short run of the hot kernels alone, for
                                        rocprofv3 counter passes
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


def local_solve_bytes(sizes, prec_bytes):
    """Algorithmic bytes of one launch of the batched local solves: every Schur
    inverse G_j (n_x^2 entries per grid line) is read twice, the right-hand
    side is gathered once in complex128 and the local solution written once."""
    total = 0
    for nx, ny in sizes:
        total += 2 * ny * nx * nx * prec_bytes + nx * ny * (16 + prec_bytes)
    return total


def arnoldi_pass_bytes(nu, k):
    """One DCGS2 streaming pass at Arnoldi step k.  Dot pass: read the k basis
    vectors, u_k and z_k, write w = A z_k and the stored z_k.  Update pass:
    read the k basis vectors, u_k and w, write v_k and w1.  Both (k + 4) N
    complex128 values."""
    return (k + 4) * nu * 16


K_TIMED = (64, 512)   # Arnoldi steps at which the two DCGS2 passes are timed


def subdomain_sizes(n, nsub, overlap):
    # owned blocks along one axis: node i -> min(nsub-1, i*nsub // (n-1))
    blocks = {}
    for i in range(n):
        s = min(nsub - 1, (i * nsub) // (n - 1))
        a, b = blocks.get(s, (i, i + 1))
        blocks[s] = (min(a, i), max(b, i + 1))
    ext = [(max(0, a - overlap), min(n, b + overlap)) for a, b in (blocks[s] for s in range(nsub))]
    return [(x1 - x0, y1 - y0) for (y0, y1) in ext for (x0, x1) in ext]


def make_problem():
    import torch

    import paper_2408_03571_amd as hs
    dev = "cuda:0"
    torch.cuda.set_device(0)
    n = N_GRID
    h = 1.0 / (n - 1)
    c = (n - 1) // 2
    b = torch.zeros(n * n, dtype=torch.complex128, device=dev)
    b[c * n + c] = 1.0 / (h * h)         # point source e_c / h^2 at the centre (Sec. 2)
    P = hs.hs_assemble(n, K_WAVE, hs.HS_BC_SOMMERFELD)
    return P, b


def kernel_times(P, prec, ws, reps=50):
    """Mean ms per launch of the hot kernels, HIP events on their streams.
    The DCGS2 passes are timed at two Arnoldi steps; their cost is linear in
    the number of basis vectors they stream."""
    import torch

    import paper_2408_03571_amd as hs
    from workloads import random_vectors
    nu = N_GRID * N_GRID
    v = torch.from_numpy(random_vectors(1, nu, seed=0)).to("cuda:0")[0].contiguous()
    M = hs.hs_setup_schwarz(P, NSUB, OVERLAP, RATIO, hs.HS_RAS2, prec)
    info = hs.hs_precond_get_info(M)
    z = torch.empty_like(v)
    for _ in range(5):
        hs.hs_apply_Minv(M, v, z)
    out = {"apply": hs.hs_time_step(M, 2, v, reps=reps), "local": hs.hs_time_step(M, 0, v, reps=reps),
           "coarse": hs.hs_time_step(M, 1, v, reps=reps), "spmv": hs.hs_time_step(M, 3, v, reps=reps),
           "info": info}
    for k in K_TIMED:
        r = max(3, reps // 10) if k > 100 else reps
        out[f"dots{k}"] = hs.hs_time_arnoldi(P, k, 0, ws, v, reps=r)
        out[f"update{k}"] = hs.hs_time_arnoldi(P, k, 1, ws, v, reps=r)
    out["small"] = hs.hs_time_arnoldi(P, K_TIMED[1], 2, ws, v, reps=reps)
    del M
    return out


def ortho_ms(kt, iters):
    """Estimated DCGS2 time of a solve: both passes, linear in the step k
    (fitted through the two timed steps), summed over the steps, plus the
    small kernels of every step."""
    k0, k1 = K_TIMED
    tot = 0.0
    for name in ("dots", "update"):
        slope = (kt[f"{name}{k1}"] - kt[f"{name}{k0}"]) / (k1 - k0)
        icpt = kt[f"{name}{k0}"] - slope * k0
        tot += (iters + 1) * icpt + slope * iters * (iters + 1) / 2
    return tot + (iters + 1) * kt["small"]


def gpu_run(args, forms_wanted):
    import torch

    import paper_2408_03571_amd as hs
    from paper_2408_03571_amd import autotune
    P, b = make_problem()
    tuned = autotune.tune_arnoldi(P, cache=None)      # timed fresh on this device, outside the timed steps
    print(f"[bench] autotuned DCGS2 shape (unknowns per lane, rows per trip) = {tuned['shape']} "
          f"in {tuned['tuning_s']:.1f} s", flush=True)
    ws = torch.empty(hs.hs_gmres_workspace_bytes(P, MAXIT), dtype=torch.uint8, device=b.device)
    x = torch.zeros_like(b)

    def one_step(prec):
        M = hs.hs_setup_schwarz(P, NSUB, OVERLAP, RATIO, hs.HS_RAS2, prec)
        st, _ = hs.hs_gmres_solve(P, M, b, x, tol=TOL, maxit=MAXIT, ws=ws, history=False)
        info = hs.hs_precond_get_info(M)
        del M
        return st, info

    precs = {"mixed": hs.HS_C64, "mixed_s": hs.HS_C64S, "fp64": hs.HS_C128}
    forms = {}
    for name in forms_wanted:
        prec = precs[name]
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
        kt = kernel_times(P, prec, ws)
        it = st["iters"]
        forms[name] = {"ms_per_solve": ms, "iters": it, "relres_true": st["relres_true"],
                       "converged": st["converged"], "steps_launched": st["steps"],
                       "host_checks": st["host_checks"], "ms_setup_local": info["ms_setup_local"],
                       "ms_setup_coarse": info["ms_setup_coarse"], "info": info, "kt": kt,
                       "applies_per_s": 1e3 / kt["apply"],
                       "est_ms": {"apply": st["steps"] * kt["apply"], "orthogonalisation": ortho_ms(kt, it),
                                  "setup": info["ms_setup_local"] + info["ms_setup_coarse"]}}
        print(f"[bench] {name}: {ms:.1f} ms/solve, {it} its ({st['steps']} steps, {st['host_checks']} host "
              f"checks), relres {st['relres_true']:.2e}; apply {kt['apply']:.3f} ms (local {kt['local']:.3f}, "
              f"coarse {kt['coarse']:.3f}), dot pass at k={K_TIMED[1]} {kt[f'dots{K_TIMED[1]}']:.3f} ms, "
              f"update pass {kt[f'update{K_TIMED[1]}']:.3f} ms, setup {forms[name]['est_ms']['setup']:.1f} ms",
              flush=True)
    forms["_autotune"] = {"shape": tuned["shape"], "tuning_s": tuned["tuning_s"]}
    return forms


def profile_kernels():
    """Short run of the hot kernels alone (no GMRES), plus a plain device copy
    of known size that calibrates the HBM byte counters."""
    import torch

    import paper_2408_03571_amd as hs
    from paper_2408_03571_amd import autotune
    P, _ = make_problem()
    print(json.dumps({"autotuned_shape": autotune.tune_arnoldi(P, cache=None)["shape"]}), flush=True)
    ws = torch.empty(hs.hs_gmres_workspace_bytes(P, K_TIMED[1] + 1), dtype=torch.uint8, device="cuda:0")
    kt = kernel_times(P, hs.HS_C64, ws, reps=20)
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")   # 256 MiB
    c = torch.empty_like(a)
    for _ in range(20):
        c.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({k: v for k, v in kt.items() if k != "info"}), flush=True)


def cpu_baseline(gpu_iters):
    """The oracle on the host cores, on a bounded sample of the same workload:
    four of the 256 local band-LU factor + solves (complex64), and the band-LU
    factor and solve of a leading block of A_0 (same bandwidth, 1/32 of its
    rows).  Band-LU cost grows linearly with the rows at fixed bandwidth, so
    both scale to the full workload; a solve is setup + (GPU iteration count)
    applications of M^{-1} (the oracle runs the same algorithm)."""
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
    return {"value": 1.0 / total_s, "unit": "solves/s", "cores": os.cpu_count(), "kind": "oracle",
            "est_setup_s": setup_s, "est_apply_s": apply_s, "est_time_to_solution_s": total_s,
            "applies_per_s": 1.0 / apply_s, "wall_s_of_sample": time.perf_counter() - t_start,
            "sample": f"oracle band-LU factor+solve of 4/256 complex64 subdomains (x64) and of the leading "
                      f"{rows}/{A0.shape[0]} rows of A_0 (x{scale_c:.0f}); time-to-solution = setup + "
                      f"{gpu_iters} applies (the GPU's iteration count; the Arnoldi work is not included); "
                      f"NumPy BLAS threads = host cores"}


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes (copy-calibrated), or None if the kernel's source changed since."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as fh:
            rec = json.load(fh)["kernels"][kernel]
        with open(os.path.join(ROOT, rec["source"]), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != rec["sha256"]:
                return None
        return rec["traffic_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def roofline(name, nbytes, ms, extra=None, traffic_key=None):
    ach = nbytes / (ms * 1e-3) / 1e9
    r = {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(traffic_key) if traffic_key else None,
         "bytes_per_launch": nbytes, "ms_per_launch": ms}
    if extra:
        r.update(extra)
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="mixed,mixed_s,fp64")
    ap.add_argument("--profile-kernels", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the solver has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.profile_kernels:
        profile_kernels()
        return
    wanted = [f for f in args.forms.split(",") if f]
    forms = gpu_run(args, wanted)
    tuned = forms.pop("_autotune")
    main_form = "mixed" if "mixed" in forms else wanted[0]
    mx = forms[main_form]
    nu = N_GRID * N_GRID
    sizes = subdomain_sizes(N_GRID, NSUB, OVERLAP)
    kt = mx["kt"]
    est = mx["est_ms"]
    share = {k: v / mx["ms_per_solve"] for k, v in est.items()}
    k1 = K_TIMED[1]
    rl = roofline(f"arn_dots_kernel (DCGS2 dot pass at Arnoldi step k={k1}, fused A z)",
                  arnoldi_pass_bytes(nu, k1), kt[f"dots{k1}"],
                  {"time_share_of_step": share["orthogonalisation"] / 2}, traffic_key=f"arn_dots_kernel@{k1}")
    others = [
        roofline(f"arn_update_kernel (DCGS2 update pass at Arnoldi step k={k1})", arnoldi_pass_bytes(nu, k1),
                 kt[f"update{k1}"], traffic_key=f"arn_update_kernel@{k1}"),
        roofline("local_solve_kernel<float,2> (all 256 subdomain solves, complex64)",
                 local_solve_bytes(sizes, 8), kt["local"], traffic_key="local_solve_kernel<float, 2>"),
        roofline("nested-dissection coarse solve (26 level launches)", mx["info"]["coarse_solve_bytes"],
                 kt["coarse"]),
        roofline("spmv_kernel", 2 * nu * 16, kt["spmv"], traffic_key="spmv_kernel"),
    ]
    cpu = None if args.no_cpu else cpu_baseline(mx["iters"])
    line = {
        "metric": "GMRES time-to-1e-6 + M^-1 applies/s, mixed vs FP64, MP-2 n=1025 k=320",
        "value": 1e3 / mx["ms_per_solve"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mx["ms_per_solve"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 local LU/solves + c128 coarse/Krylov" if main_form == "mixed" else "c128",
        "data": "synthetic",
        "config": {"workload": "MP-2 n=1025 (h=1/1024) k=320, point source at the centre, 16x16 subdomains, "
                               "overlap 2, Bezier H=2h, RAS2, flexible GMRES tol 1e-6 from x0=0",
                   "form": main_form, "unknowns": nu, "coarse_unknowns": mx["info"]["n_coarse"]},
        "time_to_solution_ms": {f: forms[f]["ms_per_solve"] for f in forms},
        "iterations": {f: forms[f]["iters"] for f in forms},
        "relres_true": {f: forms[f]["relres_true"] for f in forms},
        "applies_per_s": {f: forms[f]["applies_per_s"] for f in forms},
        "apply_ms": {f: {k: forms[f]["kt"][k] for k in ("apply", "local", "coarse")} for f in forms},
        "setup_ms": {f: {"local": forms[f]["ms_setup_local"], "coarse": forms[f]["ms_setup_coarse"]}
                     for f in forms},
        "step_breakdown_ms_est": {f: forms[f]["est_ms"] for f in forms},
        "gmres_steps_launched": {f: forms[f]["steps_launched"] for f in forms},
        "gmres_host_checks": {f: forms[f]["host_checks"] for f in forms},
        "autotuned_dcgs2_shape": {"unknowns_per_lane": tuned["shape"][0], "rows_per_trip": tuned["shape"][1],
                                  "tuning_s": tuned["tuning_s"]},
        "roofline": rl,
        "roofline_others": others,
        "cpu_baseline": cpu,
    }
    if "mixed" in forms and "fp64" in forms:
        line["speedup_mixed_vs_fp64"] = {
            "time_to_solution": forms["fp64"]["ms_per_solve"] / forms["mixed"]["ms_per_solve"],
            "applies_per_s": forms["mixed"]["applies_per_s"] / forms["fp64"]["applies_per_s"]}
    if "mixed_s" in forms and "fp64" in forms:
        line["speedup_mixed_s_vs_fp64"] = {
            "time_to_solution": forms["fp64"]["ms_per_solve"] / forms["mixed_s"]["ms_per_solve"],
            "applies_per_s": forms["mixed_s"]["applies_per_s"] / forms["fp64"]["applies_per_s"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
