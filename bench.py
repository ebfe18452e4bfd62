"""Benchmark: GMRES time-to-1e-6 and M^{-1} applies/s, mixed vs FP64, on the
MP-2 workload n = 1025 (h = 1/1024), k = 320, 16 x 16 subdomains, overlap 2,
Bezier coarse space H = 2h, two-level RAS, on one MI355X.

A step is one pass of the whole hot path: build the two-level preconditioner
(local factors + Galerkin coarse matrix + coarse factorisation) and run
flexible GMRES to a true relative residual of 1e-6 from x0 = 0.  `value` is
the mixed form's solves per second (1000 / time-to-1e-6 in ms; local factors
and solves in complex64); the line also carries the form with complex64
factor storage and complex128 solve arithmetic (mixed_s), the FP64 form, the
mixed form with the Krylov basis stored in complex64 (mixed_cb: a compressed
basis, arithmetic still complex128), the applies/s of every form, the
roofline of the dominant kernel (measured live with HIP events on its stream)
and of the other hot kernels, and the CPU oracle on a bounded sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--forms mixed,mixed_s,fp64,mixed_cb]
  python bench.py --profile-kernels     short run of the hot kernels alone (built-in
                                        DCGS2 shape, passes at k = 512, and the passes
                                        with the complex64 basis at 4 x 4), for rocprofv3
  python bench.py --workload batching   the 48-instance batching workload
  python bench.py --workload differentiation   gradients/s of the 4-source differentiation workload
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


def arnoldi_pass_bytes(nu, k, basis_bytes=16):
    """One DCGS2 streaming pass at Arnoldi step k.  Dot pass: read the k basis
    vectors, u_k and z_k, write w = A z_k and the stored z_k.  Update pass:
    read the k basis vectors, u_k and w, write v_k and w1.  Both k basis
    vectors (basis_bytes per value) and 4 N complex128 values (v_k counted as
    a vector of the working precision)."""
    return (k * basis_bytes + 4 * 16) * nu


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


def kernel_times(P, prec, ws, reps=50, depths=K_TIMED, basis=0, schedule=(0, 0)):
    """Mean ms per launch of the hot kernels, HIP events on their streams.
    The DCGS2 passes are timed at two Arnoldi steps; their cost is linear in
    the number of basis vectors they stream."""
    import torch

    import paper_2408_03571_amd as hs
    from workloads import random_vectors
    nu = N_GRID * N_GRID
    v = torch.from_numpy(random_vectors(1, nu, seed=0)).to("cuda:0")[0].contiguous()
    M = hs.hs_setup_schwarz(P, NSUB, OVERLAP, RATIO, hs.HS_RAS2, prec)
    hs.hs_precond_set_schedule(M, *schedule)
    info = hs.hs_precond_get_info(M)
    z = torch.empty_like(v)
    for _ in range(5):
        hs.hs_apply_Minv(M, v, z)
    out = {"apply": hs.hs_time_step(M, 2, v, reps=reps), "local": hs.hs_time_step(M, 0, v, reps=reps),
           "coarse": hs.hs_time_step(M, 1, v, reps=reps), "spmv": hs.hs_time_step(M, 3, v, reps=reps),
           "info": info, "levels": [hs.hs_nd_level_stats(M, lv) for lv in range(info["nd_levels"])]}
    for k in depths:
        r = max(3, reps // 10) if k > 100 else reps
        out[f"dots{k}"] = hs.hs_time_arnoldi(P, k, 0, ws, v, reps=r, basis_prec=basis)
        out[f"update{k}"] = hs.hs_time_arnoldi(P, k, 1, ws, v, reps=r, basis_prec=basis)
    if len(depths) > 1:
        out["small"] = hs.hs_time_arnoldi(P, K_TIMED[1], 2, ws, v, reps=reps, basis_prec=basis)
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

    sched = {}   # application schedule per local precision, tuned outside the timed steps

    def one_step(prec, basis):
        M = hs.hs_setup_schwarz(P, NSUB, OVERLAP, RATIO, hs.HS_RAS2, prec)
        hs.hs_precond_set_schedule(M, *sched[prec])
        st, _ = hs.hs_gmres_solve(P, M, b, x, tol=TOL, maxit=MAXIT, ws=ws, history=False, basis_prec=basis)
        info = hs.hs_precond_get_info(M)
        del M
        return st, info

    # form -> (local precision, Krylov basis storage)
    precs = {"mixed": (hs.HS_C64, hs.HS_C128), "mixed_s": (hs.HS_C64S, hs.HS_C128),
             "fp64": (hs.HS_C128, hs.HS_C128), "mixed_cb": (hs.HS_C64, hs.HS_C64)}
    forms = {}
    cb_shape = None
    for name in forms_wanted:
        prec, basis = precs[name]
        if basis != hs.HS_C128 and cb_shape is None:
            # the shape table holds one shape per size: the complex64-basis form
            # runs with the shape tuned for its own storage
            cb = autotune.tune_arnoldi(P, cache=None, basis_prec=basis)
            cb_shape = cb["shape"]
            print(f"[bench] autotuned DCGS2 shape for the complex64 basis = {cb_shape} in {cb['tuning_s']:.1f} s",
                  flush=True)
        elif basis == hs.HS_C128:
            hs.hs_set_arnoldi_config(hs.hs_problem_size(P), *tuned["shape"])
        if prec not in sched:
            Mt = hs.hs_setup_schwarz(P, NSUB, OVERLAP, RATIO, hs.HS_RAS2, prec)
            from workloads import random_vectors
            vr = torch.from_numpy(random_vectors(1, hs.hs_problem_size(P), seed=0)).to(b.device)[0].contiguous()
            ts = autotune.tune_schedule(Mt, vr)
            sched[prec] = tuple(ts["schedule"])
            del Mt
            print(f"[bench] application schedule for local precision {prec} (fork level, local grid) = "
                  f"{sched[prec]} in {ts['tuning_s']:.1f} s", flush=True)
        for _ in range(args.warmup):
            one_step(prec, basis)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(args.steps):
            stats.append(one_step(prec, basis))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        st, info = stats[-1]
        kt = kernel_times(P, prec, ws, basis=basis, schedule=sched[prec])
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
    forms["_autotune"] = {"shape": tuned["shape"], "tuning_s": tuned["tuning_s"], "shape_c64_basis": cb_shape,
                          "schedules": {str(k): list(v) for k, v in sched.items()}}
    return forms


def profile_setup():
    """Three set-ups of the n = 1025 preconditioner (complex64 local factors,
    nested-dissection coarse factor), for profiling the factor phase."""
    import torch

    import paper_2408_03571_amd as hs
    torch.cuda.set_device(0)
    P = hs.hs_assemble(N_GRID, K_WAVE, hs.HS_BC_SOMMERFELD)
    for _ in range(3):
        t0 = time.perf_counter()
        M = hs.hs_setup_schwarz(P, NSUB, OVERLAP, RATIO, hs.HS_RAS2, hs.HS_C64)
        torch.cuda.synchronize()
        print(json.dumps({"setup_ms": (time.perf_counter() - t0) * 1e3}), flush=True)
        del M


def profile_kernels():
    """Short run of the hot kernels alone (no GMRES), plus a plain device copy
    of known size that calibrates the HBM byte counters."""
    import torch

    import paper_2408_03571_amd as hs
    P, _ = make_problem()
    print(json.dumps({"dcgs2_shape": hs.hs_get_arnoldi_config(hs.hs_problem_size(P))}), flush=True)
    ws = torch.empty(hs.hs_gmres_workspace_bytes(P, K_TIMED[1] + 1), dtype=torch.uint8, device="cuda:0")
    kt = kernel_times(P, hs.HS_C64, ws, reps=20, depths=(K_TIMED[1],))
    # the two passes with the complex64 basis, at the shape tuned for it (4 unknowns per lane, 4 rows per trip)
    from workloads import random_vectors
    N = hs.hs_problem_size(P)
    v = torch.from_numpy(random_vectors(1, N, seed=0)).to("cuda:0")[0].contiguous()
    hs.hs_set_arnoldi_config(N, 4, 4)
    for which, name in ((0, "dots"), (1, "update")):
        kt[f"{name}{K_TIMED[1]}_c64basis"] = hs.hs_time_arnoldi(P, K_TIMED[1], which, ws, v, reps=20,
                                                                basis_prec=hs.HS_C64)
    hs.hs_set_arnoldi_config(N, 0, 0)
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")   # 256 MiB
    c = torch.empty_like(a)
    for _ in range(20):
        c.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({k: v for k, v in kt.items() if k != "info"}), flush=True)


def batching_run(args):
    """The batching workload: 48 MP-2 instances (n drawn from {129, 193, 257,
    385, 513}, k = 0.3/h, a point source at a random interior node, n//64 + 2
    subdomains per dimension, overlap 2, H = 4h, complex64 local solves)
    solved together by hs_batch_gmres_solve.  A step is one batched solve of
    all of them; value = instance solves per second.  Also timed: the same
    instances solved one after another (same launch shapes), and one batched
    M^{-1} application (HIP events) with its algorithmic bytes."""
    import torch

    import paper_2408_03571_amd as hs
    from workloads import batching_instances
    dev = "cuda:0"
    torch.cuda.set_device(0)
    cfgs = batching_instances(48, seed=0)
    inst = []
    for c in cfgs:
        P = hs.hs_assemble(c.n, c.k, hs.HS_BC_SOMMERFELD)
        M = hs.hs_setup_schwarz(P, c.nsub, c.overlap, c.ratio, hs.HS_RAS2, hs.HS_C64)
        inst.append((P, M, c))
    B = hs.hs_batch_create([M for _, M, _ in inst])
    off = B.offsets
    from paper_2408_03571_amd import autotune
    rt = torch.randn(off[-1], dtype=torch.complex128, device=dev)
    tuned = autotune.tune_batch(B, rt)
    del rt
    print(f"[bench] batched schedule (fork level, local-solve workgroups) = {tuned['schedule']} ({tuned['apply_ms']})",
          flush=True)
    # point sources e_src / h^2 (Sec. 2); Sommerfeld: every grid node is an unknown
    b = torch.zeros(off[-1], dtype=torch.complex128, device=dev)
    for i, (_, _, c) in enumerate(inst):
        si, sj = c.src
        b[off[i] + sj * c.n + si] = float((c.n - 1) ** 2)
    x = torch.zeros_like(b)
    maxit = 400
    ws = torch.empty(hs.hs_batch_gmres_workspace_bytes(B, maxit), dtype=torch.uint8, device=dev)
    for _ in range(max(1, args.warmup)):
        hs.hs_batch_gmres_solve(B, b, x, tol=TOL, maxit=maxit, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats = hs.hs_batch_gmres_solve(B, b, x, tol=TOL, maxit=maxit, ws=ws)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / args.steps
    assert all(s["converged"] for s in stats), "batched solve did not converge"
    # the same instances one after another, with the batch's launch shape
    ept, rows = hs.hs_get_arnoldi_config(off[-1])
    if args.batch_only:
        print(json.dumps({"batched_ms_per_step": ms_batch, "iterations_max": max(s["iters"] for s in stats)}),
              flush=True)
        return
    for N in {hs.hs_problem_size(P) for P, _, _ in inst}:
        hs.hs_set_arnoldi_config(N, ept, rows)
    wss = torch.empty(max(hs.hs_gmres_workspace_bytes(P, maxit) for P, _, _ in inst), dtype=torch.uint8,
                      device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (P, M, c) in enumerate(inst):
        xi = torch.zeros(off[i + 1] - off[i], dtype=torch.complex128, device=dev)
        hs.hs_gmres_solve(P, M, b[off[i]:off[i + 1]].contiguous(), xi, tol=TOL, maxit=maxit, ws=wss,
                          history=False)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t0) * 1e3
    del wss
    # one batched application of M^{-1}, HIP events on its stream
    r = torch.randn(off[-1], dtype=torch.complex128, device=dev)
    z = torch.empty_like(r)
    for _ in range(3):
        hs.hs_batch_apply_Minv(B, r, z)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 20
    for _ in range(reps):
        hs.hs_batch_apply_Minv(B, r, z)
    e1.record()
    torch.cuda.synchronize()
    ms_apply = e0.elapsed_time(e1) / reps
    parts = {name: hs.hs_batch_time(B, w, r, reps=reps) for w, name in
             ((0, "local_solves"), (1, "coarse_chain"), (3, "restriction_stages"), (4, "nested_dissection"))}
    nbytes = 0
    for P, M, c in inst:
        info = hs.hs_precond_get_info(M)
        N = hs.hs_problem_size(P)
        nbytes += 2 * info["local_factor_bytes"] + info["coarse_solve_bytes"] + 4 * N * 16
    its = [s["iters"] for s in stats]
    line = {
        "metric": "batched GMRES instance solves/s (48 uneven MP-2 instances, tol 1e-6)",
        "value": len(inst) * 1e3 / ms_batch, "unit": "instance solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_batch, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 local LU/solves + c128 coarse/Krylov", "data": "synthetic",
        "config": {"workload": "batching: 48 MP-2 instances, n in {129,193,257,385,513} (seed 0), k=0.3/h, "
                               "random interior point source, n//64+2 subdomains/dim, overlap 2, Bezier H=4h, "
                               "RAS2, flexible GMRES tol 1e-6", "unknowns_total": off[-1]},
        "iterations": {"min": min(its), "max": max(its), "sum": sum(its)},
        "steps_launched": stats[0]["steps"], "host_checks": stats[0]["host_checks"],
        "ms_same_instances_one_by_one": ms_single, "batch_speedup_over_one_by_one": ms_single / ms_batch,
        "dcgs2_shape": {"unknowns_per_lane": ept, "rows_per_trip": rows},
        "batched_apply_parts_ms": parts,
        "autotuned_schedule": tuned,
        "roofline": {"bound": "hbm", "kernel": "one batched M^{-1} application (all 48 instances)",
                     "achieved": nbytes / (ms_apply * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": nbytes / (ms_apply * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": nbytes, "ms_per_launch": ms_apply},
    }
    print(json.dumps(line), flush=True)


def oracle_sample(n, bc, nsub, overlap, ratio, local_dtype, pick, rows_div, k=None, k2=None):
    """Oracle set-up and apply times on a bounded sample: band-LU factor +
    solve of the subdomains in `pick` (scaled to all of them) and of the
    leading 1/rows_div rows of A_0 (same bandwidth; band-LU cost grows
    linearly with the rows at fixed bandwidth).  Returns (setup_s, apply_s,
    description)."""
    import numpy as np

    from oracle import bandlu, bezier, decomp, problem
    A = problem.assemble(n, bc, k=k, k2=k2)
    subs = decomp.decompose(n, bc, nsub, nsub, overlap)
    t_lf = t_ls = 0.0
    rng = np.random.default_rng(0)
    for s in pick:
        sub = subs[s]
        Ai = A[sub.idx][:, sub.idx]
        kl, ku = bandlu.bandwidths(Ai)
        t0 = time.perf_counter()
        lu = bandlu.BandLU(Ai, kl, ku, dtype=local_dtype).factor()
        t1 = time.perf_counter()
        lu.solve(rng.standard_normal(sub.idx.size).astype(local_dtype))
        t2 = time.perf_counter()
        t_lf += t1 - t0
        t_ls += t2 - t1
    scale_loc = len(subs) / len(pick)
    A0 = bezier.coarse_matrix(A, bezier.restriction_2d(n, bc, ratio))
    kl, ku = bandlu.bandwidths(A0)
    rows = A0.shape[0] // rows_div
    t0 = time.perf_counter()
    lu = bandlu.BandLU(A0[:rows][:, :rows], kl, ku).factor()
    t1 = time.perf_counter()
    lu.solve(rng.standard_normal(rows) + 0j)
    t2 = time.perf_counter()
    scale_c = A0.shape[0] / rows
    desc = (f"oracle band-LU factor+solve of {len(pick)}/{len(subs)} {np.dtype(local_dtype).name} subdomains "
            f"(x{scale_loc:.0f}) and of the leading {rows}/{A0.shape[0]} rows of A_0 (x{scale_c:.0f})")
    return t_lf * scale_loc + (t1 - t0) * scale_c, t_ls * scale_loc + (t2 - t1) * scale_c, desc


def cpu_baseline(gpu_iters):
    """The oracle on the host cores, on a bounded sample of the same workload:
    four of the 256 local band-LU factor + solves (complex64), and the band-LU
    factor and solve of a leading block of A_0 (same bandwidth, 1/32 of its
    rows), scaled to the full workload; a solve is setup + (GPU iteration
    count) applications of M^{-1} (the oracle runs the same algorithm)."""
    import numpy as np

    from oracle import problem
    t_start = time.perf_counter()
    setup_s, apply_s, desc = oracle_sample(N_GRID, problem.SOMMERFELD, NSUB, OVERLAP, RATIO, np.complex64,
                                           [0, 17, 120, 255], 32, k=K_WAVE)
    total_s = setup_s + gpu_iters * apply_s
    return {"value": 1.0 / total_s, "unit": "solves/s", "cores": os.cpu_count(), "kind": "oracle",
            "estimate": True,
            "est_setup_s": setup_s, "est_apply_s": apply_s, "est_time_to_solution_s": total_s,
            "applies_per_s": 1.0 / apply_s, "wall_s_of_sample": time.perf_counter() - t_start,
            "sample": f"ESTIMATE, extrapolated from a timed sample: {desc}; time-to-solution = setup + "
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


def measured_coarse_traffic():
    """HBM bytes of one whole coarse solve: the committed per-launch counter
    table summed over its launches, or None if k_nd.hip changed since."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as fh:
            rec = json.load(fh)
        src = rec["kernels"]["nd_fwd_kernel"]
        with open(os.path.join(ROOT, src["source"]), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != src["sha256"]:
                return None
        return sum(r["traffic_bytes"] for r in rec["nd_levels"]["levels"])
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


def nd_subtree_depth(levels):
    """The depth from which the coarse solve runs by subtree (len(levels): none)."""
    return min([lv for lv, s in enumerate(levels) if s["subtree_workgroups"]] or [len(levels)])


def nd_launch_plan(levels):
    """The launches of one coarse solve in order, with the levels each covers:
    the forward subtree launch, the forward levels above it (deepest first;
    the root's forward part is done by its backward launch), the backward
    levels from the root, the backward subtree launch."""
    L, Ls = len(levels), nd_subtree_depth(levels)
    seq = [("forward", list(range(Ls, L)))] if Ls < L else []
    seq += [("forward", [lv]) for lv in range(min(L, Ls) - 1, 0, -1)]
    seq += [("backward", [lv]) for lv in range(min(L, Ls))]
    seq += [("backward", list(range(Ls, L)))] if Ls < L else []
    return seq


def nd_launches(levels):
    return len(nd_launch_plan(levels))


ND_KERNELS = ("nd_fwd_kernel(", "nd_bwd_kernel(", "nd_sub_fwd_kernel<", "nd_sub_bwd_kernel<")

PMC_KERNELS = {   # key used by the bench line -> (kernel-name fragments, all required; source file)
    f"arn_dots_kernel@{K_TIMED[1]}": (("arn_dots_kernel<", "cplx<double>"), "paper_2408_03571_amd/csrc/k_arnoldi.hip"),
    f"arn_update_kernel@{K_TIMED[1]}": (("arn_update_kernel<", "cplx<double>"),
                                        "paper_2408_03571_amd/csrc/k_arnoldi.hip"),
    f"arn_dots_kernel_c64basis@{K_TIMED[1]}": (("arn_dots_kernel<", "cplx<float>"),
                                               "paper_2408_03571_amd/csrc/k_arnoldi.hip"),
    f"arn_update_kernel_c64basis@{K_TIMED[1]}": (("arn_update_kernel<", "cplx<float>"),
                                                 "paper_2408_03571_amd/csrc/k_arnoldi.hip"),
    "local_solve_kernel<float, float, 2>": (("local_solve_kernel<float, float, 2,",),
                                            "paper_2408_03571_amd/csrc/k_local.hip"),
    "spmv_kernel": (("spmv_kernel(",), "paper_2408_03571_amd/csrc/k_grid.hip"),
    "nd_fwd_kernel": (("nd_fwd_kernel(",), "paper_2408_03571_amd/csrc/k_nd.hip"),
    "nd_bwd_kernel": (("nd_bwd_kernel(",), "paper_2408_03571_amd/csrc/k_nd.hip"),
    "nd_sub_fwd_kernel": (("nd_sub_fwd_kernel<",), "paper_2408_03571_amd/csrc/k_nd.hip"),
    "nd_sub_bwd_kernel": (("nd_sub_bwd_kernel<",), "paper_2408_03571_amd/csrc/k_nd.hip"),
}


def reduce_pmc(fetch_csv, write_csv, out_json):
    """HBM bytes per dispatch of the hot kernels from two rocprofv3 --pmc runs
    of `bench.py --profile-kernels` (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch), each scaled by what the counter reads for the 256 MiB device
    copy that the same command runs."""
    import csv
    import hashlib
    from collections import defaultdict

    def per_kernel(path, counter):
        vals, grids = defaultdict(list), defaultdict(list)
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
                grids[r["Kernel_Name"]].append((int(r["Grid_Size"]), float(r["Counter_Value"])))
        return vals, grids

    fv, fg = per_kernel(fetch_csv, "FETCH_SIZE")
    wv, wg = per_kernel(write_csv, "WRITE_SIZE")
    copy_kib = 256 * 1024.0
    # the calibration copy: the copyBuffer dispatches that move the most data
    cf = max(v for g, v in fg["__amd_rocclr_copyBuffer"])
    cw = max(v for g, v in wg["__amd_rocclr_copyBuffer"])
    fscale, wscale = copy_kib / cf, copy_kib / cw
    out = {"fetch_scale": fscale, "write_scale": wscale,
           "calibration": f"__amd_rocclr_copyBuffer of 256 MiB (torch copy_): FETCH_SIZE {cf:.1f} KiB, "
                          f"WRITE_SIZE {cw:.1f} KiB per dispatch", "kernels": {}}
    nu = N_GRID * N_GRID
    algo = {f"arn_dots_kernel@{K_TIMED[1]}": arnoldi_pass_bytes(nu, K_TIMED[1]),
            f"arn_update_kernel@{K_TIMED[1]}": arnoldi_pass_bytes(nu, K_TIMED[1]),
            f"arn_dots_kernel_c64basis@{K_TIMED[1]}": arnoldi_pass_bytes(nu, K_TIMED[1], 8),
            f"arn_update_kernel_c64basis@{K_TIMED[1]}": arnoldi_pass_bytes(nu, K_TIMED[1], 8),
            "local_solve_kernel<float, float, 2>": local_solve_bytes(subdomain_sizes(N_GRID, NSUB, OVERLAP), 8),
            "spmv_kernel": 2 * nu * 16}
    for key, (frags, src) in PMC_KERNELS.items():
        names = [n for n in fv if all(fr in n for fr in frags)]
        if not names or not any(n in wv for n in names):
            continue
        f = [v for n in names for v in fv[n]]
        w = [v for n in names for v in wv.get(n, [])]
        fk, wk = sum(f) / len(f), sum(w) / len(w)
        with open(os.path.join(ROOT, src), "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()
        out["kernels"][key] = {"kernel": names[0][:120], "dispatches": len(f), "fetch_kib": fk, "write_kib": wk,
                               "traffic_bytes": (fk * fscale + wk * wscale) * 1024.0,
                               "algorithmic_bytes": algo.get(key), "source": src, "sha256": digest}
    # nested-dissection launches: the coarse solves of the command, dispatch
    # by dispatch (nd_launch_plan's order), against the algorithmic bytes of
    # the levels each covers (forward: V once; backward: G and V)
    import paper_2408_03571_amd as hs
    levels = hs.hs_nd_plan_level_stats((N_GRID - 1) // RATIO + 1, (N_GRID - 1) // RATIO + 1, 2)
    plan = nd_launch_plan(levels)

    def nd_seq(path, counter):
        rows = []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and any(k in r["Kernel_Name"] for k in ND_KERNELS):
                    rows.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        rows.sort()
        return [v for _, v in rows]

    fs, ws_ = nd_seq(fetch_csv, "FETCH_SIZE"), nd_seq(write_csv, "WRITE_SIZE")
    per = len(plan)
    nsolve = min(len(fs), len(ws_)) // per
    table = []
    if nsolve:
        for q, (direction, lvs) in enumerate(plan):
            fwd = direction == "forward"
            fk = sum(fs[i * per + q] for i in range(nsolve)) / nsolve
            wk = sum(ws_[i * per + q] for i in range(nsolve)) / nsolve
            algo = 16 * sum(levels[lv]["v_entries"] if fwd else levels[lv]["g_entries"] + levels[lv]["v_entries"]
                            for lv in lvs if not (fwd and lv == 0))
            traffic = (fk * fscale + wk * wscale) * 1024.0
            table.append({"direction": direction, "levels": lvs, "fronts": sum(levels[lv]["fronts"] for lv in lvs),
                          "subtree": len(lvs) > 1 or levels[lvs[0]]["subtree_workgroups"] > 0,
                          "fetch_kib": fk, "write_kib": wk, "traffic_bytes": traffic, "algorithmic_bytes": algo,
                          "ratio": traffic / algo if algo else None})
    out["nd_levels"] = {"solves": nsolve, "levels": table}
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))



def reduce_pmc_batch(fetch_csv, write_csv, calib_json, out_json):
    """HBM bytes per dispatch of the batched kernels from two rocprofv3 --pmc
    runs of `bench.py --workload batching --steps 1 --warmup 0 --batch-only`
    (FETCH_SIZE, then WRITE_SIZE), scaled by the copy calibration recorded by
    reduce_pmc in calib_json on the same machine; the batched local solves are
    set against their algorithmic bytes (every instance's Schur inverses read
    twice, right-hand sides gathered and solutions written once)."""
    import csv
    from collections import defaultdict

    from workloads import batching_instances

    with open(calib_json) as fh:
        cal = json.load(fh)
    fscale, wscale = cal["fetch_scale"], cal["write_scale"]

    def per_kernel(path, counter):
        vals, by_id = defaultdict(list), defaultdict(dict)
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
                    by_id[r["Kernel_Name"]][int(r["Dispatch_Id"])] = float(r["Counter_Value"])
        return vals, by_id

    (fv, fid), (wv, wid) = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    algo_local = sum(local_solve_bytes(subdomain_sizes(c.n, c.nsub, c.overlap), 8) for c in batching_instances())
    out = {"calibration": cal["calibration"], "fetch_scale": fscale, "write_scale": wscale, "kernels": {}}
    for name in sorted(fv, key=lambda n: -sum(fv[n])):
        if name not in wv or not name.lstrip("void ").startswith("hs::"):
            continue
        fk, wk = sum(fv[name]) / len(fv[name]), sum(wv[name]) / len(wv[name])
        rec = {"dispatches": len(fv[name]), "fetch_kib": fk, "write_kib": wk,
               "traffic_bytes": (fk * fscale + wk * wscale) * 1024.0}
        if "local_solve_kernel<float, float, 2" in name:
            # the solve's applications skip the instances that have converged:
            # the largest dispatch (every instance active, as in the schedule
            # tuner's applications) is the one to set against the algorithmic
            # bytes; the two runs number their dispatches alike
            full = max(fid[name][i] * fscale + wid[name].get(i, 0.0) * wscale for i in fid[name]) * 1024.0
            rec.update({"traffic_bytes_all_active": full, "algorithmic_bytes": algo_local,
                        "ratio_all_active": full / algo_local})
        out["kernels"][name[:140]] = rec
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def nd_launch_table(trace_csv, pmc_json):
    """Per-launch table of the n = 1025 coarse solve from a rocprofv3 kernel
    trace of `bench.py --profile-kernels` (median duration over the coarse
    solves that ran alone, i.e. with no local-solve dispatch beside them) and
    the counter table reduce_pmc wrote (traffic over algorithmic bytes)."""
    import csv
    from collections import defaultdict

    import paper_2408_03571_amd as hs
    with open(trace_csv) as fh:
        rows = list(csv.DictReader(fh))
    levels = hs.hs_nd_plan_level_stats((N_GRID - 1) // RATIO + 1, (N_GRID - 1) // RATIO + 1, 2)
    plan = nd_launch_plan(levels)
    per = len(plan)
    nd = sorted((r for r in rows if any(k in r["Kernel_Name"] for k in ND_KERNELS)),
                key=lambda r: int(r["Start_Timestamp"]))
    loc = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows
           if "local_solve_kernel" in r["Kernel_Name"]]
    solves = [nd[i * per:(i + 1) * per] for i in range(len(nd) // per)]

    def alone(sv):
        a, b = int(sv[0]["Start_Timestamp"]), int(sv[-1]["End_Timestamp"])
        return not any(x < b and y > a for x, y in loc)

    alone_s = [sv for sv in solves if alone(sv)]
    dur, spans = defaultdict(list), []
    for sv in alone_s:
        for q, r in enumerate(sv):
            dur[q].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        spans.append((int(sv[-1]["End_Timestamp"]) - int(sv[0]["Start_Timestamp"])) / 1e3)
    with open(pmc_json) as fh:
        pm = json.load(fh)["nd_levels"]["levels"]
    med = lambda v: sorted(v)[len(v) // 2]  # noqa: E731
    print(f"coarse solves alone in the trace: {len(alone_s)} of {len(solves)}; median span {med(spans):.1f} us\n")
    print("| launch | levels | fronts | workgroups | algorithmic MB | traffic / algorithmic | median us | GB/s |")
    print("|---|---|---:|---:|---:|---:|---:|---:|")
    tot = ta = 0.0
    for q, (d, lvs) in enumerate(plan):
        m, a = med(dur[q]), pm[q]["algorithmic_bytes"]
        tot += m
        ta += a
        sub = len(lvs) > 1 or levels[lvs[0]]["subtree_workgroups"] > 0
        wg = levels[lvs[0]]["subtree_workgroups" if sub else ("fwd_workgroups" if d == "forward" else "bwd_workgroups")]
        name = ("nd_sub_fwd_kernel" if d == "forward" else "nd_sub_bwd_kernel") if sub else \
            ("nd_fwd_kernel" if d == "forward" else "nd_bwd_kernel")
        lv = f"{lvs[0]}-{lvs[-1]}" if len(lvs) > 1 else str(lvs[0])
        print(f"| {name} | {lv} | {sum(levels[x]['fronts'] for x in lvs)} | {wg} | {a / 1e6:.1f} | "
              f"{pm[q]['ratio']:.3f} | {m:.1f} | {a / m / 1e3:.0f} |")
    print(f"\nsum of medians {tot:.1f} us for {ta / 1e9:.3f} GB ({ta / tot / 1e3:.0f} GB/s)")


DIFF_N, DIFF_K0, DIFF_NSRC, DIFF_NSUB, DIFF_TOL = 513, 150.0, 4, 8, 1e-8


def differentiation_run(args):
    """The differentiation workload: n = 513, k^2 = k0^2 (1 + 0.2 g) with
    k0 = 150 and g eight seeded Gaussian bumps, four point sources at seeded
    interior nodes (x < 0.8), receivers on the column nearest x = 0.9, data d
    from the seed-1 field.  A step is one loss L = 1/2 sum_s ||P u_s - d_s||^2
    and its gradient dL/dk^2: one preconditioner (8 x 8 subdomains, overlap
    2, Bezier H = 2h, RAS2, complex128 local factors), four forward and four
    unconjugated adjoint solves (flexible GMRES to 1e-8) and the per-node
    gradient terms, through helmholtz_solve_multi.  value = gradients per
    second.  The gradient is checked in the same run against a central
    difference along one seeded direction."""
    import numpy as np
    import torch

    import paper_2408_03571_amd as hs
    from workloads import differentiation_setup, k2_field
    dev = "cuda:0"
    torch.cuda.set_device(0)
    n, bc = DIFF_N, hs.HS_BC_SOMMERFELD
    k2 = torch.from_numpy(k2_field(n, DIFF_K0, 0)).to(dev)
    k2_true = torch.from_numpy(k2_field(n, DIFF_K0, 1)).to(dev)
    srcs, col = differentiation_setup(n, DIFF_K0, DIFF_NSRC, seed=0)
    # Sommerfeld: every grid node is an unknown, x fastest.  Receivers: the
    # grid column `col`; sources: e_s / h^2 at interior nodes (Sec. 2; an
    # interior row carries no boundary scaling)
    Pidx = torch.arange(n, device=dev) * n + col
    F = torch.zeros(len(srcs), n * n, dtype=torch.complex128, device=dev)
    for q, (si, sj) in enumerate(srcs):
        assert 0 < si < n - 1 and 0 < sj < n - 1
        F[q, sj * n + si] = float(n - 1) ** 2
    kw = dict(bc=bc, nsub=DIFF_NSUB, overlap=2, ratio=2, prec=hs.HS_C128, maxit=1000)
    with torch.no_grad():
        D = hs.helmholtz_solve_multi(k2_true, F, n, tol=1e-10, **kw)[:, Pidx].clone()

    def loss(k2_in, tol):
        U = hs.helmholtz_solve_multi(k2_in, F, n, tol=tol, **kw)
        return 0.5 * ((U[:, Pidx] - D).abs() ** 2).sum(), U

    def step():
        k2_t = k2.clone().requires_grad_(True)
        L, U = loss(k2_t, DIFF_TOL)
        L.backward()
        return L.item(), k2_t.grad, U.grad_fn

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        L, g, fn = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    fwd_its = [st["iters"] for st in fn.stats]
    adj_its = [st["iters"] for st in fn.adjoint_stats]
    # central difference along one seeded unit direction (outside the timed steps)
    rng = np.random.default_rng(2)
    d = rng.standard_normal((n, n))
    d /= np.linalg.norm(d)
    d_t = torch.from_numpy(d).to(dev)
    eps = 1e-4 * float(k2.abs().max()) * n
    with torch.no_grad():
        Lp = loss(k2 + eps * d_t, 1e-11)[0].item()
        Lm = loss(k2 - eps * d_t, 1e-11)[0].item()
    fd = (Lp - Lm) / (2 * eps)
    an = float((g * d_t).sum())
    # the dominant kernels: the DCGS2 dot pass at the mean Arnoldi step and one application of M^{-1}
    P = hs.hs_assemble(n, 1.0, bc, k2.reshape(-1).contiguous())
    M = hs.hs_setup_schwarz(P, DIFF_NSUB, 2, 2, hs.HS_RAS2, hs.HS_C128)
    N = hs.hs_problem_size(P)
    kmid = int(np.mean(fwd_its + adj_its) / 2)
    ws = torch.empty(hs.hs_gmres_workspace_bytes(P, kmid + 1), dtype=torch.uint8, device=dev)
    from workloads import random_vectors
    v = torch.from_numpy(random_vectors(1, N, seed=0)).to(dev)[0].contiguous()
    t_dots = hs.hs_time_arnoldi(P, kmid, 0, ws, v, reps=20)
    t_apply = hs.hs_time_step(M, 2, v, reps=20)
    # one application of M^{-1} to all sources at once (the batch repeats M)
    B = hs.hs_batch_create([M] * DIFF_NSRC)
    vs = torch.from_numpy(random_vectors(DIFF_NSRC, N, seed=0)).to(dev).reshape(-1).contiguous()
    t_apply_all = hs.hs_batch_time(B, 2, vs, reps=20)
    del B
    rl = roofline(f"arn_dots_kernel (DCGS2 dot pass at the mean Arnoldi step k={kmid})",
                  arnoldi_pass_bytes(N, kmid), t_dots)
    cpu = None
    if not args.no_cpu:
        t_s = time.perf_counter()
        setup_s, apply_s, desc = oracle_sample(n, bc, DIFF_NSUB, 2, 2, np.complex128, [0, 9, 36, 63], 8,
                                               k2=k2_field(n, DIFF_K0, 0))
        total_s = setup_s + sum(fwd_its + adj_its) * apply_s
        cpu = {"value": 1.0 / total_s, "unit": "gradients/s", "cores": os.cpu_count(), "kind": "oracle",
               "estimate": True, "est_setup_s": setup_s, "est_apply_s": apply_s, "est_gradient_s": total_s,
               "wall_s_of_sample": time.perf_counter() - t_s,
               "sample": f"ESTIMATE, extrapolated from a timed sample: {desc}; a gradient = setup + "
                         f"{sum(fwd_its + adj_its)} applies (the GPU's forward and adjoint iteration counts; the "
                         f"Arnoldi work is not included)"}
    line = {
        "metric": "dL/d(k^2) gradients/s (4 sources, forward + adjoint solves, MP-2 n=513 heterogeneous k)",
        "value": 1e3 / ms, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "differentiation: MP-2 n=513, k^2 = 150^2 (1 + 0.2 g), 4 sources, receivers at "
                               "x = 0.9, 8x8 subdomains, overlap 2, Bezier H=2h, RAS2, FGMRES tol 1e-8"},
        "loss": L, "forward_iterations": fwd_its, "adjoint_iterations": adj_its,
        "fd_check": {"central_difference": fd, "adjoint": an, "rel_err": abs(fd - an) / abs(an)},
        "apply_ms": t_apply, f"apply_ms_{DIFF_NSRC}_sources_together": t_apply_all, "roofline": rl,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="mixed,mixed_s,fp64,mixed_cb")
    ap.add_argument("--profile-kernels", action="store_true")
    ap.add_argument("--profile-setup", action="store_true", help="three n=1025 set-ups (factor phase)")
    ap.add_argument("--workload", default="precision", choices=["precision", "batching", "differentiation"])
    ap.add_argument("--batch-only", action="store_true",
                    help="batching workload: only the batched solves (for a kernel trace)")
    ap.add_argument("--reduce-pmc", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON"),
                    help="reduce two rocprofv3 --pmc runs of --profile-kernels to HBM bytes per dispatch")
    ap.add_argument("--nd-launch-table", nargs=2, metavar=("TRACE_CSV", "PMC_JSON"),
                    help="per-launch table of the coarse solve from a kernel trace of --profile-kernels and a "
                         "--reduce-pmc output")
    ap.add_argument("--reduce-pmc-batch", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "CALIB_JSON", "OUT_JSON"),
                    help="the same for two --pmc runs of the batching workload (--batch-only), calibrated by the "
                         "copy factors of a --reduce-pmc output")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the solver has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.reduce_pmc:
        reduce_pmc(*args.reduce_pmc)
        return
    if args.nd_launch_table:
        nd_launch_table(*args.nd_launch_table)
        return
    if args.reduce_pmc_batch:
        reduce_pmc_batch(*args.reduce_pmc_batch)
        return
    if args.profile_kernels:
        profile_kernels()
        return
    if args.profile_setup:
        profile_setup()
        return
    if args.workload == "batching":
        batching_run(args)
        return
    if args.workload == "differentiation":
        differentiation_run(args)
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
    # the two DCGS2 passes run once per iteration over the same rows; the
    # slower one is the dominant kernel of the step (headline), each credited
    # with its share of the orthogonalisation time
    d_ms, u_ms = kt[f"dots{k1}"], kt[f"update{k1}"]
    passes = [
        (u_ms, f"arn_update_kernel (DCGS2 update pass at Arnoldi step k={k1})", f"arn_update_kernel@{k1}"),
        (d_ms, f"arn_dots_kernel (DCGS2 dot pass at Arnoldi step k={k1}, fused A z)", f"arn_dots_kernel@{k1}"),
    ]
    passes.sort(key=lambda p: -p[0])
    pass_rl = [roofline(name, arnoldi_pass_bytes(nu, k1), ms,
                        {"time_share_of_step": share["orthogonalisation"] * ms / (d_ms + u_ms)}, traffic_key=key)
               for ms, name, key in passes]
    rl = pass_rl[0]
    others = [
        pass_rl[1],
        roofline("local_solve_kernel<float,2> (all 256 subdomain solves, complex64)",
                 local_solve_bytes(sizes, 8), kt["local"], traffic_key="local_solve_kernel<float, float, 2>"),
        roofline(f"nested-dissection coarse solve ({nd_launches(kt['levels'])} launches)",
                 mx["info"]["coarse_solve_bytes"], kt["coarse"], {"traffic": measured_coarse_traffic()}),
        roofline("spmv_kernel", 2 * nu * 16, kt["spmv"], traffic_key="spmv_kernel"),
    ]
    if "mixed_cb" in forms:
        kc = forms["mixed_cb"]["kt"]
        others += [
            roofline(f"arn_dots_kernel, complex64 basis (mixed_cb form, k={k1})", arnoldi_pass_bytes(nu, k1, 8),
                     kc[f"dots{k1}"], traffic_key=f"arn_dots_kernel_c64basis@{k1}"),
            roofline(f"arn_update_kernel, complex64 basis (mixed_cb form, k={k1})", arnoldi_pass_bytes(nu, k1, 8),
                     kc[f"update{k1}"], traffic_key=f"arn_update_kernel_c64basis@{k1}"),
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
                                  "tuning_s": tuned["tuning_s"], "complex64_basis": tuned.get("shape_c64_basis")},
        "apply_schedule_fork_level_local_grid": tuned.get("schedules"),
        "roofline": rl,
        "roofline_others": others,
        "cpu_baseline": cpu,
    }
    if "mixed" in forms and "fp64" in forms:
        line["speedup_mixed_vs_fp64"] = {
            "time_to_solution": forms["fp64"]["ms_per_solve"] / forms["mixed"]["ms_per_solve"],
            "applies_per_s": forms["mixed"]["applies_per_s"] / forms["fp64"]["applies_per_s"]}
    if "mixed_cb" in forms and "fp64" in forms:
        line["speedup_mixed_cb_vs_fp64"] = {
            "time_to_solution": forms["fp64"]["ms_per_solve"] / forms["mixed_cb"]["ms_per_solve"],
            "applies_per_s": forms["mixed_cb"]["applies_per_s"] / forms["fp64"]["applies_per_s"]}
    if "mixed_s" in forms and "fp64" in forms:
        line["speedup_mixed_s_vs_fp64"] = {
            "time_to_solution": forms["fp64"]["ms_per_solve"] / forms["mixed_s"]["ms_per_solve"],
            "applies_per_s": forms["mixed_s"]["applies_per_s"] / forms["fp64"]["applies_per_s"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
