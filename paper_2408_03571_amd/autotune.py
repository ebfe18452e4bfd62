"""Autotuner for the launch shapes of the hot kernels.

Orthogonalisation (tune_arnoldi):

The two streaming passes of the DCGS2 Arnoldi step (dot pass and update pass)
take a shape per problem size: unknowns per lane of a wave (1, 2, 4, 8: the
tile each wave streams from every basis vector) and basis vectors per loop
trip (2, 4: the band of rows whose loads are in flight together).  The tuner
times every shape on the device with HIP events through hs_time_arnoldi at
two Krylov depths, picks the one with the least summed time, installs it with
hs_set_arnoldi_config and records it in a JSON cache keyed by device name and
problem size, so a later process can install the same table without timing
(a fixed table makes solves reproducible: the unknowns per lane fix how the
dot products are partitioned).  The table holds one shape per problem size;
the best shape depends on how the basis is stored (a complex64 basis moves
half the bytes per trip), so the tuner takes the storage to time with and the
cache keeps one record per size and storage.

Batches (tune_batch): the persistent launch that runs every subdomain solve
of a batch takes a workgroup count; fewer workgroups than the subdomains
leave CU slots to the coarse sweeps running beside it.  The tuner times one
whole batched application of M^{-1} for each candidate count and installs
the fastest (the count changes no result).

Application schedule (tune_schedule): the local solves of one application
of M^{-1} run beside the coarse branch; forking them after the first few
forward levels of the coarse solve keeps them away from its bandwidth-bound
leaf levels, and fewer local workgroups leave CUs to the level sweeps.  The
tuner times whole applications for a few (fork level, local grid) pairs and
installs the fastest (the schedule changes no result).

Argument marshalling and timing only; every timed step runs in the HIP
library.
"""
from __future__ import annotations

import json
import os
import time

from . import (HS_C128, hs_batch_set_schedule, hs_batch_time, hs_gmres_workspace_bytes, hs_precond_set_schedule,
               hs_problem_size, hs_set_arnoldi_config, hs_time_arnoldi, hs_time_step)

SHAPES = [(e, r) for e in (1, 2, 4, 8) for r in (2, 4)]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "helmschwarz", "tune.json")


def _device_key():
    import torch
    return torch.cuda.get_device_name(0)


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(path, table):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_arnoldi(P, depths=(32, 256), reps=5, cache=DEFAULT_CACHE, force=False, basis_prec=HS_C128):
    """Pick the launch shape of the DCGS2 passes for the size of problem P,
    timed with the basis stored as basis_prec.

    Returns a dict with the chosen shape, the timings of every shape (ms per
    pass at each depth) and whether it came from the cache.  The shape is
    installed for this process either way."""
    import torch
    N = hs_problem_size(P)
    key = f"{_device_key()}|arnoldi|{N}" + ("" if basis_prec == HS_C128 else f"|basis{basis_prec}")
    table = _load(cache) if cache else {}
    if not force and key in table:
        e, r = table[key]["shape"]
        hs_set_arnoldi_config(N, e, r)
        return dict(table[key], cached=True)
    kmax = max(depths)
    ws = torch.empty(hs_gmres_workspace_bytes(P, kmax + 1), dtype=torch.uint8, device="cuda")
    g = torch.Generator(device="cpu").manual_seed(0)
    v = torch.complex(torch.randn(N, generator=g, dtype=torch.float64),
                      torch.randn(N, generator=g, dtype=torch.float64)).to("cuda")
    t0 = time.perf_counter()
    times = {}
    for e, r in SHAPES:
        hs_set_arnoldi_config(N, e, r)
        tot = 0.0
        per = {}
        for k in depths:
            td = hs_time_arnoldi(P, k, 0, ws, v, reps=reps, basis_prec=basis_prec)
            tu = hs_time_arnoldi(P, k, 1, ws, v, reps=reps, basis_prec=basis_prec)
            per[str(k)] = [td, tu]
            tot += td + tu
        times[f"{e},{r}"] = {"per_depth_ms": per, "total_ms": tot}
    best = min(SHAPES, key=lambda s: times[f"{s[0]},{s[1]}"]["total_ms"])
    hs_set_arnoldi_config(N, *best)
    rec = {"shape": list(best), "n_unknowns": N, "basis_prec": basis_prec, "depths": list(depths),
           "times": times, "tuning_s": time.perf_counter() - t0}
    if cache:
        table[key] = rec
        _save(cache, table)
    del ws
    return dict(rec, cached=False)


def apply_cache(cache=DEFAULT_CACHE):
    """Install every shape recorded for this device; returns how many."""
    dev = _device_key()
    count = 0
    for key, rec in _load(cache).items():
        parts = key.split("|")
        if len(parts) != 3:   # records of another basis storage are not installed
            continue
        d, kind, n = parts
        if d == dev and kind == "arnoldi":
            hs_set_arnoldi_config(int(n), *rec["shape"])
            count += 1
    return count


BATCH_SCHEDULES = [(f, g) for f in (0, 4, 8, 12) for g in (0, 1024)]   # g = 0: one workgroup per subdomain


def tune_batch(B, r, reps=10, schedules=BATCH_SCHEDULES):
    """Pick the schedule of the batched application (fork level of the local
    solves, workgroups of their launch) by timing whole batched applications
    on the batch vector r; returns the choice and the timings (ms per
    application)."""
    t0 = time.perf_counter()
    times = {}
    for f, g in schedules:
        hs_batch_set_schedule(B, f, g)
        times[(f, g)] = hs_batch_time(B, 2, r, reps=reps)
    best = min(times, key=times.get)
    hs_batch_set_schedule(B, *best)
    return {"schedule": list(best), "local_grid": best[1], "apply_ms": {f"{f},{g}": t for (f, g), t in times.items()},
            "tuning_s": time.perf_counter() - t0}


SCHEDULES = [(f, g) for f in (0, 1, 2, 3, 4, 6) for g in (0, 128, 192)]


def tune_schedule(M, r, reps=20, schedules=SCHEDULES):
    """Pick the application schedule of preconditioner M by timing whole
    applications on the vector r; returns the choice and the timings (ms per
    application)."""
    t0 = time.perf_counter()
    times = {}
    for f, g in schedules:
        hs_precond_set_schedule(M, f, g)
        times[f"{f},{g}"] = hs_time_step(M, 2, r, reps=reps)
    best = min(schedules, key=lambda s: times[f"{s[0]},{s[1]}"])
    hs_precond_set_schedule(M, *best)
    return {"schedule": list(best), "apply_ms": times, "tuning_s": time.perf_counter() - t0}
