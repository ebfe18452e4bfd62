"""Batched instances: one launch per stage of M^{-1} over every instance, and
lockstep flexible GMRES over all of them (hs_batch_*).

The batched launches run each instance's arithmetic unchanged (same kernels,
same per-instance partition of every reduction), so each instance's M^{-1} r
is bitwise equal to its own single application, and with the same DCGS2
launch shape each instance's GMRES iterate is bitwise equal to its single
solve.  The batch mixes coarse ratios 2 and 4 (different numbers of
restriction / prolongation stages and different nested-dissection depths),
sizes and precisions.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2408_03571_amd as hs  # noqa: E402
from oracle import problem  # noqa: E402
from workloads import batching_instances, random_vector  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"

# (n, ns, ratio, source)
MIX = [(129, 4, 4, (30, 70)), (65, 4, 2, (32, 32)), (193, 5, 4, (100, 40)), (129, 4, 2, (64, 64)),
       (97, 3, 2, (20, 75))]


def build(mix, prec, variant=hs.HS_RAS2):
    out = []
    for n, ns, ratio, src in mix:
        k = 0.3 * (n - 1)
        P = hs.hs_assemble(n, k, problem.SOMMERFELD)
        M = hs.hs_setup_schwarz(P, ns, 2, ratio, variant=variant, prec=prec)
        out.append((P, M, n, src))
    return out


def batch_vector(parts):
    return torch.cat([torch.from_numpy(np.ascontiguousarray(p)) for p in parts]).to(DEV)


@pytest.mark.parametrize("prec,variant", [(hs.HS_C64, hs.HS_RAS2), (hs.HS_C128, hs.HS_RAS2), (hs.HS_C64S, hs.HS_RAS2),
                                          (hs.HS_C64, hs.HS_SHS2), (hs.HS_C128, hs.HS_AS2)])
def test_batch_apply_matches_single(prec, variant):
    inst = build(MIX, prec, variant)
    B = hs.hs_batch_create([M for _, M, _, _ in inst])
    rs = [random_vector(hs.hs_problem_size(P), seed=20 + i) for i, (P, _, _, _) in enumerate(inst)]
    r = batch_vector(rs)
    z = torch.empty_like(r)
    hs.hs_batch_apply_Minv(B, r, z)
    off = B.offsets
    assert off[-1] == r.numel()
    for i, (P, M, _, _) in enumerate(inst):
        zi = torch.empty(hs.hs_problem_size(P), dtype=torch.complex128, device=DEV)
        hs.hs_apply_Minv(M, dev_vec(rs[i]), zi)
        assert torch.equal(z[off[i]:off[i + 1]], zi), i
    # a second application on other data reuses the batch state
    r2 = batch_vector([random_vector(hs.hs_problem_size(P), seed=40 + i) for i, (P, _, _, _) in enumerate(inst)])
    z2 = torch.empty_like(r2)
    hs.hs_batch_apply_Minv(B, r2, z2)
    P0, M0, _, _ = inst[0]
    zi = torch.empty(hs.hs_problem_size(P0), dtype=torch.complex128, device=DEV)
    hs.hs_apply_Minv(M0, r2[off[0]:off[1]].contiguous(), zi)
    assert torch.equal(z2[off[0]:off[1]], zi)


def dev_vec(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


@pytest.mark.parametrize("graph,basis,variant", [(True, hs.HS_C128, hs.HS_RAS2), (False, hs.HS_C128, hs.HS_RAS2),
                                                (True, hs.HS_C64, hs.HS_RAS2), (True, hs.HS_C128, hs.HS_SHS2)])
def test_batch_gmres_matches_single(graph, basis, variant):
    inst = build(MIX, hs.HS_C64, variant)
    B = hs.hs_batch_create([M for _, M, _, _ in inst])
    total = B.offsets[-1]
    ept, rows = hs.hs_get_arnoldi_config(total)
    bs = [problem.rhs(n, problem.SOMMERFELD, [src]) for _, _, n, src in inst]
    b = batch_vector(bs)
    x = torch.zeros_like(b)
    stats = hs.hs_batch_gmres_solve(B, b, x, tol=1e-6, maxit=400, graph=graph, basis_prec=basis)
    off = B.offsets
    sizes = sorted({hs.hs_problem_size(P) for P, _, _, _ in inst})
    try:
        for N in sizes:
            hs.hs_set_arnoldi_config(N, ept, rows)
        for i, (P, M, n, src) in enumerate(inst):
            xi = torch.zeros(hs.hs_problem_size(P), dtype=torch.complex128, device=DEV)
            st, _ = hs.hs_gmres_solve(P, M, dev_vec(bs[i]), xi, tol=1e-6, maxit=400, basis_prec=basis)
            assert stats[i]["converged"] and st["converged"], i
            assert stats[i]["iters"] == st["iters"], (i, stats[i]["iters"], st["iters"])
            assert stats[i]["relres_true"] == st["relres_true"]
            assert torch.equal(x[off[i]:off[i + 1]], xi), i
    finally:
        for N in sizes:
            hs.hs_set_arnoldi_config(N, 0, 0)


def test_array_form_equals_the_handle_form():
    # hs_gmres_solve_batch takes plain arrays of problems, preconditioners and
    # vectors and one workspace for everything; it must return the handle
    # form's solutions bit for bit (same batch, same options)
    inst = build(MIX, hs.HS_C64)
    Ms = [M for _, M, _, _ in inst]
    B = hs.hs_batch_create(Ms)
    bs = [problem.rhs(n, problem.SOMMERFELD, [src]) for _, _, n, src in inst]
    b = batch_vector(bs)
    x = torch.zeros_like(b)
    ref = hs.hs_batch_gmres_solve(B, b, x, tol=1e-6, maxit=400)
    xs = [torch.full((hs.hs_problem_size(P),), complex(np.nan, np.nan), dtype=torch.complex128, device=DEV)
          for P, _, _, _ in inst]
    stats = hs.hs_gmres_solve_batch([P for P, _, _, _ in inst], Ms, [dev_vec(v) for v in bs], xs, tol=1e-6,
                                    maxit=400)
    off = B.offsets
    for i in range(len(inst)):
        assert stats[i]["converged"] and stats[i]["iters"] == ref[i]["iters"], i
        assert stats[i]["relres_true"] == ref[i]["relres_true"]
        assert torch.equal(xs[i], x[off[i]:off[i + 1]]), i
    # the array form refuses a preconditioner that is not built on its problem
    with pytest.raises(hs.HSError) as e:
        hs.hs_gmres_solve_batch([inst[1][0], inst[0][0]], Ms[:2], [dev_vec(v) for v in bs[:2]], xs[:2])
    assert e.value.status == hs.HS_EINVAL


def test_batch_zero_rhs_and_noconv():
    inst = build(MIX[:3], hs.HS_C64)
    B = hs.hs_batch_create([M for _, M, _, _ in inst])
    bs = [problem.rhs(n, problem.SOMMERFELD, [src]) for _, _, n, src in inst]
    bs[1] = np.zeros_like(bs[1])
    b = batch_vector(bs)
    x = torch.full_like(b, 7.0)
    stats = hs.hs_batch_gmres_solve(B, b, x, tol=1e-6, maxit=400)
    off = B.offsets
    assert stats[1]["converged"] and stats[1]["iters"] == 0
    assert float(x[off[1]:off[2]].abs().max()) == 0.0
    assert stats[0]["converged"] and stats[2]["converged"]
    stats = hs.hs_batch_gmres_solve(B, b, x, tol=1e-12, maxit=3)
    assert stats[0]["status"] == hs.HS_ENOCONV
    assert stats[0]["iters"] == 3 and not stats[0]["converged"]
    with pytest.raises(hs.HSError):
        hs.hs_batch_gmres_solve(B, b, x, tol=1e-12, maxit=3, raise_on_noconv=True)


def test_batch_rejects_mixed_precisions_and_variants():
    a = build(MIX[:1], hs.HS_C64)
    c = build(MIX[1:2], hs.HS_C128)
    with pytest.raises(hs.HSError):
        hs.hs_batch_create([a[0][1], c[0][1]])
    P = hs.hs_assemble(65, 19.2, problem.SOMMERFELD)
    M = hs.hs_setup_schwarz(P, 4, 2, 2, variant=hs.HS_SHS2, prec=hs.HS_C64)
    with pytest.raises(hs.HSError):
        hs.hs_batch_create([a[0][1], M])


def test_batching_workload_subset():
    """A 12-instance slice of the batching workload (sizes up to 257): every
    instance converges to 1e-6 true residual; each equals its single solve."""
    cfgs = [c for c in batching_instances(48, seed=0) if c.n <= 257][:12]
    inst = []
    for c in cfgs:
        P = hs.hs_assemble(c.n, c.k, problem.SOMMERFELD)
        M = hs.hs_setup_schwarz(P, c.nsub, c.overlap, c.ratio, variant=hs.HS_RAS2, prec=hs.HS_C64)
        inst.append((P, M, c))
    B = hs.hs_batch_create([M for _, M, _ in inst])
    bs = [problem.rhs(c.n, problem.SOMMERFELD, [c.src]) for _, _, c in inst]
    b = batch_vector(bs)
    x = torch.zeros_like(b)
    stats = hs.hs_batch_gmres_solve(B, b, x, tol=1e-6, maxit=600)
    assert all(s["converged"] and s["relres_true"] <= 1e-6 for s in stats)
    ept, rows = hs.hs_get_arnoldi_config(B.offsets[-1])
    off = B.offsets
    sizes = sorted({hs.hs_problem_size(P) for P, _, _ in inst})
    try:
        for N in sizes:
            hs.hs_set_arnoldi_config(N, ept, rows)
        for i in (0, len(inst) // 2, len(inst) - 1):
            P, M, c = inst[i]
            xi = torch.zeros(hs.hs_problem_size(P), dtype=torch.complex128, device=DEV)
            st, _ = hs.hs_gmres_solve(P, M, dev_vec(bs[i]), xi, tol=1e-6, maxit=600)
            assert stats[i]["iters"] == st["iters"]
            assert torch.equal(x[off[i]:off[i + 1]], xi)
    finally:
        for N in sizes:
            hs.hs_set_arnoldi_config(N, 0, 0)


def test_batch_local_grid_changes_nothing():
    """The persistent local-solve launch gives the same bits for any
    workgroup count (each subdomain is solved by one workgroup, in the same
    arithmetic order)."""
    inst = build(MIX, hs.HS_C64)
    B = hs.hs_batch_create([M for _, M, _, _ in inst])
    r = batch_vector([random_vector(hs.hs_problem_size(P), seed=60 + i) for i, (P, _, _, _) in enumerate(inst)])
    ref = None
    for g in (0, 1, 7, 64, 256):
        hs.hs_batch_set_local_grid(B, g)
        z = torch.empty_like(r)
        hs.hs_batch_apply_Minv(B, r, z)
        if ref is None:
            ref = z
        assert torch.equal(z, ref), g
    # the fork level of the local solves (before, inside or after the forward
    # coarse levels) changes nothing either, in a graph-replayed solve too
    bs = [problem.rhs(n, problem.SOMMERFELD, [src]) for _, _, n, src in inst]
    b = batch_vector(bs)
    xs = []
    for f, g in ((0, 0), (2, 0), (4, 64), (50, 0)):
        hs.hs_batch_set_schedule(B, f, g)
        z = torch.empty_like(r)
        hs.hs_batch_apply_Minv(B, r, z)
        assert torch.equal(z, ref), (f, g)
        x = torch.zeros_like(b)
        hs.hs_batch_gmres_solve(B, b, x, tol=1e-6, maxit=400)
        xs.append(x)
    assert all(torch.equal(x, xs[0]) for x in xs[1:])


@pytest.mark.parametrize("variant", [hs.HS_RAS2, hs.HS_SHS2])
def test_batch_repeated_handle_is_a_multi_rhs_solve(variant):
    """A handle repeated in a batch stands for several right-hand sides of one
    problem: the repeats get scratch of their own, so every right-hand side's
    M^{-1} r and GMRES iterate are bitwise those of its own single solve, also
    beside another problem in the same batch."""
    (P0, M0, n0, _), (P1, M1, n1, _) = build(MIX[:2], hs.HS_C64, variant)
    Ps, Ms = [P0, P1, P0, P0], [M0, M1, M0, M0]
    B = hs.hs_batch_create(Ms)
    off = B.offsets
    rs = [random_vector(hs.hs_problem_size(P), seed=60 + i) for i, P in enumerate(Ps)]
    r = batch_vector(rs)
    z = torch.empty_like(r)
    hs.hs_batch_apply_Minv(B, r, z)
    for i, (P, M) in enumerate(zip(Ps, Ms)):
        zi = torch.empty(hs.hs_problem_size(P), dtype=torch.complex128, device=DEV)
        hs.hs_apply_Minv(M, dev_vec(rs[i]), zi)
        assert torch.equal(z[off[i]:off[i + 1]], zi), i
    srcs = [(40, 60), (32, 32), (90, 20), (64, 64)]
    ns = [n0, n1, n0, n0]
    bs = [problem.rhs(n, problem.SOMMERFELD, [src]) for n, src in zip(ns, srcs)]
    b = batch_vector(bs)
    x = torch.zeros_like(b)
    ept, rows = hs.hs_get_arnoldi_config(off[-1])
    stats = hs.hs_batch_gmres_solve(B, b, x, tol=1e-6, maxit=400)
    sizes = sorted({hs.hs_problem_size(P) for P in Ps})
    try:
        for N in sizes:
            hs.hs_set_arnoldi_config(N, ept, rows)
        for i, (P, M) in enumerate(zip(Ps, Ms)):
            xi = torch.zeros(hs.hs_problem_size(P), dtype=torch.complex128, device=DEV)
            st, _ = hs.hs_gmres_solve(P, M, dev_vec(bs[i]), xi, tol=1e-6, maxit=400)
            assert stats[i]["converged"] and st["converged"], i
            assert stats[i]["iters"] == st["iters"], (i, stats[i]["iters"], st["iters"])
            assert torch.equal(x[off[i]:off[i + 1]], xi), i
    finally:
        for N in sizes:
            hs.hs_set_arnoldi_config(N, 0, 0)


def test_block_coarse_lds_limit_outlives_a_smaller_batch():
    """The dynamic-LDS limit of the block coarse kernels belongs to the kernel,
    not to a batch: a batch created later, with smaller fronts, leaves the
    earlier batch's launches valid and its results unchanged."""
    (Pb, Mb, _, _), = build([(193, 5, 2, (100, 40))], hs.HS_C64)
    (Ps, Ms, _, _), = build([(65, 4, 2, (32, 32))], hs.HS_C64)
    Bbig = hs.hs_batch_create([Mb] * 4)
    Bsmall = hs.hs_batch_create([Ms] * 4)
    N = hs.hs_problem_size(Pb)
    rs = [random_vector(N, seed=80 + i) for i in range(4)]
    r = batch_vector(rs)
    z = torch.empty_like(r)
    hs.hs_batch_apply_Minv(Bbig, r, z)
    rsm = batch_vector([random_vector(hs.hs_problem_size(Ps), seed=90 + i) for i in range(4)])
    hs.hs_batch_apply_Minv(Bsmall, rsm, torch.empty_like(rsm))
    for i in range(4):
        zi = torch.empty(N, dtype=torch.complex128, device=DEV)
        hs.hs_apply_Minv(Mb, dev_vec(rs[i]), zi)
        assert torch.equal(z[i * N:(i + 1) * N], zi), i
