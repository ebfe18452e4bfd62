/*
 * helmschwarz.h -- C ABI of the MI355X (gfx950) two-level Schwarz / Bezier
 * coarse-space GMRES solver for the 2-D Helmholtz equation.
 *
 * Method: arXiv 2408.03571 (Sieburgh, Heinlein, Dwarka, Vuik).
 *   Sec. 2  model problems MP-1 (Dirichlet) / MP-2 (Sommerfeld), five-point
 *           finite differences on the unit square, A u = f (eq. LS_final);
 *   Sec. 3  two-level additive (AS2, eq. DDM:SO_AS) and scaled/restricted
 *           (SAS2, eq. DDM:SO_SAS, here RAS2 with Boolean D_i) Schwarz with
 *           exact local and coarse solves;
 *   Sec. 4  Bezier coarse restriction R_0 (eq. GCS:HO_R_0), A_0 = R_0 A R_0^T;
 *   Sec. 5  GMRES to a relative tolerance.
 *
 * Conventions common to every call
 *   - Vectors are complex128, interleaved (re, im) == torch.complex128, on the
 *     device, x-fastest over the unknowns: Sommerfeld uses all n*n grid nodes,
 *     Dirichlet the (n-2)*(n-2) interior nodes.
 *   - All pointers named *_dev are device pointers owned by the caller; the
 *     library never frees them and never keeps them past the call, except
 *     k2_dev (see hs_assemble).
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream). Work
 *     is enqueued on it; calls documented as asynchronous return before the
 *     device work finishes.
 *   - Every call returns hs_status; on failure hs_last_error() gives a
 *     thread-local message. Arguments are validated on the host before any
 *     device work; no C++ exception crosses the ABI.
 *   - Handles (hs_problem, hs_precond, hs_batch) are host objects created by
 *     the library and released by hs_destroy_* / hs_batch_destroy.
 *   - All device memory is caller-owned.  A preconditioner lives in the
 *     workspace handed to hs_setup_schwarz (size: hs_schwarz_workspace_bytes),
 *     a batch in the one handed to hs_batch_create (hs_batch_workspace_bytes),
 *     a GMRES solve in its own (hs_gmres_workspace_bytes and the batch
 *     forms); workspaces are 256-byte aligned and must outlive the handle
 *     built in them.  The library calls no hipMalloc / hipFree anywhere.
 */
#ifndef HELMSCHWARZ_H
#define HELMSCHWARZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HS_OK = 0,
  HS_EINVAL = -1,    /* bad argument (checked on the host, nothing enqueued) */
  HS_ENOMEM = -2,    /* device allocation failed                             */
  HS_ESINGULAR = -3, /* zero pivot in a local or coarse factorisation        */
  HS_ENOCONV = -4,   /* GMRES hit maxit; x holds the last iterate            */
  HS_ENAN = -5,      /* non-finite norm in the right-hand side or Arnoldi    */
  HS_EHIP = -6       /* a HIP runtime call failed                            */
} hs_status;

enum { HS_BC_DIRICHLET = 0, HS_BC_SOMMERFELD = 1 };
enum { HS_AS2 = 0, HS_RAS2 = 1, HS_SHS2 = 2 };
enum { HS_C128 = 0, HS_C64 = 1, HS_C64X = 2, HS_C64S = 3 };
/* coarse basis: Bezier (Sec. 4, eq. GCS:HO_R_0) or linear (the P1 basis the
 * paper compares it with in Sec. 5) */
enum { HS_COARSE_BEZIER = 0, HS_COARSE_P1 = 1 };

typedef struct { double re, im; } hs_c128;
typedef struct hs_problem hs_problem;
typedef struct hs_precond hs_precond;

/* ---------------------------------------------------------------- problem
 * Sec. 2: -Laplace(u) - k^2 u = f on [0,1]^2, h = 1/(n-1), n odd >= 5.
 * bc = HS_BC_DIRICHLET (MP-1, u = 0) or HS_BC_SOMMERFELD (MP-2,
 * du/dn - i k u = 0 by a centred ghost node, edge rows scaled 1/2 and corner
 * rows 1/4 so that A is complex symmetric).
 * k2_dev: NULL for constant k, else an n*n double array of k^2 on every grid
 * node ([j][i], x fastest) in device memory; it is referenced, not copied,
 * and must outlive the problem and every preconditioner built on it.
 * No device work.  Errors: HS_EINVAL (n even or < 5, k <= 0 with NULL field,
 * bad bc, out == NULL). */
hs_status hs_assemble(int n, double k, int bc, const double* k2_dev, hs_problem** out);

/* Number of unknowns: n*n (Sommerfeld) or (n-2)*(n-2) (Dirichlet). */
int64_t hs_problem_size(const hs_problem* P);

/* y = A x (eq. LS_final), the complex five-point operator generated on the
 * fly from (h, k or k^2 field, bc).  Asynchronous.  x and y must not alias. */
hs_status hs_spmv(const hs_problem* P, const hs_c128* x_dev, hs_c128* y_dev, void* stream);

/* ------------------------------------------------------- preconditioner
 * Sec. 3-4: builds the two-level preconditioner on P.
 *   nsub_x, nsub_y  subdomains along x and y; per dimension node i belongs to
 *            block min(nsub-1, floor(i*nsub/(n-1))) (interface nodes go up)
 *   overlap  node layers added on each side of every owned block
 *   ratio    coarse ratio H/h, a power of two >= 2 with (n-1) % ratio == 0;
 *            R_0 is eq. (GCS:HO_R_0) for ratio 2 and the product of ratio-2
 *            stages otherwise
 *   variant  HS_AS2 (eq. DDM:SO_AS), HS_RAS2 (eq. DDM:SO_SAS, Boolean D_i)
 *            or HS_SHS2 (eq. DDM:SO_SHS, the same D_i: the coarse
 *            correction e = Q r first, then the local solves of r - A e;
 *            the two branches no longer run side by side)
 *   prec     precision of the local factors and solves (the coarse
 *            factor/solve is always complex128):
 *              HS_C128  factored, stored and solved in complex128
 *              HS_C64   factored, stored and solved in complex64
 *              HS_C64X  factored in complex128, rounded once to complex64,
 *                       stored and solved in complex64
 *              HS_C64S  factored in complex128, rounded once to complex64
 *                       and stored so (the bytes the solves stream); the
 *                       solves widen each entry and run in complex128, so
 *                       M^{-1} is a fixed linear operator up to FP64
 *                       rounding (no complex64 rounding of r or of the
 *                       local solutions)
 *   ws_dev   caller-owned device memory of ws_bytes >=
 *            hs_schwarz_workspace_bytes(...) bytes, 256-byte aligned.  It
 *            holds everything the preconditioner keeps on the device (tables,
 *            local and coarse factors, A_0, the vectors of an application)
 *            followed by the set-up scratch (the fronts of the coarse
 *            factorisation; hs_precond_info.setup_scratch_bytes), which is
 *            read only while hs_setup_schwarz runs.  The buffer must stay
 *            allocated, and must not be written by the caller, until
 *            hs_destroy_precond.
 * Factors on `stream` and synchronises it before returning.
 * Errors: HS_EINVAL (nsub_x or nsub_y < 1, a block narrower than
 * overlap+1, bad ratio, variant or prec, ws_dev NULL, misaligned or smaller
 * than needed: all checked before any device work), HS_ESINGULAR (message
 * names the subdomain or "coarse"), HS_EHIP. */
hs_status hs_setup_schwarz(const hs_problem* P, int nsub_x, int nsub_y, int overlap, int ratio, int variant,
                           int prec, void* ws_dev, size_t ws_bytes, void* stream, hs_precond** out);

/* Device bytes hs_setup_schwarz needs for these sizes, for any variant and
 * coarse basis (the largest: SHS2 keeps two more fine-grid vectors, the
 * Bezier basis has the widest coarse stencil).  Host only; plans the
 * decomposition and the nested dissection.  Errors: as hs_setup_schwarz. */
hs_status hs_schwarz_workspace_bytes(const hs_problem* P, int nsub_x, int nsub_y, int overlap, int ratio,
                                     int prec, size_t* bytes);
/* The exact figure for one variant and basis. */
hs_status hs_schwarz_workspace_bytes_ex(const hs_problem* P, int nsub_x, int nsub_y, int overlap, int ratio,
                                        int variant, int prec, int basis, size_t* bytes);

/* hs_setup_schwarz with a choice of coarse basis (Sec. 4-5):
 *   basis  HS_COARSE_BEZIER  R_0 of eq. (GCS:HO_R_0) per ratio-2 stage
 *                            (what hs_setup_schwarz builds; A_0 has 25-point
 *                            rows for H = 2h, 49-point for H >= 4h)
 *          HS_COARSE_P1      linear interpolation: each ratio-2 stage of
 *                            R_0^T puts 1 on the coincident fine node and 1/2
 *                            on its two neighbours per axis (composite: the
 *                            bilinear hat of width H), so A_0 keeps 9-point
 *                            rows at every ratio
 * Everything else as hs_setup_schwarz.  Errors: as hs_setup_schwarz, and
 * HS_EINVAL for an unknown basis. */
hs_status hs_setup_schwarz_ex(const hs_problem* P, int nsub_x, int nsub_y, int overlap, int ratio, int variant,
                              int prec, int basis, void* ws_dev, size_t ws_bytes, void* stream,
                              hs_precond** out);

/* Schedule of one application of M^{-1} (AS2 / RAS2; SHS2 runs its branches
 * in order): the local solves run on an internal second stream beside the
 * coarse branch on the caller's stream, and fork after the first fork_level
 * forward level launches of the nested-dissection coarse solve (0: before
 * the coarse branch starts).  The leaf levels of the coarse solve stream
 * their factors and starve when they share the memory system with the local
 * solves; the upper levels are latency-bound and leave it idle.
 * local_grid: workgroups of the persistent local-solve launch (0: one per
 * subdomain).  Changes no result.  A captured GMRES step is re-captured.
 * Errors: HS_EINVAL (negative values). */
hs_status hs_precond_set_schedule(hs_precond* M, int fork_level, int local_grid);
hs_status hs_precond_get_schedule(const hs_precond* M, int* fork_level, int* local_grid);

/* z = M^{-1} r (AS2 or RAS2).  Asynchronous; uses the preconditioner's
 * internal scratch, so two applies of the same handle must not overlap in
 * time (enqueue them on one stream).  r and z must not alias. */
hs_status hs_apply_Minv(hs_precond* M, const hs_c128* r_dev, hs_c128* z_dev, void* stream);

/* z = M^{-1} r exactly as hs_apply_Minv (the same kernels, in the same order,
 * so the same bits), for callers that cannot allocate device memory: code
 * being captured into a HIP graph, tight serving loops, harnesses that
 * forbid allocation.  The buffers one application writes and reads back
 * (hs_precond_info.apply_work_bytes: local solutions, coarse vectors, the
 * coarse solve's per-front work vectors) come from a static device array of
 * 64 MiB that the library holds on every GPU it runs on until the process
 * ends, instead of the preconditioner's own; the factors are read in place.
 * This call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  Limit: apply_work_bytes <= 64 MiB, which covers AS2 / RAS2 at
 * n = 1025 with 16 x 16 subdomains in either local precision; larger
 * preconditioners are rejected with HS_EINVAL before any device work.
 * The array is shared by every call on one GPU and keeps the last call's
 * contents (every byte is written before it is read within a call): two
 * calls that overlap in time on one GPU race, whatever their handles and
 * streams, so enqueue them on one stream or order them.  The current device
 * must be the one the preconditioner was built on.  Asynchronous.
 * Errors: HS_EINVAL (null or aliasing pointers, scratch above the limit),
 * HS_EHIP. */
hs_status hs_apply_Minv_noalloc(hs_precond* M, const hs_c128* r_dev, hs_c128* z_dev, void* stream);

/* ------------------------------------------------------------------ GMRES
 * Sec. 5: unrestarted right-preconditioned flexible GMRES, x_0 = 0; stops
 * when the implicit residual drops below tol*||b|| and the recomputed true
 * residual ||b - A x||/||b|| confirms it (otherwise it keeps iterating).
 * Arnoldi, Givens and the true residual are complex128.
 *
 * Orthogonalisation (the paper does not fix it; both give A Z = V Hbar with
 * V orthonormal to working precision):
 *   HS_ORTHO_DCGS2  classical Gram-Schmidt with one reorthogonalisation pass,
 *                   delayed by one step and fused with the next projection:
 *                   two streaming passes over V per iteration.  The
 *                   Hessenberg columns, Givens rotations and the stop test
 *                   live on the device, so the host only checks a state word
 *                   every few iterations, and one iteration can be replayed
 *                   as a HIP graph.  The stop test on column j runs after the
 *                   (j+1)-th M^{-1} application has been formed, so a
 *                   converged solve spends one extra application.
 *   HS_ORTHO_MGS    modified Gram-Schmidt, one kernel per projection, Givens
 *                   on the host, one stream synchronisation per iteration.
 *
 * ws_dev: caller-owned device workspace of at least
 * hs_gmres_workspace_bytes(P, maxit) bytes (holds V, Z and the Hessenberg
 * matrix; large enough for either method).  history_host: NULL or a host
 * array of maxit+1 doubles receiving the implicit relative residual after
 * each iteration.  Errors: HS_EINVAL, HS_ENOCONV (x = last iterate, stats
 * filled), HS_ENAN. */
enum { HS_ORTHO_DCGS2 = 0, HS_ORTHO_MGS = 1 };

typedef struct {
  int ortho;        /* HS_ORTHO_DCGS2 or HS_ORTHO_MGS                            */
  int graph;        /* DCGS2: 1 = capture one iteration once per (workspace,
                       maxit) and replay it as a HIP graph; 0 = plain launches   */
  int check_every;  /* DCGS2: iterations between host checks of the device
                       state; 0 = adaptive (from the observed residual decay)    */
  int basis_prec;   /* DCGS2: storage of the Krylov basis V.  HS_C128 (default)
                       or HS_C64: each basis vector is rounded once to
                       complex64 when it is formed and read back widened, all
                       arithmetic stays complex128 (a compressed basis: the two
                       streaming passes move half the bytes).  The Arnoldi
                       relation then holds to complex64 rounding, so the
                       implicit residual is trusted to ~1e-7 relative; the
                       stop is still confirmed by the complex128 true
                       residual.  HS_ORTHO_MGS accepts only HS_C128.      */
} hs_gmres_opts;

typedef struct {
  int iters;             /* Krylov dimension of the returned x (M^{-1} columns) */
  int converged;         /* 1 if relres_true <= tol                      */
  double relres_implicit;
  double relres_true;    /* ||b - A x|| / ||b||, recomputed in complex128 */
  double ms_solve;       /* wall time of the call                        */
  int steps;             /* iterations launched (DCGS2: includes the ones
                            enqueued after the stop test fired)           */
  int host_checks;       /* host synchronisations on the solve's stream   */
} hs_gmres_stats;

hs_status hs_gmres_workspace_bytes(const hs_problem* P, int maxit, size_t* bytes);
/* opts == NULL: DCGS2, graph replay, adaptive checks. */
hs_status hs_gmres_solve_ex(const hs_problem* P, hs_precond* M, const hs_c128* b_dev, hs_c128* x_dev,
                            double tol, int maxit, const hs_gmres_opts* opts, void* ws_dev, size_t ws_bytes,
                            double* history_host, void* stream, hs_gmres_stats* stats);
/* hs_gmres_solve_ex with opts == NULL. */
hs_status hs_gmres_solve(const hs_problem* P, hs_precond* M, const hs_c128* b_dev, hs_c128* x_dev,
                         double tol, int maxit, void* ws_dev, size_t ws_bytes,
                         double* history_host, void* stream, hs_gmres_stats* stats);

/* Timing of the DCGS2 orthogonalisation at Arnoldi step k (k basis vectors
 * already in V), HIP events on `stream` around `reps` launches after one
 * untimed launch; fills the workspace's vectors from r_dev first.
 *   which = 0: the dot pass (w = A z fused; V^H u and V^H w over k rows)
 *           1: the update pass (v_k and w1 over k rows)
 *           2: fold + Hessenberg column + scale (the small kernels of a step)
 * ws_dev as for hs_gmres_solve with maxit >= k + 1.  Synchronises `stream`.
 * Errors: HS_EINVAL. */
hs_status hs_time_arnoldi(const hs_problem* P, int k, int which, void* ws_dev, size_t ws_bytes,
                          const hs_c128* r_dev, int reps, void* stream, double* avg_ms);
/* hs_time_arnoldi with the basis stored as basis_prec (HS_C128 or HS_C64,
 * see hs_gmres_opts.basis_prec).  Errors: as hs_time_arnoldi, and HS_EINVAL
 * for another basis_prec. */
hs_status hs_time_arnoldi_ex(const hs_problem* P, int k, int which, int basis_prec, void* ws_dev, size_t ws_bytes,
                             const hs_c128* r_dev, int reps, void* stream, double* avg_ms);

/* ------------------------------------------------------------- batches
 * Many independent instances (each an hs_problem with its own hs_precond)
 * advanced together on one GPU.  One application of M^{-1} to all of them
 * is a fixed set of launches, each over all instances: one launch runs every
 * subdomain solve of every instance, then one per restriction stage, one per
 * nested-dissection depth and direction (the instances' coarse trees aligned
 * by depth), one per prolongation stage and one final combination.  One
 * flexible-GMRES iteration of all instances adds one launch per DCGS2
 * kernel; hs_batch_gmres_solve captures it as a HIP graph and replays it, so
 * the instances iterate in lockstep; the launches of a step skip the
 * instances that no longer iterate (their workgroups return at once, the
 * Arnoldi kernels and the M^{-1} stages alike).  For SHS2 (eq. DDM:SO_SHS) the coarse launches come first, then
 * one launch forms every instance's residual r - A e_0, then the subdomain
 * solves of that residual and the combination; AS2 / RAS2 run the subdomain
 * solves beside the coarse launches.
 *
 * Batch vectors concatenate the instances' unknowns in order:
 * hs_batch_offsets fills count+1 offsets (instance i is [off[i], off[i+1])).
 * The preconditioners must share variant and prec and outlive the batch
 * (the batch reads their factors and scratch in place, so a preconditioner
 * must not be applied on its own, or by another batch, while a batch call
 * using it is in flight).
 * A handle may appear several times: several right-hand sides of one
 * problem (the sources of the differentiation workload, Sec. 2's problem with
 * several f).  Its repeats get scratch of their own, in the batch's
 * workspace; their subdomain solves and coarse tasks are interleaved, so the
 * launches that read a factor block serve every right-hand side together
 * and the coarse levels' latency is paid once.
 * ws_dev: caller-owned device memory of ws_bytes >=
 * hs_batch_workspace_bytes(count, M) bytes, 256-byte aligned (the batch's
 * launch tables and the repeats' scratch), kept until hs_batch_destroy.
 * Errors: HS_EINVAL (also a workspace that is NULL, misaligned or too
 * small), HS_EHIP. */
typedef struct hs_batch hs_batch;
hs_status hs_batch_workspace_bytes(int count, hs_precond* const* M, size_t* bytes);
hs_status hs_batch_create(int count, hs_precond* const* M, void* ws_dev, size_t ws_bytes, hs_batch** out);
void hs_batch_destroy(hs_batch* B);
hs_status hs_batch_offsets(const hs_batch* B, int64_t* offsets);
/* z = M_i^{-1} r for every instance at once (batch vectors). Asynchronous. */
hs_status hs_batch_apply_Minv(hs_batch* B, const hs_c128* r_dev, hs_c128* z_dev, void* stream);
hs_status hs_batch_gmres_workspace_bytes(const hs_batch* B, int maxit, size_t* bytes);
/* Workgroups of the persistent launch that runs every subdomain solve of the
 * batch (each takes subdomains g, g + grid, ... in order); 0 = one per
 * subdomain.  A grid below the CU count's worth of resident workgroups
 * leaves room for the coarse sweeps that run beside it.  Meant for the
 * autotuner; changes no result.  Errors: HS_EINVAL. */
hs_status hs_batch_set_local_grid(hs_batch* B, int grid);
/* Schedule of one batched application of M^{-1} (AS2 / RAS2), as
 * hs_precond_set_schedule for one preconditioner: the subdomain solves of
 * every instance fork onto a second stream after the first fork_level
 * forward levels of the batched coarse solve (0: before the coarse
 * branch), in local_grid persistent workgroups (0: one per subdomain).
 * Changes no result.  Errors: HS_EINVAL. */
hs_status hs_batch_set_schedule(hs_batch* B, int fork_level, int local_grid);

/* Timing of one batched step with HIP events on `stream` (reps launches after
 * one untimed one; synchronises): which = 0 the local solves of every
 * instance (one launch), 1 the coarse chain (restriction stages, nested
 * dissection, prolongation stages), 2 the whole application, 3 the
 * restriction stages, 4 the nested-dissection solves.  r_dev: a batch
 * vector; z_dev: a batch vector the whole application writes (which = 2;
 * may be NULL otherwise).  Errors: HS_EINVAL. */
hs_status hs_batch_time(hs_batch* B, int which, const hs_c128* r_dev, hs_c128* z_dev, int reps, void* stream,
                        double* avg_ms);
/* Flexible GMRES (DCGS2) on every instance, each to tol relative to its own
 * right-hand side, the same stop rule as hs_gmres_solve (true residual
 * confirmed; a rejected stop resumes that instance alone).  stats: count
 * entries.  The launch shape of the DCGS2 passes is the one set for the
 * batch's total unknowns (hs_set_arnoldi_config).  Returns HS_ENOCONV (or
 * HS_ENAN) if any instance did not converge; x holds every instance's last
 * iterate. */
hs_status hs_batch_gmres_solve(hs_batch* B, const hs_c128* b_dev, hs_c128* x_dev, double tol, int maxit,
                               const hs_gmres_opts* opts, void* ws_dev, size_t ws_bytes, void* stream,
                               hs_gmres_stats* stats);

/* The same solve for instances given as plain arrays, in one call with one
 * workspace: b[i], x[i] are instance i's right-hand side and solution
 * (device, hs_problem_size(P[i]) unknowns each), M[i] its preconditioner,
 * built on P[i].  ws_dev (256-byte aligned, >= hs_gmres_batch_workspace_bytes
 * bytes) holds the batch's tables, its GMRES workspace and two concatenated
 * batch vectors; the call builds the batch there, gathers the b[i], solves
 * with the default options, scatters the solutions into the x[i] and
 * synchronises `stream`.  stats: count entries.  Returns HS_ENOCONV (or
 * HS_ENAN) if any instance did not converge (x[i] holds its last iterate).
 * Errors: HS_EINVAL (also P[i] != M[i]'s problem), HS_EHIP. */
hs_status hs_gmres_batch_workspace_bytes(int count, const hs_problem* const* P, hs_precond* const* M, int maxit,
                                         size_t* bytes);
hs_status hs_gmres_solve_batch(int count, const hs_problem* const* P, hs_precond* const* M,
                               const hs_c128* const* b, hs_c128* const* x, double tol, int maxit, void* ws_dev,
                               size_t ws_bytes, void* stream, hs_gmres_stats* stats);

/* Launch shape of the two DCGS2 streaming passes for problems with
 * n_unknowns unknowns, process-wide: ept = unknowns per lane per wave
 * (1, 2, 4, 8), rows = basis vectors streamed per loop trip (2 or 4).
 * ept and rows both 0 restore the built-in choice.  ept fixes how the dot
 * products are partitioned (so results are reproducible for a fixed table);
 * rows does not change any result.  Meant for the autotuner; a solve picks
 * the shape up when it starts (a captured step is re-captured).
 * Errors: HS_EINVAL. */
hs_status hs_set_arnoldi_config(int64_t n_unknowns, int ept, int rows);
hs_status hs_get_arnoldi_config(int64_t n_unknowns, int* ept, int* rows);

/* ------------------------------------------------- k^2 sensitivity
 * For a problem built on a k^2 field (k2_dev != NULL) and vectors u, lam on
 * the unknowns:  grad[j*n + i] += scale * Re( dA_ll/dk^2_l * u_l * lam_l )
 * for every unknown l at grid node (i, j); other nodes are untouched.
 * dA_ll/dk^2_l is the exact derivative of the assembled diagonal: -1 inside,
 * and for Sommerfeld edge / corner rows the scaled volume term plus the
 * derivative of the boundary term -2 i w e k / h with k = sqrt(k^2).
 * With g = 2 dL/du* (the gradient torch hands a complex tensor for a real
 * loss L(u)) and lam = A^{-1} conj(g) (one unconjugated adjoint solve,
 * A = A^T, Sec. 2), scale = -1 accumulates dL/dk^2.
 * grad_dev: n*n doubles on the device.  Asynchronous.  Errors: HS_EINVAL. */
hs_status hs_k2_gradient(const hs_problem* P, const hs_c128* u_dev, const hs_c128* lam_dev, double scale,
                         double* grad_dev, void* stream);

/* --------------------------------------------- components of M^{-1}
 * The steps of one application, exposed so that each can be checked on its
 * own.  All asynchronous; all use the preconditioner's sizes.           */
typedef struct {
  int64_t n_fine;        /* unknowns of the problem                          */
  int64_t n_coarse;      /* coarse unknowns (Sec. 4, |G_H| minus Dirichlet)  */
  int coarse_per_dim;    /* coarse unknowns per dimension                    */
  int coarse_reach;      /* stencil reach of A_0: Bezier 2 for H = 2h, 3 for
                            4h+; linear 1                                    */
  int nsub_total;        /* nsub * nsub                                      */
  int64_t local_total;   /* sum of subdomain sizes (overlap counted)         */
  int64_t local_factor_bytes;  /* bytes of the local factors G_j one local
                                  solve reads once, counted as ny * nx^2
                                  entries per subdomain (the algorithmic
                                  figure: the zero columns a line stores past
                                  nx when nx % 4 != 0 are not counted)       */
  int64_t coarse_factor_bytes;
  int nd_fronts;         /* nested-dissection fronts of the coarse solver    */
  int nd_levels;
  double ms_setup_local; /* device time of the local factorisation           */
  double ms_setup_coarse;/* device time of A_0 assembly + coarse factorisation */
  int64_t coarse_solve_bytes; /* factor bytes one coarse solve must read      */
  int coarse_basis;      /* HS_COARSE_BEZIER or HS_COARSE_P1                 */
  int64_t workspace_bytes;     /* bytes of ws_dev the preconditioner uses      */
  int64_t setup_scratch_bytes; /* the last part of them, read only during the
                                  set-up (fronts of the coarse factorisation,
                                  complex128 factors before rounding); the
                                  timing helpers write their outputs there
                                  afterwards                                 */
  int64_t apply_work_bytes; /* device bytes one application of M^{-1} writes
                               and reads back (local solutions, coarse
                               vectors, the coarse solve's work vectors); the
                               scratch hs_apply_Minv_noalloc needs          */
} hs_precond_info;

hs_status hs_precond_get_info(const hs_precond* M, hs_precond_info* info);

/* r0 = R_0 r (Sec. 4, eq. GCS:HO_R_0; composite for ratio > 2). */
hs_status hs_coarse_restrict(hs_precond* M, const hs_c128* r_dev, hs_c128* r0_dev, void* stream);
/* z = R_0^T e0 (overwrites z). */
hs_status hs_coarse_prolong(hs_precond* M, const hs_c128* e0_dev, hs_c128* z_dev, void* stream);
/* e0 = A_0^{-1} r0 with A_0 = R_0 A R_0^T (exact coarse solve). */
hs_status hs_coarse_solve(hs_precond* M, const hs_c128* r0_dev, hs_c128* e0_dev, void* stream);
/* A_0 as a (2R+1)^2-point stencil: stencil_dev[c*(2R+1)^2 + (dy+R)*(2R+1) + (dx+R)]
 * = A_0[c, c + dx + dy*ncu] (zero where the neighbour is not an unknown),
 * R = coarse_reach, ncu = coarse_per_dim. */
hs_status hs_coarse_matrix(hs_precond* M, hs_c128* stencil_dev, void* stream);
/* Local solves A_i^{-1} R_i r for every subdomain i, concatenated in
 * subdomain order (x-major over the subdomain grid), each x-fastest over its
 * extended block; returned in complex128 whatever the local precision. */
hs_status hs_local_solve(hs_precond* M, const hs_c128* r_dev, hs_c128* zloc_dev, void* stream);

/* Timing of one step of M^{-1} with HIP events recorded on `stream` around
 * `reps` back-to-back launches (after one untimed launch); synchronises the
 * stream and returns the mean milliseconds per launch in *avg_ms.
 *   which = 0: the batched local solves (one launch, all subdomains)
 *           1: the nested-dissection coarse solve (all level launches)
 *           2: the whole M^{-1} application
 *           3: the five-point SpMV (r -> scratch)
 *           4: one modified Gram-Schmidt projection of flexible GMRES
 *              (w -= h v_prev, then the partial sums of v_cur^H w)
 * r_dev: an input vector of hs_problem_size unknowns.  Uses the
 * preconditioner's scratch; the outputs go to the set-up scratch at the end
 * of its workspace.  Errors: HS_EINVAL. */
hs_status hs_time_step(hs_precond* M, int which, const hs_c128* r_dev, int reps, void* stream, double* avg_ms);

/* Host-only structural check of the nested-dissection plan used for A_0^{-1}
 * on an ncx x ncy coarse grid with stencil reach `reach` and leaf boxes of at
 * most `leaf` nodes a side: the eliminated sets partition the grid, and every
 * front's boundary equals the set of uneliminated nodes within Chebyshev
 * distance `reach` of its subtree (the support of its Schur complement).
 * stats (8 int64, may be NULL): fronts, levels, entries of G stored (|I|^2
 * per front, |I|(|I|+1)/2 for a front of at most 64 unknowns, which keeps
 * one triangle of its complex-symmetric G), sum |I||B|, sum |F|^2, max |I|,
 * max |B|, max |F|.  No device work.
 * Errors: HS_EINVAL (bad sizes or a structural violation, named in the
 * message). */
hs_status hs_nd_plan_check(int ncx, int ncy, int reach, int leaf, int64_t* stats);

/* Per-level figures of the nested-dissection coarse solve of M (level 0 is
 * the root, hs_precond_info.nd_levels levels): stats (8 int64) = fronts,
 * entries of G read by the backward sweep (|I|^2 per front, |I|(|I|+1)/2
 * for a front that keeps one triangle, as in hs_nd_plan_check), sum |I||B| (entries
 * of V, read once by each sweep), forward and backward workgroups of the
 * level's own launches, max |I|, max |B|, and, for the deepest levels, which
 * are solved by subtree (one workgroup per front at the shallowest of them
 * with all its descendants, one launch per direction for all of them), the
 * workgroups of those launches (0 for a level with launches of its own).
 * Host only.  Errors: HS_EINVAL. */
hs_status hs_nd_level_stats(const hs_precond* M, int level, int64_t* stats);
/* The same figures for the plan of an ncx x ncy coarse grid of stencil reach
 * `reach` with leaf boxes of at most `leaf` nodes a side (the plan
 * hs_setup_schwarz builds uses leaf 8), without a preconditioner.  Host only.
 * Errors: HS_EINVAL. */
hs_status hs_nd_plan_level_stats(int ncx, int ncy, int reach, int leaf, int level, int64_t* stats);

void hs_destroy_problem(hs_problem* P);
void hs_destroy_precond(hs_precond* M);
const char* hs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HELMSCHWARZ_H */
