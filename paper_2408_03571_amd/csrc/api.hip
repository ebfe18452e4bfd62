// C ABI of libhelmschwarz: argument validation, preconditioner set-up, the
// application of M^{-1} (Sec. 3, eqs. DDM:SO_AS / DDM:SO_SAS) and the
// flexible GMRES driver (Sec. 5).  Every entry point catches internally and
// returns an hs_status; the message is kept per thread.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include <mutex>

#include "hs_internal.h"

namespace hs {

thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

size_t local_factor_lds_bytes(int prec, int nx);
size_t local_solve_lds_bytes(int prec, int nx, int ny);
void launch_local_factor(const ProblemDev& P, int prec, int nsub, const SubDesc* desc, void* G, int* status,
                         size_t lds, bool pair, hipStream_t s);
NDDev* nd_create(const NDPlan& plan, Arena& A);
void nd_destroy(NDDev* d);
void nd_level_stats(const NDPlan& plan, const NDDev& d, int lv, int64_t* out);
int nd_factor_run(const NDPlan& plan, NDDev& d, const c128* A0, c128* F, hipStream_t s);
// after (if set) is called once, after the first after_levels forward level
// launches (or after all of them); cbuf / ubuf: the per-front work vectors
// (nullptr: the plan's own)
void nd_solve_run(const NDPlan& plan, NDDev& d, const c128* r0, c128* e0, hipStream_t s,
                  const Callback& after = Callback{}, int after_levels = 0, c128* cbuf = nullptr,
                  c128* ubuf = nullptr);
void k_mgs(const ProblemDev& P, const c128* z, int64_t n, c128* w, const c128* vprev, const c128* pprev, c128* hout,
           const c128* vcur, c128* pout, double* pnorm, hipStream_t s);
void k_norm2(int64_t n, const c128* a, double* pnorm, hipStream_t s);
void k_scale(int64_t n, const c128* in, c128* out, const double* pnorm, double* nrm_out, hipStream_t s);
void k_combo(int64_t n, int m, const c128* y, const c128* Z, int64_t ld, c128* x, hipStream_t s,
             const c128* x0 = nullptr);
void k_bminus(int64_t n, const c128* b, c128* r, hipStream_t s);
void k_fold_norm(const double* pnorm, double* out, hipStream_t s);
int k_red_blocks();


constexpr int kLeaf = 8;

}  // namespace hs

using namespace hs;

struct hs_precond {
  const hs_problem* P = nullptr;
  int nsx = 0, nsy = 0, overlap = 0, ratio = 2, variant = HS_RAS2;
  int prec = HS_C128;   // arithmetic of the local solves and type of the local solutions
  int gprec = HS_C128;  // storage type of the local factors
  int fprec = HS_C128;  // arithmetic of the local factorisation
  int basis = HS_COARSE_BEZIER;
  std::vector<SubDesc> desc_h;     // subdomain order (x-major): factor and combination
  std::vector<SubDesc> sdesc_h;    // the same subdomains in solve classes
  std::vector<int> xmap_h, ymap_h; // grid index -> [owner, cover0..2] per dimension
  SubDesc* desc = nullptr;
  LocalLaunch lsolve;
  int* xmap = nullptr;
  int* ymap = nullptr;
  void* G = nullptr;
  void* sol = nullptr;
  int* lstatus = nullptr;
  int64_t g_elems = 0, sol_elems = 0, g_algo = 0;
  size_t factor_lds = 0, solve_lds = 0;
  int solve_threads = 256;
  std::vector<GridLevel> levels;   // 0 = fine, back() = coarse
  std::vector<int> lreach;         // stencil reach of the operator on each level
  int reach = 2;
  std::vector<c128*> stage;        // Galerkin operators of levels 1..L (A0 = the last)
  c128* A0 = nullptr;
  std::vector<c128*> rbuf;         // restriction results, levels 1..L
  std::vector<c128*> pbuf;         // prolongation results, levels 1..L-1
  c128* e0 = nullptr;
  c128* efine = nullptr;           // SHS2: e = Q r on the fine grid
  c128* tres = nullptr;            // SHS2: r - A e
  // set-up scratch: the tail of the workspace, read only while the set-up
  // runs; the timing helpers write their outputs there afterwards
  c128* Gf = nullptr;              // HS_C64X / HS_C64S: complex128 factors before rounding
  c128* F = nullptr;               // nested-dissection fronts
  c128* tout = nullptr;            // timing helper output (2 vectors)
  c128* mgs_part = nullptr;        // timing helper partial sums
  size_t ws_used = 0, ws_scratch = 0;
  hipStream_t side = nullptr;      // local branch of M^{-1} runs here
  int fork_level = 0;              // AS2/RAS2: forward ND levels launched before the local branch forks
  int local_grid = 0;              // workgroups of the local-solve launch (0: one per subdomain)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t cap = nullptr;       // capture stream of the GMRES step graph
  hipGraphExec_t gexec = nullptr;  // one DCGS2 iteration, for (g_ws, g_maxit)
  const void* g_ws = nullptr;
  int g_maxit = 0, g_ept = 0, g_rpi = 0, g_vprec = 0;
  NDPlan plan;
  NDDev* nd = nullptr;
  hs_precond_info info{};
  ~hs_precond() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap) (void)hipStreamDestroy(cap);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    nd_destroy(nd);
  }
};

namespace {

template <typename F>
hs_status guarded(F&& f) {
  try {
    f();
    return HS_OK;
  } catch (const Failure& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HS_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return HS_EINVAL;
  }
}

inline hipStream_t S(void* s) { return (hipStream_t)s; }

// per-dimension owned blocks: grid index i -> min(ns-1, floor(i*ns/(n-1)))
std::vector<std::pair<int, int>> owner_blocks(int n, int lo, int nu, int ns) {
  std::vector<std::pair<int, int>> b(ns, {-1, -1});
  for (int i = lo; i < lo + nu; ++i) {
    const int s = std::min(ns - 1, (int)(((int64_t)i * ns) / (n - 1)));
    if (b[s].first < 0) b[s].first = i;
    b[s].second = i + 1;
  }
  return b;
}

// The buffers one application of M^{-1} writes and reads back: local
// solutions, restriction and prolongation results, the coarse solution, the
// SHS2 vectors and the coarse solve's per-front work vectors.  A
// preconditioner owns one set (own_work); hs_apply_Minv_noalloc lays another
// over the library's static scratch array.  Every one of them is written
// before it is read within an application, so none needs clearing.
constexpr int kMaxStages = 32;  // ratio-2 stages of R_0 (ratio < 2^31)
struct ApplyWork {
  void* sol = nullptr;
  c128* rbuf[kMaxStages] = {};  // level l at rbuf[l - 1], l = 1..L
  c128* pbuf[kMaxStages] = {};  // level l at pbuf[l - 1], l = 1..L-1
  c128 *e0 = nullptr, *efine = nullptr, *tres = nullptr;
  c128 *cbuf = nullptr, *ubuf = nullptr;  // nullptr: the coarse plan's own
};

ApplyWork own_work(const hs_precond* M) {
  ApplyWork w;
  w.sol = M->sol;
  for (size_t l = 0; l < M->rbuf.size(); ++l) w.rbuf[l] = M->rbuf[l];
  for (size_t l = 0; l < M->pbuf.size(); ++l) w.pbuf[l] = M->pbuf[l];
  w.e0 = M->e0;
  w.efine = M->efine;
  w.tres = M->tres;
  return w;
}

void restrict_chain(hs_precond* M, const ApplyWork& w, const c128* r, hipStream_t s, c128* last_out) {
  const int L = (int)M->levels.size() - 1;
  const c128* in = r;
  for (int l = 1; l <= L; ++l) {
    c128* out = (l == L && last_out) ? last_out : w.rbuf[l - 1];
    launch_restrict2(M->levels[l - 1], M->levels[l], in, out, s);
    in = out;
  }
}

// coarse correction up to level 1 (the last stage is fused into combine);
// returns the level-1 vector
const c128* coarse_to_level1(hs_precond* M, const ApplyWork& w, const c128* r, hipStream_t s,
                             const Callback& fork = Callback{}, int fork_level = 0) {
  const int L = (int)M->levels.size() - 1;
  restrict_chain(M, w, r, s, nullptr);
  nd_solve_run(M->plan, *M->nd, w.rbuf[L - 1], w.e0, s, fork, fork_level, w.cbuf, w.ubuf);
  const c128* cur = w.e0;
  for (int l = L - 1; l >= 1; --l) {
    launch_prolong2(M->levels[l], M->levels[l + 1], cur, w.pbuf[l - 1], 0, s);
    cur = w.pbuf[l - 1];
  }
  return cur;
}

// The coarse and local branches of AS2 / RAS2 are independent: the local
// solves (bandwidth-bound) run on a second stream while the coarse branch
// (restriction, then the level sweeps of the nested-dissection solve) runs
// on the caller's stream; the combination waits for both.  The leaf levels
// of the coarse solve are bandwidth-bound too and starve when they share the
// memory system with the local solves, so the local branch forks after the
// first fork_level forward levels, to run beside the latency-bound upper
// levels (hs_precond_set_schedule).
void apply_minv(hs_precond* M, const ApplyWork& w, const c128* r, c128* z, hipStream_t s) {
  const hs_problem* P = M->P;
  if (M->variant == HS_SHS2) {
    // eq. (DDM:SO_SHS): e = Q r, local solves of the deflated residual r - A e,
    // z = e + sum_i R_i^T D_i A_i^{-1} R_i (r - A e)
    const c128* c1 = coarse_to_level1(M, w, r, s);
    launch_prolong2(M->levels[0], M->levels[1], c1, w.efine, 0, s);
    launch_residual(P->dev, r, w.efine, w.tres, s);
    launch_local_solve(M->lsolve, P->dev, M->gprec, M->prec, M->G, w.tres, w.sol, M->solve_lds, M->solve_threads,
                       s);
    launch_combine(P->dev, M->variant, M->prec, M->nsx, M->desc, M->xmap, M->ymap, w.sol, &M->levels[0],
                   &M->levels[1], nullptr, z, s, w.efine);
    return;
  }
  auto fork = [&]() {
    HS_HIP(hipEventRecord(M->ev_fork, s));
    HS_HIP(hipStreamWaitEvent(M->side, M->ev_fork, 0));
    launch_local_solve(M->lsolve, P->dev, M->gprec, M->prec, M->G, r, w.sol, M->solve_lds, M->solve_threads,
                       M->side, M->local_grid);
    HS_HIP(hipEventRecord(M->ev_join, M->side));
  };
  if (M->fork_level <= 0) fork();
  const c128* c1 = coarse_to_level1(M, w, r, s, M->fork_level > 0 ? callback_of(fork) : Callback{},
                                    M->fork_level);
  HS_HIP(hipStreamWaitEvent(s, M->ev_join, 0));
  launch_combine(P->dev, M->variant, M->prec, M->nsx, M->desc, M->xmap, M->ymap, w.sol, &M->levels[0],
                 &M->levels[1], c1, z, s);
}

void apply_minv(hs_precond* M, const c128* r, c128* z, hipStream_t s) { apply_minv(M, own_work(M), r, z, s); }

// Lays one application's buffers out from `base` (256-byte aligned pieces)
// and returns the bytes they take; base == nullptr only counts.
size_t apply_work_layout(const hs_precond* M, unsigned char* base, ApplyWork* w) {
  size_t o = 0;
  auto take = [&](size_t bytes) -> unsigned char* {
    unsigned char* p = base ? base + o : nullptr;
    o = (o + bytes + 255) & ~(size_t)255;
    return p;
  };
  const int L = (int)M->levels.size() - 1;
  w->sol = take((size_t)M->sol_elems * (M->prec == HS_C64 ? sizeof(c64) : sizeof(c128)));
  for (int l = 1; l <= L; ++l)
    w->rbuf[l - 1] = (c128*)take((size_t)M->levels[l].nu * M->levels[l].nu * sizeof(c128));
  for (int l = 1; l < L; ++l)
    w->pbuf[l - 1] = (c128*)take((size_t)M->levels[l].nu * M->levels[l].nu * sizeof(c128));
  w->e0 = (c128*)take((size_t)M->levels[L].nu * M->levels[L].nu * sizeof(c128));
  if (M->variant == HS_SHS2) {
    w->efine = (c128*)take((size_t)M->P->N * sizeof(c128));
    w->tres = (c128*)take((size_t)M->P->N * sizeof(c128));
  }
  w->cbuf = (c128*)take((size_t)std::max<int64_t>(1, M->plan.c_elems) * sizeof(c128));
  w->ubuf = (c128*)take((size_t)std::max<int64_t>(1, M->plan.u_elems) * sizeof(c128));
  return o;
}

// Static scratch of hs_apply_Minv_noalloc: one array per GPU, in the code
// object's zero-initialised data, held until the process ends.  Host code
// reaches it only through the per-device address hipGetSymbolAddress
// returns (the array's name is a host-side stand-in, not a device address).
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};

// address of the current device's scratch array, looked up once per device
unsigned char* static_scratch() {
  int dev = -1;
  HS_HIP(hipGetDevice(&dev));
  HS_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range for the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = (unsigned char*)p;
  }
  return g_scratch_dev[dev];
}

}  // namespace

// ===================================================================== ABI
extern "C" {

const char* hs_last_error(void) { return g_err.c_str(); }

hs_status hs_assemble(int n, double k, int bc, const double* k2_dev, hs_problem** out) {
  return guarded([&] {
    HS_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    HS_REQUIRE(n >= 5 && (n % 2) == 1, "n must be odd and >= 5");
    HS_REQUIRE(bc == HS_BC_DIRICHLET || bc == HS_BC_SOMMERFELD, "bc must be HS_BC_DIRICHLET or HS_BC_SOMMERFELD");
    HS_REQUIRE(k2_dev != nullptr || (k > 0.0 && std::isfinite(k)), "k must be positive and finite");
    hs_problem* P = new hs_problem();
    P->dev.n = n;
    P->dev.bc = bc;
    P->dev.lo = (bc == HS_BC_SOMMERFELD) ? 0 : 1;
    P->dev.nu = n - 2 * P->dev.lo;
    P->dev.h = 1.0 / (n - 1);
    P->dev.inv_h2 = (double)(n - 1) * (double)(n - 1);
    P->dev.k2c = k * k;
    P->dev.k2 = k2_dev;
    P->k = k;
    P->N = (int64_t)P->dev.nu * P->dev.nu;
    *out = P;
  });
}

int64_t hs_problem_size(const hs_problem* P) { return P ? P->N : -1; }

void hs_destroy_problem(hs_problem* P) { delete P; }

hs_status hs_spmv(const hs_problem* P, const hs_c128* x, hs_c128* y, void* stream) {
  return guarded([&] {
    HS_REQUIRE(P && x && y, "null argument");
    HS_REQUIRE((const void*)x != (const void*)y, "x and y must not alias");
    launch_spmv(P->dev, (const c128*)x, (c128*)y, S(stream));
  });
}

hs_status hs_k2_gradient(const hs_problem* P, const hs_c128* u, const hs_c128* lam, double scale, double* grad,
                         void* stream) {
  return guarded([&] {
    HS_REQUIRE(P && u && lam && grad, "null argument");
    HS_REQUIRE(P->dev.k2 != nullptr, "the problem has no k^2 field");
    launch_k2_grad(P->dev, (const c128*)u, (const c128*)lam, scale, grad, S(stream));
  });
}

}  // extern "C"

namespace {

// ------------------------------------------------- preconditioner set-up
// Host planning (no device work): validation, the decomposition (Sec. 3),
// the coarse grids (Sec. 4) and the nested-dissection plan of A_0.
void setup_plan(hs_precond* M, const hs_problem* P, int nsx, int nsy, int overlap, int ratio, int variant, int prec,
                int basis) {
  HS_REQUIRE(nsx >= 1 && nsy >= 1, "nsub_x and nsub_y must be >= 1");
  HS_REQUIRE(overlap >= 0, "overlap must be >= 0");
  HS_REQUIRE(ratio >= 2 && (ratio & (ratio - 1)) == 0, "ratio must be a power of two >= 2");
  HS_REQUIRE((P->dev.n - 1) % ratio == 0, "(n-1) must be divisible by ratio");
  HS_REQUIRE(variant == HS_AS2 || variant == HS_RAS2 || variant == HS_SHS2,
             "variant must be HS_AS2, HS_RAS2 or HS_SHS2");
  HS_REQUIRE(prec == HS_C128 || prec == HS_C64 || prec == HS_C64X || prec == HS_C64S,
             "prec must be HS_C128, HS_C64, HS_C64X or HS_C64S");
  HS_REQUIRE(basis == HS_COARSE_BEZIER || basis == HS_COARSE_P1, "basis must be HS_COARSE_BEZIER or HS_COARSE_P1");
  const ProblemDev& D = P->dev;
  M->P = P;
  M->nsx = nsx;
  M->nsy = nsy;
  M->overlap = overlap;
  M->ratio = ratio;
  M->variant = variant;
  M->basis = basis;
  // arithmetic of the local factorisation, storage of the factors, and
  // arithmetic / local-solution type of the solves
  M->fprec = (prec == HS_C64) ? HS_C64 : HS_C128;
  M->gprec = (prec == HS_C128) ? HS_C128 : HS_C64;
  M->prec = (prec == HS_C64 || prec == HS_C64X) ? HS_C64 : HS_C128;
  // ------------------------------------------------------ decomposition
  struct Axis {
    std::vector<std::pair<int, int>> blocks;
    std::vector<int> ext0, ext1, map;
  };
  auto axis = [&](int ns) {
    Axis a;
    a.blocks = owner_blocks(D.n, D.lo, D.nu, ns);
    for (const auto& b : a.blocks) {
      HS_REQUIRE(b.first >= 0, "empty subdomain block (nsub too large for n)");
      HS_REQUIRE(b.second - b.first >= overlap + 1, "subdomain block narrower than overlap + 1");
    }
    a.ext0.resize(ns);
    a.ext1.resize(ns);
    for (int q = 0; q < ns; ++q) {
      a.ext0[q] = std::max(D.lo, a.blocks[q].first - overlap);
      a.ext1[q] = std::min(D.lo + D.nu, a.blocks[q].second + overlap);
    }
    // grid index -> [owner, cover0..2]
    a.map.assign(4 * (size_t)D.n, -1);
    for (int i = D.lo; i < D.lo + D.nu; ++i) {
      int c = 1;
      for (int q = 0; q < ns; ++q) {
        if (i >= a.blocks[q].first && i < a.blocks[q].second) a.map[4 * i] = q;
        if (i >= a.ext0[q] && i < a.ext1[q]) {
          HS_REQUIRE(c < 4, "a node lies in more than three extended blocks along one axis");
          a.map[4 * i + c++] = q;
        }
      }
    }
    return a;
  };
  const Axis ax = axis(nsx), ay = axis(nsy);
  int64_t gofs = 0, sofs = 0, gent = 0;  // gent: the G_j entries, ny * nx^2 per subdomain (no layout padding)
  int max_nx = 0, max_ny = 0;
  for (int sy = 0; sy < nsy; ++sy)
    for (int sx = 0; sx < nsx; ++sx) {
      SubDesc d{};
      d.ex0 = ax.ext0[sx];
      d.ey0 = ay.ext0[sy];
      d.nx = ax.ext1[sx] - ax.ext0[sx];
      d.ny = ay.ext1[sy] - ay.ext0[sy];
      d.ox0 = ax.blocks[sx].first;
      d.ox1 = ax.blocks[sx].second;
      d.oy0 = ay.blocks[sy].first;
      d.oy1 = ay.blocks[sy].second;
      d.gofs = gofs;
      d.sofs = sofs;
      HS_REQUIRE(d.nx <= 96, "subdomain line longer than 96 nodes");
      gofs += (int64_t)d.ny * local_line_entries(d.nx);
      gent += (int64_t)d.ny * d.nx * d.nx;
      sofs += (int64_t)d.nx * d.ny;
      max_nx = std::max(max_nx, d.nx);
      max_ny = std::max(max_ny, d.ny);
      M->desc_h.push_back(d);
    }
  M->g_elems = gofs;
  M->g_algo = gent;
  M->sol_elems = sofs;
  M->factor_lds = local_factor_lds_bytes(M->fprec, max_nx);
  M->solve_lds = local_solve_lds_bytes(M->prec, max_nx, max_ny);
  M->solve_threads = local_solve_threads(max_nx);
  HS_REQUIRE(M->factor_lds <= 160 * 1024 && M->solve_lds <= 160 * 1024,
             "subdomain too large for the LDS-resident local kernels");
  M->xmap_h = ax.map;
  M->ymap_h = ay.map;
  M->sdesc_h = M->desc_h;
  M->lsolve.cls = local_classes(M->sdesc_h);
  // --------------------------------------------------------- coarse grids
  M->levels.push_back(GridLevel{D.n, D.lo, D.nu, basis});
  for (int r = ratio; r > 1; r /= 2) {
    const GridLevel& f = M->levels.back();
    GridLevel c{(f.n - 1) / 2 + 1, D.lo, 0, basis};
    c.nu = c.n - 2 * D.lo;
    M->levels.push_back(c);
  }
  const int L = (int)M->levels.size() - 1;
  HS_REQUIRE(L <= kMaxStages, "ratio too large");
  HS_REQUIRE(M->levels.back().nu >= 1, "no coarse unknowns for this n and ratio");
  M->lreach.assign(L + 1, 1);
  for (int l = 1; l <= L; ++l) M->lreach[l] = galerkin_reach(basis, M->lreach[l - 1]);
  M->reach = M->lreach[L];
  const int ncu = M->levels.back().nu;
  M->plan = build_nd_plan(ncu, ncu, M->reach, kLeaf);
}

// Device memory of M, carved from A in a fixed order: the persistent part,
// then the set-up scratch.  Uploads the tables when A has a base; with a
// counting arena it only sizes.
void setup_carve(hs_precond* M, Arena& A) {
  const hs_problem* P = M->P;
  const int L = (int)M->levels.size() - 1;
  M->desc = A.put(M->desc_h);
  M->lsolve.desc = A.put(M->sdesc_h);
  M->xmap = A.put(M->xmap_h);
  M->ymap = A.put(M->ymap_h);
  M->rbuf.clear();
  M->pbuf.clear();
  for (int l = 1; l <= L; ++l) M->rbuf.push_back(A.take<c128>((int64_t)M->levels[l].nu * M->levels[l].nu));
  for (int l = 1; l < L; ++l) M->pbuf.push_back(A.take<c128>((int64_t)M->levels[l].nu * M->levels[l].nu));
  M->e0 = A.take<c128>((int64_t)M->levels[L].nu * M->levels[L].nu);
  M->efine = M->tres = nullptr;
  if (M->variant == HS_SHS2) {
    M->efine = A.take<c128>(P->N);
    M->tres = A.take<c128>(P->N);
  }
  const int64_t gall = M->g_elems + local_factor_pad();
  M->G = (M->gprec == HS_C64) ? (void*)A.take<c64>(gall) : (void*)A.take<c128>(gall);
  M->sol = (M->prec == HS_C64) ? (void*)A.take<c64>(M->sol_elems) : (void*)A.take<c128>(M->sol_elems);
  M->lstatus = A.take<int>((int64_t)M->nsx * M->nsy);
  M->stage.clear();
  for (int l = 1; l <= L; ++l) {
    const int W = 2 * M->lreach[l] + 1;
    M->stage.push_back(A.take<c128>((int64_t)M->levels[l].nu * M->levels[l].nu * W * W));
  }
  M->A0 = M->stage.back();
  nd_destroy(M->nd);
  M->nd = nullptr;
  M->nd = nd_create(M->plan, A);
  M->ws_used = A.off;
  // set-up scratch
  const size_t s0 = A.off;
  M->Gf = (M->fprec != M->gprec) ? A.take<c128>(gall) : nullptr;
  const int64_t tail = std::max<int64_t>(M->plan.f_elems, 2 * P->N + 2 * k_red_blocks() + 2);
  M->F = A.take<c128>(tail);
  M->tout = M->F;
  M->mgs_part = M->F + 2 * P->N;
  M->ws_scratch = A.off - s0;
  M->ws_used = A.off;
}

size_t setup_bytes(hs_precond* M) {
  Arena cnt;
  setup_carve(M, cnt);
  return cnt.off;
}

// The factorisations (Sec. 3 local, Sec. 4 coarse) on stream s, then the
// pivot checks; fills M->info.
void setup_run(hs_precond* M, hipStream_t s) {
  const hs_problem* P = M->P;
  const ProblemDev& D = P->dev;
  const int L = (int)M->levels.size() - 1;
  const int ns = M->nsx * M->nsy;
  const int64_t gall = M->g_elems + local_factor_pad();
  prepare_local_solve(M->gprec, M->prec, M->solve_lds);
  HS_HIP(hipStreamCreateWithFlags(&M->side, hipStreamNonBlocking));
  HS_HIP(hipEventCreateWithFlags(&M->ev_fork, hipEventDisableTiming));
  HS_HIP(hipEventCreateWithFlags(&M->ev_join, hipEventDisableTiming));
  // ------------------------------------------------------- local factor
  hipEvent_t ev[4] = {};
  struct Events {
    hipEvent_t* e;
    ~Events() {
      for (int q = 0; q < 4; ++q)
        if (e[q]) (void)hipEventDestroy(e[q]);
    }
  } evs{ev};
  for (auto& e : ev) HS_HIP(hipEventCreate(&e));
  HS_HIP(hipMemsetAsync(M->G, 0, (size_t)gall * (M->gprec == HS_C64 ? 8 : 16), s));
  HS_HIP(hipMemsetAsync(M->lstatus, 0, sizeof(int) * ns, s));
  void* Gf = M->G;
  if (M->Gf) {  // HS_C64X / HS_C64S: factor in complex128, round once
    Gf = M->Gf;
    HS_HIP(hipMemsetAsync(Gf, 0, (size_t)gall * 16, s));
  }
  HS_HIP(hipEventRecord(ev[0], s));
  launch_local_factor(D, M->fprec, ns, M->desc, Gf, M->lstatus, M->factor_lds, M->gprec == HS_C64, s);
  if (M->Gf) launch_round_c64(gall, (const c128*)Gf, (c64*)M->G, s);
  HS_HIP(hipEventRecord(ev[1], s));
  // -------------------------------------------- coarse matrix + factor
  HS_HIP(hipEventRecord(ev[2], s));
  launch_galerkin_first(D, M->levels[1], M->stage[0], s);
  for (int l = 2; l <= L; ++l)
    launch_galerkin_next(M->levels[l - 1], M->lreach[l - 1], M->stage[l - 2], M->levels[l], M->stage[l - 1], s);
  const int cst = nd_factor_run(M->plan, *M->nd, M->A0, M->F, s);
  HS_HIP(hipEventRecord(ev[3], s));
  HS_HIP(hipStreamSynchronize(s));
  std::vector<int> lst((size_t)ns);
  HS_HIP(hipMemcpy(lst.data(), M->lstatus, lst.size() * sizeof(int), hipMemcpyDeviceToHost));
  for (size_t q = 0; q < lst.size(); ++q)
    if (lst[q]) throw Failure{HS_ESINGULAR, "zero pivot in the local factor of subdomain " + std::to_string(q)};
  if (cst) throw Failure{HS_ESINGULAR, "zero pivot in the coarse factor (front " + std::to_string(cst - 1) + ")"};
  float ms_loc = 0.f, ms_crs = 0.f;
  HS_HIP(hipEventElapsedTime(&ms_loc, ev[0], ev[1]));
  HS_HIP(hipEventElapsedTime(&ms_crs, ev[2], ev[3]));
  const GridLevel& cg = M->levels.back();
  hs_precond_info& I = M->info;
  I.n_fine = P->N;
  I.n_coarse = (int64_t)cg.nu * cg.nu;
  I.coarse_per_dim = cg.nu;
  I.coarse_reach = M->reach;
  I.coarse_basis = M->basis;
  I.nsub_total = ns;
  I.local_total = M->sol_elems;
  I.local_factor_bytes = M->g_algo * (M->gprec == HS_C64 ? 8 : 16);
  I.coarse_factor_bytes = (M->plan.g_algo + M->plan.v_algo) * 16;
  I.coarse_solve_bytes = (M->plan.g_algo + 2 * M->plan.v_algo) * 16;
  I.nd_fronts = (int)M->plan.fronts.size();
  I.nd_levels = M->plan.max_depth + 1;
  I.ms_setup_local = ms_loc;
  I.ms_setup_coarse = ms_crs;
  {
    ApplyWork w;
    I.apply_work_bytes = (int64_t)apply_work_layout(M, nullptr, &w);
  }
  I.workspace_bytes = (int64_t)M->ws_used;
  I.setup_scratch_bytes = (int64_t)M->ws_scratch;
}

size_t query_bytes(const hs_problem* P, int nsx, int nsy, int overlap, int ratio, int variant, int prec, int basis) {
  hs_precond M;
  setup_plan(&M, P, nsx, nsy, overlap, ratio, variant, prec, basis);
  return setup_bytes(&M);
}

}  // namespace

extern "C" {

hs_status hs_schwarz_workspace_bytes_ex(const hs_problem* P, int nsub_x, int nsub_y, int overlap, int ratio,
                                        int variant, int prec, int basis, size_t* bytes) {
  return guarded([&] {
    HS_REQUIRE(P && bytes, "null argument");
    *bytes = query_bytes(P, nsub_x, nsub_y, overlap, ratio, variant, prec, basis);
  });
}

hs_status hs_schwarz_workspace_bytes(const hs_problem* P, int nsub_x, int nsub_y, int overlap, int ratio, int prec,
                                     size_t* bytes) {
  // the largest layout over the variants and bases: SHS2 adds two fine-grid
  // vectors, the Bezier basis has the widest coarse stencil
  return hs_schwarz_workspace_bytes_ex(P, nsub_x, nsub_y, overlap, ratio, HS_SHS2, prec, HS_COARSE_BEZIER, bytes);
}

hs_status hs_setup_schwarz_ex(const hs_problem* P, int nsub_x, int nsub_y, int overlap, int ratio, int variant,
                              int prec, int basis, void* ws, size_t ws_bytes, void* stream, hs_precond** out) {
  return guarded([&] {
    HS_REQUIRE(out != nullptr && P != nullptr, "null argument");
    *out = nullptr;
    HS_REQUIRE(ws != nullptr, "ws_dev is NULL");
    HS_REQUIRE(((uintptr_t)ws & 255) == 0, "ws_dev must be 256-byte aligned");
    hs_precond* M = new hs_precond();
    try {
      setup_plan(M, P, nsub_x, nsub_y, overlap, ratio, variant, prec, basis);
      const size_t need = setup_bytes(M);
      if (ws_bytes < need)
        throw Failure{HS_EINVAL, "workspace too small: the preconditioner needs " + std::to_string(need) +
                                     " bytes (hs_schwarz_workspace_bytes)"};
      // all host-side validation is done: device work starts here
      Arena A{(unsigned char*)ws, 0, ws_bytes};
      setup_carve(M, A);
      setup_run(M, S(stream));
    } catch (...) {
      delete M;
      throw;
    }
    *out = M;
  });
}

hs_status hs_setup_schwarz(const hs_problem* P, int nsub_x, int nsub_y, int overlap, int ratio, int variant,
                           int prec, void* ws, size_t ws_bytes, void* stream, hs_precond** out) {
  return hs_setup_schwarz_ex(P, nsub_x, nsub_y, overlap, ratio, variant, prec, HS_COARSE_BEZIER, ws, ws_bytes,
                             stream, out);
}

void hs_destroy_precond(hs_precond* M) { delete M; }

hs_status hs_precond_get_info(const hs_precond* M, hs_precond_info* info) {
  return guarded([&] {
    HS_REQUIRE(M && info, "null argument");
    *info = M->info;
  });
}

hs_status hs_precond_set_schedule(hs_precond* M, int fork_level, int local_grid) {
  return guarded([&] {
    HS_REQUIRE(M, "null argument");
    HS_REQUIRE(fork_level >= 0 && local_grid >= 0, "fork_level and local_grid must be >= 0");
    M->fork_level = fork_level;
    M->local_grid = local_grid;
    if (M->gexec) {  // the captured step holds the old schedule
      HS_HIP(hipGraphExecDestroy(M->gexec));
      M->gexec = nullptr;
    }
  });
}

hs_status hs_precond_get_schedule(const hs_precond* M, int* fork_level, int* local_grid) {
  return guarded([&] {
    HS_REQUIRE(M && fork_level && local_grid, "null argument");
    *fork_level = M->fork_level;
    *local_grid = M->local_grid;
  });
}

hs_status hs_apply_Minv(hs_precond* M, const hs_c128* r, hs_c128* z, void* stream) {
  return guarded([&] {
    HS_REQUIRE(M && r && z, "null argument");
    HS_REQUIRE((const void*)r != (const void*)z, "r and z must not alias");
    apply_minv(M, (const c128*)r, (c128*)z, S(stream));
  });
}

hs_status hs_apply_Minv_noalloc(hs_precond* M, const hs_c128* r, hs_c128* z, void* stream) {
  return guarded([&] {
    HS_REQUIRE(M && r && z, "null argument");
    HS_REQUIRE((const void*)r != (const void*)z, "r and z must not alias");
    ApplyWork w;
    const size_t need = apply_work_layout(M, nullptr, &w);
    if (need > kStaticScratchBytes)
      throw Failure{HS_EINVAL, "hs_apply_Minv_noalloc: the preconditioner needs " + std::to_string(need) +
                                   " bytes of scratch, above the static limit of " +
                                   std::to_string(kStaticScratchBytes)};
    apply_work_layout(M, static_scratch(), &w);
    apply_minv(M, w, (const c128*)r, (c128*)z, S(stream));
  });
}

hs_status hs_nd_plan_level_stats(int ncx, int ncy, int reach, int leaf, int level, int64_t* stats) {
  return guarded([&] {
    HS_REQUIRE(stats != nullptr, "null argument");
    HS_REQUIRE(ncx >= 1 && ncy >= 1 && reach >= 1 && leaf >= 1, "bad plan sizes");
    const NDPlan plan = build_nd_plan(ncx, ncy, reach, leaf);
    HS_REQUIRE(level >= 0 && level <= plan.max_depth, "level out of range");
    Arena cnt;  // counting only: the task tables are built on the host, nothing is uploaded
    NDDev* d = nd_create(plan, cnt);
    nd_level_stats(plan, *d, level, stats);
    nd_destroy(d);
  });
}

hs_status hs_nd_level_stats(const hs_precond* M, int level, int64_t* stats) {
  return guarded([&] {
    HS_REQUIRE(M && stats, "null argument");
    HS_REQUIRE(level >= 0 && level <= M->plan.max_depth, "level out of range");
    nd_level_stats(M->plan, *M->nd, level, stats);
  });
}

hs_status hs_coarse_restrict(hs_precond* M, const hs_c128* r, hs_c128* r0, void* stream) {
  return guarded([&] {
    HS_REQUIRE(M && r && r0, "null argument");
    restrict_chain(M, own_work(M), (const c128*)r, S(stream), (c128*)r0);
  });
}

hs_status hs_coarse_prolong(hs_precond* M, const hs_c128* e0, hs_c128* z, void* stream) {
  return guarded([&] {
    HS_REQUIRE(M && e0 && z, "null argument");
    const int L = (int)M->levels.size() - 1;
    const c128* cur = (const c128*)e0;
    for (int l = L - 1; l >= 1; --l) {
      launch_prolong2(M->levels[l], M->levels[l + 1], cur, M->pbuf[l - 1], 0, S(stream));
      cur = M->pbuf[l - 1];
    }
    launch_prolong2(M->levels[0], M->levels[1], cur, (c128*)z, 0, S(stream));
  });
}

hs_status hs_coarse_solve(hs_precond* M, const hs_c128* r0, hs_c128* e0, void* stream) {
  return guarded([&] {
    HS_REQUIRE(M && r0 && e0, "null argument");
    HS_REQUIRE((const void*)r0 != (const void*)e0, "r0 and e0 must not alias");
    nd_solve_run(M->plan, *M->nd, (const c128*)r0, (c128*)e0, S(stream));
  });
}

hs_status hs_coarse_matrix(hs_precond* M, hs_c128* stencil, void* stream) {
  return guarded([&] {
    HS_REQUIRE(M && stencil, "null argument");
    const int W = 2 * M->reach + 1;
    const int64_t n = M->info.n_coarse * W * W;
    HS_HIP(hipMemcpyAsync(stencil, M->A0, n * sizeof(c128), hipMemcpyDeviceToDevice, S(stream)));
  });
}

hs_status hs_local_solve(hs_precond* M, const hs_c128* r, hs_c128* zloc, void* stream) {
  return guarded([&] {
    HS_REQUIRE(M && r && zloc, "null argument");
    launch_local_solve(M->lsolve, M->P->dev, M->gprec, M->prec, M->G, (const c128*)r, M->sol,
                       M->solve_lds, M->solve_threads, S(stream));
    launch_local_to_c128(M->prec, M->sol_elems, M->sol, (c128*)zloc, S(stream));
  });
}

hs_status hs_time_step(hs_precond* M, int which, const hs_c128* r_, int reps, void* stream, double* avg_ms) {
  return guarded([&] {
    HS_REQUIRE(M && r_ && avg_ms, "null argument");
    HS_REQUIRE(reps >= 1, "reps must be >= 1");
    HS_REQUIRE(which >= 0 && which <= 4, "which must be 0..4");
    const hipStream_t s = S(stream);
    const c128* r = (const c128*)r_;
    const int L = (int)M->levels.size() - 1;
    auto once = [&]() {
      switch (which) {
        case 0:
          launch_local_solve(M->lsolve, M->P->dev, M->gprec, M->prec, M->G, r, M->sol, M->solve_lds, M->solve_threads,
                             s);
          break;
        case 1:
          nd_solve_run(M->plan, *M->nd, M->rbuf[L - 1], M->e0, s);
          break;
        case 2:
          apply_minv(M, r, M->tout, s);
          break;
        case 3:
          launch_spmv(M->P->dev, r, M->tout, s);
          break;
        default:  // one modified Gram-Schmidt projection (w -= h v_prev; dot with v_cur)
          k_mgs(M->P->dev, nullptr, M->P->N, M->tout, r, M->mgs_part, M->mgs_part + 2 * k_red_blocks(),
                M->tout + M->P->N, M->mgs_part + k_red_blocks(), nullptr, s);
      }
    };
    if (which == 1) restrict_chain(M, own_work(M), r, s, nullptr);
    if (which == 4) {
      HS_HIP(hipMemsetAsync(M->mgs_part, 0, (2 * k_red_blocks() + 2) * sizeof(c128), s));
      HS_HIP(hipMemcpyAsync(M->tout, r, M->P->N * sizeof(c128), hipMemcpyDeviceToDevice, s));
      HS_HIP(hipMemcpyAsync(M->tout + M->P->N, r, M->P->N * sizeof(c128), hipMemcpyDeviceToDevice, s));
    }
    once();
    hipEvent_t e0, e1;
    HS_HIP(hipEventCreate(&e0));
    HS_HIP(hipEventCreate(&e1));
    HS_HIP(hipEventRecord(e0, s));
    for (int q = 0; q < reps; ++q) once();
    HS_HIP(hipEventRecord(e1, s));
    HS_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    HS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
  });
}

}  // extern "C"

// ------------------------------------------------------------------ GMRES
namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// workspace of the modified Gram-Schmidt driver
struct MgsLayout {
  size_t V, Z, part, pnorm, hcol, scal, y, r, total;
};

MgsLayout mgs_layout(int64_t N, int maxit) {
  MgsLayout L{};
  const int kb = k_red_blocks();
  size_t o = 0;
  auto take = [&](size_t& f, size_t bytes) {
    f = o;
    o = align_up(o + bytes);
  };
  take(L.V, (size_t)(maxit + 1) * N * sizeof(c128));
  take(L.Z, (size_t)maxit * N * sizeof(c128));
  take(L.part, (size_t)(maxit + 1) * kb * sizeof(c128));
  take(L.pnorm, (size_t)kb * sizeof(double));
  take(L.hcol, (size_t)(maxit + 2) * sizeof(c128));
  take(L.scal, 4 * sizeof(double));
  take(L.y, (size_t)(maxit + 1) * sizeof(c128));
  take(L.r, (size_t)N * sizeof(c128));
  L.total = o;
  return L;
}

// workspace of the DCGS2 driver
struct ArnLayout {
  size_t V, Z, U, Zc, W, r, x0, part, fold, dots, pn, R, cs, sn, g, hist, y, st, pnorm, scal, tab, bstart, total;
  int ept, rpi, nw;
};

// The partial-sum rows are sized for one element per lane (the most waves),
// so the workspace fits every launch shape the table may hold.
ArnLayout arn_layout(int64_t N, int maxit, int ept = 0, int rpi = 0) {
  ArnLayout L{};
  arn_config(N, &L.ept, &L.rpi);
  if (ept) L.ept = ept;
  if (rpi) L.rpi = rpi;
  L.nw = arn_waves(N, L.ept);
  const int nw_max = arn_waves(N, 1);
  size_t o = 0;
  auto take = [&](size_t& f, size_t bytes) {
    f = o;
    o = align_up(o + bytes);
  };
  const size_t vec = (size_t)N * sizeof(c128);
  // tile-major basis: maxit rows of ceil(N / (64 ept)) tiles; sized for the
  // widest tile (64 * 8) so the workspace fits every launch shape
  take(L.V, (size_t)maxit * (size_t)(N + 64 * 8) * sizeof(c128));
  take(L.Z, (size_t)(maxit + 1) * vec);
  take(L.U, vec);
  take(L.Zc, vec);
  take(L.W, vec);
  take(L.r, vec);
  take(L.x0, vec);  // start of a correction cycle (complex64 basis)
  take(L.part, (size_t)(2 * maxit + 2) * ((nw_max + 3) / 4) * sizeof(c128));  // one slab per 4-wave block
  take(L.fold, (size_t)(2 * maxit + 2) * FOLD_CHUNKS * sizeof(c128));
  take(L.dots, (size_t)(2 * maxit + 2) * sizeof(c128));
  take(L.pn, (size_t)nw_max * sizeof(double));
  take(L.R, (size_t)(maxit + 1) * (maxit + 1) * sizeof(c128));
  take(L.cs, (size_t)(maxit + 1) * sizeof(double));
  take(L.sn, (size_t)(maxit + 1) * sizeof(c128));
  take(L.g, (size_t)(maxit + 2) * sizeof(c128));
  take(L.hist, (size_t)(maxit + 2) * sizeof(double));
  take(L.y, (size_t)(maxit + 1) * sizeof(c128));
  take(L.st, sizeof(ArnState));
  take(L.pnorm, (size_t)k_red_blocks() * sizeof(double));
  take(L.scal, 4 * sizeof(double));
  take(L.tab, sizeof(ArnDev));
  take(L.bstart, 2 * sizeof(int));
  L.total = o;
  return L;
}

// The one-instance table of the streaming kernels, uploaded into the
// workspace (the host copies must stay alive until the stream synchronises).
struct ArnSingle {
  ArnDev a;
  int bstart[2];
  ArnBatch b;
};

void arn_single(ArnSingle& S1, const ArnLayout& L, char* base, hipStream_t s, int vprec) {
  S1.bstart[0] = 0;
  S1.bstart[1] = arn_stream_blocks(S1.a.nw);
  HS_HIP(hipMemcpyAsync(base + L.tab, &S1.a, sizeof(ArnDev), hipMemcpyHostToDevice, s));
  HS_HIP(hipMemcpyAsync(base + L.bstart, S1.bstart, 2 * sizeof(int), hipMemcpyHostToDevice, s));
  S1.b = ArnBatch{(const ArnDev*)(base + L.tab), (const int*)(base + L.bstart), 1, S1.bstart[1], S1.a.ept, S1.a.rpi,
                  S1.a.maxit, vprec};
}

ArnDev arn_dev(const hs_problem* P, int maxit, const ArnLayout& L, char* base) {
  ArnDev a{};
  a.P = P->dev;
  a.N = P->N;
  a.maxit = maxit;
  a.ept = L.ept;
  a.rpi = L.rpi;
  a.nw = L.nw;
  a.V = base + L.V;
  a.Z = (c128*)(base + L.Z);
  a.U = (c128*)(base + L.U);
  a.Zc = (c128*)(base + L.Zc);
  a.W = (c128*)(base + L.W);
  a.part = (c128*)(base + L.part);
  a.fold = (c128*)(base + L.fold);
  a.dots = (c128*)(base + L.dots);
  a.pn = (double*)(base + L.pn);
  a.R = (c128*)(base + L.R);
  a.cs = (double*)(base + L.cs);
  a.sn = (c128*)(base + L.sn);
  a.g = (c128*)(base + L.g);
  a.hist = (double*)(base + L.hist);
  a.y = (c128*)(base + L.y);
  a.st = (ArnState*)(base + L.st);
  return a;
}

// one flexible-GMRES iteration: z_k = M^{-1} u_k, then the DCGS2 kernels
void arn_step(hs_precond* M, const ArnDev& a, const ArnBatch& b, hipStream_t s) {
  apply_minv(M, a.U, a.Zc, s);
  k_arn_dots(b, s);
  k_arn_fold(b, s);
  k_arn_column(b, s);
  k_arn_update(b, s);
  k_arn_scale(b, s);
}

// The step as a HIP graph, captured once per (workspace, maxit) on an
// internal non-blocking stream; the local branch of M^{-1} joins the capture
// through the fork / join events.  The step holds no memset or host call.
hipGraphExec_t arn_graph(hs_precond* M, const ArnDev& a, const ArnBatch& b, const void* ws, int maxit) {
  if (M->gexec && M->g_ws == ws && M->g_maxit == maxit && M->g_ept == a.ept && M->g_rpi == a.rpi &&
      M->g_vprec == b.vprec)
    return M->gexec;
  if (M->gexec) {
    (void)hipGraphExecDestroy(M->gexec);
    M->gexec = nullptr;
  }
  if (!M->cap) HS_HIP(hipStreamCreateWithFlags(&M->cap, hipStreamNonBlocking));
  HS_HIP(hipStreamBeginCapture(M->cap, hipStreamCaptureModeThreadLocal));
  hipGraph_t g = nullptr;
  try {
    arn_step(M, a, b, M->cap);
  } catch (...) {
    (void)hipStreamEndCapture(M->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HS_HIP(hipStreamEndCapture(M->cap, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HS_HIP(e);
  M->gexec = ex;
  M->g_ws = ws;
  M->g_maxit = maxit;
  M->g_ept = a.ept;
  M->g_rpi = a.rpi;
  M->g_vprec = b.vprec;
  return ex;
}

struct SolveCtx {
  const hs_problem* P;
  hs_precond* M;
  const c128* b;
  c128* x;
  double tol;
  int maxit;
  void* ws;
  size_t ws_bytes;
  double* history;
  hipStream_t s;
};

// returns true when converged; fills out
bool solve_dcgs2(const SolveCtx& c, const hs_gmres_opts& o, hs_gmres_stats& out) {
  const int64_t N = c.P->N;
  const ArnLayout L = arn_layout(N, c.maxit);
  HS_REQUIRE(c.ws_bytes >= L.total, "workspace too small (see hs_gmres_workspace_bytes)");
  char* base = (char*)c.ws;
  const hipStream_t s = c.s;
  ArnSingle S1;
  S1.a = arn_dev(c.P, c.maxit, L, base);
  const ArnDev& a = S1.a;
  arn_single(S1, L, base, s, o.basis_prec);
  const ArnBatch& bt = S1.b;
  double* pnorm = (double*)(base + L.pnorm);
  double* scal = (double*)(base + L.scal);
  c128* rtmp = (c128*)(base + L.r);

  k_norm2(N, c.b, pnorm, s);
  k_scale(N, c.b, a.U, pnorm, scal, s);
  double beta0 = 0.0;
  HS_HIP(hipMemcpyAsync(&beta0, scal, sizeof(double), hipMemcpyDeviceToHost, s));
  HS_HIP(hipStreamSynchronize(s));
  out.host_checks++;
  if (!std::isfinite(beta0)) throw Failure{HS_ENAN, "non-finite norm of b"};
  if (c.history) c.history[0] = 1.0;
  if (beta0 == 0.0) {
    HS_HIP(hipMemsetAsync(c.x, 0, N * sizeof(c128), s));
    HS_HIP(hipStreamSynchronize(s));
    out.relres_implicit = out.relres_true = 0.0;
    return true;
  }
  k_arn_init(a, beta0, c.tol * beta0, s);
  const hipGraphExec_t ex = o.graph ? arn_graph(c.M, a, bt, c.ws, c.maxit) : nullptr;

  // x = x0 + Z y; x0 is the start of the current correction cycle (none in
  // the first)
  c128* x0 = (c128*)(base + L.x0);
  int cycles = 0;
  auto true_residual = [&](int m) {
    k_arn_backsub(a, m, s);
    k_combo(N, m, a.y, a.Z, N, c.x, s, cycles > 0 ? x0 : nullptr);
    launch_spmv(c.P->dev, c.x, rtmp, s);
    k_bminus(N, c.b, rtmp, s);
    k_norm2(N, rtmp, pnorm, s);
    k_fold_norm(pnorm, scal + 1, s);
    double rn = 0.0;
    HS_HIP(hipMemcpyAsync(&rn, scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    HS_HIP(hipStreamSynchronize(s));
    out.host_checks++;
    return rn / beta0;
  };
  // implicit residuals of a cycle are relative to its start; the history is
  // kept relative to ||b||
  auto save_history = [&](int done_iters, int m, double scale) {
    if (!c.history || m <= 0) return;
    std::vector<double> hh(m);
    HS_HIP(hipMemcpyAsync(hh.data(), a.hist + 1, m * sizeof(double), hipMemcpyDeviceToHost, s));
    HS_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < m; ++q) c.history[done_iters + 1 + q] = hh[q] * scale;
  };

  int K = o.check_every > 0 ? o.check_every : 4;
  int next_k = 0;  // step index of the next launch
  int prev_m = 0;
  double prev_rel = 1.0;
  ArnState h{};
  double relres_true = 1.0;
  bool converged = false;
  int done_iters = 0;          // iterations of the finished correction cycles
  double beta_cycle = beta0;   // ||r|| at the start of the current cycle
  int limit = c.maxit;         // iteration limit of the current cycle
  for (;;) {
    const int cnt = std::min(K, limit + 1 - next_k);
    for (int q = 0; q < cnt; ++q) {
      if (ex)
        HS_HIP(hipGraphLaunch(ex, s));
      else
        arn_step(c.M, a, bt, s);
    }
    next_k += cnt;
    out.steps += cnt;
    HS_HIP(hipMemcpyAsync(&h, a.st, sizeof(ArnState), hipMemcpyDeviceToHost, s));
    HS_HIP(hipStreamSynchronize(s));
    out.host_checks++;
    if (h.done == 0 && next_k <= limit) {
      if (o.check_every <= 0) {  // aim the next check at the predicted stop
        const double target = c.tol * beta0 / beta_cycle;
        if (h.m > prev_m && h.relres > 0.0 && h.relres < prev_rel) {
          const double rate = (std::log(h.relres) - std::log(prev_rel)) / (h.m - prev_m);
          const double need = (std::log(target) - std::log(h.relres)) / rate;
          K = (int)std::min(64.0, std::max(1.0, std::ceil(need)));
        } else {
          K = std::min(2 * K, 64);
        }
        prev_m = h.m;
        prev_rel = h.relres;
      }
      continue;
    }
    if (h.done < 0)
      throw Failure{HS_ENAN, "non-finite value in the Arnoldi process at iteration " +
                                 std::to_string(done_iters + h.k)};
    relres_true = true_residual(h.m);
    if (relres_true <= c.tol || h.done != 1 || done_iters + h.k >= c.maxit) {
      converged = relres_true <= c.tol;
      break;
    }
    if (o.basis_prec == HS_C64) {
      // A complex64 basis bounds the attainable accuracy of one Krylov
      // space (its Arnoldi relation holds to complex64 rounding): start a
      // correction cycle on r = b - A x, which the check just formed in
      // complex128, and add its solution to x.
      save_history(done_iters, h.m, beta_cycle / beta0);
      done_iters += h.m;
      HS_HIP(hipMemcpyAsync(x0, c.x, N * sizeof(c128), hipMemcpyDeviceToDevice, s));
      k_scale(N, rtmp, a.U, pnorm, scal, s);
      beta_cycle = relres_true * beta0;
      limit = c.maxit - done_iters;
      k_arn_init(a, beta_cycle, c.tol * beta0, s, limit);
      cycles++;
      next_k = 0;
      prev_m = 0;
      prev_rel = 1.0;
      continue;
    }
    // the implicit residual met tol but the true one did not: finish step k
    // (its column k is already written) and go on
    k_arn_resume(a, s);
    k_arn_update(bt, s);
    k_arn_scale(bt, s);
    next_k = h.k + 1;
  }
  out.iters = done_iters + h.m;
  out.relres_implicit = h.relres * beta_cycle / beta0;
  out.relres_true = relres_true;
  save_history(done_iters, h.m, beta_cycle / beta0);
  return converged;
}

bool solve_mgs(const SolveCtx& c, hs_gmres_stats& out) {
  const int64_t N = c.P->N;
  const MgsLayout Lw = mgs_layout(N, c.maxit);
  HS_REQUIRE(c.ws_bytes >= Lw.total, "workspace too small (see hs_gmres_workspace_bytes)");
  const hipStream_t s = c.s;
  const int maxit = c.maxit;
  char* base = (char*)c.ws;
  c128* V = (c128*)(base + Lw.V);
  c128* Z = (c128*)(base + Lw.Z);
  c128* part = (c128*)(base + Lw.part);
  double* pnorm = (double*)(base + Lw.pnorm);
  c128* hcol = (c128*)(base + Lw.hcol);
  double* scal = (double*)(base + Lw.scal);
  c128* ydev = (c128*)(base + Lw.y);
  c128* rtmp = (c128*)(base + Lw.r);
  const c128* b = c.b;
  c128* x = c.x;
  using cd = std::complex<double>;
  const int kb = k_red_blocks();

  k_norm2(N, b, pnorm, s);
  k_scale(N, b, V, pnorm, scal, s);
  double beta = 0.0;
  HS_HIP(hipMemcpyAsync(&beta, scal, sizeof(double), hipMemcpyDeviceToHost, s));
  HS_HIP(hipStreamSynchronize(s));
  out.host_checks++;
  if (!std::isfinite(beta)) throw Failure{HS_ENAN, "non-finite norm of b"};
  if (c.history) c.history[0] = 1.0;
  if (beta == 0.0) {
    HS_HIP(hipMemsetAsync(x, 0, N * sizeof(c128), s));
    HS_HIP(hipStreamSynchronize(s));
    out.relres_implicit = out.relres_true = 0.0;
    return true;
  }
  std::vector<std::vector<cd>> R(maxit + 1, std::vector<cd>(maxit, 0.0));
  std::vector<double> cs(maxit, 0.0);
  std::vector<cd> sn(maxit, 0.0), g(maxit + 1, 0.0), hh(maxit + 2);
  g[0] = beta;
  int iters = 0;
  bool converged = false;
  double relres_true = 1.0, relres_impl = 1.0;
  auto solve_and_residual = [&](int m) {
    std::vector<cd> y(m);
    for (int i = m - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int q = i + 1; q < m; ++q) acc -= R[i][q] * y[q];
      y[i] = acc / R[i][i];
    }
    HS_HIP(hipMemcpyAsync(ydev, y.data(), m * sizeof(c128), hipMemcpyHostToDevice, s));
    k_combo(N, m, ydev, Z, N, x, s);
    launch_spmv(c.P->dev, x, rtmp, s);
    k_bminus(N, b, rtmp, s);
    k_norm2(N, rtmp, pnorm, s);
    k_fold_norm(pnorm, scal + 1, s);
    double rn = 0.0;
    HS_HIP(hipMemcpyAsync(&rn, scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    HS_HIP(hipStreamSynchronize(s));
    out.host_checks++;
    return rn / beta;
  };
  for (int j = 0; j < maxit; ++j) {
    c128* vj = V + (int64_t)j * N;
    c128* zj = Z + (int64_t)j * N;
    c128* w = V + (int64_t)(j + 1) * N;
    apply_minv(c.M, vj, zj, s);
    // w = A z_j fused into the first projection; modified Gram-Schmidt
    // against V_0..V_j (each kernel finishes projection i-1 and forms the
    // dot product of projection i); then V_{j+1} = w / ||w||
    for (int i = 0; i <= j; ++i) {
      const c128* vprev = (i == 0) ? nullptr : V + (int64_t)(i - 1) * N;
      const c128* pprev = (i == 0) ? nullptr : part + (int64_t)(i - 1) * kb;
      c128* hout = (i == 0) ? nullptr : hcol + (i - 1);
      k_mgs(c.P->dev, i == 0 ? zj : nullptr, N, w, vprev, pprev, hout, V + (int64_t)i * N, part + (int64_t)i * kb,
            nullptr, s);
    }
    k_mgs(c.P->dev, nullptr, N, w, vj, part + (int64_t)j * kb, hcol + j, nullptr, nullptr, pnorm, s);
    k_scale(N, w, w, pnorm, scal + 2, s);
    HS_HIP(hipMemcpyAsync(hh.data(), hcol, (j + 1) * sizeof(c128), hipMemcpyDeviceToHost, s));
    double hn = 0.0;
    HS_HIP(hipMemcpyAsync(&hn, scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    HS_HIP(hipStreamSynchronize(s));
    out.host_checks++;
    out.steps++;
    if (!std::isfinite(hn)) throw Failure{HS_ENAN, "non-finite Arnoldi norm at iteration " + std::to_string(j + 1)};
    std::vector<cd> col(j + 2);
    for (int i = 0; i <= j; ++i) col[i] = hh[i];
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const cd t = cs[i] * col[i] + sn[i] * col[i + 1];
      col[i + 1] = -std::conj(sn[i]) * col[i] + cs[i] * col[i + 1];
      col[i] = t;
    }
    const cd a = col[j], bb = col[j + 1];
    if (std::abs(a) == 0.0) {
      cs[j] = 0.0;
      sn[j] = 1.0;
    } else {
      const double na = std::abs(a), nrm = std::hypot(na, std::abs(bb));
      cs[j] = na / nrm;
      sn[j] = (a / na) * std::conj(bb) / nrm;
    }
    col[j] = cs[j] * col[j] + sn[j] * col[j + 1];
    col[j + 1] = 0.0;
    for (int i = 0; i <= j; ++i) R[i][j] = col[i];
    g[j + 1] = -std::conj(sn[j]) * g[j];
    g[j] = cs[j] * g[j];
    iters = j + 1;
    relres_impl = std::abs(g[j + 1]) / beta;
    if (c.history) c.history[j + 1] = relres_impl;
    const bool breakdown = (hn == 0.0);
    if (relres_impl <= c.tol || breakdown) {
      relres_true = solve_and_residual(j + 1);
      if (relres_true <= c.tol || breakdown) {
        converged = relres_true <= c.tol;
        break;
      }
    }
    if (j == maxit - 1) relres_true = solve_and_residual(j + 1);
  }
  out.iters = iters;
  out.relres_implicit = relres_impl;
  out.relres_true = relres_true;
  return converged;
}

}  // namespace

extern "C" {

hs_status hs_gmres_workspace_bytes(const hs_problem* P, int maxit, size_t* bytes) {
  return guarded([&] {
    HS_REQUIRE(P && bytes, "null argument");
    HS_REQUIRE(maxit >= 1, "maxit must be >= 1");
    *bytes = std::max(mgs_layout(P->N, maxit).total, arn_layout(P->N, maxit).total);
  });
}

hs_status hs_gmres_solve_ex(const hs_problem* P, hs_precond* M, const hs_c128* b_, hs_c128* x_, double tol,
                            int maxit, const hs_gmres_opts* opts, void* ws, size_t ws_bytes, double* history,
                            void* stream, hs_gmres_stats* stats) {
  hs_status result = HS_OK;
  hs_status st = guarded([&] {
    const auto t0 = std::chrono::steady_clock::now();
    HS_REQUIRE(P && M && b_ && x_ && ws, "null argument");
    HS_REQUIRE(M->P == P, "preconditioner was built on another problem");
    HS_REQUIRE(maxit >= 1, "maxit must be >= 1");
    HS_REQUIRE(tol > 0.0, "tol must be positive");
    hs_gmres_opts o{HS_ORTHO_DCGS2, 1, 0, HS_C128};
    if (opts) o = *opts;
    HS_REQUIRE(o.ortho == HS_ORTHO_DCGS2 || o.ortho == HS_ORTHO_MGS, "ortho must be HS_ORTHO_DCGS2 or HS_ORTHO_MGS");
    HS_REQUIRE(o.check_every >= 0, "check_every must be >= 0");
    HS_REQUIRE(o.basis_prec == HS_C128 || o.basis_prec == HS_C64, "basis_prec must be HS_C128 or HS_C64");
    HS_REQUIRE(o.ortho == HS_ORTHO_DCGS2 || o.basis_prec == HS_C128, "HS_ORTHO_MGS keeps a complex128 basis");
    const SolveCtx c{P, M, (const c128*)b_, (c128*)x_, tol, maxit, ws, ws_bytes, history, S(stream)};
    hs_gmres_stats out{};
    const bool converged = (o.ortho == HS_ORTHO_MGS) ? solve_mgs(c, out) : solve_dcgs2(c, o, out);
    out.converged = converged ? 1 : 0;
    out.ms_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = out;
    if (!converged) result = HS_ENOCONV;
  });
  if (st != HS_OK) return st;
  if (result == HS_ENOCONV) set_error("GMRES reached maxit without converging");
  return result;
}

hs_status hs_gmres_solve(const hs_problem* P, hs_precond* M, const hs_c128* b, hs_c128* x, double tol, int maxit,
                         void* ws, size_t ws_bytes, double* history, void* stream, hs_gmres_stats* stats) {
  return hs_gmres_solve_ex(P, M, b, x, tol, maxit, nullptr, ws, ws_bytes, history, stream, stats);
}

hs_status hs_set_arnoldi_config(int64_t n_unknowns, int ept, int rows) {
  return guarded([&] {
    HS_REQUIRE(n_unknowns >= 1, "n_unknowns must be >= 1");
    const bool reset = (ept == 0 && rows == 0);
    HS_REQUIRE(reset || ept == 1 || ept == 2 || ept == 4 || ept == 8, "ept must be 1, 2, 4 or 8");
    HS_REQUIRE(reset || rows == 2 || rows == 4, "rows must be 2 or 4");
    arn_set_config(n_unknowns, ept, rows);
  });
}

hs_status hs_get_arnoldi_config(int64_t n_unknowns, int* ept, int* rows) {
  return guarded([&] {
    HS_REQUIRE(ept && rows, "null argument");
    HS_REQUIRE(n_unknowns >= 1, "n_unknowns must be >= 1");
    arn_config(n_unknowns, ept, rows);
  });
}

hs_status hs_time_arnoldi(const hs_problem* P, int k, int which, void* ws, size_t ws_bytes, const hs_c128* r_,
                          int reps, void* stream, double* avg_ms) {
  return hs_time_arnoldi_ex(P, k, which, HS_C128, ws, ws_bytes, r_, reps, stream, avg_ms);
}

hs_status hs_time_arnoldi_ex(const hs_problem* P, int k, int which, int basis_prec, void* ws, size_t ws_bytes,
                             const hs_c128* r_, int reps, void* stream, double* avg_ms) {
  return guarded([&] {
    HS_REQUIRE(P && ws && r_ && avg_ms, "null argument");
    HS_REQUIRE(basis_prec == HS_C128 || basis_prec == HS_C64, "basis_prec must be HS_C128 or HS_C64");
    HS_REQUIRE(k >= 0, "k must be >= 0");
    HS_REQUIRE(which >= 0 && which <= 2, "which must be 0..2");
    HS_REQUIRE(reps >= 1, "reps must be >= 1");
    const int maxit = k + 1;
    const ArnLayout L = arn_layout(P->N, maxit);
    HS_REQUIRE(ws_bytes >= L.total, "workspace too small (see hs_gmres_workspace_bytes with maxit >= k + 1)");
    const hipStream_t s = S(stream);
    ArnSingle S1;
    S1.a = arn_dev(P, maxit, L, (char*)ws);
    const ArnDev& a = S1.a;
    arn_single(S1, L, (char*)ws, s, basis_prec);
    const ArnBatch& bt = S1.b;
    const c128* r = (const c128*)r_;
    const size_t vb = (size_t)P->N * sizeof(c128);
    for (c128* dst : {a.U, a.Zc, a.W}) HS_HIP(hipMemcpyAsync(dst, r, vb, hipMemcpyDeviceToDevice, s));
    k_arn_fill_basis(bt, r, k, s);
    k_arn_init(a, 1.0, 0.0, s);
    k_arn_set_step(a, k, s);
    k_arn_dots(bt, s);
    k_arn_fold(bt, s);
    auto once = [&]() {
      switch (which) {
        case 0:
          k_arn_dots(bt, s);
          break;
        case 1:
          k_arn_update(bt, s);
          break;
        default:
          k_arn_set_step(a, k, s);
          k_arn_fold(bt, s);
          k_arn_column(bt, s);
          k_arn_scale(bt, s);
      }
    };
    once();
    hipEvent_t e0, e1;
    HS_HIP(hipEventCreate(&e0));
    HS_HIP(hipEventCreate(&e1));
    HS_HIP(hipEventRecord(e0, s));
    for (int q = 0; q < reps; ++q) once();
    HS_HIP(hipEventRecord(e1, s));
    HS_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    HS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
  });
}

}  // extern "C"

// ================================================================ batches
// Many instances (each a problem with its own preconditioner) advanced
// together: one launch per stage of M^{-1} for all of them (all subdomain
// solves of all instances in one launch, each restriction / prolongation
// stage and each nested-dissection depth over all instances, one final
// combination) and one launch per kernel of the DCGS2 Arnoldi step.
struct hs_batch {
  int count = 0;
  std::vector<hs_precond*> M;
  std::vector<int64_t> offs;  // count + 1: instance i is [offs[i], offs[i+1]) of the batch vectors
  int variant = HS_RAS2, prec = HS_C128, gprec = HS_C128;
  // local solves
  LocalLaunch lsolve;
  LocalArgs* local_tab = nullptr;
  int nsub_total = 0, solve_threads = 0;
  int local_grid = 0;  // workgroups of the persistent local-solve launch (0: one per subdomain)
  int fork_level = 0;  // AS2/RAS2: forward coarse levels launched before the local solves fork
  size_t solve_lds = 0;
  // coarse chain
  struct Stage {
    StageArgs* tab = nullptr;
    int* start = nullptr;
    int tiles = 0;
  };
  std::vector<Stage> restrict_st, prolong_st;  // prolong_st[l - 1]: level l+1 -> l
  NDBatch* nd = nullptr;
  Stage fine_st;                     // SHS2: level 1 -> fine grid into each instance's e
  ResidualArgs* res_tab = nullptr;   // SHS2: t = r - A e per instance
  int* res_start = nullptr;
  int res_tiles = 0;
  CombineArgs* comb_tab = nullptr;
  int* comb_start = nullptr;
  int comb_tiles = 0;
  hipStream_t side = nullptr, cap = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* g_ws = nullptr;
  int g_maxit = 0, g_ept = 0, g_rpi = 0, g_vprec = 0;
  size_t ws_used = 0;
  ~hs_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap) (void)hipStreamDestroy(cap);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    nd_batch_destroy(nd);
  }
};

namespace {

std::vector<int> prefix(const std::vector<int>& n) {
  std::vector<int> s(n.size() + 1, 0);
  for (size_t i = 0; i < n.size(); ++i) s[i + 1] = s[i] + n[i];
  return s;
}

// st: inside a GMRES step, the instances' Arnoldi states; the launches skip
// the instances that no longer iterate.  nullptr: apply to every instance.
void batch_apply(hs_batch* B, const c128* r, c128* z, hipStream_t s, const ArnState* st = nullptr) {
  if (B->variant == HS_SHS2) {  // coarse correction first, then the local solves of r - A e (in order)
    for (const auto& sg : B->restrict_st) launch_restrict2_batch(B->count, sg.tab, sg.start, sg.tiles, r, s, st);
    nd_batch_solve_run(*B->nd, s, Callback{}, 0, st);
    for (int l = (int)B->prolong_st.size(); l >= 1; --l) {
      const auto& sg = B->prolong_st[l - 1];
      launch_prolong2_batch(B->count, sg.tab, sg.start, sg.tiles, s, st);
    }
    launch_prolong2_batch(B->count, B->fine_st.tab, B->fine_st.start, B->fine_st.tiles, s, st);
    launch_residual_batch(B->count, B->res_tab, B->res_start, B->res_tiles, r, s, st);
    launch_local_solve_batch(B->lsolve, B->gprec, B->prec, B->local_tab, r, B->solve_lds,
                             B->solve_threads, B->local_grid, s, st);
    launch_combine_batch(B->variant, B->prec, B->count, B->comb_tab, B->comb_start, B->comb_tiles, z, s, st);
    return;
  }
  // as for one preconditioner: the local solves fork after the first
  // fork_level forward coarse levels (hs_batch_set_schedule)
  auto fork = [&]() {
    HS_HIP(hipEventRecord(B->ev_fork, s));
    HS_HIP(hipStreamWaitEvent(B->side, B->ev_fork, 0));
    launch_local_solve_batch(B->lsolve, B->gprec, B->prec, B->local_tab, r, B->solve_lds,
                             B->solve_threads, B->local_grid, B->side, st);
    HS_HIP(hipEventRecord(B->ev_join, B->side));
  };
  if (B->fork_level <= 0) fork();
  for (const auto& sg : B->restrict_st) launch_restrict2_batch(B->count, sg.tab, sg.start, sg.tiles, r, s, st);
  nd_batch_solve_run(*B->nd, s, B->fork_level > 0 ? callback_of(fork) : Callback{}, B->fork_level, st);
  for (int l = (int)B->prolong_st.size(); l >= 1; --l) {
    const auto& sg = B->prolong_st[l - 1];
    launch_prolong2_batch(B->count, sg.tab, sg.start, sg.tiles, s, st);
  }
  HS_HIP(hipStreamWaitEvent(s, B->ev_join, 0));
  launch_combine_batch(B->variant, B->prec, B->count, B->comb_tab, B->comb_start, B->comb_tiles, z, s, st);
}

// workspace of a batched solve: the batch vectors U and Zc, one DCGS2 region
// per instance, the instance table, the block prefix sums, the per-instance
// one-entry prefixes (for resuming one instance) and the states.
struct BatchLayout {
  int ept = 0, rpi = 0;
  size_t U = 0, Zc = 0, tab = 0, bstart = 0, bone = 0, states = 0, total = 0;
  std::vector<size_t> inst;
  std::vector<ArnLayout> L;
};

BatchLayout batch_layout(const hs_batch* B, int maxit) {
  BatchLayout BL;
  arn_config(B->offs.back(), &BL.ept, &BL.rpi);
  size_t o = 0;
  auto take = [&](size_t& f, size_t bytes) {
    f = o;
    o = align_up(o + bytes);
  };
  const size_t vec = (size_t)B->offs.back() * sizeof(c128);
  take(BL.U, vec);
  take(BL.Zc, vec);
  take(BL.tab, (size_t)B->count * sizeof(ArnDev));
  take(BL.bstart, (size_t)(B->count + 1) * sizeof(int));
  take(BL.bone, (size_t)B->count * 2 * sizeof(int));
  take(BL.states, (size_t)B->count * sizeof(ArnState));
  BL.inst.resize(B->count);
  for (int i = 0; i < B->count; ++i) {
    BL.L.push_back(arn_layout(B->offs[i + 1] - B->offs[i], maxit, BL.ept, BL.rpi));
    take(BL.inst[i], BL.L.back().total);
  }
  BL.total = o;
  return BL;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Tables and the repeats' scratch of a batch, carved from A (a counting
// arena only sizes them).
void batch_build(hs_batch* B, int count, hs_precond* const* Ms, Arena& A) {
  B->count = count;
  B->M.assign(Ms, Ms + count);
  B->variant = Ms[0]->variant;
  B->prec = Ms[0]->prec;
  B->gprec = Ms[0]->gprec;
  B->offs.assign(1, 0);
  for (int i = 0; i < count; ++i) B->offs.push_back(B->offs.back() + Ms[i]->P->N);
  // Scratch of each instance's application (local solutions, coarse
  // vectors, SHS2 vectors): the handle's own at its first occurrence; a
  // repeated handle (another right-hand side of the same problem) gets
  // buffers of its own, owned by the batch.
  struct Scratch {
    void* sol;
    std::vector<c128*> rbuf, pbuf;
    c128 *e0, *efine, *tres;
  };
  std::vector<Scratch> sc(count);
  {
    std::vector<const hs_precond*> seen;
    for (int i = 0; i < count; ++i) {
      const hs_precond* M = Ms[i];
      if (std::find(seen.begin(), seen.end(), M) == seen.end()) {
        seen.push_back(M);
        sc[i] = Scratch{M->sol, M->rbuf, M->pbuf, M->e0, M->efine, M->tres};
        continue;
      }
      Scratch& t = sc[i];
      t.sol = (M->prec == HS_C64) ? (void*)A.take<c64>(M->sol_elems)
                                  : (void*)A.take<c128>(M->sol_elems);
      const int L = (int)M->levels.size() - 1;
      for (int l = 1; l <= L; ++l)
        t.rbuf.push_back(A.take<c128>((int64_t)M->levels[l].nu * M->levels[l].nu));
      for (int l = 1; l < L; ++l)
        t.pbuf.push_back(A.take<c128>((int64_t)M->levels[l].nu * M->levels[l].nu));
      t.e0 = A.take<c128>((int64_t)M->levels[L].nu * M->levels[L].nu);
      t.efine = M->efine ? A.take<c128>(M->P->N) : nullptr;
      t.tres = M->tres ? A.take<c128>(M->P->N) : nullptr;
    }
  }
  // local solves: every subdomain of every instance, in instance order;
  // the instances on one handle interleaved subdomain by subdomain, so
  // that the workgroups reading one factor run together
  std::vector<SubDesc> desc;
  std::vector<LocalArgs> ltab(count);
  for (int i = 0; i < count; ++i) {
    const hs_precond* M = Ms[i];
    if (std::find(Ms, Ms + i, M) != Ms + i) continue;  // placed with its first occurrence
    for (SubDesc d : M->desc_h)
      for (int j = i; j < count; ++j)
        if (Ms[j] == M) {
          d.inst = j;
          desc.push_back(d);
        }
  }
  for (int i = 0; i < count; ++i) {
    const hs_precond* M = Ms[i];
    // SHS2: the local solves take the deflated residual r - A e of the instance
    ltab[i] = LocalArgs{M->P->dev, M->G, sc[i].sol, B->offs[i], M->variant == HS_SHS2 ? sc[i].tres : nullptr};
    B->solve_lds = std::max(B->solve_lds, M->solve_lds);
    B->solve_threads = std::max(B->solve_threads, M->solve_threads);
  }
  // largest subdomains first (work ~ ny nx^2): the last round of
  // workgroups then holds the short solves
  std::stable_sort(desc.begin(), desc.end(), [](const SubDesc& x, const SubDesc& y) {
    return (int64_t)x.ny * x.nx * x.nx > (int64_t)y.ny * y.nx * y.nx;
  });
  B->nsub_total = (int)desc.size();
  if (A.base) prepare_local_solve(B->gprec, B->prec, B->solve_lds);
  B->lsolve.cls = local_classes(desc);
  B->lsolve.desc = A.put(desc);
  B->local_tab = A.put(ltab);
  // restriction stages
  int maxL = 0;
  for (int i = 0; i < count; ++i) maxL = std::max(maxL, (int)Ms[i]->levels.size() - 1);
  for (int st = 0; st < maxL; ++st) {
    std::vector<StageArgs> tab(count);
    std::vector<int> tiles(count, 0);
    for (int i = 0; i < count; ++i) {
      const hs_precond* M = Ms[i];
      const int L = (int)M->levels.size() - 1;
      StageArgs a{};
      if (st < L) {
        a.f = M->levels[st];
        a.c = M->levels[st + 1];
        a.in = st == 0 ? nullptr : sc[i].rbuf[st - 1];
        a.out = sc[i].rbuf[st];
        a.voff = B->offs[i];
        a.tiles = grid_tiles(a.c.nu, a.c.nu);
      }
      tab[i] = a;
      tiles[i] = a.tiles;
    }
    const std::vector<int> pre = prefix(tiles);
    B->restrict_st.push_back({A.put(tab), A.put(pre), pre.back()});
  }
  // nested-dissection coarse solves
  std::vector<const NDPlan*> plans;
  std::vector<NDDev*> devs;
  std::vector<const c128*> r0;
  std::vector<c128*> e0;
  for (int i = 0; i < count; ++i) {
    hs_precond* M = Ms[i];
    plans.push_back(&M->plan);
    devs.push_back(M->nd);
    r0.push_back(sc[i].rbuf[M->levels.size() - 2]);
    e0.push_back(sc[i].e0);
  }
  B->nd = nd_batch_create(plans, devs, r0, e0, A);
  // prolongation stages l+1 -> l for l = maxL-1 .. 1 (l = 0 is fused into the combination)
  for (int l = 1; l < maxL; ++l) {
    std::vector<StageArgs> tab(count);
    std::vector<int> tiles(count, 0);
    for (int i = 0; i < count; ++i) {
      const hs_precond* M = Ms[i];
      const int L = (int)M->levels.size() - 1;
      StageArgs a{};
      if (l <= L - 1) {
        a.f = M->levels[l];
        a.c = M->levels[l + 1];
        a.in = (l == L - 1) ? sc[i].e0 : sc[i].pbuf[l];
        a.out = sc[i].pbuf[l - 1];
        a.voff = 0;
        a.tiles = grid_tiles(a.f.nu, a.f.nu);
      }
      tab[i] = a;
      tiles[i] = a.tiles;
    }
    const std::vector<int> pre = prefix(tiles);
    B->prolong_st.push_back({A.put(tab), A.put(pre), pre.back()});
  }
  const bool shs = B->variant == HS_SHS2;
  if (shs) {
    // eq. (DDM:SO_SHS): the coarse correction on the fine grid, then the
    // deflated residual that the local solves take
    std::vector<StageArgs> tab(count);
    std::vector<ResidualArgs> rtab(count);
    std::vector<int> tiles(count);
    for (int i = 0; i < count; ++i) {
      const hs_precond* M = Ms[i];
      const int L = (int)M->levels.size() - 1;
      StageArgs a{};
      a.f = M->levels[0];
      a.c = M->levels[1];
      a.in = L > 1 ? sc[i].pbuf[0] : sc[i].e0;
      a.out = sc[i].efine;
      a.voff = 0;
      a.tiles = grid_tiles(a.f.nu, a.f.nu);
      tab[i] = a;
      tiles[i] = a.tiles;
      rtab[i] = ResidualArgs{M->P->dev, B->offs[i], sc[i].efine, sc[i].tres};
    }
    const std::vector<int> pre = prefix(tiles);
    B->fine_st = {A.put(tab), A.put(pre), pre.back()};
    B->res_tab = A.put(rtab);
    B->res_start = A.put(pre);
    B->res_tiles = pre.back();
  }
  // final combination (SHS2: local solutions plus e, no coarse prolongation)
  std::vector<CombineArgs> ctab(count);
  std::vector<int> ctiles(count);
  for (int i = 0; i < count; ++i) {
    const hs_precond* M = Ms[i];
    const int L = (int)M->levels.size() - 1;
    ctab[i] = CombineArgs{M->P->dev, M->nsx, M->desc, M->xmap, M->ymap, sc[i].sol, M->levels[0], M->levels[1],
                          shs ? nullptr : (L > 1 ? sc[i].pbuf[0] : sc[i].e0), B->offs[i],
                          shs ? sc[i].efine : nullptr};
    ctiles[i] = grid_tiles(M->P->dev.nu, M->P->dev.nu);
  }
  const std::vector<int> cpre = prefix(ctiles);
  B->comb_tab = A.put(ctab);
  B->comb_start = A.put(cpre);
  B->comb_tiles = cpre.back();
  B->ws_used = A.off;
}

size_t batch_bytes(int count, hs_precond* const* Ms) {
  hs_batch B;
  Arena cnt;
  batch_build(&B, count, Ms, cnt);
  return cnt.off;
}

void batch_check(int count, hs_precond* const* Ms) {
  HS_REQUIRE(count >= 1 && Ms != nullptr, "count must be >= 1 and M non-NULL");
  for (int i = 0; i < count; ++i) HS_REQUIRE(Ms[i] != nullptr, "NULL preconditioner in the batch");
  for (int i = 1; i < count; ++i) {
    HS_REQUIRE(Ms[i]->variant == Ms[0]->variant, "all preconditioners of a batch need one variant");
    HS_REQUIRE(Ms[i]->prec == Ms[0]->prec && Ms[i]->gprec == Ms[0]->gprec,
               "all preconditioners of a batch need one precision");
  }
}

}  // namespace

extern "C" {

hs_status hs_batch_workspace_bytes(int count, hs_precond* const* Ms, size_t* bytes) {
  return guarded([&] {
    HS_REQUIRE(bytes != nullptr, "null argument");
    batch_check(count, Ms);
    *bytes = batch_bytes(count, Ms);
  });
}

hs_status hs_batch_create(int count, hs_precond* const* Ms, void* ws, size_t ws_bytes, hs_batch** out) {
  return guarded([&] {
    HS_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    batch_check(count, Ms);
    HS_REQUIRE(ws != nullptr, "ws_dev is NULL");
    HS_REQUIRE(((uintptr_t)ws & 255) == 0, "ws_dev must be 256-byte aligned");
    const size_t need = batch_bytes(count, Ms);
    if (ws_bytes < need)
      throw Failure{HS_EINVAL, "workspace too small: the batch needs " + std::to_string(need) +
                                   " bytes (hs_batch_workspace_bytes)"};
    hs_batch* B = new hs_batch();
    try {
      Arena A{(unsigned char*)ws, 0, ws_bytes};
      batch_build(B, count, Ms, A);
      HS_HIP(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
      HS_HIP(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
      HS_HIP(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
    } catch (...) {
      delete B;
      throw;
    }
    *out = B;
  });
}

void hs_batch_destroy(hs_batch* B) { delete B; }

hs_status hs_batch_offsets(const hs_batch* B, int64_t* offsets) {
  return guarded([&] {
    HS_REQUIRE(B && offsets, "null argument");
    for (int i = 0; i <= B->count; ++i) offsets[i] = B->offs[i];
  });
}

hs_status hs_batch_set_local_grid(hs_batch* B, int grid) {
  return guarded([&] {
    HS_REQUIRE(B != nullptr, "null argument");
    HS_REQUIRE(grid >= 0, "grid must be >= 0");
    B->local_grid = grid;
    if (B->gexec) {  // the captured step holds the old launch
      (void)hipGraphExecDestroy(B->gexec);
      B->gexec = nullptr;
    }
  });
}

hs_status hs_batch_set_schedule(hs_batch* B, int fork_level, int local_grid) {
  return guarded([&] {
    HS_REQUIRE(B != nullptr, "null argument");
    HS_REQUIRE(fork_level >= 0 && local_grid >= 0, "fork_level and local_grid must be >= 0");
    B->fork_level = fork_level;
    B->local_grid = local_grid;
    if (B->gexec) {  // the captured step holds the old launches
      (void)hipGraphExecDestroy(B->gexec);
      B->gexec = nullptr;
    }
  });
}

hs_status hs_batch_time(hs_batch* B, int which, const hs_c128* r_, hs_c128* z_, int reps, void* stream,
                        double* avg_ms) {
  return guarded([&] {
    HS_REQUIRE(B && r_ && avg_ms, "null argument");
    HS_REQUIRE(which >= 0 && which <= 4, "which must be 0..4");
    HS_REQUIRE(reps >= 1, "reps must be >= 1");
    HS_REQUIRE(which != 2 || (z_ != nullptr && (const void*)z_ != (const void*)r_),
               "the whole application needs an output z_dev that does not alias r_dev");
    const hipStream_t s = S(stream);
    const c128* r = (const c128*)r_;
    c128* z = (c128*)z_;
    auto once = [&]() {
      switch (which) {
        case 0:
          launch_local_solve_batch(B->lsolve, B->gprec, B->prec, B->local_tab, r, B->solve_lds,
                                   B->solve_threads, B->local_grid, s);
          break;
        case 1:
          for (const auto& st : B->restrict_st) launch_restrict2_batch(B->count, st.tab, st.start, st.tiles, r, s);
          nd_batch_solve_run(*B->nd, s);
          for (int l = (int)B->prolong_st.size(); l >= 1; --l) {
            const auto& st = B->prolong_st[l - 1];
            launch_prolong2_batch(B->count, st.tab, st.start, st.tiles, s);
          }
          break;
        case 2:
          batch_apply(B, r, z, s);
          break;
        case 3:
          for (const auto& st : B->restrict_st) launch_restrict2_batch(B->count, st.tab, st.start, st.tiles, r, s);
          break;
        default:
          nd_batch_solve_run(*B->nd, s);
      }
    };
    once();
    hipEvent_t e0, e1;
    HS_HIP(hipEventCreate(&e0));
    HS_HIP(hipEventCreate(&e1));
    HS_HIP(hipEventRecord(e0, s));
    for (int q = 0; q < reps; ++q) once();
    HS_HIP(hipEventRecord(e1, s));
    HS_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    HS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
  });
}

hs_status hs_batch_apply_Minv(hs_batch* B, const hs_c128* r, hs_c128* z, void* stream) {
  return guarded([&] {
    HS_REQUIRE(B && r && z, "null argument");
    HS_REQUIRE((const void*)r != (const void*)z, "r and z must not alias");
    batch_apply(B, (const c128*)r, (c128*)z, S(stream));
  });
}

}  // extern "C"

namespace {

// one batched flexible-GMRES iteration
void batch_step(hs_batch* B, const c128* U, c128* Zc, const ArnBatch& bt, const ArnState* states, hipStream_t s) {
  batch_apply(B, U, Zc, s, states);
  k_arn_dots(bt, s);
  k_arn_fold(bt, s);
  k_arn_column(bt, s);
  k_arn_update(bt, s);
  k_arn_scale(bt, s);
}

hipGraphExec_t batch_graph(hs_batch* B, const c128* U, c128* Zc, const ArnBatch& bt, const ArnState* states,
                           const void* ws, int maxit) {
  if (B->gexec && B->g_ws == ws && B->g_maxit == maxit && B->g_ept == bt.ept && B->g_rpi == bt.rpi &&
      B->g_vprec == bt.vprec)
    return B->gexec;
  if (B->gexec) {
    (void)hipGraphExecDestroy(B->gexec);
    B->gexec = nullptr;
  }
  if (!B->cap) HS_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
  HS_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
  hipGraph_t g = nullptr;
  try {
    batch_step(B, U, Zc, bt, states, B->cap);
  } catch (...) {
    (void)hipStreamEndCapture(B->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HS_HIP(hipStreamEndCapture(B->cap, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HS_HIP(e);
  B->gexec = ex;
  B->g_ws = ws;
  B->g_maxit = maxit;
  B->g_ept = bt.ept;
  B->g_rpi = bt.rpi;
  B->g_vprec = bt.vprec;
  return ex;
}

}  // namespace

extern "C" {

hs_status hs_batch_gmres_workspace_bytes(const hs_batch* B, int maxit, size_t* bytes) {
  return guarded([&] {
    HS_REQUIRE(B && bytes, "null argument");
    HS_REQUIRE(maxit >= 1, "maxit must be >= 1");
    *bytes = batch_layout(B, maxit).total;
  });
}

hs_status hs_batch_gmres_solve(hs_batch* B, const hs_c128* b_, hs_c128* x_, double tol, int maxit,
                               const hs_gmres_opts* opts, void* ws, size_t ws_bytes, void* stream,
                               hs_gmres_stats* stats) {
  hs_status result = HS_OK;
  hs_status st = guarded([&] {
    const auto t0 = std::chrono::steady_clock::now();
    HS_REQUIRE(B && b_ && x_ && ws && stats, "null argument");
    HS_REQUIRE(maxit >= 1, "maxit must be >= 1");
    HS_REQUIRE(tol > 0.0, "tol must be positive");
    hs_gmres_opts o{HS_ORTHO_DCGS2, 1, 0, HS_C128};
    if (opts) o = *opts;
    HS_REQUIRE(o.ortho == HS_ORTHO_DCGS2, "a batch solves with HS_ORTHO_DCGS2");
    HS_REQUIRE(o.check_every >= 0, "check_every must be >= 0");
    HS_REQUIRE(o.basis_prec == HS_C128 || o.basis_prec == HS_C64, "basis_prec must be HS_C128 or HS_C64");
    const BatchLayout BL = batch_layout(B, maxit);
    HS_REQUIRE(ws_bytes >= BL.total, "workspace too small (see hs_batch_gmres_workspace_bytes)");
    const hipStream_t s = S(stream);
    const int count = B->count;
    const c128* b = (const c128*)b_;
    c128* x = (c128*)x_;
    char* base = (char*)ws;
    c128* U = (c128*)(base + BL.U);
    c128* Zc = (c128*)(base + BL.Zc);
    ArnState* states = (ArnState*)(base + BL.states);
    // per-instance tables
    std::vector<ArnDev> tab(count);
    std::vector<int> nblk(count), bone(2 * count);
    for (int i = 0; i < count; ++i) {
      const hs_problem* P = B->M[i]->P;
      ArnDev a = arn_dev(P, maxit, BL.L[i], base + BL.inst[i]);
      a.U = U + B->offs[i];
      a.Zc = Zc + B->offs[i];
      a.st = states + i;
      tab[i] = a;
      nblk[i] = arn_stream_blocks(a.nw);
      bone[2 * i] = 0;
      bone[2 * i + 1] = nblk[i];
    }
    const std::vector<int> bstart = prefix(nblk);
    HS_HIP(hipMemcpyAsync(base + BL.tab, tab.data(), count * sizeof(ArnDev), hipMemcpyHostToDevice, s));
    HS_HIP(hipMemcpyAsync(base + BL.bstart, bstart.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    HS_HIP(hipMemcpyAsync(base + BL.bone, bone.data(), 2 * count * sizeof(int), hipMemcpyHostToDevice, s));
    const ArnDev* tab_dev = (const ArnDev*)(base + BL.tab);
    const int* bone_dev = (const int*)(base + BL.bone);
    const ArnBatch all{tab_dev, (const int*)(base + BL.bstart), count, bstart.back(), BL.ept, BL.rpi, maxit,
                       o.basis_prec};
    auto one = [&](int i) {
      return ArnBatch{tab_dev + i, bone_dev + 2 * i, 1, nblk[i], BL.ept, BL.rpi, maxit, o.basis_prec};
    };
    // ||b_i||, u_0 = b_i / ||b_i||
    std::vector<double> beta0(count);
    for (int i = 0; i < count; ++i) {
      const ArnDev& a = tab[i];
      double* pnorm = (double*)(base + BL.inst[i] + BL.L[i].pnorm);
      double* scal = (double*)(base + BL.inst[i] + BL.L[i].scal);
      k_norm2(a.N, b + B->offs[i], pnorm, s);
      k_scale(a.N, b + B->offs[i], a.U, pnorm, scal, s);
      HS_HIP(hipMemcpyAsync(&beta0[i], scal, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HS_HIP(hipStreamSynchronize(s));
    std::vector<hs_gmres_stats> out(count);
    std::vector<int> finished(count, 0), failed(count, 0);
    int host_checks = 1;
    for (int i = 0; i < count; ++i) {
      const ArnDev& a = tab[i];
      if (!std::isfinite(beta0[i])) {
        failed[i] = HS_ENAN;
        finished[i] = 1;
        k_arn_init(a, 1.0, 0.0, s);
        k_arn_set_done(a, 4, s);
        continue;
      }
      k_arn_init(a, beta0[i], tol * beta0[i], s);
      if (beta0[i] == 0.0) {
        HS_HIP(hipMemsetAsync(x + B->offs[i], 0, a.N * sizeof(c128), s));
        k_arn_set_done(a, 4, s);
        finished[i] = 1;
        out[i].converged = 1;
      }
    }
    const hipGraphExec_t ex = o.graph ? batch_graph(B, U, Zc, all, states, ws, maxit) : nullptr;
    // per instance: correction cycles of a complex64 basis (as in the single
    // solve), iterations of the finished cycles, ||r|| at the cycle start,
    // iteration limit of the cycle
    std::vector<int> cycles(count, 0), done_iters(count, 0), limit(count, maxit);
    std::vector<double> beta_cycle(beta0);
    auto true_residual = [&](int i, int m) {
      const ArnDev& a = tab[i];
      char* ib = base + BL.inst[i];
      double* pnorm = (double*)(ib + BL.L[i].pnorm);
      double* scal = (double*)(ib + BL.L[i].scal);
      c128* rtmp = (c128*)(ib + BL.L[i].r);
      c128* xi = x + B->offs[i];
      k_arn_backsub(a, m, s);
      k_combo(a.N, m, a.y, a.Z, a.N, xi, s, cycles[i] > 0 ? (const c128*)(ib + BL.L[i].x0) : nullptr);
      launch_spmv(B->M[i]->P->dev, xi, rtmp, s);
      k_bminus(a.N, b + B->offs[i], rtmp, s);
      k_norm2(a.N, rtmp, pnorm, s);
      k_fold_norm(pnorm, scal + 1, s);
      double rn = 0.0;
      HS_HIP(hipMemcpyAsync(&rn, scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
      HS_HIP(hipStreamSynchronize(s));
      ++host_checks;
      return rn / beta0[i];
    };
    std::vector<ArnState> h(count);
    int K = o.check_every > 0 ? o.check_every : 4;
    int steps = 0;
    std::vector<int> prev_m(count, 0);
    std::vector<double> prev_rel(count, 1.0);
    for (;;) {
      int left = 0, room = maxit + 1;
      for (int i = 0; i < count; ++i)
        if (!finished[i]) {
          ++left;
          room = std::min(room, limit[i] + 1 - h[i].k);
        }
      if (!left) break;
      const int cnt = std::max(1, std::min(K, room));
      for (int q = 0; q < cnt; ++q) {
        if (ex)
          HS_HIP(hipGraphLaunch(ex, s));
        else
          batch_step(B, U, Zc, all, states, s);
      }
      steps += cnt;
      HS_HIP(hipMemcpyAsync(h.data(), states, count * sizeof(ArnState), hipMemcpyDeviceToHost, s));
      HS_HIP(hipStreamSynchronize(s));
      ++host_checks;
      int want = 64;
      for (int i = 0; i < count; ++i) {
        if (finished[i]) continue;
        if (h[i].done == 0) {
          if (o.check_every <= 0 && h[i].m > prev_m[i] && h[i].relres > 0.0 && h[i].relres < prev_rel[i]) {
            const double rate = (std::log(h[i].relres) - std::log(prev_rel[i])) / (h[i].m - prev_m[i]);
            const double target = tol * beta0[i] / beta_cycle[i];
            const double need = (std::log(target) - std::log(h[i].relres)) / rate;
            want = std::min(want, (int)std::min(64.0, std::max(1.0, std::ceil(need))));
          }
          prev_m[i] = h[i].m;
          prev_rel[i] = h[i].relres;
          continue;
        }
        if (h[i].done < 0) {
          failed[i] = HS_ENAN;
          finished[i] = 1;
          out[i].iters = done_iters[i] + h[i].m;
          continue;
        }
        const double rt = true_residual(i, h[i].m);
        if (rt <= tol || h[i].done != 1 || done_iters[i] + h[i].k >= maxit) {
          finished[i] = 1;
          out[i].iters = done_iters[i] + h[i].m;
          out[i].relres_implicit = h[i].relres * beta_cycle[i] / beta0[i];
          out[i].relres_true = rt;
          out[i].converged = rt <= tol;
          k_arn_set_done(tab[i], 4, s);  // no later step touches it
          continue;
        }
        if (o.basis_prec == HS_C64) {  // a correction cycle on r_i (see the single solve)
          char* ib = base + BL.inst[i];
          const ArnDev& a = tab[i];
          done_iters[i] += h[i].m;
          HS_HIP(hipMemcpyAsync(ib + BL.L[i].x0, x + B->offs[i], a.N * sizeof(c128), hipMemcpyDeviceToDevice, s));
          k_scale(a.N, (const c128*)(ib + BL.L[i].r), a.U, (const double*)(ib + BL.L[i].pnorm),
                  (double*)(ib + BL.L[i].scal), s);
          beta_cycle[i] = rt * beta0[i];
          limit[i] = maxit - done_iters[i];
          k_arn_init(a, beta_cycle[i], tol * beta0[i], s, limit[i]);
          cycles[i]++;
          h[i] = ArnState{};
          prev_m[i] = 0;
          prev_rel[i] = 1.0;
          want = 1;
          continue;
        }
        // the implicit residual met tol but the true one did not: finish
        // this instance's step k alone and let it go on
        const ArnBatch bi = one(i);
        k_arn_resume(tab[i], s);
        k_arn_update(bi, s);
        k_arn_scale(bi, s);
        h[i].k += 1;
        h[i].done = 0;
        want = 1;
      }
      if (o.check_every <= 0) K = want;
    }
    HS_HIP(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < count; ++i) {
      out[i].ms_solve = ms;
      out[i].steps = steps;
      out[i].host_checks = host_checks;
      stats[i] = out[i];
      if (failed[i] && result == HS_OK) result = (hs_status)failed[i];
      else if (!out[i].converged && result == HS_OK) result = HS_ENOCONV;
    }
  });
  if (st != HS_OK) return st;
  if (result == HS_ENOCONV) set_error("GMRES reached maxit without converging on at least one instance");
  if (result == HS_ENAN) set_error("non-finite value in at least one instance");
  return result;
}

}  // extern "C"

// ------------------------------------------------ batches as plain arrays
namespace {

// workspace of the array form: the batch's tables, its GMRES workspace and
// the two concatenated batch vectors (b, x), in that order
struct ArrayLayout {
  size_t batch = 0, gmres = 0, bvec = 0, xvec = 0, total = 0, gmres_bytes = 0;
};

ArrayLayout array_layout(int count, hs_precond* const* Ms, int maxit, hs_batch* B) {
  Arena cnt;
  batch_build(B, count, Ms, cnt);
  ArrayLayout L;
  size_t o = align_up(cnt.off);
  L.gmres = o;
  L.gmres_bytes = batch_layout(B, maxit).total;
  o = align_up(o + L.gmres_bytes);
  L.bvec = o;
  o = align_up(o + (size_t)B->offs.back() * sizeof(c128));
  L.xvec = o;
  o = align_up(o + (size_t)B->offs.back() * sizeof(c128));
  L.total = o;
  return L;
}

void array_check(int count, const hs_problem* const* P, hs_precond* const* Ms, int maxit) {
  batch_check(count, Ms);
  HS_REQUIRE(P != nullptr, "P is NULL");
  HS_REQUIRE(maxit >= 1, "maxit must be >= 1");
  for (int i = 0; i < count; ++i) HS_REQUIRE(Ms[i]->P == P[i], "M[i] was not built on P[i]");
}

}  // namespace

extern "C" {

hs_status hs_gmres_batch_workspace_bytes(int count, const hs_problem* const* P, hs_precond* const* M, int maxit,
                                         size_t* bytes) {
  return guarded([&] {
    HS_REQUIRE(bytes != nullptr, "null argument");
    array_check(count, P, M, maxit);
    hs_batch B;
    *bytes = array_layout(count, M, maxit, &B).total;
  });
}

hs_status hs_gmres_solve_batch(int count, const hs_problem* const* P, hs_precond* const* M,
                               const hs_c128* const* b, hs_c128* const* x, double tol, int maxit, void* ws,
                               size_t ws_bytes, void* stream, hs_gmres_stats* stats) {
  hs_status result = HS_OK;
  const hs_status st = guarded([&] {
    HS_REQUIRE(b && x && stats, "null argument");
    array_check(count, P, M, maxit);
    for (int i = 0; i < count; ++i) HS_REQUIRE(b[i] && x[i], "NULL vector in b or x");
    HS_REQUIRE(tol > 0.0, "tol must be positive");
    HS_REQUIRE(ws != nullptr, "ws_dev is NULL");
    HS_REQUIRE(((uintptr_t)ws & 255) == 0, "ws_dev must be 256-byte aligned");
    ArrayLayout L;
    {
      hs_batch sizing;
      L = array_layout(count, M, maxit, &sizing);
    }
    if (ws_bytes < L.total)
      throw Failure{HS_EINVAL, "workspace too small: the batch solve needs " + std::to_string(L.total) +
                                   " bytes (hs_gmres_batch_workspace_bytes)"};
    const hipStream_t s = S(stream);
    unsigned char* base = (unsigned char*)ws;
    hs_batch B;
    Arena A{base, 0, L.gmres};
    batch_build(&B, count, M, A);
    HS_HIP(hipStreamCreateWithFlags(&B.side, hipStreamNonBlocking));
    HS_HIP(hipEventCreateWithFlags(&B.ev_fork, hipEventDisableTiming));
    HS_HIP(hipEventCreateWithFlags(&B.ev_join, hipEventDisableTiming));
    c128* bv = (c128*)(base + L.bvec);
    c128* xv = (c128*)(base + L.xvec);
    for (int i = 0; i < count; ++i)
      HS_HIP(hipMemcpyAsync(bv + B.offs[i], b[i], (size_t)(B.offs[i + 1] - B.offs[i]) * sizeof(c128),
                            hipMemcpyDeviceToDevice, s));
    result = hs_batch_gmres_solve(&B, (const hs_c128*)bv, (hs_c128*)xv, tol, maxit, nullptr, base + L.gmres,
                                  L.gmres_bytes, stream, stats);
    if (result != HS_OK && result != HS_ENOCONV && result != HS_ENAN) throw Failure{result, hs_last_error()};
    const std::string msg = result == HS_OK ? std::string() : std::string(hs_last_error());
    for (int i = 0; i < count; ++i)
      HS_HIP(hipMemcpyAsync(x[i], xv + B.offs[i], (size_t)(B.offs[i + 1] - B.offs[i]) * sizeof(c128),
                            hipMemcpyDeviceToDevice, s));
    HS_HIP(hipStreamSynchronize(s));
    if (result != HS_OK) set_error(msg);
  });
  return st != HS_OK ? st : result;
}

}  // extern "C"
