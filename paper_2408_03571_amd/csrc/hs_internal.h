// Internal declarations shared by the HIP translation units of libhelmschwarz.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/helmschwarz.h"

// ----------------------------------------------------------------- errors
namespace hs {

void set_error(const std::string& msg);

struct Failure {
  hs_status st;
  std::string msg;
};

#define HS_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::hs::Failure{HS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define HS_REQUIRE(cond, msg)                                   \
  do {                                                          \
    if (!(cond)) throw ::hs::Failure{HS_EINVAL, std::string(msg)}; \
  } while (0)

// Device memory carved out of one caller-owned buffer, in 256-byte aligned
// pieces.  With base == nullptr it only counts (the size queries run the
// same carving as the set-ups they size).  put() uploads a host table.
struct Arena {
  unsigned char* base = nullptr;
  size_t off = 0;
  size_t cap = ~(size_t)0;
  template <typename X>
  X* take(int64_t n) {
    if (n < 1) n = 1;
    const size_t at = off;
    off = (off + (size_t)n * sizeof(X) + 255) & ~(size_t)255;
    if (base && off > cap) throw Failure{HS_EINVAL, "workspace too small for this preconditioner or batch"};
    return base ? reinterpret_cast<X*>(base + at) : nullptr;
  }
  template <typename X>
  X* put(const std::vector<X>& h) {
    X* p = take<X>((int64_t)h.size());
    if (base && !h.empty()) {
      const hipError_t e = hipMemcpy(p, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice);
      if (e != hipSuccess) throw Failure{HS_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e)};
    }
    return p;
  }
};

// A non-owning reference to a callable (no heap allocation, unlike
// std::function): the schedule hook of the coarse solves.
struct Callback {
  void (*fn)(void*) = nullptr;
  void* ctx = nullptr;
  explicit operator bool() const { return fn != nullptr; }
  void operator()() const { fn(ctx); }
};
template <typename F>
Callback callback_of(F& f) {
  return Callback{[](void* c) { (*static_cast<F*>(c))(); }, &f};
}

// ---------------------------------------------------------- complex maths
template <typename T> struct cplx { T x, y; };
using c64 = cplx<float>;
using c128 = cplx<double>;

template <typename T> __host__ __device__ inline cplx<T> cmk(T a, T b) { return {a, b}; }
template <typename T> __host__ __device__ inline cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __host__ __device__ inline cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __host__ __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __host__ __device__ inline cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
// acc += a * b
template <typename T> __host__ __device__ inline void cfma(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc -= a * b
template <typename T> __host__ __device__ inline void cfms(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}
template <typename T> __host__ __device__ inline T cabs2(cplx<T> a) { return a.x * a.x + a.y * a.y; }
template <typename T> __host__ __device__ inline cplx<T> cinv(cplx<T> a) {
  // 1/a with scaling against overflow
  T s = fabs(a.x) > fabs(a.y) ? fabs(a.x) : fabs(a.y);
  T ax = a.x / s, ay = a.y / s;
  T d = (ax * ax + ay * ay) * s;
  return {ax / d, -ay / d};
}
template <typename To, typename Ti> __host__ __device__ inline cplx<To> ccast(cplx<Ti> a) {
  return {(To)a.x, (To)a.y};
}

// -------------------------------------------------------------- problem
// Device-side view of the five-point problem: stencil coefficients are
// generated on the fly from (n, h, k or k^2[], bc).
struct ProblemDev {
  int n;         // grid nodes per dimension
  int bc;        // HS_BC_*
  int lo;        // first grid index carrying an unknown (0 or 1)
  int nu;        // unknowns per dimension
  double h, inv_h2, k2c;  // k2c: constant k^2 (used when k2 == nullptr)
  const double* k2;       // optional k^2 per grid node [j*n + i]
};

// Five-point row of unknown (i, j) (grid indices).  Off-diagonal entries are
// real; a missing neighbour (outside the grid, or a Dirichlet boundary node)
// has coefficient zero.
struct Row5 {
  c128 d;
  double w, e, s, n;  // west (i-1), east (i+1), south (j-1), north (j+1)
};

__host__ __device__ inline Row5 row5(const ProblemDev& P, int i, int j) {
  const double k2 = P.k2 ? P.k2[(int64_t)j * P.n + i] : P.k2c;
  Row5 r;
  if (P.bc == HS_BC_DIRICHLET) {
    r.d = {4.0 * P.inv_h2 - k2, 0.0};
    r.w = (i - 1 >= 1) ? -P.inv_h2 : 0.0;
    r.e = (i + 1 <= P.n - 2) ? -P.inv_h2 : 0.0;
    r.s = (j - 1 >= 1) ? -P.inv_h2 : 0.0;
    r.n = (j + 1 <= P.n - 2) ? -P.inv_h2 : 0.0;
    return r;
  }
  // Sommerfeld: centred ghost node u_g = u_mirror + 2 i k h u_b on each
  // outward normal; the mirror neighbour doubles, the row is scaled by 2^-e.
  const int gl = (i == 0), gr = (i == P.n - 1), gs = (j == 0), gn = (j == P.n - 1);
  const int e = gl + gr + gs + gn;
  const double sc = e == 0 ? 1.0 : (e == 1 ? 0.5 : 0.25);
  const double kk = sqrt(k2);
  r.d = {sc * (4.0 * P.inv_h2 - k2), -sc * 2.0 * kk * (double)e / P.h};
  r.w = gl ? 0.0 : -sc * P.inv_h2 * (gr ? 2.0 : 1.0);
  r.e = gr ? 0.0 : -sc * P.inv_h2 * (gl ? 2.0 : 1.0);
  r.s = gs ? 0.0 : -sc * P.inv_h2 * (gn ? 2.0 : 1.0);
  r.n = gn ? 0.0 : -sc * P.inv_h2 * (gs ? 2.0 : 1.0);
  return r;
}

// (A x)_l for unknown l (x fastest over the nu x nu unknown grid).
__device__ inline c128 spmv_at(const ProblemDev& P, const c128* __restrict__ x, int64_t l) {
  const int iu = (int)(l % P.nu), ju = (int)(l / P.nu);
  const Row5 r = row5(P, iu + P.lo, ju + P.lo);
  c128 acc = cmul(r.d, x[l]);
  if (r.w != 0.0) { const c128 v = x[l - 1]; acc.x += r.w * v.x; acc.y += r.w * v.y; }
  if (r.e != 0.0) { const c128 v = x[l + 1]; acc.x += r.e * v.x; acc.y += r.e * v.y; }
  if (r.s != 0.0) { const c128 v = x[l - P.nu]; acc.x += r.s * v.x; acc.y += r.s * v.y; }
  if (r.n != 0.0) { const c128 v = x[l + P.nu]; acc.x += r.n * v.x; acc.y += r.n * v.y; }
  return acc;
}

}  // namespace hs

// ------------------------------------------------------------ handles
struct hs_problem {
  hs::ProblemDev dev;
  double k;
  int64_t N;
};

namespace hs {

// One grid level of the coarse hierarchy (fine grid = level 0).
struct GridLevel {
  int n;      // nodes per dimension
  int lo;     // first unknown grid index
  int nu;     // unknowns per dimension
  int basis;  // coarse basis of the ratio-2 transfer from the next finer
              // level into this one (HS_COARSE_BEZIER or HS_COARSE_P1)
};

// Per-subdomain descriptor (device and host).
struct SubDesc {
  int ex0, ey0;     // first grid index of the extended block
  int nx, ny;       // extended block size
  int ox0, ox1;     // owned x range [ox0, ox1)
  int oy0, oy1;     // owned y range
  int64_t gofs;     // element offset of G_0 in the factor array
  int64_t sofs;     // element offset in the local-solution array
  int inst;         // instance of a batch (0 for a single preconditioner)
  int pad;
};

// Nested-dissection front (device and host).
struct Rect { int x0, x1, y0, y1, base; };
constexpr int kMaxRects = 24;

// G = F_II^-1 of a front is complex symmetric, as A_0 = A_0^T (Sec. 2-4).
// Fronts of at most kNDTri unknowns -- the size a subtree workgroup takes
// whole, where one pass over a stored entry serves its row and its column
// (level launches, which split a front's rows over workgroups, read such a
// front's lines twice) -- keep only the lower triangle, rows packed: G[k][c]
// (c <= k) at entry k(k+1)/2 + c.  Larger fronts keep all of G, rows ldg
// entries apart.
constexpr int kNDTri = 64;
__host__ __device__ inline bool nd_tri(int nI) { return nI <= kNDTri; }
// offset of G[k][c] in its front's block
__host__ __device__ inline int64_t nd_g_index(int nI, int ldg, int k, int c) {
  if (nd_tri(nI)) {
    const int hi = k > c ? k : c, lo = k > c ? c : k;
    return (int64_t)hi * (hi + 1) / 2 + lo;
  }
  return (int64_t)k * ldg + c;
}
// entries a solve reads from G (the stored ones)
__host__ __device__ inline int64_t nd_g_entries(int nI, int ldg) {
  return nd_tri(nI) ? (int64_t)nI * (nI + 1) / 2 : (int64_t)nI * ldg;
}

struct NDFront {
  int nI, nB, nF;
  int ldg, ldv;              // row strides of G (full storage) and V: |I| and |B| rounded up to 8 entries (128 bytes)
  int depth;
  int child[2];
  int nrect;
  Rect rect[kMaxRects];      // position lookup: rect[0] = I, rest = B pieces
  int64_t Iid, Bid;          // offsets into the id arrays
  int64_t inv[2];            // offsets into the inverse-map array (|F| ints per child) or -1
  int64_t gofs, vofs;        // G (|I|^2, or its packed lower triangle) and V (|I| x |B|) in the factor array
  int64_t fofs;              // F (|F|^2) in the front workspace
  int64_t cofs, uofs;        // c (|I|) and u (|B|) vectors of the solve
  int64_t pofs;              // rho (|I|) pivot rows
  int64_t ppofs;             // positions of this front's B nodes in the parent front
};

struct NDPlan {
  int ncx, ncy, reach, leaf;
  std::vector<NDFront> fronts;
  std::vector<int> Iid, Bid, inv, ppos;
  std::vector<std::vector<int>> levels;  // front ids per depth
  int64_t g_elems = 0, v_elems = 0, f_elems = 0, c_elems = 0, u_elems = 0, p_elems = 0;  // storage
  int64_t g_algo = 0, v_algo = 0;  // entries of G (|I|^2 or |I|(|I|+1)/2) and of V (|I||B|) a solve reads
  int max_depth = 0;
};

NDPlan build_nd_plan(int ncx, int ncy, int reach, int leaf);
struct NDDev;  // device copy of a plan (k_nd.hip)

}  // namespace hs

namespace hs {
// ------------------------------------------------------------ batching
// Launches over many instances map a block to its instance through the
// prefix sums `start` (count + 1 entries) of the per-instance block counts.
__host__ __device__ inline int batch_locate(const int* start, int count, int b) {
  int lo = 0, hi = count - 1;  // largest i with start[i] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// per-instance data of the batched local solves
struct LocalArgs {
  ProblemDev P;
  const void* G;    // local factors (storage type of the batch)
  void* sol;        // local solutions
  int64_t voff;     // offset of the instance in the batch vectors
  const c128* rhs;  // right-hand side of the local solves; nullptr: the batch vector at voff
};

// per-instance data of the batched grid sweeps (restrict / prolong stages
// and the final combination)
struct StageArgs {
  GridLevel f, c;   // fine and coarse level of the stage
  const c128* in;   // nullptr: the batch input vector at voff
  c128* out;
  int64_t voff;
  int tiles;        // launch tiles of this instance (0: not in this stage)
};

struct CombineArgs {
  ProblemDev P;
  int nsx;
  const SubDesc* desc;
  const int* xmap;
  const int* ymap;
  const void* sol;
  GridLevel f, c;
  const c128* e0;   // level-1 coarse correction (or the coarse solution when H = 2h); nullptr: none
  int64_t voff;
  const c128* addv; // added on the fine grid (SHS2: the coarse correction e = Q r); nullptr: none
};

// per-instance data of the batched residual t = r - A e (SHS2)
struct ResidualArgs {
  ProblemDev P;
  int64_t voff;     // offset of r in the batch vector
  const c128* e;
  c128* t;
};

}  // namespace hs

// ------------------------------------------------------------ kernels
// launchers (defined in the k_*.hip files)
namespace hs {
void launch_spmv(const ProblemDev& P, const c128* x, c128* y, hipStream_t s);
void launch_k2_grad(const ProblemDev& P, const c128* u, const c128* lam, double scale, double* grad, hipStream_t s);
void launch_restrict2(const GridLevel& f, const GridLevel& c, const c128* in, c128* out, hipStream_t s);
void launch_prolong2(const GridLevel& f, const GridLevel& c, const c128* in, c128* out, int accumulate,
                     hipStream_t s);
// reach of the coarse stencil after one Galerkin stage of a reach-rin operator
int galerkin_reach(int basis, int rin);
void launch_galerkin_first(const ProblemDev& P, const GridLevel& c, c128* A0, hipStream_t s);
void launch_galerkin_next(const GridLevel& f, int rin, const c128* Af, const GridLevel& c, c128* Ac,
                          hipStream_t s);
// addv != nullptr: z also gains addv (a fine-grid vector)
void launch_combine(const ProblemDev& P, int variant, int prec, int nsx, const SubDesc* desc_dev,
                    const int* xmap_dev, const int* ymap_dev, const void* sol, const GridLevel* f,
                    const GridLevel* c, const c128* e0, c128* z, hipStream_t s, const c128* addv = nullptr);
void launch_residual(const ProblemDev& P, const c128* r, const c128* e, c128* t, hipStream_t s);
// batched grid sweeps: `start` holds the prefix sums of the per-instance tiles
int grid_tiles(int nx, int ny);
// st: the instances' Arnoldi states (skip the idle ones) or nullptr
struct ArnState;
void launch_residual_batch(int count, const ResidualArgs* tab, const int* start, int total_tiles, const c128* r,
                           hipStream_t s, const ArnState* st = nullptr);
void launch_restrict2_batch(int count, const StageArgs* tab, const int* start, int total_tiles, const c128* in,
                            hipStream_t s, const ArnState* st = nullptr);
void launch_prolong2_batch(int count, const StageArgs* tab, const int* start, int total_tiles, hipStream_t s,
                           const ArnState* st = nullptr);
void launch_combine_batch(int variant, int prec, int count, const CombineArgs* tab, const int* start,
                          int total_tiles, c128* z, hipStream_t s, const ArnState* st = nullptr);

void launch_local_factor(const ProblemDev& P, int prec, int nsub, const SubDesc* desc, void* G, int* status,
                         size_t lds, bool pair, hipStream_t s);
void prepare_local_solve(int gprec, int cprec, size_t lds);
// The subdomains of a local-solve launch, grouped into classes of segment
// counts (one kernel instantiation each; usually a single class).
struct LocalClass {
  int first, count, range;
};
struct LocalLaunch {
  const SubDesc* desc = nullptr;  // device, class by class
  std::vector<LocalClass> cls;
};
// reorders desc class by class (stable within a class) and returns the classes
std::vector<LocalClass> local_classes(std::vector<SubDesc>& desc);
// grid: persistent workgroups per class (each takes subdomains g, g + grid,
// ...); 0 = one per subdomain
void launch_local_solve(const LocalLaunch& L, const ProblemDev& P, int gprec, int cprec, const void* G,
                        const c128* r, void* sol, size_t lds, int threads, hipStream_t s, int grid = 0);
// all subdomains of a batch: desc[b].inst selects tab[]
void launch_local_solve_batch(const LocalLaunch& L, int gprec, int cprec, const LocalArgs* tab, const c128* r,
                              size_t lds, int threads, int grid, hipStream_t s, const ArnState* st = nullptr);
int local_solve_threads(int max_nx);
// factor entries stored per grid line (both layouts): the segment rows times
// TPR * nx, zero columns past nx included
int64_t local_line_entries(int nx);
int64_t local_factor_pad();
void launch_local_to_c128(int prec, int64_t count, const void* sol, c128* out, hipStream_t s);
void launch_round_c64(int64_t count, const c128* in, c64* out, hipStream_t s);

// ---------------------------------------------- low-synchronisation Arnoldi
// Device-resident state of one flexible-GMRES solve (k_arnoldi.hip).
struct ArnState {
  int k;          // Arnoldi step in progress: u_k (normalised, not yet reorthogonalised) sits in U
  int done;       // 0 running, 1 implicit residual <= tol, 2 breakdown, 3 maxit, -1 non-finite
  int m;          // columns of the Hessenberg matrix that are final
  int maxit;
  double beta0;   // ||b||
  double tol_abs; // tol * ||b||
  double beta;    // norm of the last classical Gram-Schmidt residual: u_k = w1 / beta
  double alpha;   // ||u_k - V s||, the reorthogonalisation norm of the current step
  c128 c;         // v_k^H w of the current step
  double relres;  // |g_m| / ||b||
  double pad;
};

// A batched application of M^{-1} inside a GMRES step skips the instances
// whose Arnoldi state is no longer running (converged, stopped or failed):
// their result would not be read.  st == nullptr: every instance runs.
__device__ inline bool inst_idle(const ArnState* st, int inst) { return st != nullptr && st[inst].done != 0; }


constexpr int FOLD_CHUNKS = 16;  // first-level ranges of the dot-partial fold

struct ArnDev {
  ProblemDev P;            // operator, for the fused A z
  int64_t N;               // unknowns
  int maxit;               // rows reserved in V / columns of R
  int ept, nw;             // elements per lane, waves of the streaming kernels
  int rpi;                 // basis rows per loop trip of the streaming kernels (2 or 4)
  void* V;                 // final basis, maxit rows, tile-major, complex128 or complex64
  c128* Z;                 // preconditioned vectors (maxit+1 rows)
  c128 *U, *Zc, *W;        // current u_k, M^{-1} u_k, A z_k
  c128* part;              // dot partials: one slab of 2 maxit + 2 entries per block of the dot pass
  c128* fold;              // first-level sums of the slabs: FOLD_CHUNKS x (2 maxit + 2)
  c128* dots;              // folded dots: s [0,maxit), t [maxit, 2 maxit), u^H u, u^H w
  double* pn;              // per-wave partials of ||w1||^2
  c128* R;                 // rotated Hessenberg columns, (maxit+1) x (maxit+1), column-major
  double* cs;              // Givens cosines
  c128* sn;                // Givens sines
  c128* g;                 // rotated right-hand side
  double* hist;            // implicit relative residual per finalised column
  c128* y;                 // least-squares solution
  ArnState* st;
};

// The streaming kernels run over one or many instances: block b belongs to
// instance batch_locate(bstart, count, b) and is that instance's block
// b - bstart[inst].  All instances share the launch shape (ept, rpi) and maxit.
struct ArnBatch {
  const ArnDev* tab;   // device, count entries
  const int* bstart;   // device, count + 1 prefix sums of the per-instance blocks
  int count;
  int blocks;          // bstart[count]
  int ept, rpi, maxit;
  int vprec;           // storage type of the basis V: HS_C128 or HS_C64
};

int arn_stream_blocks(int nw);
int arn_ept(int64_t N);
void arn_config(int64_t N, int* ept, int* rpi);  // tuned or built-in launch shape
void arn_set_config(int64_t N, int ept, int rpi);
int arn_waves(int64_t N, int ept);
// limit > 0: the cycle stops (done = 3) after that many iterations (<= maxit)
void k_arn_init(const ArnDev& a, double beta0, double tol_abs, hipStream_t s, int limit = 0);
void k_arn_dots(const ArnBatch& b, hipStream_t s);
// basis vectors 0..k-1 of the (single) instance := r, in the tile-major layout
void k_arn_fill_basis(const ArnBatch& b, const c128* r, int k, hipStream_t s);
void k_arn_fold(const ArnBatch& b, hipStream_t s);
void k_arn_column(const ArnBatch& b, hipStream_t s);
void k_arn_update(const ArnBatch& b, hipStream_t s);
void k_arn_scale(const ArnBatch& b, hipStream_t s);
void k_arn_resume(const ArnDev& a, hipStream_t s);
void k_arn_backsub(const ArnDev& a, int m, hipStream_t s);
void k_arn_set_step(const ArnDev& a, int k, hipStream_t s);
void k_arn_set_done(const ArnDev& a, int code, hipStream_t s);

struct NDBatch;
// tables and the repeats' work vectors come from the arena
NDBatch* nd_batch_create(const std::vector<const NDPlan*>& plans, const std::vector<NDDev*>& devs,
                         const std::vector<const c128*>& r0, const std::vector<c128*>& e0, Arena& A);
void nd_batch_destroy(NDBatch* B);
// after (if set) is called once, after the first after_levels forward levels
// have been launched (or after all of them)
void nd_batch_solve_run(const NDBatch& B, hipStream_t s, const Callback& after = Callback{},
                        int after_levels = 0, const ArnState* st = nullptr);

}  // namespace hs
