// Grid kernels: five-point operator, coarse restriction / prolongation
// (Bezier or linear basis), Galerkin coarse operator and the final
// combination of M^{-1} r.
//
// All of them are HBM-streaming stencil sweeps: a 2-D launch with threadIdx.x
// along x (the fastest index of every vector) keeps each wave's loads and
// stores coalesced; neighbour reuse is left to L1/L2.
#include "hs_internal.h"

namespace hs {

namespace {

constexpr int TX = 64, TY = 4;

// Ratio-2 stage taps of the two coarse bases along one axis, offset -2..2:
// Bezier (Sec. 4, eq. GCS:HO_R_0) and linear interpolation (the P1 basis the
// paper compares against, Sec. 4-5), whose prolongation puts 1 on the
// coincident fine node and 1/2 on its two neighbours.
__constant__ double kTaps[2][5] = {{1.0 / 8, 4.0 / 8, 6.0 / 8, 4.0 / 8, 1.0 / 8}, {0.0, 0.5, 1.0, 0.5, 0.0}};

__device__ inline double tap(int basis, int d) { return (d >= -2 && d <= 2) ? kTaps[basis][d + 2] : 0.0; }

// ------------------------------------------------------------------ A x
// eq. (LS_final): y = A x with the stencil generated from (h, k^2, bc).
// One TX x TY tile per workgroup.  Workgroups go to the 8 XCDs in turn (each
// with its own L2), so tiles are handed out XCD by XCD: workgroup b takes
// tile (b mod 8) * per + b / 8 of the row-major tile order, and each XCD
// sweeps a contiguous run of tile rows, whose halo rows are then mostly
// still in its L2 (launched with 8 * per workgroups, per = ceil(tiles / 8)).
constexpr int kXcds = 8;
__global__ void __launch_bounds__(TX* TY) spmv_kernel(ProblemDev P, const c128* __restrict__ x,
                                                      c128* __restrict__ y, int tiles_x, int tiles, int per) {
  const int t = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
  if (t >= tiles) return;
  const int by = t / tiles_x, bx = t - by * tiles_x;
  const int iu = bx * TX + threadIdx.x;
  const int ju = by * TY + threadIdx.y;
  if (iu >= P.nu || ju >= P.nu) return;
  const int i = iu + P.lo, j = ju + P.lo;
  const Row5 r = row5(P, i, j);
  const int64_t l = (int64_t)ju * P.nu + iu;
  c128 acc = cmul(r.d, x[l]);
  if (r.w != 0.0) { const c128 v = x[l - 1]; acc.x += r.w * v.x; acc.y += r.w * v.y; }
  if (r.e != 0.0) { const c128 v = x[l + 1]; acc.x += r.e * v.x; acc.y += r.e * v.y; }
  if (r.s != 0.0) { const c128 v = x[l - P.nu]; acc.x += r.s * v.x; acc.y += r.s * v.y; }
  if (r.n != 0.0) { const c128 v = x[l + P.nu]; acc.x += r.n * v.x; acc.y += r.n * v.y; }
  y[l] = acc;
}

// ------------------------------------------------- R_0 (one ratio-2 stage)
// Sec. 4, eq. (GCS:HO_R_0): coarse node c sits on fine node 2c and takes
// (1,4,6,4,1)/8 of its fine neighbours along each axis (linear basis:
// (1/2,1,1/2)); taps that fall on a node that is not an unknown (outside the
// grid / Dirichlet boundary) drop.
// One TX x TY tile of coarse nodes: the (2 TY + 3) x (2 TX + 3) window of
// fine values it reads is staged in LDS with coalesced loads (nodes outside
// the unknowns read as zero, which drops their taps), then every coarse node
// takes its 5 x 5 taps from LDS (a weighted sum along x per fine row, then
// the weighted sum of the rows).
constexpr int RWX = 2 * TX + 3, RWY = 2 * TY + 3;

__device__ inline void restrict_tile(const GridLevel& f, const GridLevel& c, const c128* __restrict__ in, int tx0,
                                     int ty0, c128* __restrict__ out, c128 (*win)[RWX]) {
  const int tid = threadIdx.y * TX + threadIdx.x;
  const int gx0 = 2 * (tx0 + c.lo) - 2 - f.lo, gy0 = 2 * (ty0 + c.lo) - 2 - f.lo;  // fine unknown index of win[0][0]
  for (int q = tid; q < RWX * RWY; q += TX * TY) {
    const int r = q / RWX, cc = q - r * RWX;
    const int x = gx0 + cc, y = gy0 + r;
    win[r][cc] = (x >= 0 && x < f.nu && y >= 0 && y < f.nu) ? in[(int64_t)y * f.nu + x] : c128{0.0, 0.0};
  }
  __syncthreads();
  const int Iu = tx0 + threadIdx.x, Ju = ty0 + threadIdx.y;
  if (Iu >= c.nu || Ju >= c.nu) return;
  c128 acc = {0.0, 0.0};
  for (int b = -2; b <= 2; ++b) {
    const c128* row = win[2 * threadIdx.y + 2 + b] + 2 * threadIdx.x + 2;
    c128 rs = {0.0, 0.0};
    for (int a = -2; a <= 2; ++a) {
      const c128 v = row[a];
      rs.x += tap(c.basis, a) * v.x;
      rs.y += tap(c.basis, a) * v.y;
    }
    acc.x += tap(c.basis, b) * rs.x;
    acc.y += tap(c.basis, b) * rs.y;
  }
  out[(int64_t)Ju * c.nu + Iu] = acc;
}

__global__ void __launch_bounds__(TX* TY) restrict2_kernel(GridLevel f, GridLevel c,
                                                           const c128* __restrict__ in,
                                                           c128* __restrict__ out) {
  __shared__ c128 win[RWY][RWX];
  restrict_tile(f, c, in, blockIdx.x * TX, blockIdx.y * TY, out, win);
}

// Batched launches: block b belongs to instance batch_locate(start, b) and
// covers tile b - start[inst] of that instance's row-major tile grid.
__device__ inline int tile_of(const int* start, int count, int& t) {
  const int inst = batch_locate(start, count, blockIdx.x);
  t = blockIdx.x - start[inst];
  return inst;
}

__global__ void __launch_bounds__(TX* TY) restrict2_batch_kernel(const StageArgs* __restrict__ tab,
                                                                 const int* __restrict__ start, int count,
                                                                 const c128* __restrict__ in_batch,
                                                                 const ArnState* __restrict__ st) {
  __shared__ c128 win[RWY][RWX];
  int t;
  const int inst = tile_of(start, count, t);
  if (inst_idle(st, inst)) return;
  const StageArgs A = tab[inst];
  const int tpr = (A.c.nu + TX - 1) / TX;
  const c128* in = A.in ? A.in : in_batch + A.voff;
  restrict_tile(A.f, A.c, in, (t % tpr) * TX, (t / tpr) * TY, A.out, win);
}

// ---------------------------------------------- R_0^T (one ratio-2 stage)
// Gather form: a fine node receives from the <= 3 coarse nodes per axis
// whose taps cover it, so no two threads write the same output.
__device__ inline c128 prolong_at(const GridLevel& f, const GridLevel& c, const c128* __restrict__ in,
                                  int i, int j) {
  c128 acc = {0.0, 0.0};
  const int J0 = (j - 1) >> 1, I0 = (i - 1) >> 1;  // floor((j-2)/2) + ... covered below
  for (int J = J0; J <= J0 + 2; ++J) {
    const int Ju = J - c.lo;
    const double wy = tap(c.basis, j - 2 * J);
    if (Ju < 0 || Ju >= c.nu || wy == 0.0) continue;
    for (int I = I0; I <= I0 + 2; ++I) {
      const int Iu = I - c.lo;
      const double wx = tap(c.basis, i - 2 * I);
      if (Iu < 0 || Iu >= c.nu || wx == 0.0) continue;
      const c128 v = in[(int64_t)Ju * c.nu + Iu];
      acc.x += wx * wy * v.x;
      acc.y += wx * wy * v.y;
    }
  }
  return acc;
}

__global__ void __launch_bounds__(TX* TY) prolong2_kernel(GridLevel f, GridLevel c,
                                                          const c128* __restrict__ in,
                                                          c128* __restrict__ out, int accumulate) {
  const int iu = blockIdx.x * TX + threadIdx.x;
  const int ju = blockIdx.y * TY + threadIdx.y;
  if (iu >= f.nu || ju >= f.nu) return;
  c128 v = prolong_at(f, c, in, iu + f.lo, ju + f.lo);
  const int64_t l = (int64_t)ju * f.nu + iu;
  if (accumulate) v = cadd(v, out[l]);
  out[l] = v;
}

__global__ void __launch_bounds__(TX* TY) prolong2_batch_kernel(const StageArgs* __restrict__ tab,
                                                                const int* __restrict__ start, int count,
                                                                const ArnState* __restrict__ st) {
  int t;
  const int inst = tile_of(start, count, t);
  if (inst_idle(st, inst)) return;
  const StageArgs A = tab[inst];
  const int tpr = (A.f.nu + TX - 1) / TX;
  const int iu = (t % tpr) * TX + threadIdx.x, ju = (t / tpr) * TY + threadIdx.y;
  if (iu >= A.f.nu || ju >= A.f.nu) return;
  A.out[(int64_t)ju * A.f.nu + iu] = prolong_at(A.f, A.c, A.in, iu + A.f.lo, ju + A.f.lo);
}

// ------------------------------------------------ Galerkin A_0 = R A R^T
// One ratio-2 Galerkin stage of a (2*RIN+1)^2-point fine operator to a
// (2*ROUT+1)^2-point coarse operator, ROUT = (2*RT + RIN) / 2 for taps of
// reach RT (2: Bezier, 1: linear).  Each thread owns one coarse node and
// accumulates its row in LDS:
//   A0[c, c+d] = sum_{p in supp(c)} t(p-2c) sum_e A(p, p+e) t(p+e-2(c+d)).
constexpr int GAL_WG = 64;

template <int RIN, int ROUT, int RT, bool FIRST>
__global__ void __launch_bounds__(GAL_WG) galerkin_kernel(ProblemDev P, GridLevel f, const c128* __restrict__ Af,
                                                          GridLevel c, c128* __restrict__ Ac) {
  constexpr int WO = 2 * ROUT + 1, NO = WO * WO;
  constexpr int WI = 2 * RIN + 1;
  __shared__ c128 acc_s[GAL_WG][NO];
  c128* acc = acc_s[threadIdx.x];
  const int64_t node = (int64_t)blockIdx.x * GAL_WG + threadIdx.x;
  const int64_t Nc = (int64_t)c.nu * c.nu;
  if (node >= Nc) return;
  for (int q = 0; q < NO; ++q) acc[q] = {0.0, 0.0};
  const int Iu = (int)(node % c.nu), Ju = (int)(node / c.nu);
  const int I = Iu + c.lo, J = Ju + c.lo;
  const int basis = (RT == 2) ? HS_COARSE_BEZIER : HS_COARSE_P1;
  for (int ay = -RT; ay <= RT; ++ay) {
    const int pj = 2 * J + ay;
    if (pj - f.lo < 0 || pj - f.lo >= f.nu) continue;
    for (int ax = -RT; ax <= RT; ++ax) {
      const int pi = 2 * I + ax;
      if (pi - f.lo < 0 || pi - f.lo >= f.nu) continue;
      const double wp = tap(basis, ax) * tap(basis, ay);
      // fine row p
      c128 arow[WI * WI];
      if (FIRST) {
        const Row5 r = row5(P, pi, pj);
        for (int q = 0; q < WI * WI; ++q) arow[q] = {0.0, 0.0};
        arow[RIN * WI + RIN] = r.d;
        arow[RIN * WI + RIN - 1] = {r.w, 0.0};
        arow[RIN * WI + RIN + 1] = {r.e, 0.0};
        arow[(RIN - 1) * WI + RIN] = {r.s, 0.0};
        arow[(RIN + 1) * WI + RIN] = {r.n, 0.0};
      } else {
        const int64_t pl = (int64_t)(pj - f.lo) * f.nu + (pi - f.lo);
        for (int q = 0; q < WI * WI; ++q) arow[q] = Af[pl * (WI * WI) + q];
      }
      for (int ey = -RIN; ey <= RIN; ++ey) {
        for (int ex = -RIN; ex <= RIN; ++ex) {
          const c128 a = arow[(ey + RIN) * WI + (ex + RIN)];
          if (a.x == 0.0 && a.y == 0.0) continue;
          const c128 wa = cscale(a, wp);
          const int sy = ay + ey, sx = ax + ex;  // q - 2c
          // coarse neighbours d with |s - 2d| <= RT
          const int dy0 = (sy - RT + 1 + 64) / 2 - 32, dy1 = (sy + RT + 64) / 2 - 32;
          const int dx0 = (sx - RT + 1 + 64) / 2 - 32, dx1 = (sx + RT + 64) / 2 - 32;
          for (int dy = dy0; dy <= dy1; ++dy) {
            const double ty = tap(basis, sy - 2 * dy);
            for (int dx = dx0; dx <= dx1; ++dx) {
              const double w = ty * tap(basis, sx - 2 * dx);
              c128& o = acc[(dy + ROUT) * WO + (dx + ROUT)];
              o.x += w * wa.x;
              o.y += w * wa.y;
            }
          }
        }
      }
    }
  }
  for (int dy = -ROUT; dy <= ROUT; ++dy)
    for (int dx = -ROUT; dx <= ROUT; ++dx) {
      const int Nx = Iu + dx, Ny = Ju + dy;
      c128 v = acc[(dy + ROUT) * WO + (dx + ROUT)];
      if (Nx < 0 || Nx >= c.nu || Ny < 0 || Ny >= c.nu) v = {0.0, 0.0};
      Ac[node * NO + (dy + ROUT) * WO + (dx + ROUT)] = v;
    }
}

// ---------------------------------------------------- z = coarse + local
// z = R_0^T e0 (last ratio-2 stage, gather form) plus the local part:
// RAS2 takes the owner subdomain's solution (Boolean D_i), AS2 sums the
// solutions of every subdomain whose extended block holds the node, in a
// fixed order (deterministic, no atomics).
template <typename T>
__device__ inline c128 combine_at(const ProblemDev& P, int variant, int nsx, const SubDesc* __restrict__ desc,
                                  const int* __restrict__ xmap, const int* __restrict__ ymap,
                                  const cplx<T>* __restrict__ sol, const GridLevel& f, const GridLevel& c,
                                  const c128* __restrict__ e0, int has_coarse, const c128* __restrict__ addv,
                                  int iu, int ju) {
  const int i = iu + P.lo, j = ju + P.lo;
  c128 acc = has_coarse ? prolong_at(f, c, e0, i, j) : c128{0.0, 0.0};
  if (addv) acc = cadd(acc, addv[(int64_t)ju * P.nu + iu]);
  // maps: per grid index 4 ints: owner, cover0, cover1, cover2 (-1 = none)
  const int* xm = xmap + 4 * i;
  const int* ym = ymap + 4 * j;
  if (variant == HS_RAS2 || variant == HS_SHS2) {
    const SubDesc& d = desc[ym[0] * nsx + xm[0]];
    const cplx<T> v = sol[d.sofs + (int64_t)(j - d.ey0) * d.nx + (i - d.ex0)];
    acc.x += (double)v.x;
    acc.y += (double)v.y;
  } else {
    for (int b = 1; b < 4; ++b) {
      const int sy = ym[b];
      if (sy < 0) break;
      for (int a = 1; a < 4; ++a) {
        const int sx = xm[a];
        if (sx < 0) break;
        const SubDesc& d = desc[sy * nsx + sx];
        const cplx<T> v = sol[d.sofs + (int64_t)(j - d.ey0) * d.nx + (i - d.ex0)];
        acc.x += (double)v.x;
        acc.y += (double)v.y;
      }
    }
  }
  return acc;
}

template <typename T>
__global__ void __launch_bounds__(TX* TY) combine_kernel(ProblemDev P, int variant, int nsx,
                                                         const SubDesc* __restrict__ desc,
                                                         const int* __restrict__ xmap,
                                                         const int* __restrict__ ymap,
                                                         const cplx<T>* __restrict__ sol, GridLevel f,
                                                         GridLevel c, const c128* __restrict__ e0,
                                                         c128* __restrict__ z, int has_coarse,
                                                         const c128* __restrict__ addv) {
  const int iu = blockIdx.x * TX + threadIdx.x;
  const int ju = blockIdx.y * TY + threadIdx.y;
  if (iu >= P.nu || ju >= P.nu) return;
  z[(int64_t)ju * P.nu + iu] =
      combine_at<T>(P, variant, nsx, desc, xmap, ymap, sol, f, c, e0, has_coarse, addv, iu, ju);
}

template <typename T>
__global__ void __launch_bounds__(TX* TY) combine_batch_kernel(int variant, const CombineArgs* __restrict__ tab,
                                                               const int* __restrict__ start, int count,
                                                               c128* __restrict__ z, const ArnState* __restrict__ st) {
  int t;
  const int inst = tile_of(start, count, t);
  if (inst_idle(st, inst)) return;
  const CombineArgs& A = tab[inst];
  const ProblemDev P = A.P;
  const int tpr = (P.nu + TX - 1) / TX;
  const int iu = (t % tpr) * TX + threadIdx.x, ju = (t / tpr) * TY + threadIdx.y;
  if (iu >= P.nu || ju >= P.nu) return;
  z[A.voff + (int64_t)ju * P.nu + iu] = combine_at<T>(P, variant, A.nsx, A.desc, A.xmap, A.ymap,
                                                      (const cplx<T>*)A.sol, A.f, A.c, A.e0, A.e0 != nullptr,
                                                      A.addv, iu, ju);
}

// t = r - A e  (the deflated residual of SHS2, eq. DDM:SO_SHS)
__global__ void __launch_bounds__(TX* TY) residual_kernel(ProblemDev P, const c128* __restrict__ r,
                                                          const c128* __restrict__ e, c128* __restrict__ t) {
  const int iu = blockIdx.x * TX + threadIdx.x;
  const int ju = blockIdx.y * TY + threadIdx.y;
  if (iu >= P.nu || ju >= P.nu) return;
  const int64_t l = (int64_t)ju * P.nu + iu;
  t[l] = csub(r[l], spmv_at(P, e, l));
}

// t_i = r_i - A_i e_i for every instance of a batch (SHS2)
__global__ void __launch_bounds__(TX* TY) residual_batch_kernel(const ResidualArgs* __restrict__ tab,
                                                                const int* __restrict__ start, int count,
                                                                const c128* __restrict__ r,
                                                                const ArnState* __restrict__ st) {
  int t;
  const int inst = tile_of(start, count, t);
  if (inst_idle(st, inst)) return;
  const ResidualArgs A = tab[inst];
  const int tpr = (A.P.nu + TX - 1) / TX;
  const int iu = (t % tpr) * TX + threadIdx.x, ju = (t / tpr) * TY + threadIdx.y;
  if (iu >= A.P.nu || ju >= A.P.nu) return;
  const int64_t l = (int64_t)ju * A.P.nu + iu;
  A.t[l] = csub(r[A.voff + l], spmv_at(A.P, A.e, l));
}

// grad[node] += scale * Re(dA_ll/dk^2 * u_l * lam_l)
__global__ void __launch_bounds__(TX* TY) k2_grad_kernel(ProblemDev P, const c128* __restrict__ u,
                                                         const c128* __restrict__ lam, double scale,
                                                         double* __restrict__ grad) {
  const int iu = blockIdx.x * TX + threadIdx.x;
  const int ju = blockIdx.y * TY + threadIdx.y;
  if (iu >= P.nu || ju >= P.nu) return;
  const int i = iu + P.lo, j = ju + P.lo;
  const int64_t l = (int64_t)ju * P.nu + iu;
  c128 d = {-1.0, 0.0};
  if (P.bc == HS_BC_SOMMERFELD) {
    const int e = (i == 0) + (i == P.n - 1) + (j == 0) + (j == P.n - 1);
    const double w = e == 0 ? 1.0 : (e == 1 ? 0.5 : 0.25);
    const double k2 = P.k2 ? P.k2[(int64_t)j * P.n + i] : P.k2c;
    d = {-w, -w * (double)e / (sqrt(k2) * P.h)};
  }
  const c128 t = cmul(cmul(d, u[l]), lam[l]);
  grad[(int64_t)j * P.n + i] += scale * t.x;
}

inline dim3 grid2(int nx, int ny) { return dim3((nx + TX - 1) / TX, (ny + TY - 1) / TY); }

}  // namespace

void launch_spmv(const ProblemDev& P, const c128* x, c128* y, hipStream_t s) {
  const dim3 g = grid2(P.nu, P.nu);
  const int tiles = (int)(g.x * g.y), per = (tiles + kXcds - 1) / kXcds;
  spmv_kernel<<<kXcds * per, dim3(TX, TY), 0, s>>>(P, x, y, (int)g.x, tiles, per);
  HS_HIP(hipGetLastError());
}

void launch_residual(const ProblemDev& P, const c128* r, const c128* e, c128* t, hipStream_t s) {
  residual_kernel<<<grid2(P.nu, P.nu), dim3(TX, TY), 0, s>>>(P, r, e, t);
  HS_HIP(hipGetLastError());
}

void launch_k2_grad(const ProblemDev& P, const c128* u, const c128* lam, double scale, double* grad, hipStream_t s) {
  k2_grad_kernel<<<grid2(P.nu, P.nu), dim3(TX, TY), 0, s>>>(P, u, lam, scale, grad);
  HS_HIP(hipGetLastError());
}

int grid_tiles(int nx, int ny) { return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY); }

void launch_restrict2_batch(int count, const StageArgs* tab, const int* start, int total_tiles, const c128* in,
                            hipStream_t s, const ArnState* st) {
  if (total_tiles <= 0) return;
  restrict2_batch_kernel<<<total_tiles, dim3(TX, TY), 0, s>>>(tab, start, count, in, st);
  HS_HIP(hipGetLastError());
}

void launch_residual_batch(int count, const ResidualArgs* tab, const int* start, int total_tiles, const c128* r,
                           hipStream_t s, const ArnState* st) {
  if (total_tiles <= 0) return;
  residual_batch_kernel<<<total_tiles, dim3(TX, TY), 0, s>>>(tab, start, count, r, st);
  HS_HIP(hipGetLastError());
}

void launch_prolong2_batch(int count, const StageArgs* tab, const int* start, int total_tiles, hipStream_t s,
                           const ArnState* st) {
  if (total_tiles <= 0) return;
  prolong2_batch_kernel<<<total_tiles, dim3(TX, TY), 0, s>>>(tab, start, count, st);
  HS_HIP(hipGetLastError());
}

void launch_combine_batch(int variant, int prec, int count, const CombineArgs* tab, const int* start,
                          int total_tiles, c128* z, hipStream_t s, const ArnState* st) {
  if (prec == HS_C64)
    combine_batch_kernel<float><<<total_tiles, dim3(TX, TY), 0, s>>>(variant, tab, start, count, z, st);
  else
    combine_batch_kernel<double><<<total_tiles, dim3(TX, TY), 0, s>>>(variant, tab, start, count, z, st);
  HS_HIP(hipGetLastError());
}

void launch_restrict2(const GridLevel& f, const GridLevel& c, const c128* in, c128* out, hipStream_t s) {
  restrict2_kernel<<<grid2(c.nu, c.nu), dim3(TX, TY), 0, s>>>(f, c, in, out);
  HS_HIP(hipGetLastError());
}

void launch_prolong2(const GridLevel& f, const GridLevel& c, const c128* in, c128* out, int accumulate,
                     hipStream_t s) {
  prolong2_kernel<<<grid2(f.nu, f.nu), dim3(TX, TY), 0, s>>>(f, c, in, out, accumulate);
  HS_HIP(hipGetLastError());
}

int galerkin_reach(int basis, int rin) {
  const int rt = (basis == HS_COARSE_P1) ? 1 : 2;
  return (2 * rt + rin) / 2;
}

void launch_galerkin_first(const ProblemDev& P, const GridLevel& c, c128* A0, hipStream_t s) {
  const GridLevel f{P.n, P.lo, P.nu, 0};
  const int64_t Nc = (int64_t)c.nu * c.nu;
  const int blocks = (int)((Nc + GAL_WG - 1) / GAL_WG);
  if (c.basis == HS_COARSE_P1)
    galerkin_kernel<1, 1, 1, true><<<blocks, GAL_WG, 0, s>>>(P, f, nullptr, c, A0);
  else
    galerkin_kernel<1, 2, 2, true><<<blocks, GAL_WG, 0, s>>>(P, f, nullptr, c, A0);
  HS_HIP(hipGetLastError());
}

void launch_galerkin_next(const GridLevel& f, int rin, const c128* Af, const GridLevel& c, c128* Ac,
                          hipStream_t s) {
  const int64_t Nc = (int64_t)c.nu * c.nu;
  const int blocks = (int)((Nc + GAL_WG - 1) / GAL_WG);
  ProblemDev dummy{};
  if (c.basis == HS_COARSE_P1 && rin == 1)
    galerkin_kernel<1, 1, 1, false><<<blocks, GAL_WG, 0, s>>>(dummy, f, Af, c, Ac);
  else if (c.basis == HS_COARSE_BEZIER && rin == 2)
    galerkin_kernel<2, 3, 2, false><<<blocks, GAL_WG, 0, s>>>(dummy, f, Af, c, Ac);
  else if (c.basis == HS_COARSE_BEZIER && rin == 3)
    galerkin_kernel<3, 3, 2, false><<<blocks, GAL_WG, 0, s>>>(dummy, f, Af, c, Ac);
  else
    throw Failure{HS_EINVAL, "unsupported coarse stencil reach"};
  HS_HIP(hipGetLastError());
}

void launch_combine(const ProblemDev& P, int variant, int prec, int nsx, const SubDesc* desc_dev,
                    const int* xmap_dev, const int* ymap_dev, const void* sol, const GridLevel* f,
                    const GridLevel* c, const c128* e0, c128* z, hipStream_t s, const c128* addv) {
  const GridLevel ff = f ? *f : GridLevel{P.n, P.lo, P.nu, 0};
  const GridLevel cc = c ? *c : GridLevel{0, 0, 0, 0};
  const int has_coarse = (e0 != nullptr);
  if (prec == HS_C64)
    combine_kernel<float><<<grid2(P.nu, P.nu), dim3(TX, TY), 0, s>>>(
        P, variant, nsx, desc_dev, xmap_dev, ymap_dev, (const c64*)sol, ff, cc, e0, z, has_coarse, addv);
  else
    combine_kernel<double><<<grid2(P.nu, P.nu), dim3(TX, TY), 0, s>>>(
        P, variant, nsx, desc_dev, xmap_dev, ymap_dev, (const c128*)sol, ff, cc, e0, z, has_coarse, addv);
  HS_HIP(hipGetLastError());
}

}  // namespace hs
