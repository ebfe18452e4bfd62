// Exact coarse solve A_0^{-1} (Sec. 3: the coarse problem R_0 A R_0^T is
// solved with a sparse direct method) by nested dissection.
//
// Factorisation, level by level from the leaves up.  Each front
// F = [[F_II, F_IB], [F_BI, F_BB]] is assembled from A_0 and the children's
// update matrices, then swept by in-place Gauss-Jordan on its I pivots with
// partial pivoting restricted to the I rows.  The sweep leaves
//   rows rho(I) x cols I : F_II^{-1} (rows and columns permuted by rho)
//   rows rho(I) x cols B : V = F_II^{-1} F_IB
//   rows B      x cols B : U = F_BB - F_BI F_II^{-1} F_IB  (to the parent)
// The sweep is blocked: a panel of NB pivots is chosen and inverted by one
// workgroup per front (K1), the rest of the front takes the rank-NB update
// F -= F[:,C] Y F[rho C,:] in 64 x 64 tiles on the FP64 matrix cores (K2),
// then the pivot rows and the
// panel columns are finalised (K3).
//
// Solve: forward sweep leaves -> root, c_I = r0[I] + children's updates,
// u_B = (children's updates on B) - V^T c_I (V^T = F_BI F_II^{-1} because
// the front is complex symmetric); backward sweep root -> leaves,
// x_I = G c_I - V x_B.
#include <algorithm>
#include <array>
#include <functional>
#include <mutex>
#include <unordered_map>

#include "hs_internal.h"
#include "hs_wave.h"

namespace hs {

constexpr int NB = 8;       // panel width
constexpr int TILE = 64;
typedef double d4 __attribute__((ext_vector_type(4)));

struct Task { int f, a, b, c; };  // solve tasks: front, chunk, instance of a batch

// per-instance pointers of a batched coarse solve
struct NDSolveArgs {
  const NDFront* fronts;
  const int *Iid, *Bid, *inv;
  const c128 *G, *V, *r0;
  c128 *cbuf, *ubuf, *e0;
};

struct NDDev {
  NDFront* fronts = nullptr;
  int* Iid = nullptr;
  int* Bid = nullptr;
  int* inv = nullptr;
  int* ppos = nullptr;
  c128* G = nullptr;
  c128* V = nullptr;
  c128* F = nullptr;
  c128* cbuf = nullptr;
  c128* ubuf = nullptr;
  int* rho = nullptr;
  int* rinv = nullptr;
  int* used = nullptr;
  c128* Y = nullptr;
  int* status = nullptr;
  // per level task lists (device) and counts
  std::vector<int*> lvl_fronts;
  std::vector<Task*> asm_t, upd_t, fix_t, ext_t;
  std::vector<void*> fwd_t, bwd_t;  // solve tasks (k_nd.hip: STask)
  std::vector<int> n_fronts, n_asm, n_upd, n_fix, n_ext, n_fwd, n_bwd, max_nI, max_nB;
  // the levels from depth sub_lv down are solved by subtree (k_nd.hip: SubTask)
  int sub_lv = 0, n_sub = 0;
  void* sub_t = nullptr;
  void* sub_f = nullptr;
  size_t sub_lds_f = 0, sub_lds_b = 0;
};

namespace {

__device__ inline int front_pos(const NDFront& f, int ncx, int gid) {
  const int x = gid % ncx, y = gid / ncx;
  for (int q = 0; q < f.nrect; ++q) {
    const Rect r = f.rect[q];
    if (x >= r.x0 && x < r.x1 && y >= r.y0 && y < r.y1) return r.base + (y - r.y0) * (r.x1 - r.x0) + (x - r.x0);
  }
  return -1;
}

// --------------------------------------------------------------- assemble
// One single-wave workgroup per front row: zero it, add the A_0 entries that
// belong to this front (pairs with at least one end in I and both ends still
// uneliminated), then extend-add the children's update rows through the
// precomputed child -> parent position map.
__global__ void __launch_bounds__(64) nd_assemble_kernel(const NDFront* __restrict__ fronts, const Task* __restrict__ tasks,
                                                         const int* __restrict__ Iid, const int* __restrict__ Bid,
                                                         const int* __restrict__ inv, const int* __restrict__ ppos,
                                                         const c128* __restrict__ A0, int ncx, int ncy, int R,
                                                         c128* __restrict__ F) {
  const int lane = threadIdx.x;
  const Task tk = tasks[blockIdx.x];
  const NDFront& f = fronts[tk.f];
  const int r = tk.a;
  const int nF = f.nF;
  c128* row = F + f.fofs + (int64_t)r * nF;
  for (int c = lane; c < nF; c += 64) row[c] = {0.0, 0.0};
  __syncthreads();
  const int W = 2 * R + 1;
  const int u = (r < f.nI) ? Iid[f.Iid + r] : Bid[f.Bid + (r - f.nI)];
  const int ux = u % ncx, uy = u / ncx;
  for (int q = lane; q < W * W; q += 64) {
    const int dy = q / W - R, dx = q % W - R;
    const int vx = ux + dx, vy = uy + dy;
    if (vx < 0 || vx >= ncx || vy < 0 || vy >= ncy) continue;
    const c128 a = A0[(int64_t)u * (W * W) + q];
    if (a.x == 0.0 && a.y == 0.0) continue;
    const int p = front_pos(f, ncx, vy * ncx + vx);
    if (p < 0) continue;
    if (r >= f.nI && p >= f.nI) continue;  // B x B pairs belong to an ancestor
    row[p] = cadd(row[p], a);
  }
  __syncthreads();
  for (int ch = 0; ch < 2; ++ch) {
    if (f.child[ch] < 0) break;
    const int b = inv[f.inv[ch] + r];
    if (b >= 0) {
      const NDFront& fc = fronts[f.child[ch]];
      const c128* urow = F + fc.fofs + (int64_t)(fc.nI + b) * fc.nF + fc.nI;
      const int* pp = ppos + fc.ppofs;
      for (int bb = lane; bb < fc.nB; bb += 64) {
        const int p = pp[bb];
        row[p] = cadd(row[p], urow[bb]);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ K1: panel
// One workgroup per front: Gauss-Jordan on the panel columns [k0, k0+nbp)
// restricted to the I rows not pivoted yet; pivot = largest modulus.
constexpr int K1_WG = 1024;

__global__ void __launch_bounds__(K1_WG) nd_panel_kernel(const NDFront* __restrict__ fronts,
                                                         const int* __restrict__ lvl, int nlvl, int k0,
                                                         c128* __restrict__ F, int* __restrict__ used_g,
                                                         int* __restrict__ rho_g, int* __restrict__ rinv_g,
                                                         c128* __restrict__ Ybuf, int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int fi = lvl[blockIdx.x];
  const NDFront& f = fronts[fi];
  const int nI = f.nI;
  if (k0 >= nI) return;
  const int nbp = min(NB, nI - k0);
  c128* Pn = (c128*)smem;                 // nI x NB
  int* cand = (int*)(Pn + (size_t)nI * NB);  // nI flags: 1 = candidate
  __shared__ double s_best[16];
  __shared__ int s_bi[16];
  __shared__ int s_piv;
  __shared__ c128 s_prow[NB];
  __shared__ int s_rho[NB];
  const int tid = threadIdx.x;
  const c128* Fr = F + f.fofs;
  int* used = used_g + f.pofs;
  for (int r = tid; r < nI; r += K1_WG) {
    cand[r] = used[r] ? 0 : 1;
    for (int c = 0; c < nbp; ++c) Pn[r * NB + c] = Fr[(int64_t)r * f.nF + k0 + c];
  }
  __syncthreads();
  for (int s = 0; s < nbp; ++s) {
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int r = tid; r < nI; r += K1_WG) {
      if (cand[r] != 1) continue;
      const double m = cabs2(Pn[r * NB + s]);
      if (m > best || (m == best && r < bi)) { best = m; bi = r; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_down(best, off, 64);
      const int oi = __shfl_down(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if ((tid & 63) == 0) { s_best[tid >> 6] = best; s_bi[tid >> 6] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = s_best[0];
      int i = s_bi[0];
      for (int w = 1; w < K1_WG / 64; ++w)
        if (s_best[w] > b || (s_best[w] == b && s_bi[w] < i)) { b = s_best[w]; i = s_bi[w]; }
      if (!(b > 0.0)) {
        atomicCAS(status, 0, fi + 1);
        if (i >= nI) {  // no finite candidate: take the first candidate row
          i = 0;
          while (i < nI - 1 && cand[i] != 1) ++i;
        }
      }
      s_piv = i;
      s_rho[s] = i;
      cand[i] = 2;  // pivoted in this panel: still updated, no longer a candidate
    }
    __syncthreads();
    const int p = s_piv;
    c128 piv = Pn[p * NB + s];
    if (!(cabs2(piv) > 0.0)) piv = {1.0, 0.0};
    const c128 ip = cinv(piv);
    if (tid < nbp) s_prow[tid] = (tid == s) ? ip : cmul(Pn[p * NB + tid], ip);
    __syncthreads();
    for (int r = tid; r < nI; r += K1_WG) {
      if (cand[r] == 0) continue;
      if (r == p) {
        for (int c = 0; c < nbp; ++c) Pn[r * NB + c] = s_prow[c];
      } else {
        const c128 fct = Pn[r * NB + s];
        for (int c = 0; c < nbp; ++c) {
          if (c == s) continue;
          c128 v = Pn[r * NB + c];
          cfms(v, fct, s_prow[c]);
          Pn[r * NB + c] = v;
        }
        Pn[r * NB + s] = {-(fct.x * ip.x - fct.y * ip.y), -(fct.x * ip.y + fct.y * ip.x)};
      }
    }
    __syncthreads();
  }
  // Y[c][c'] = panel values of pivot row rho(c)
  c128* Y = Ybuf + (int64_t)blockIdx.x * NB * NB;
  for (int q = tid; q < nbp * nbp; q += K1_WG) {
    const int c = q / nbp, cc = q - c * nbp;
    Y[c * NB + cc] = Pn[s_rho[c] * NB + cc];
  }
  if (tid < nbp) {
    used[s_rho[tid]] = 1;
    rho_g[f.pofs + k0 + tid] = s_rho[tid];
    rinv_g[f.pofs + s_rho[tid]] = k0 + tid;
  }
}

// ------------------------------------------------------- K2: rank-NB update
// F[i][j] -= F[i][C] (Y F[rhoC][j]) for rows i not in rhoC, columns j not in C.
__global__ void __launch_bounds__(256) nd_update_kernel(const NDFront* __restrict__ fronts,
                                                        const Task* __restrict__ tasks, int k0,
                                                        const int* __restrict__ rho_g,
                                                        const c128* __restrict__ Ybuf,
                                                        c128* __restrict__ F) {
  const Task tk = tasks[blockIdx.x];
  const NDFront& f = fronts[tk.f];
  if (k0 >= f.nI) return;
  const int nbp = min(NB, f.nI - k0);
  const int nF = f.nF;
  const int i0 = tk.a * TILE, j0 = tk.b * TILE;
  __shared__ c128 A[TILE][NB];
  __shared__ c128 YZ[NB][TILE];
  __shared__ c128 Z[NB][TILE];
  __shared__ c128 Ys[NB][NB];
  __shared__ int prows[NB];
  const int tid = threadIdx.x;
  const c128* Y = Ybuf + (int64_t)tk.c * NB * NB;
  c128* Fr = F + f.fofs;
  if (tid < nbp) prows[tid] = rho_g[f.pofs + k0 + tid];
  if (tid < nbp * nbp) Ys[tid / nbp][tid % nbp] = Y[(tid / nbp) * NB + tid % nbp];
  __syncthreads();
  for (int q = tid; q < NB * TILE; q += 256) {
    const int c = q / TILE, jj = q % TILE;
    const int j = j0 + jj;
    Z[c][jj] = (c < nbp && j < nF) ? Fr[(int64_t)prows[c] * nF + j] : c128{0.0, 0.0};
    const int ii = q / NB, cc = q % NB;
    const int i = i0 + ii;
    A[ii][cc] = (cc < nbp && i < nF) ? Fr[(int64_t)i * nF + k0 + cc] : c128{0.0, 0.0};
  }
  __syncthreads();
  for (int q = tid; q < NB * TILE; q += 256) {
    const int c = q / TILE, jj = q % TILE;
    c128 acc = {0.0, 0.0};
    if (c < nbp)  // rows past a short last panel stay zero (they meet zero columns of A)
      for (int cc = 0; cc < nbp; ++cc) cfma(acc, Ys[c][cc], Z[cc][jj]);
    YZ[c][jj] = acc;
  }
  __syncthreads();
  // P = A YZ on the FP64 matrix cores: v_mfma_f64_16x16x4f64 takes A[l%16][k]
  // and B[k][l%16] from lane l (k = l/16) and leaves D[l/16 + 4r][l%16] in
  // register r.  A complex product is four real ones; NB = 8 is two k-steps.
  // Wave w takes rows 16w .. 16w+15 of the tile, all four 16-column blocks.
  static_assert(NB == 8 && TILE == 64, "two k-steps of 4, four 16 x 16 blocks per wave");
  const int lane = tid & 63, w = tid >> 6;
  d4 cre[4], cim[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) cre[cb] = cim[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < NB / 4; ++ks) {
    const c128 av = A[16 * w + (lane & 15)][4 * ks + (lane >> 4)];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const c128 bv = YZ[4 * ks + (lane >> 4)][16 * cb + (lane & 15)];
      cre[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, cre[cb], 0, 0, 0);
      cre[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bv.y, cre[cb], 0, 0, 0);
      cim[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y, cim[cb], 0, 0, 0);
      cim[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x, cim[cb], 0, 0, 0);
    }
  }
  // F -= P outside the pivot rows and the panel's columns.  The 16 entries of
  // a lane are loaded together (entries that stay, or lie outside the front,
  // load F[0] instead), then the ones to update are stored.
  int64_t at[4][4];
  c128 v[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 16 * w + (lane >> 4) + 4 * r;
    bool row_ok = i < nF;
    for (int c = 0; c < nbp; ++c) row_ok &= (prows[c] != i);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int j = j0 + 16 * cb + (lane & 15);
      const bool ok = row_ok && j < nF && !(j >= k0 && j < k0 + nbp);
      at[r][cb] = ok ? (int64_t)i * nF + j : -1;
      v[r][cb] = Fr[ok ? at[r][cb] : 0];
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
      if (at[r][cb] >= 0) Fr[at[r][cb]] = {v[r][cb].x - cre[cb][r], v[r][cb].y - cim[cb][r]};
}

// ----------------------------------------------------------- K3: finalise
// kind 0 (column chunk): pivot rows  F[rhoC][j] = Y F[rhoC][j] (j not in C),
//                                     F[rhoC][C] = Y
// kind 1 (row chunk):    other rows  F[i][C]    = -F[i][C] Y
__global__ void __launch_bounds__(256) nd_fix_kernel(const NDFront* __restrict__ fronts, const Task* __restrict__ tasks,
                                                     int k0, const int* __restrict__ rho_g,
                                                     const c128* __restrict__ Ybuf, c128* __restrict__ F) {
  const Task tk = tasks[blockIdx.x];
  const NDFront& f = fronts[tk.f];
  if (k0 >= f.nI) return;
  const int nbp = min(NB, f.nI - k0);
  const int nF = f.nF;
  __shared__ c128 Ys[NB][NB];
  __shared__ c128 T[NB][TILE];
  __shared__ int prows[NB];
  const int tid = threadIdx.x;
  const c128* Y = Ybuf + (int64_t)tk.c * NB * NB;
  c128* Fr = F + f.fofs;
  if (tid < nbp) prows[tid] = rho_g[f.pofs + k0 + tid];
  if (tid < nbp * nbp) Ys[tid / nbp][tid % nbp] = Y[(tid / nbp) * NB + tid % nbp];
  __syncthreads();
  if (tk.b == 0) {
    const int j0 = tk.a * TILE;
    for (int q = tid; q < NB * TILE; q += 256) {
      const int c = q / TILE, jj = q % TILE, j = j0 + jj;
      T[c][jj] = (c < nbp && j < nF) ? Fr[(int64_t)prows[c] * nF + j] : c128{0.0, 0.0};
    }
    __syncthreads();
    for (int q = tid; q < NB * TILE; q += 256) {
      const int c = q / TILE, jj = q % TILE, j = j0 + jj;
      if (c >= nbp || j >= nF) continue;
      c128 v;
      if (j >= k0 && j < k0 + nbp) {
        v = Ys[c][j - k0];
      } else {
        v = {0.0, 0.0};
        for (int cc = 0; cc < nbp; ++cc) cfma(v, Ys[c][cc], T[cc][jj]);
      }
      Fr[(int64_t)prows[c] * nF + j] = v;
    }
  } else {
    const int i0 = tk.a * TILE;
    // rows i0..i0+63, one thread per (row, panel column)
    for (int q = tid; q < TILE * NB; q += 256) {
      const int ii = q / NB, c = q % NB, i = i0 + ii;
      if (c >= nbp || i >= nF) continue;
      bool piv = false;
      for (int cc = 0; cc < nbp; ++cc) piv |= (prows[cc] == i);
      if (piv) continue;
      c128 acc = {0.0, 0.0};
      for (int cc = 0; cc < nbp; ++cc) cfma(acc, Fr[(int64_t)i * nF + k0 + cc], Ys[cc][c]);
      // every read of the panel entries precedes every write (staged in LDS)
      T[c][ii] = {-acc.x, -acc.y};
    }
    __syncthreads();
    for (int q = tid; q < TILE * NB; q += 256) {
      const int ii = q / NB, c = q % NB, i = i0 + ii;
      if (c >= nbp || i >= nF) continue;
      bool piv = false;
      for (int cc = 0; cc < nbp; ++cc) piv |= (prows[cc] == i);
      if (piv) continue;
      Fr[(int64_t)i * nF + k0 + c] = T[c][ii];
    }
  }
}

// ---------------------------------------------------------- extract G, V
__global__ void __launch_bounds__(256) nd_extract_kernel(const NDFront* __restrict__ fronts,
                                                         const Task* __restrict__ tasks,
                                                         const int* __restrict__ rho_g,
                                                         const int* __restrict__ rinv_g,
                                                         const c128* __restrict__ F, c128* __restrict__ G,
                                                         c128* __restrict__ V) {
  const Task tk = tasks[blockIdx.x];
  const NDFront& f = fronts[tk.f];
  const int k = tk.a;
  const int nI = f.nI, nB = f.nB, nF = f.nF;
  const c128* src = F + f.fofs + (int64_t)rho_g[f.pofs + k] * nF;
  // row k of G: all of it, or, for a front that keeps one triangle, the part
  // left of the diagonal of the symmetric part (G + G^T) / 2.  The computed
  // inverse is symmetric only up to rounding; its symmetric part is at least
  // as close to the exact inverse (in the Frobenius norm), whereas copying
  // one triangle of it over the other can raise the residual of a solve
  // through a near-singular front by orders of magnitude.
  c128* g = G + f.gofs + nd_g_index(nI, f.ldg, k, 0);
  if (nd_tri(nI)) {
    const int ck = rinv_g[f.pofs + k];  // column of G[:, k] in the factored front
    for (int c = threadIdx.x; c <= k; c += 256) {
      const c128 a = src[rinv_g[f.pofs + c]];
      const c128 b = F[f.fofs + (int64_t)rho_g[f.pofs + c] * nF + ck];
      g[c] = c128{0.5 * (a.x + b.x), 0.5 * (a.y + b.y)};
    }
  } else {
    for (int c = threadIdx.x; c < nI; c += 256) g[c] = src[rinv_g[f.pofs + c]];
  }
  c128* v = V + f.vofs + (int64_t)k * f.ldv;
  for (int b = threadIdx.x; b < nB; b += 256) v[b] = src[nI + b];
}

// --------------------------------------------------------------- solve
constexpr int SOLVE_MAX = 2048;
constexpr int BWD_ROWS = 8;    // 4 waves x 2 interleaved rows
constexpr int FWD_UNR = 8;     // rows of V per thread per round (loads in flight)

// Forward task shape, fixed by |I| alone (so a front is summed in the same
// order by whichever launch serves it): RG row groups x 256/RG columns of
// u_B, about eight rows of V per thread.  Small fronts take one wide chunk
// of B in a single round of loads; large ones narrow chunks of many rows,
// down to 8 columns (one 128-byte line of a row of V) for the few fronts of
// more than 256 unknowns, whose levels then spread over twice the workgroups.
__host__ __device__ inline int fwd_groups(int nI) {
  return nI <= 16 ? 2 : (nI <= 32 ? 4 : (nI <= 64 ? 8 : (nI <= 256 ? 16 : 32)));
}
__host__ __device__ inline int fwd_cols(int nI) { return 256 / fwd_groups(nI); }

// the backward sums of a wave (rows ka and kb of NR right-hand sides) into
// e0: value 4q + c is (a0.x, a0.y, a1.x, a1.y)[c] of right-hand side q
template <int NR, typename E0>
__device__ inline void store_bwd_rows(const c128 (&a0)[NR], const c128 (&a1)[NR], int nr, bool hb, int ka, int kb,
                                      const int* __restrict__ Iid, int64_t iofs, int lane, E0 e0_of) {
  double v[4 * NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    v[4 * q + 0] = a0[q].x;
    v[4 * q + 1] = a0[q].y;
    v[4 * q + 2] = a1[q].x;
    v[4 * q + 3] = a1[q].y;
  }
  const double sum = wave::sum<4 * NR>(v, lane);
  constexpr int G = 64 / (4 * NR);  // lanes holding each value
  if (lane % G == 0) {
    const int j = lane / G, q = j >> 2, c = j & 3;
    if (q < nr && (c < 2 || hb))
      reinterpret_cast<double*>(e0_of(q))[2 * (int64_t)Iid[iofs + (c < 2 ? ka : kb)] + (c & 1)] = sum;
  }
}

// A task serves a group of up to NR right-hand sides on one factor (several
// right-hand sides of one problem; a single solve or a lone instance is a
// group of one): every entry of V and G is loaded once and applied to all of
// them, each right-hand side's arithmetic in the same order, so a batched
// instance's result equals its single solve bit for bit.
constexpr int ND_NR = 4;
struct NDGroup {
  int n;
  int inst[ND_NR];
};

// The fields of a front that its solve tasks read, copied into every task,
// so that a task's first scalar loads bring all of them: no further round
// trip for the front's record, nor for its children's.
struct SolveFront {
  int nI, nB, ldg, ldv;
  int64_t Iid, Bid, inv[2], gofs, vofs, cofs, uofs;
  int64_t cu[2];  // the children's u_B offsets in ubuf; -1: no such child
};
// solve task: front f, c consecutive chunks from chunk a, instance group g
struct STask {
  SolveFront f;
  int a, c, g, pad;
};

// c_I of every right-hand side of the group into LDS (rhs q at cIs + q *
// stride): r0 on I plus the children's updates, gathered for all of them at
// once so the loads of the group are in flight together; optionally kept in
// cbuf for the backward sweep.
template <int NR>
__device__ inline void stage_cI(const SolveFront& f, const NDSolveArgs& A0,
                                const NDSolveArgs* __restrict__ tab, const NDGroup& g, c128* cIs, int stride,
                                bool keep) {
  const int nI = f.nI, nr = g.n;
  const c128 *r0[NR], *ub[NR];
  c128* cb[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const NDSolveArgs& A = tab[g.inst[q < nr ? q : 0]];  // spare slots read the first instance
    r0[q] = A.r0;
    ub[q] = A.ubuf;
    cb[q] = A.cbuf + f.cofs;
  }
#pragma unroll 4
  for (int r = threadIdx.x; r < nI; r += 256) {
    const int id = A0.Iid[f.Iid + r];
    c128 acc[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = r0[q][id];
    for (int ch = 0; ch < 2; ++ch) {
      if (f.cu[ch] < 0) break;
      const int b = A0.inv[f.inv[ch] + r];
      if (b >= 0) {
        const int64_t o = f.cu[ch] + b;
        c128 u[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) u[q] = ub[q][o];
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] = cadd(acc[q], u[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (q < nr) {
        cIs[q * stride + r] = acc[q];
        if (keep) cb[q][r] = acc[q];
      }
  }
}

// Forward, one level: task = (front, tk.c consecutive chunks of C = 256/RG
// columns of B, from chunk tk.a).
//   u_B = (children's updates on B) - V^T c_I
// Thread (row group g, column c) sums rows g, g + RG, ... of its column of V
// (a row of a chunk is one contiguous C-wide read); the RG partial sums of a
// column meet in LDS in order.  The first round of V is loaded before c_I is
// staged (it does not depend on it), so the factor loads and the staging
// gathers are in flight together.
template <int NR, int RG>
__device__ inline void fwd_front_rg(const STask& tk, const NDSolveArgs* __restrict__ tab, const NDGroup& g, int max_nI,
                                    c128* __restrict__ part) {
  constexpr int C = 256 / RG;
  const NDSolveArgs& A0 = tab[g.inst[0]];  // index maps and V are shared by the group
  const SolveFront& f = tk.f;
  extern __shared__ __align__(16) unsigned char smem[];
  c128* cIs = (c128*)smem;  // NR x |I| of the level's largest front
  const int tid = threadIdx.x, col = tid % C, grp = tid / C;
  const int nI = f.nI, nB = f.nB, nr = g.n;
  const int nch = tk.c > 0 ? tk.c : 1;
  const c128* __restrict__ Vf = A0.V + f.vofs;
  c128 v[FWD_UNR];
  auto load_round = [&](int b, int m0) {
    const bool okb = b < nB;
#pragma unroll
    for (int u = 0; u < FWD_UNR; ++u) {
      const int k = grp + RG * (m0 + u);
      v[u] = (okb && k < nI) ? Vf[(int64_t)k * f.ldv + b] : c128{0.0, 0.0};
    }
  };
  // the children's updates on B for output e = (rhs, column) of chunk cc:
  // gathers independent of V and c_I, issued with them
  auto child_b = [&](int e, int cc) -> c128 {
    const int q = NR == 1 ? 0 : e / C, c = NR == 1 ? e : e % C;  // (NR == 1: a static index)
    const int bq = (tk.a + cc) * C + c;
    c128 sb = {0.0, 0.0};
    if (bq < nB) {
      const NDSolveArgs& A = tab[g.inst[q]];
      for (int ch = 0; ch < 2; ++ch) {
        if (f.cu[ch] < 0) break;
        const int bc = A0.inv[f.inv[ch] + nI + bq];
        if (bc >= 0) sb = cadd(sb, A.ubuf[f.cu[ch] + bc]);
      }
    }
    return sb;
  };
  load_round(tk.a * C + col, 0);
  c128 s_pre = (tid < nr * C) ? child_b(tid, 0) : c128{0.0, 0.0};
  stage_cI<NR>(f, A0, tab, g, cIs, max_nI, tk.a == 0);
  __syncthreads();
  if (nB == 0) return;
  for (int cc = 0; cc < nch; ++cc) {
    const int b = (tk.a + cc) * C + col;
    if (cc > 0) {
      load_round(b, 0);
      if (tid < nr * C) s_pre = child_b(tid, cc);
    }
    c128 acc[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = {0.0, 0.0};
    for (int m0 = 0;; m0 += FWD_UNR) {
#pragma unroll
      for (int u = 0; u < FWD_UNR; ++u) {
        const int k = grp + RG * (m0 + u);
        if (k < nI) {
#pragma unroll
          for (int q = 0; q < NR; ++q)
            if (q < nr) cfma(acc[q], v[u], cIs[q * max_nI + k]);
        }
      }
      if (grp + RG * (m0 + FWD_UNR) >= nI) break;
      load_round(b, m0 + FWD_UNR);
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) part[(q * RG + grp) * C + col] = acc[q];
    __syncthreads();
    // nr * C outputs (up to 4 x 128): the workgroup's 256 threads loop over them
    for (int e = tid; e < nr * C; e += 256) {
      const int q = NR == 1 ? 0 : e / C, c = NR == 1 ? e : e % C;  // (NR == 1: a static index)
      const int bq = (tk.a + cc) * C + c;
      if (bq < nB) {
        const NDSolveArgs& A = tab[g.inst[q]];
        const c128 s = e == tid ? s_pre : child_b(e, cc);
        c128 t = part[(q * RG) * C + c];
        for (int gg = 1; gg < RG; ++gg) t = cadd(t, part[(q * RG + gg) * C + c]);
        A.ubuf[f.uofs + bq] = csub(s, t);
      }
    }
    __syncthreads();  // part is rewritten by the next chunk
  }
}

template <int NR>
__device__ inline void fwd_front(const STask& tk, const NDSolveArgs* __restrict__ tab, const NDGroup& g, int max_nI) {
  __shared__ c128 part[NR * 256];
  switch (fwd_groups(tk.f.nI)) {  // workgroup-uniform
    case 2: fwd_front_rg<NR, 2>(tk, tab, g, max_nI, part); break;
    case 4: fwd_front_rg<NR, 4>(tk, tab, g, max_nI, part); break;
    case 8: fwd_front_rg<NR, 8>(tk, tab, g, max_nI, part); break;
    case 16: fwd_front_rg<NR, 16>(tk, tab, g, max_nI, part); break;
    default: fwd_front_rg<NR, 32>(tk, tab, g, max_nI, part);
  }
}

// Backward, one level: task = (front, tk.c consecutive chunks of BWD_ROWS
// rows of I, from chunk tk.a).  c_I and x_B are staged in LDS once per task;
// each wave forms two rows x_k = G[k,:] c_I - V[k,:] x_B at once (lanes over
// columns, coalesced, four columns per lane per round: eight loads in
// flight), then sums them over the wave (DPP and permlane swaps, one tree for
// any number of right-hand sides).  The first round of G is loaded before
// the staging.  The root (no B) stages its c_I itself from r0 and its
// children's updates: the forward sweep has nothing else to do there and
// skips it.
// Small fronts (|I| <= 64, |B| <= 64 NV: the leaves and the levels above
// them): a row is one round of loads (G[k, lane] and NV segments of 64
// entries of V[k, :]), so each wave takes the rows of two chunks at once and
// issues the loads of four rows together, then sums them in two wave
// reductions.
template <int NR, int NV>
__device__ inline void bwd_small(const STask& tk, const NDSolveArgs* __restrict__ tab, const NDGroup& g,
                                 const SolveFront& f, const c128* base, int stride, int max_nI, int nch) {
  const NDSolveArgs& A0 = tab[g.inst[0]];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nI = f.nI, nB = f.nB, nr = g.n;
  const c128* __restrict__ Gf = A0.G + f.gofs;
  const c128* __restrict__ Vf = A0.V + f.vofs;
  for (int cc = 0; cc < nch; cc += 2) {
    int kr[4];
    bool h[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      kr[i] = (tk.a + cc + (i >> 1)) * BWD_ROWS + 2 * wv + (i & 1);
      h[i] = kr[i] < nI && (i < 2 || cc + 1 < nch);
    }
    if (!h[0]) break;  // wave-uniform; no barrier follows
    c128 gv[4], vv[4][NV];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = h[i] ? kr[i] : kr[0];
      gv[i] = lane < nI ? Gf[nd_g_index(nI, f.ldg, r, lane)] : c128{0.0, 0.0};
#pragma unroll
      for (int p = 0; p < NV; ++p)
        vv[i][p] = lane + 64 * p < nB ? Vf[(int64_t)r * f.ldv + lane + 64 * p] : c128{0.0, 0.0};
    }
    c128 a[4][NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const c128* cI = base + q * stride;
      const c128* xB = cI + max_nI;
      const c128 x = (q < nr && lane < nI) ? cI[lane] : c128{0.0, 0.0};
      c128 y[NV];
#pragma unroll
      for (int p = 0; p < NV; ++p) y[p] = (q < nr && lane + 64 * p < nB) ? xB[lane + 64 * p] : c128{0.0, 0.0};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i][q] = {0.0, 0.0};
        cfma(a[i][q], gv[i], x);
#pragma unroll
        for (int p = 0; p < NV; ++p) cfms(a[i][q], vv[i][p], y[p]);
      }
    }
    store_bwd_rows<NR>(a[0], a[1], nr, h[1], kr[0], kr[1], A0.Iid, f.Iid, lane,
                       [&](int q) { return tab[g.inst[NR == 1 ? 0 : q]].e0; });
    if (h[2])
      store_bwd_rows<NR>(a[2], a[3], nr, h[3], kr[2], kr[3], A0.Iid, f.Iid, lane,
                         [&](int q) { return tab[g.inst[NR == 1 ? 0 : q]].e0; });
  }
}

template <int NR>
__device__ inline void bwd_front(const STask& tk, const NDSolveArgs* __restrict__ tab, const NDGroup& g, int max_nI,
                                 int max_nB) {
  const NDSolveArgs& A0 = tab[g.inst[0]];
  const SolveFront& f = tk.f;
  extern __shared__ __align__(16) unsigned char smem[];
  c128* base = (c128*)smem;  // per right-hand side: c_I (max_nI), then x_B (max_nB)
  const int stride = max_nI + max_nB;
  const int tid = threadIdx.x;
  const int nI = f.nI, nB = f.nB, nr = g.n;
  const int lane = tid & 63, wv = tid >> 6;
  const int nch = tk.c > 0 ? tk.c : 1;
  const bool small = nI <= 64 && nB <= 256;  // workgroup-uniform
  // first round of G for the first chunk (wave-uniform rows)
  c128 u0[4], w0[4];
  const c128* __restrict__ Gf = A0.G + f.gofs;
  if (!small) {
    const int ka = tk.a * BWD_ROWS + 2 * wv, kb = ka + 1;
    const bool ha = ka < nI, hb = kb < nI;
    const int ra = ha ? ka : 0, rb = hb ? kb : ra;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int c = lane + 64 * p;
      const bool ok = ha && c < nI;
      u0[p] = ok ? Gf[nd_g_index(nI, f.ldg, ra, c)] : c128{0.0, 0.0};
      w0[p] = ok ? Gf[nd_g_index(nI, f.ldg, rb, c)] : c128{0.0, 0.0};
    }
  }
  if (nB == 0) {
    stage_cI<NR>(f, A0, tab, g, base, stride, false);
  } else {
    const c128* cb[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) cb[q] = tab[g.inst[q < nr ? q : 0]].cbuf + f.cofs;
#pragma unroll 4
    for (int r = tid; r < nI; r += 256) {
      c128 v[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) v[q] = cb[q][r];
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nr) base[q * stride + r] = v[q];
    }
  }
  {
    const c128* xe[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) xe[q] = tab[g.inst[q < nr ? q : 0]].e0;
#pragma unroll 4
    for (int b = tid; b < nB; b += 256) {
      const int id = A0.Bid[f.Bid + b];
      c128 v[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) v[q] = xe[q][id];
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nr) base[q * stride + max_nI + b] = v[q];
    }
  }
  __syncthreads();
  if (small) {
    if (nB <= 128)
      bwd_small<NR, 2>(tk, tab, g, f, base, stride, max_nI, nch);
    else
      bwd_small<NR, 4>(tk, tab, g, f, base, stride, max_nI, nch);
    return;
  }
  for (int cc = 0; cc < nch; ++cc) {
    const int ka = (tk.a + cc) * BWD_ROWS + 2 * wv, kb = ka + 1;
    if (ka >= nI) break;  // wave-uniform; no barrier follows
    const bool hb = kb < nI;
    c128 a0[NR], a1[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) a0[q] = a1[q] = {0.0, 0.0};
    const int rb = hb ? kb : ka;
    for (int c0 = lane; c0 < nI; c0 += 256) {
      c128 u[4], w[4];
      if (cc == 0 && c0 == lane) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          u[p] = u0[p];
          w[p] = w0[p];
        }
      } else {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int c = c0 + 64 * p;
          const bool ok = c < nI;
          u[p] = ok ? Gf[nd_g_index(nI, f.ldg, ka, c)] : c128{0.0, 0.0};
          w[p] = ok ? Gf[nd_g_index(nI, f.ldg, rb, c)] : c128{0.0, 0.0};
        }
      }
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        if (q >= nr) break;
        const c128* cI = base + q * stride;
        c128 x[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int c = c0 + 64 * p;
          x[p] = c < nI ? cI[c] : c128{0.0, 0.0};
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          cfma(a0[q], u[p], x[p]);
          cfma(a1[q], w[p], x[p]);
        }
      }
    }
    const c128* va = A0.V + f.vofs + (int64_t)ka * f.ldv;
    const c128* vb = A0.V + f.vofs + (int64_t)(hb ? kb : ka) * f.ldv;
    for (int c0 = lane; c0 < nB; c0 += 256) {
      c128 u[4], w[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int c = c0 + 64 * p;
        const bool ok = c < nB;
        u[p] = ok ? va[c] : c128{0.0, 0.0};
        w[p] = ok ? vb[c] : c128{0.0, 0.0};
      }
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        if (q >= nr) break;
        const c128* xB = base + q * stride + max_nI;
        c128 x[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int c = c0 + 64 * p;
          x[p] = c < nB ? xB[c] : c128{0.0, 0.0};
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          cfms(a0[q], u[p], x[p]);
          cfms(a1[q], w[p], x[p]);
        }
      }
    }
    store_bwd_rows<NR>(a0, a1, nr, hb, ka, kb, A0.Iid, f.Iid, lane,
                       [&](int q) { return tab[g.inst[NR == 1 ? 0 : q]].e0; });
  }
}

// single solves: a group of one right-hand side
__global__ void __launch_bounds__(256) nd_fwd_kernel(const STask* __restrict__ tasks, const int* __restrict__ Iid,
                                                     const int* __restrict__ inv, const c128* __restrict__ V,
                                                     const c128* __restrict__ r0, c128* __restrict__ cbuf,
                                                     c128* __restrict__ ubuf, int max_nI) {
  const NDSolveArgs A{nullptr, Iid, nullptr, inv, nullptr, V, r0, cbuf, ubuf, nullptr};
  const NDGroup g{1, {0, 0, 0, 0}};
  fwd_front<1>(tasks[blockIdx.x], &A, g, max_nI);
}

__global__ void __launch_bounds__(256) nd_bwd_kernel(const STask* __restrict__ tasks, const int* __restrict__ Iid,
                                                     const int* __restrict__ Bid, const int* __restrict__ inv,
                                                     const c128* __restrict__ G, const c128* __restrict__ V,
                                                     const c128* __restrict__ r0, const c128* __restrict__ ubuf,
                                                     const c128* __restrict__ cbuf, c128* __restrict__ e0, int max_nI,
                                                     int max_nB) {
  const NDSolveArgs A{nullptr, Iid, Bid, inv, G, V, r0, const_cast<c128*>(cbuf), const_cast<c128*>(ubuf), e0};
  const NDGroup g{1, {0, 0, 0, 0}};
  bwd_front<1>(tasks[blockIdx.x], &A, g, max_nI, max_nB);
}

// a group is skipped when every instance of it is idle
__device__ inline bool group_idle(const ArnState* st, const NDGroup& g) {
  if (!st) return false;
  for (int q = 0; q < g.n; ++q)
    if (!inst_idle(st, g.inst[q])) return false;
  return true;
}

template <int NR>
__global__ void __launch_bounds__(256) nd_fwd_batch_kernel(const STask* __restrict__ tasks,
                                                           const NDSolveArgs* __restrict__ tab,
                                                           const NDGroup* __restrict__ groups, int max_nI,
                                                           const ArnState* __restrict__ st) {
  const STask& tk = tasks[blockIdx.x];
  const NDGroup& g = groups[tk.g];  // read in place (a private copy would be indexed dynamically)
  if (group_idle(st, g)) return;
  fwd_front<NR>(tk, tab, g, max_nI);
}

template <int NR>
__global__ void __launch_bounds__(256) nd_bwd_batch_kernel(const STask* __restrict__ tasks,
                                                           const NDSolveArgs* __restrict__ tab,
                                                           const NDGroup* __restrict__ groups, int max_nI,
                                                           int max_nB, const ArnState* __restrict__ st) {
  const STask& tk = tasks[blockIdx.x];
  const NDGroup& g = groups[tk.g];  // read in place (a private copy would be indexed dynamically)
  if (group_idle(st, g)) return;
  bwd_front<NR>(tk, tab, g, max_nI, max_nB);
}

// -------------------------------------------------------------- subtrees
// From a depth Ls down, the tree is solved by subtree: one workgroup takes a
// front at depth Ls together with all its descendants, level by level with
// workgroup barriers in between.  The children's updates u_B stay in LDS;
// only c_I (kept for the backward sweep), the subtree root's u_B and x reach
// memory.  One launch per direction replaces the levels it covers, and the
// fronts of a level of a subtree are served together, so their loads are in
// flight at once.  Each front gets the level kernels' arithmetic (the same
// sums in the same order), so its results do not depend on which launch
// solved it.
// Workgroups of 512 threads, or of 1024 where a launch has at most one
// subtree per CU (kSubWide).
constexpr int kSubLevels = 5;               // depths in a subtree at most
constexpr int kSubNI = 64, kSubNB = 320;    // front limits: one round of G and V loads per backward row
constexpr int kSubNV = kSubNB / 64;         // segments of 64 entries of a row of V
constexpr size_t kSubLdsMax = 80 * 1024;    // two 512-thread subtree workgroups per CU
constexpr int kSubWide = 256;               // launches of at most this many subtrees take 1024 threads each

struct SubFront {
  int nI, nB, ldg, ldv;
  int c, u;          // LDS offsets (entries per right-hand side) of c_I and, below the subtree root, u_B
  int uch[2];        // LDS offsets of the children's u_B (-1: no such child)
  int pI, pB, pP, pS;  // prefix sums over the fronts before it at its depth: |I|, |B|, row pairs, |I| + |B|
  int64_t Iid, Bid, inv[2], gofs, vofs, cofs, uofs;
};
struct SubTask {
  int first, nlev, grp, ctot, utot, stot;
  int quad;  // bit d: every front at subtree depth d has |B| <= 128 (two row pairs per wave backward)
  int lev[kSubLevels + 1];  // fronts at subtree depth d (0: its root): records first + lev[d] .. first + lev[d + 1]
  int sI[kSubLevels], sB[kSubLevels], sP[kSubLevels], sS[kSubLevels];  // per depth: sums of |I|, |B|, pairs, |I|+|B|
};

__host__ __device__ inline size_t sub_rec_bytes(int nsf) { return ((size_t)nsf * sizeof(SubFront) + 15) & ~(size_t)15; }

// the front of a depth's list that item e falls in (K: which prefix sum)
template <int K>
__device__ inline int sub_find(const SubFront* lf, int nf, int e) {
  int k = 0;
  while (k + 1 < nf) {
    const SubFront& s = lf[k + 1];
    const int p = K == 0 ? s.pI : (K == 1 ? s.pB : (K == 2 ? s.pP : s.pS));
    if (p > e) break;
    ++k;
  }
  return k;
}

// the task's front records into LDS
template <int WG>
__device__ inline SubFront* sub_records(const SubTask& t, const SubFront* __restrict__ gsf, unsigned char* smem) {
  SubFront* sf = reinterpret_cast<SubFront*>(smem);
  const int words = t.lev[t.nlev] * (int)(sizeof(SubFront) / 4);
  const int* src = reinterpret_cast<const int*>(gsf + t.first);
  for (int i = threadIdx.x; i < words; i += WG) reinterpret_cast<int*>(sf)[i] = src[i];
  return sf;
}

// V^T c_I for column j of front s: the level kernel's RG partial sums (rows
// g, g + RG, ... in order), then added in order of g
template <int NR, int RG>
__device__ inline void sub_col(const SubFront& s, int j, const c128* __restrict__ V, const c128* cl, int ctot, int nr,
                               c128 (&tv)[NR]) {
  constexpr int U = 8;  // rows in flight
  c128 part[RG][NR];
#pragma unroll
  for (int gg = 0; gg < RG; ++gg)
#pragma unroll
    for (int q = 0; q < NR; ++q) part[gg][q] = {0.0, 0.0};
  const c128* __restrict__ v = V + s.vofs + j;
  for (int k0 = 0; k0 < s.nI; k0 += U) {
    c128 vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) vv[u] = k0 + u < s.nI ? v[(int64_t)(k0 + u) * s.ldv] : c128{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u < s.nI) {
#pragma unroll
        for (int q = 0; q < NR; ++q)
          if (q < nr) cfma(part[u % RG][q], vv[u], cl[q * ctot + s.c + k0 + u]);
      }
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    tv[q] = part[0][q];
#pragma unroll
    for (int gg = 1; gg < RG; ++gg) tv[q] = cadd(tv[q], part[gg][q]);
  }
}

// Forward sweep of one subtree, deepest level first:
//   c_I = r0[I] + children's updates (from LDS), kept in cbuf;
//   u_B = (children's updates on B) - V^T c_I, into LDS (the subtree root's
//   into ubuf, for the level above).
template <int WG, int NR>
__device__ inline void sub_fwd(const SubTask& t, const SubFront* __restrict__ gsf, const NDSolveArgs* __restrict__ tab,
                               const NDGroup& g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const SubFront* sf = sub_records<WG>(t, gsf, smem);
  c128* cl = reinterpret_cast<c128*>(smem + sub_rec_bytes(t.lev[t.nlev]));
  c128* ul = cl + NR * t.ctot;
  const NDSolveArgs& A0 = tab[g.inst[0]];  // index maps and V are shared by the group
  const int nr = g.n, tid = threadIdx.x;
  const c128* r0[NR];
  c128 *cb[NR], *ub[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const NDSolveArgs& A = tab[g.inst[q < nr ? q : 0]];
    r0[q] = A.r0;
    cb[q] = A.cbuf;
    ub[q] = A.ubuf;
  }
  __syncthreads();
  for (int d = t.nlev - 1; d >= 0; --d) {
    const SubFront* lf = sf + t.lev[d];
    const int nf = t.lev[d + 1] - t.lev[d];
    for (int e = tid; e < t.sI[d]; e += WG) {
      const SubFront& s = lf[sub_find<0>(lf, nf, e)];
      const int r = e - s.pI;
      const int id = A0.Iid[s.Iid + r];
      c128 acc[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[q] = r0[q][id];
      for (int ch = 0; ch < 2; ++ch) {
        if (s.uch[ch] < 0) break;
        const int b = A0.inv[s.inv[ch] + r];
        if (b >= 0) {
#pragma unroll
          for (int q = 0; q < NR; ++q) acc[q] = cadd(acc[q], ul[q * t.utot + s.uch[ch] + b]);
        }
      }
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nr) {
          cl[q * t.ctot + s.c + r] = acc[q];
          cb[q][s.cofs + r] = acc[q];
        }
    }
    __syncthreads();
    for (int e = tid; e < t.sB[d]; e += WG) {
      const SubFront& s = lf[sub_find<1>(lf, nf, e)];
      const int j = e - s.pB;
      c128 sb[NR], tv[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) sb[q] = {0.0, 0.0};
      for (int ch = 0; ch < 2; ++ch) {
        if (s.uch[ch] < 0) break;
        const int bc = A0.inv[s.inv[ch] + s.nI + j];
        if (bc >= 0) {
#pragma unroll
          for (int q = 0; q < NR; ++q) sb[q] = cadd(sb[q], ul[q * t.utot + s.uch[ch] + bc]);
        }
      }
      switch (fwd_groups(s.nI)) {  // |I| <= 64: 2, 4 or 8 row groups
        case 2: sub_col<NR, 2>(s, j, A0.V, cl, t.ctot, nr, tv); break;
        case 4: sub_col<NR, 4>(s, j, A0.V, cl, t.ctot, nr, tv); break;
        default: sub_col<NR, 8>(s, j, A0.V, cl, t.ctot, nr, tv);
      }
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nr) {
          const c128 u = csub(sb[q], tv[q]);
          if (s.u >= 0)
            ul[q * t.utot + s.u + j] = u;
          else
            ub[q][s.uofs + j] = u;
        }
    }
    __syncthreads();
  }
}

// The row pairs of a subtree depth whose fronts all have |B| <= 128: a row's
// V is at most two 64-wide segments, so each wave takes two row pairs at once
// (the loads of four rows in flight together) and sums each pair as the
// general loop does (the V segments it leaves out are zero in both).
template <int WG, int NR>
__device__ inline void sub_bwd_quad(const SubTask& t, const SubFront* lf, int nf, int d, const c128* base,
                                    const NDSolveArgs* __restrict__ tab, const NDGroup& g) {
  const NDSolveArgs& A0 = tab[g.inst[0]];
  const int nr = g.n, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int npq = (t.sP[d] + 1) >> 1;
  for (int pq = wv; pq < npq; pq += WG / 64) {  // wave-uniform
    int ka[2], pS[2], nI[2], nB[2];
    int64_t iofs[2];
    bool hb[2];
    const bool has1 = 2 * pq + 1 < t.sP[d];
    c128 gv[4], vv[4][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int pr = j == 0 || has1 ? 2 * pq + j : 2 * pq;
      const SubFront& s = lf[sub_find<2>(lf, nf, pr)];
      ka[j] = 2 * (pr - s.pP);
      hb[j] = ka[j] + 1 < s.nI;
      pS[j] = s.pS;
      nI[j] = s.nI;
      nB[j] = s.nB;
      iofs[j] = s.Iid;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = i == 0 || hb[j] ? ka[j] + i : ka[j];
        gv[2 * j + i] = lane < s.nI ? A0.G[s.gofs + nd_g_index(s.nI, s.ldg, r, lane)] : c128{0.0, 0.0};
#pragma unroll
        for (int p = 0; p < 2; ++p)
          vv[2 * j + i][p] =
              lane + 64 * p < s.nB ? A0.V[s.vofs + (int64_t)r * s.ldv + lane + 64 * p] : c128{0.0, 0.0};
      }
    }
    c128 a[4][NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const c128* cI = base + q * t.stot + pS[j];
        const c128 x = (q < nr && lane < nI[j]) ? cI[lane] : c128{0.0, 0.0};
        c128 y[2];
#pragma unroll
        for (int p = 0; p < 2; ++p)
          y[p] = (q < nr && lane + 64 * p < nB[j]) ? cI[nI[j] + lane + 64 * p] : c128{0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          c128& acc = a[2 * j + i][q];
          acc = {0.0, 0.0};
          cfma(acc, gv[2 * j + i], x);
#pragma unroll
          for (int p = 0; p < 2; ++p) cfms(acc, vv[2 * j + i][p], y[p]);
        }
      }
    }
    store_bwd_rows<NR>(a[0], a[1], nr, hb[0], ka[0], ka[0] + 1, A0.Iid, iofs[0], lane,
                       [&](int q) { return tab[g.inst[NR == 1 ? 0 : q]].e0; });
    if (has1)
      store_bwd_rows<NR>(a[2], a[3], nr, hb[1], ka[1], ka[1] + 1, A0.Iid, iofs[1], lane,
                         [&](int q) { return tab[g.inst[NR == 1 ? 0 : q]].e0; });
  }
}

// Backward sweep of one subtree, its root first: per level, c_I (cbuf) and
// x_B (e0: the ancestors' solutions, from this launch or the levels above)
// of every front are staged in LDS, then each wave takes a row pair at a
// time, x_k = G[k, :] c_I - V[k, :] x_B with lanes over columns (the level
// kernels' small-front rows) and one wave sum per pair.
// QUAD: depths whose fronts all have |B| <= 128 take two row pairs per wave
// (single solves; the batch kernels keep one, which already fills their
// registers: the sums are the same either way).
template <int WG, int NR, bool QUAD>
__device__ inline void sub_bwd(const SubTask& t, const SubFront* __restrict__ gsf, const NDSolveArgs* __restrict__ tab,
                               const NDGroup& g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const SubFront* sf = sub_records<WG>(t, gsf, smem);
  c128* base = reinterpret_cast<c128*>(smem + sub_rec_bytes(t.lev[t.nlev]));
  const NDSolveArgs& A0 = tab[g.inst[0]];
  const int nr = g.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const c128* cb[NR];
  const c128* xe[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const NDSolveArgs& A = tab[g.inst[q < nr ? q : 0]];
    cb[q] = A.cbuf;
    xe[q] = A.e0;
  }
  __syncthreads();
  for (int d = 0; d < t.nlev; ++d) {
    const SubFront* lf = sf + t.lev[d];
    const int nf = t.lev[d + 1] - t.lev[d];
    for (int e = tid; e < t.sS[d]; e += WG) {
      const SubFront& s = lf[sub_find<3>(lf, nf, e)];
      const int r = e - s.pS;
      c128 v[NR];
      if (r < s.nI) {
#pragma unroll
        for (int q = 0; q < NR; ++q) v[q] = cb[q][s.cofs + r];
      } else {
        const int id = A0.Bid[s.Bid + r - s.nI];
#pragma unroll
        for (int q = 0; q < NR; ++q) v[q] = xe[q][id];
      }
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nr) base[q * t.stot + e] = v[q];
    }
    __syncthreads();
    if (QUAD && ((t.quad >> d) & 1)) {  // workgroup-uniform
      sub_bwd_quad<WG, NR>(t, lf, nf, d, base, tab, g);
      __syncthreads();
      continue;
    }
    for (int pr = wv; pr < t.sP[d]; pr += WG / 64) {  // wave-uniform
      const SubFront& s = lf[sub_find<2>(lf, nf, pr)];
      const int ka = 2 * (pr - s.pP), kb = ka + 1;
      const bool hb = kb < s.nI;
      c128 gv[2], vv[2][kSubNV];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = i == 0 || hb ? ka + i : ka;
        gv[i] = lane < s.nI ? A0.G[s.gofs + nd_g_index(s.nI, s.ldg, r, lane)] : c128{0.0, 0.0};
#pragma unroll
        for (int p = 0; p < kSubNV; ++p)
          vv[i][p] = lane + 64 * p < s.nB ? A0.V[s.vofs + (int64_t)r * s.ldv + lane + 64 * p] : c128{0.0, 0.0};
      }
      c128 a[2][NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const c128* cI = base + q * t.stot + s.pS;
        const c128 x = (q < nr && lane < s.nI) ? cI[lane] : c128{0.0, 0.0};
        c128 y[kSubNV];
#pragma unroll
        for (int p = 0; p < kSubNV; ++p) y[p] = (q < nr && lane + 64 * p < s.nB) ? cI[s.nI + lane + 64 * p] : c128{0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[i][q] = {0.0, 0.0};
          cfma(a[i][q], gv[i], x);
#pragma unroll
          for (int p = 0; p < kSubNV; ++p) cfms(a[i][q], vv[i][p], y[p]);
        }
      }
      store_bwd_rows<NR>(a[0], a[1], nr, hb, ka, kb, A0.Iid, s.Iid, lane,
                         [&](int q) { return tab[g.inst[NR == 1 ? 0 : q]].e0; });
    }
    __syncthreads();
  }
}

template <int WG>
__global__ void __launch_bounds__(WG) nd_sub_fwd_kernel(const SubTask* __restrict__ tasks,
                                                        const SubFront* __restrict__ sf, NDSolveArgs A) {
  const NDGroup g{1, {0, 0, 0, 0}};
  sub_fwd<WG, 1>(tasks[blockIdx.x], sf, &A, g);
}

template <int WG>
__global__ void __launch_bounds__(WG) nd_sub_bwd_kernel(const SubTask* __restrict__ tasks,
                                                        const SubFront* __restrict__ sf, NDSolveArgs A) {
  const NDGroup g{1, {0, 0, 0, 0}};
  sub_bwd<WG, 1, true>(tasks[blockIdx.x], sf, &A, g);
}

template <int WG, int NR>
__global__ void __launch_bounds__(WG) nd_sub_fwd_batch_kernel(const SubTask* __restrict__ tasks,
                                                              const SubFront* __restrict__ sf,
                                                              const NDSolveArgs* __restrict__ tab,
                                                              const NDGroup* __restrict__ groups,
                                                              const ArnState* __restrict__ st) {
  const SubTask& t = tasks[blockIdx.x];
  const NDGroup& g = groups[t.grp];
  if (group_idle(st, g)) return;
  sub_fwd<WG, NR>(t, sf, tab, g);
}

template <int WG, int NR>
__global__ void __launch_bounds__(WG) nd_sub_bwd_batch_kernel(const SubTask* __restrict__ tasks,
                                                              const SubFront* __restrict__ sf,
                                                              const NDSolveArgs* __restrict__ tab,
                                                              const NDGroup* __restrict__ groups,
                                                              const ArnState* __restrict__ st) {
  const SubTask& t = tasks[blockIdx.x];
  const NDGroup& g = groups[t.grp];
  if (group_idle(st, g)) return;
  sub_bwd<WG, NR, false>(t, sf, tab, g);
}

// Solve tasks of one level: each front's chunks (column chunks of B forward,
// row chunks of I backward) are grouped into tasks of up to `group`
// consecutive chunks, group chosen so that a level launches about `target`
// workgroups: small fronts then share one workgroup's staging of c_I / x_B
// instead of paying it per chunk.  A single solve targets 1024 (at n = 1025
// the levels of 1400-2000 chunks then take two per task: 0.396 -> 0.390 ms;
// 512 and 768 did worse), a batch 2048.  The grouping does not change any
// sum.
constexpr int kSolveTasks = 2048;
constexpr int kSolveTasksSingle = 1024;
SolveFront solve_front(const NDPlan& p, int t) {
  const NDFront& F = p.fronts[t];
  SolveFront s{};
  s.nI = F.nI;
  s.nB = F.nB;
  s.ldg = F.ldg;
  s.ldv = F.ldv;
  s.Iid = F.Iid;
  s.Bid = F.Bid;
  s.gofs = F.gofs;
  s.vofs = F.vofs;
  s.cofs = F.cofs;
  s.uofs = F.uofs;
  for (int ch = 0; ch < 2; ++ch) {
    s.inv[ch] = F.inv[ch];
    s.cu[ch] = F.child[ch] >= 0 ? p.fronts[F.child[ch]].uofs : -1;
  }
  return s;
}

struct ChunkList {
  struct Entry {
    SolveFront f;
    int chunks, grp;
  };
  std::vector<Entry> fronts;
  int64_t total = 0;
  void add(const SolveFront& f, int chunks, int grp) {
    fronts.push_back({f, chunks, grp});
    total += chunks;
  }
  std::vector<STask> tasks(int target) const {
    const int group = (int)std::max<int64_t>(1, (total + target - 1) / target);
    std::vector<STask> out;
    for (const Entry& e : fronts)
      for (int a = 0; a < e.chunks; a += group) out.push_back({e.f, a, std::min(group, e.chunks - a), e.grp, 0});
    return out;
  }
};

// Subtrees rooted at depth Ls: front records and tasks (group `grp`),
// appended; the LDS bytes of the largest forward and backward task for nr
// right-hand sides.
struct SubBuild {
  std::vector<SubFront> fr;
  std::vector<SubTask> tasks;
  size_t lds_f = 0, lds_b = 0;
};

void sub_build(const NDPlan& p, int Ls, int nr, int grp, SubBuild& out) {
  for (int root : p.levels[Ls]) {
    std::vector<std::vector<int>> dep(1, std::vector<int>{root});
    for (;;) {
      std::vector<int> nx;
      for (int f : dep.back())
        for (int ch = 0; ch < 2; ++ch)
          if (p.fronts[f].child[ch] >= 0) nx.push_back(p.fronts[f].child[ch]);
      if (nx.empty()) break;
      dep.push_back(nx);
    }
    if ((int)dep.size() > kSubLevels) throw Failure{HS_EINVAL, "nested-dissection subtree deeper than its limit"};
    std::unordered_map<int, int> uo;  // front -> LDS offset of its u_B (below the subtree root)
    int u = 0;
    for (size_t d = 1; d < dep.size(); ++d)
      for (int f : dep[d]) {
        uo[f] = u;
        u += p.fronts[f].nB;
      }
    SubTask t{};
    t.first = (int)out.fr.size();
    t.nlev = (int)dep.size();
    t.grp = grp;
    int c = 0, stot = 0;
    for (size_t d = 0; d < dep.size(); ++d) {
      t.lev[d] = (int)out.fr.size() - t.first;
      int sI = 0, sB = 0, sP = 0, sS = 0;
      for (int f : dep[d]) {
        const NDFront& F = p.fronts[f];
        SubFront s{};
        s.nI = F.nI;
        s.nB = F.nB;
        s.ldg = F.ldg;
        s.ldv = F.ldv;
        s.c = c;
        c += F.nI;
        s.u = d > 0 ? uo.at(f) : -1;
        for (int ch = 0; ch < 2; ++ch) {
          s.uch[ch] = F.child[ch] >= 0 ? uo.at(F.child[ch]) : -1;
          s.inv[ch] = F.inv[ch];
        }
        s.pI = sI;
        s.pB = sB;
        s.pP = sP;
        s.pS = sS;
        sI += F.nI;
        sB += F.nB;
        sP += (F.nI + 1) / 2;
        sS += F.nI + F.nB;
        s.Iid = F.Iid;
        s.Bid = F.Bid;
        s.gofs = F.gofs;
        s.vofs = F.vofs;
        s.cofs = F.cofs;
        s.uofs = F.uofs;
        out.fr.push_back(s);
      }
      t.sI[d] = sI;
      t.sB[d] = sB;
      t.sP[d] = sP;
      t.sS[d] = sS;
      int mB = 0;
      for (int f : dep[d]) mB = std::max(mB, p.fronts[f].nB);
      if (mB <= 128) t.quad |= 1 << d;
      stot = std::max(stot, sS);
    }
    t.lev[t.nlev] = (int)out.fr.size() - t.first;
    t.ctot = c;
    t.utot = u;
    t.stot = stot;
    const size_t rec = sub_rec_bytes(t.lev[t.nlev]);
    out.lds_f = std::max(out.lds_f, rec + (size_t)nr * (c + u) * sizeof(c128));
    out.lds_b = std::max(out.lds_b, rec + (size_t)nr * stot * sizeof(c128));
    out.tasks.push_back(t);
  }
}

// The depth from which a plan is solved by subtree, for groups of nr
// right-hand sides: the shallowest depth whose subtrees fit (every front
// from it down within kSubNI / kSubNB, at most kSubLevels depths, LDS within
// kSubLdsMax) and number at least min_count; if none is that many, the
// deepest that fits.  max_depth + 1: no subtrees.
int sub_level(const NDPlan& p, int nr, int min_count) {
  const int D = p.max_depth;
  int lo = D + 1;
  for (int lv = D; lv >= std::max(0, D - kSubLevels + 1); --lv) {
    bool ok = true;
    for (int f : p.levels[lv]) ok = ok && p.fronts[f].nI <= kSubNI && p.fronts[f].nB <= kSubNB;
    if (!ok) break;
    lo = lv;
  }
  int pick = D + 1;
  for (int lv = lo; lv <= D; ++lv) {
    SubBuild b;
    sub_build(p, lv, nr, 0, b);
    if (b.lds_f > kSubLdsMax || b.lds_b > kSubLdsMax) continue;
    if ((int)p.levels[lv].size() >= min_count) return lv;
    pick = lv;
  }
  return pick;
}

constexpr int kSubMinSingle = 256;  // subtrees of a single solve: at least one per CU (1024 threads each)

// Dynamic-LDS limits of the subtree kernels, only ever raised (as for the
// panel kernel).
template <int NR>
void raise_sub_lds(size_t lds) {
  static std::mutex mu;
  static size_t raised = 0;
  std::lock_guard<std::mutex> lk(mu);
  if (lds <= raised) return;
  auto set = [&](const void* k) { HS_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); };
  if constexpr (NR == 1) {
    set((const void*)nd_sub_fwd_kernel<512>);
    set((const void*)nd_sub_bwd_kernel<512>);
    set((const void*)nd_sub_fwd_kernel<1024>);
    set((const void*)nd_sub_bwd_kernel<1024>);
    set((const void*)nd_sub_fwd_batch_kernel<1024, 1>);
    set((const void*)nd_sub_bwd_batch_kernel<1024, 1>);
  }
  set((const void*)nd_sub_fwd_batch_kernel<512, NR>);
  set((const void*)nd_sub_bwd_batch_kernel<512, NR>);
  raised = lds;
}


}  // namespace

NDDev* nd_create(const NDPlan& plan, Arena& A) {
  NDDev* d = new NDDev();
  try {
    int max_nI = 0, max_nB = 0;
    for (const NDFront& f : plan.fronts) {
      max_nI = std::max(max_nI, f.nI);
      max_nB = std::max(max_nB, f.nB);
    }
    if (max_nI > SOLVE_MAX || max_nB > SOLVE_MAX || (size_t)max_nI * NB * 16 + max_nI * 4 > 150 * 1024)
      throw Failure{HS_EINVAL, "coarse grid too large for the nested-dissection front limits"};
    d->fronts = A.put(plan.fronts);
    d->Iid = A.put(plan.Iid);
    d->Bid = A.put(plan.Bid);
    d->inv = A.put(plan.inv);
    d->ppos = A.put(plan.ppos);
    d->G = A.take<c128>(plan.g_elems);
    d->V = A.take<c128>(plan.v_elems);
    d->cbuf = A.take<c128>(plan.c_elems);
    d->ubuf = A.take<c128>(plan.u_elems);
    d->rho = A.take<int>(plan.p_elems);
    d->rinv = A.take<int>(plan.p_elems);
    d->used = A.take<int>(plan.p_elems);
    d->status = A.take<int>(1);
    size_t maxlvl = 0;
    for (const auto& l : plan.levels) maxlvl = std::max(maxlvl, l.size());
    d->Y = A.take<c128>((int64_t)maxlvl * NB * NB);
    d->sub_lv = sub_level(plan, 1, kSubMinSingle);
    if (d->sub_lv <= plan.max_depth) {
      SubBuild b;
      sub_build(plan, d->sub_lv, 1, 0, b);
      d->sub_f = A.put(b.fr);
      d->sub_t = A.put(b.tasks);
      d->n_sub = (int)b.tasks.size();
      d->sub_lds_f = b.lds_f;
      d->sub_lds_b = b.lds_b;
      if (A.base) raise_sub_lds<1>(std::max(b.lds_f, b.lds_b));  // (a counting pass touches no device)
    }
    const int L = (int)plan.levels.size();
    for (int lv = 0; lv < L; ++lv) {
      const std::vector<int>& fl = plan.levels[lv];
      std::vector<Task> ta, tu, tf, te;
      std::vector<STask> tw, tb;
      ChunkList cw, cb;
      int mI = 0, mB = 0;
      size_t na = 0, nu = 0, nx = 0, ne = 0;
      for (const int t : fl) {
        const NDFront& f = plan.fronts[t];
        const size_t nt = (f.nF + TILE - 1) / TILE;
        na += f.nF;
        nu += nt * nt;
        nx += 2 * nt;
        ne += f.nI;
      }
      ta.reserve(na);
      tu.reserve(nu);
      tf.reserve(nx);
      te.reserve(ne);
      for (int q = 0; q < (int)fl.size(); ++q) {
        const int t = fl[q];
        const NDFront& f = plan.fronts[t];
        mI = std::max(mI, f.nI);
        mB = std::max(mB, f.nB);
        const int nt = (f.nF + TILE - 1) / TILE;
        for (int r = 0; r < f.nF; ++r) ta.push_back({t, r, 0, 0});
        for (int a = 0; a < nt; ++a)
          for (int b = 0; b < nt; ++b) tu.push_back({t, a, b, q});
        for (int a = 0; a < nt; ++a) tf.push_back({t, a, 0, q});
        for (int a = 0; a < nt; ++a) tf.push_back({t, a, 1, q});
        for (int k = 0; k < f.nI; ++k) te.push_back({t, k, 0, 0});
        if (lv < d->sub_lv) {
          const SolveFront sf = solve_front(plan, t);
          cw.add(sf, std::max(1, (f.nB + fwd_cols(f.nI) - 1) / fwd_cols(f.nI)), 0);
          cb.add(sf, (f.nI + BWD_ROWS - 1) / BWD_ROWS, 0);
        }
      }
      tw = cw.tasks(kSolveTasksSingle);
      tb = cb.tasks(kSolveTasksSingle);
      d->lvl_fronts.push_back(A.put(fl));
      d->n_fronts.push_back((int)fl.size());
      d->asm_t.push_back(A.put(ta));
      d->n_asm.push_back((int)ta.size());
      d->upd_t.push_back(A.put(tu));
      d->n_upd.push_back((int)tu.size());
      d->fix_t.push_back(A.put(tf));
      d->n_fix.push_back((int)tf.size());
      d->ext_t.push_back(A.put(te));
      d->n_ext.push_back((int)te.size());
      d->fwd_t.push_back(A.put(tw));
      d->n_fwd.push_back((int)tw.size());
      d->bwd_t.push_back(A.put(tb));
      d->n_bwd.push_back((int)tb.size());
      d->max_nI.push_back(mI);
      d->max_nB.push_back(mB);
    }
  } catch (...) {
    delete d;
    throw;
  }
  return d;
}

// per-level figures of the solve: fronts, entries of G read (sum |I|^2, or
// |I|(|I|+1)/2 for a front keeping one triangle), sum |I||B|, forward
// and backward workgroups, max |I|, max |B|
void nd_level_stats(const NDPlan& plan, const NDDev& d, int lv, int64_t* out) {
  int64_t gi = 0, vb = 0;
  for (int t : plan.levels[lv]) {
    const NDFront& f = plan.fronts[t];
    gi += nd_tri(f.nI) ? nd_g_entries(f.nI, f.ldg) : (int64_t)f.nI * f.nI;
    vb += (int64_t)f.nI * f.nB;
  }
  out[0] = (int64_t)plan.levels[lv].size();
  out[1] = gi;
  out[2] = vb;
  out[3] = lv >= 1 ? d.n_fwd[lv] : 0;  // the root's forward part is done by its backward task
  out[4] = d.n_bwd[lv];
  out[5] = d.max_nI[lv];
  out[6] = d.max_nB[lv];
  out[7] = lv >= d.sub_lv ? d.n_sub : 0;  // solved by subtree: the subtree launches' workgroups
}

void nd_destroy(NDDev* d) { delete d; }

// The panel kernel's dynamic-LDS limit is only ever raised, so a set-up on
// another host thread never lowers it under a pending launch.
void raise_panel_lds(size_t lds) {
  static std::mutex mu;
  static size_t raised = 0;
  std::lock_guard<std::mutex> lk(mu);
  if (lds <= raised) return;
  HS_HIP(hipFuncSetAttribute((const void*)nd_panel_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  raised = lds;
}

int nd_factor_run(const NDPlan& plan, NDDev& d, const c128* A0, c128* F, hipStream_t s) {
  d.F = F;
  HS_HIP(hipMemsetAsync(d.used, 0, (size_t)std::max<int64_t>(1, plan.p_elems) * sizeof(int), s));
  HS_HIP(hipMemsetAsync(d.status, 0, sizeof(int), s));
  const int R = plan.reach;
  for (int lv = plan.max_depth; lv >= 0; --lv) {
    if (d.n_asm[lv] > 0) {
      nd_assemble_kernel<<<d.n_asm[lv], 64, 0, s>>>(d.fronts, d.asm_t[lv], d.Iid, d.Bid, d.inv, d.ppos, A0,
                                                    plan.ncx, plan.ncy, R, d.F);
      HS_HIP(hipGetLastError());
    }
    const int mI = d.max_nI[lv];
    const size_t lds = (size_t)mI * NB * sizeof(c128) + (size_t)mI * sizeof(int) + 64;
    raise_panel_lds(lds);
    for (int k0 = 0; k0 < mI; k0 += NB) {
      nd_panel_kernel<<<d.n_fronts[lv], K1_WG, lds, s>>>(d.fronts, d.lvl_fronts[lv], d.n_fronts[lv], k0, d.F,
                                                         d.used, d.rho, d.rinv, d.Y, d.status);
      HS_HIP(hipGetLastError());
      nd_update_kernel<<<d.n_upd[lv], 256, 0, s>>>(d.fronts, d.upd_t[lv], k0, d.rho, d.Y, d.F);
      HS_HIP(hipGetLastError());
      nd_fix_kernel<<<d.n_fix[lv], 256, 0, s>>>(d.fronts, d.fix_t[lv], k0, d.rho, d.Y, d.F);
      HS_HIP(hipGetLastError());
    }
    nd_extract_kernel<<<d.n_ext[lv], 256, 0, s>>>(d.fronts, d.ext_t[lv], d.rho, d.rinv, d.F, d.G, d.V);
    HS_HIP(hipGetLastError());
  }
  int st = 0;
  HS_HIP(hipMemcpyAsync(&st, d.status, sizeof(int), hipMemcpyDeviceToHost, s));
  HS_HIP(hipStreamSynchronize(s));
  d.F = nullptr;
  return st;
}

void nd_solve_run(const NDPlan& plan, NDDev& d, const c128* r0, c128* e0, hipStream_t s,
                  const Callback& after, int after_levels, c128* cbuf, c128* ubuf) {
  if (!cbuf) cbuf = d.cbuf;
  if (!ubuf) ubuf = d.ubuf;
  // level 0 holds the root only (no B): its forward part is staged by the
  // backward sweep
  int launched = 0;
  const NDSolveArgs args{d.fronts, d.Iid, d.Bid, d.inv, d.G, d.V, r0, cbuf, ubuf, e0};
  if (d.n_sub) {
    if (after && launched == after_levels) after();
    if (d.n_sub <= kSubWide)
      nd_sub_fwd_kernel<1024><<<d.n_sub, 1024, d.sub_lds_f, s>>>((const SubTask*)d.sub_t,
                                                                  (const SubFront*)d.sub_f, args);
    else
      nd_sub_fwd_kernel<512><<<d.n_sub, 512, d.sub_lds_f, s>>>((const SubTask*)d.sub_t, (const SubFront*)d.sub_f,
                                                                args);
    HS_HIP(hipGetLastError());
    ++launched;
  }
  for (int lv = std::min(plan.max_depth, d.sub_lv - 1); lv >= 1; --lv) {
    if (after && launched == after_levels) after();
    const size_t lds = (size_t)d.max_nI[lv] * sizeof(c128);
    nd_fwd_kernel<<<d.n_fwd[lv], 256, lds, s>>>((const STask*)d.fwd_t[lv], d.Iid, d.inv, d.V, r0, cbuf, ubuf,
                                                d.max_nI[lv]);
    HS_HIP(hipGetLastError());
    ++launched;
  }
  if (after && after_levels >= launched) after();  // after all forward levels
  for (int lv = 0; lv <= std::min(plan.max_depth, d.sub_lv - 1); ++lv) {
    const size_t lds = (size_t)(d.max_nI[lv] + d.max_nB[lv]) * sizeof(c128);
    nd_bwd_kernel<<<d.n_bwd[lv], 256, lds, s>>>((const STask*)d.bwd_t[lv], d.Iid, d.Bid, d.inv, d.G, d.V, r0,
                                                ubuf, cbuf, e0, d.max_nI[lv], d.max_nB[lv]);
    HS_HIP(hipGetLastError());
  }
  if (d.n_sub) {
    if (d.n_sub <= kSubWide)
      nd_sub_bwd_kernel<1024><<<d.n_sub, 1024, d.sub_lds_b, s>>>((const SubTask*)d.sub_t,
                                                                  (const SubFront*)d.sub_f, args);
    else
      nd_sub_bwd_kernel<512><<<d.n_sub, 512, d.sub_lds_b, s>>>((const SubTask*)d.sub_t, (const SubFront*)d.sub_f,
                                                                args);
    HS_HIP(hipGetLastError());
  }
}

// --------------------------------------------------------- batched solve
// The coarse solves of many instances: the level task lists of all
// instances, aligned by depth from the root, one launch per depth and
// direction.  Each task carries its instance.  Instances on one factor
// (several right-hand sides of one problem) get work vectors of their own
// after the first, and their tasks of a front are consecutive, so that
// neighbouring workgroups read the same factor blocks together and the
// repeats are served from cache.
struct NDBatch {
  NDSolveArgs* tab = nullptr;
  NDGroup* groups = nullptr;  // tasks name a group of instances on one factor
  int nr = 1;                 // largest group
  std::vector<void*> fwd_t, bwd_t;  // solve tasks (STask)
  std::vector<int> n_fwd, n_bwd, max_nI, max_nB;
  void* sub_t = nullptr;  // subtree tasks of every instance group (SubTask)
  void* sub_f = nullptr;
  int n_sub = 0;
  size_t sub_lds_f = 0, sub_lds_b = 0;
};

namespace {

constexpr size_t kBlockLdsMax = 150 * 1024;  // dynamic LDS of one block-solve workgroup

// The limit is a property of the kernel, shared by every batch: it is only
// ever raised, so an earlier batch's launches stay within it.
template <int NR>
void nd_block_lds_limits(size_t fwd, size_t bwd) {
  static std::mutex mu;  // batches created on several host threads
  std::lock_guard<std::mutex> lk(mu);
  static size_t raised_f = 0, raised_b = 0;
  if (fwd > raised_f) {
    HS_HIP(hipFuncSetAttribute((const void*)nd_fwd_batch_kernel<NR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)fwd));
    raised_f = fwd;
  }
  if (bwd > raised_b) {
    HS_HIP(hipFuncSetAttribute((const void*)nd_bwd_batch_kernel<NR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bwd));
    raised_b = bwd;
  }
}

}  // namespace

NDBatch* nd_batch_create(const std::vector<const NDPlan*>& plans, const std::vector<NDDev*>& devs,
                         const std::vector<const c128*>& r0, const std::vector<c128*>& e0, Arena& A) {
  NDBatch* B = new NDBatch();
  try {
    int depth = 0;
    for (const NDPlan* p : plans) depth = std::max(depth, p->max_depth);
    // instances on one factor, in order of first appearance; the repeats get
    // work vectors of their own
    std::vector<std::vector<int>> same;
    std::vector<NDSolveArgs> tab(plans.size());
    for (size_t i = 0; i < plans.size(); ++i) {
      const NDDev& d = *devs[i];
      c128 *cbuf = d.cbuf, *ubuf = d.ubuf;
      bool repeat = false;
      for (auto& g : same)
        if (devs[g[0]] == devs[i]) {
          g.push_back((int)i);
          repeat = true;
          break;
        }
      if (!repeat) {
        same.push_back({(int)i});
      } else {
        cbuf = A.take<c128>(plans[i]->c_elems);
        ubuf = A.take<c128>(plans[i]->u_elems);
      }
      tab[i] = NDSolveArgs{d.fronts, d.Iid, d.Bid, d.inv, d.G, d.V, r0[i], cbuf, ubuf, e0[i]};
    }
    B->tab = A.put(tab);
    // level extents over all instances, aligned by depth from the root
    std::vector<int> mI(depth + 1, 0), mB(depth + 1, 0);
    size_t widest = 0;
    for (const NDPlan* p : plans)
      for (int lv = 0; lv < (int)p->levels.size(); ++lv)
        for (int t : p->levels[lv]) {
          mI[lv] = std::max(mI[lv], p->fronts[t].nI);
          mB[lv] = std::max(mB[lv], p->fronts[t].nB);
          widest = std::max(widest, (size_t)(mI[lv] + mB[lv]));
        }
    // groups of up to ND_NR right-hand sides on one factor, as many as the
    // block solve's staging fits in LDS
    int cap = ND_NR;
    while (cap > 1 && (size_t)cap * widest * sizeof(c128) > kBlockLdsMax) cap /= 2;
    std::vector<NDGroup> grp;
    std::vector<std::vector<int>> grp_of(same.size());  // group indices per factor
    for (size_t s = 0; s < same.size(); ++s)
      for (size_t a = 0; a < same[s].size(); a += cap) {
        NDGroup g{};
        g.n = (int)std::min<size_t>(cap, same[s].size() - a);
        for (int q = 0; q < g.n; ++q) g.inst[q] = same[s][a + q];
        B->nr = std::max(B->nr, g.n);
        grp_of[s].push_back((int)grp.size());
        grp.push_back(g);
      }
    B->groups = A.put(grp);
    // the depth from which each factor is solved by subtree, and the
    // subtree tasks (a subtree's groups side by side)
    std::vector<int> sub_lv(same.size());
    SubBuild sb;
    const int min_count = std::max<int>(1, kSubMinSingle / (int)grp.size());
    for (size_t s = 0; s < same.size(); ++s) {
      const NDPlan& plan = *plans[same[s][0]];
      sub_lv[s] = sub_level(plan, B->nr, min_count);
      if (sub_lv[s] > plan.max_depth) continue;
      SubBuild one;
      sub_build(plan, sub_lv[s], B->nr, 0, one);
      const int f0 = (int)sb.fr.size();
      sb.fr.insert(sb.fr.end(), one.fr.begin(), one.fr.end());
      for (const SubTask& t : one.tasks)
        for (int gi : grp_of[s]) {
          SubTask tg = t;
          tg.first += f0;
          tg.grp = gi;
          sb.tasks.push_back(tg);
        }
      sb.lds_f = std::max(sb.lds_f, one.lds_f);
      sb.lds_b = std::max(sb.lds_b, one.lds_b);
    }
    if (!sb.tasks.empty()) {
      B->sub_f = A.put(sb.fr);
      B->sub_t = A.put(sb.tasks);
      B->n_sub = (int)sb.tasks.size();
      B->sub_lds_f = sb.lds_f;
      B->sub_lds_b = sb.lds_b;
    }
    auto up = [&](const std::vector<STask>& v) -> void* { return v.empty() ? nullptr : (void*)A.put(v); };
    for (int lv = 0; lv <= depth; ++lv) {
      ChunkList cw, cb;
      for (size_t s = 0; s < same.size(); ++s) {
        const NDPlan& plan = *plans[same[s][0]];
        if (lv >= (int)plan.levels.size() || lv >= sub_lv[s]) continue;
        for (int t : plan.levels[lv]) {  // a front's groups side by side
          const NDFront& f = plan.fronts[t];
          const SolveFront sf = solve_front(plan, t);
          for (int gi : grp_of[s]) {
            cw.add(sf, std::max(1, (f.nB + fwd_cols(f.nI) - 1) / fwd_cols(f.nI)), gi);
            cb.add(sf, (f.nI + BWD_ROWS - 1) / BWD_ROWS, gi);
          }
        }
      }
      const std::vector<STask> tw = cw.tasks(kSolveTasks), tb = cb.tasks(kSolveTasks);
      B->fwd_t.push_back(up(tw));
      B->n_fwd.push_back((int)tw.size());
      B->bwd_t.push_back(up(tb));
      B->n_bwd.push_back((int)tb.size());
      B->max_nI.push_back(mI[lv]);
      B->max_nB.push_back(mB[lv]);
    }
    size_t lf = 0, lb = 0;
    for (int lv = 0; lv <= depth; ++lv) {
      lf = std::max(lf, (size_t)B->nr * mI[lv] * sizeof(c128));
      lb = std::max(lb, (size_t)B->nr * (mI[lv] + mB[lv]) * sizeof(c128));
    }
    const size_t ls = std::max(B->sub_lds_f, B->sub_lds_b);
    if (A.base) {  // (a counting pass touches no device)
      if (B->nr == 1) {
        nd_block_lds_limits<1>(lf, lb);
        raise_sub_lds<1>(ls);
      } else if (B->nr == 2) {
        nd_block_lds_limits<2>(lf, lb);
        raise_sub_lds<2>(ls);
      } else {
        nd_block_lds_limits<4>(lf, lb);
        raise_sub_lds<4>(ls);
      }
    }
  } catch (...) {
    delete B;
    throw;
  }
  return B;
}

void nd_batch_destroy(NDBatch* B) { delete B; }

namespace {

template <int NR>
void nd_batch_levels(const NDBatch& B, hipStream_t s, const Callback& after, int after_levels, const ArnState* st) {
  const int L = (int)B.n_fwd.size();
  int launched = 0;
  if (B.n_sub) {
    if (after && launched == after_levels) after();
    const SubTask* t = (const SubTask*)B.sub_t;
    const SubFront* f = (const SubFront*)B.sub_f;
    if (NR == 1 && B.n_sub <= kSubWide)  // (1024-thread batch kernels only for single right-hand sides)
      nd_sub_fwd_batch_kernel<1024, 1><<<B.n_sub, 1024, B.sub_lds_f, s>>>(t, f, B.tab, B.groups, st);
    else
      nd_sub_fwd_batch_kernel<512, NR><<<B.n_sub, 512, B.sub_lds_f, s>>>(t, f, B.tab, B.groups, st);
    HS_HIP(hipGetLastError());
    ++launched;
  }
  for (int lv = L - 1; lv >= 1; --lv) {  // level 0: the roots, staged by the backward sweep
    if (!B.n_fwd[lv]) continue;
    if (after && launched == after_levels) after();
    const size_t lds = (size_t)B.nr * B.max_nI[lv] * sizeof(c128);
    nd_fwd_batch_kernel<NR><<<B.n_fwd[lv], 256, lds, s>>>((const STask*)B.fwd_t[lv], B.tab, B.groups,
                                                          B.max_nI[lv], st);
    HS_HIP(hipGetLastError());
    ++launched;
  }
  if (after && after_levels >= launched) after();  // after all forward levels
  for (int lv = 0; lv < L; ++lv) {
    if (!B.n_bwd[lv]) continue;
    const size_t lds = (size_t)B.nr * (B.max_nI[lv] + B.max_nB[lv]) * sizeof(c128);
    nd_bwd_batch_kernel<NR><<<B.n_bwd[lv], 256, lds, s>>>((const STask*)B.bwd_t[lv], B.tab, B.groups,
                                                          B.max_nI[lv], B.max_nB[lv], st);
    HS_HIP(hipGetLastError());
  }
  if (B.n_sub) {
    const SubTask* t = (const SubTask*)B.sub_t;
    const SubFront* f = (const SubFront*)B.sub_f;
    if (NR == 1 && B.n_sub <= kSubWide)
      nd_sub_bwd_batch_kernel<1024, 1><<<B.n_sub, 1024, B.sub_lds_b, s>>>(t, f, B.tab, B.groups, st);
    else
      nd_sub_bwd_batch_kernel<512, NR><<<B.n_sub, 512, B.sub_lds_b, s>>>(t, f, B.tab, B.groups, st);
    HS_HIP(hipGetLastError());
  }
}

}  // namespace

void nd_batch_solve_run(const NDBatch& B, hipStream_t s, const Callback& after, int after_levels,
                        const ArnState* st) {
  if (B.nr == 1)
    nd_batch_levels<1>(B, s, after, after_levels, st);
  else if (B.nr == 2)
    nd_batch_levels<2>(B, s, after, after_levels, st);
  else
    nd_batch_levels<4>(B, s, after, after_levels, st);
}

}  // namespace hs
