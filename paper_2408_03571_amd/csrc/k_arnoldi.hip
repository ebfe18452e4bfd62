// Low-synchronisation Arnoldi for flexible GMRES (Sec. 5), complex128.
//
// Classical Gram-Schmidt with one reorthogonalisation pass that is delayed by
// one step and fused with the next step's projection (DCGS2).  Step k starts
// from u_k = w1_{k-1} / beta_{k-1}, the once-orthogonalised residual of step
// k-1, forms z_k = M^{-1} u_k (stored: flexible GMRES keeps Z) and w = A z_k,
// and in ONE streaming pass over the final basis V_{<k} computes
//     s = V^H u_k,   t = V^H w,   u_k^H u_k,   u_k^H w.
// One block then takes
//     alpha = ||u_k - V s|| = sqrt(u^H u - |s|^2),   v_k = (u_k - V s) / alpha,
// makes column k-1 of the Hessenberg matrix final (its entries gain
// beta_{k-1} s, its subdiagonal is beta_{k-1} alpha), rotates it, and writes
// the first-pass entries of column k: t and c = v_k^H w = (u^H w - s^H t)/alpha.
// A second pass over V writes v_k and w1 = w - V t - c v_k; normalising w1
// gives u_{k+1}.  Two reads of V per step replace the k dependent
// projections of modified Gram-Schmidt (each of which reads v_i and reads
// and writes w).  A Z = V Hbar holds with z_k = M^{-1} u_k, which is all the
// flexible variant needs for x = Z y to minimise the residual.
//
// The convergence test of column k-1 runs in step k, after z_k is formed, so
// a converged solve spends one extra preconditioner application.  Every
// kernel reads the step index and the stop flag from the device state: one
// step is a fixed launch sequence that a HIP graph can replay, and the host
// only looks at the state every few steps.
//
// Reductions use per-wave partials in a fixed tree, folded in index order;
// there are no atomics, so two solves are bitwise identical.
//
// Basis layout (tile-major): the unknowns are cut into tiles of 64*EPT, one
// per wave, and tile w of basis vector i sits at V + (w*M + i)*64*EPT, M the
// row capacity.  A wave's slice of every basis vector is then one contiguous
// stream (a row-major basis interleaves k streams 16.8 MB apart, which costs
// about 5% of the bandwidth at n = 1025).  The tail of the last tile is
// padding that is never read.
#include <map>
#include <type_traits>
#include <mutex>

#include "hs_internal.h"
#include "hs_wave.h"

namespace hs {

namespace {

constexpr int AWG = 256;      // threads per block
constexpr int WPB = AWG / 64; // waves per block

__device__ inline double bfly(double v) {
  v += __shfl_xor(v, 32, 64);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 8, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 1, 64);
  return v;
}

__host__ __device__ inline int stream_blocks(const ArnDev& a) { return (a.nw + WPB - 1) / WPB; }

// instance and instance-local block of a streaming block
#define HS_ARN_BLOCK(bt)                                            \
  const int inst_ = batch_locate(bt.bstart, bt.count, blockIdx.x);  \
  const int blk = blockIdx.x - bt.bstart[inst_];                    \
  const ArnDev a = bt.tab[inst_]

// value of lane l (l wave-uniform) in every lane
__device__ inline double rl(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Basis vectors are streamed once per pass and exceed every cache level:
// non-temporal loads keep them from evicting the vectors that are reused.
typedef double dbl2 __attribute__((ext_vector_type(2)));
__device__ inline c128 ld_stream(const c128* p) {
  const dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(p));
  return {v.x, v.y};
}
__device__ inline void st_stream(c128* p, c128 v) {
  dbl2 t;
  t.x = v.x;
  t.y = v.y;
  __builtin_nontemporal_store(t, reinterpret_cast<dbl2*>(p));
}

// Basis element loads and stores by storage type: complex128, or complex64
// widened to complex128 on load (a compressed basis: half the bytes per pass,
// all arithmetic in complex128).
typedef float flt2 __attribute__((ext_vector_type(2)));
__device__ inline c128 ld_basis(const c128* p) { return ld_stream(p); }
__device__ inline c128 ld_basis(const c64* p) {
  const flt2 v = __builtin_nontemporal_load(reinterpret_cast<const flt2*>(p));
  return {(double)v.x, (double)v.y};
}
// round to the storage type (identity for complex128)
__device__ inline c128 to_basis(c128 v, const c128*) { return v; }
__device__ inline c128 to_basis(c128 v, const c64*) { return {(double)(float)v.x, (double)(float)v.y}; }
__device__ inline void st_basis(c128* p, c128 v) { *p = v; }
__device__ inline void st_basis(c64* p, c128 v) { *p = {(float)v.x, (float)v.y}; }

// Element of register q of a lane within its wave's tile of 64*EPT unknowns.
// Complex128 basis: 64 q + lane (one 16-byte load per element).  Complex64
// basis: lanes own adjacent pairs, 128 (q/2) + 2 lane + q%2, so that one
// 16-byte load fetches two elements (8-byte loads halve the rate).
template <int EPT, typename TV>
struct TileMap {
  static constexpr bool kPair = std::is_same<TV, c64>::value && (EPT % 2 == 0);
  __device__ static int off(int q, int lane) { return kPair ? 128 * (q >> 1) + 2 * lane + (q & 1) : 64 * q + lane; }
};

typedef float flt4 __attribute__((ext_vector_type(4)));

// A basis row is always stored over its whole tile, with zeros at unknowns
// >= N (st_row), so a tile can be loaded without bounds checks or selects.

// One basis vector's slice (row = the tile's base) as loaded, in the storage
// precision; get(q) is the value of register q of the tile map in complex128.
// Keeping a prefetched trip in this form halves its registers for the
// complex64 basis.
template <int EPT, typename TV, bool PAIR = TileMap<EPT, TV>::kPair>
struct RawRow {
  c128 v[EPT];
  __device__ void load(const TV* __restrict__ row, int lane) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) v[q] = ld_basis(row + 64 * q + lane);
  }
  __device__ c128 get(int q) const { return v[q]; }
};
template <int EPT>
struct RawRow<EPT, c64, true> {
  flt4 v[EPT / 2];
  __device__ void load(const c64* __restrict__ row, int lane) {
#pragma unroll
    for (int p = 0; p < EPT / 2; ++p)
      v[p] = __builtin_nontemporal_load(reinterpret_cast<const flt4*>(row + 128 * p + 2 * lane));
  }
  __device__ c128 get(int q) const {
    const flt4 t = v[q >> 1];
    return (q & 1) ? c128{(double)t.z, (double)t.w} : c128{(double)t.x, (double)t.y};
  }
};

template <int EPT, typename TV>
__device__ inline void ld_row(const TV* __restrict__ row, int lane, c128 (&x)[EPT]) {
  RawRow<EPT, TV> r;
  r.load(row, lane);
#pragma unroll
  for (int q = 0; q < EPT; ++q) x[q] = r.get(q);
}

// Store a slice in the tile map (values already in the storage precision),
// the whole tile: entries at unknowns >= N must hold zero.
template <int EPT, typename TV>
__device__ inline void st_row(TV* __restrict__ row, int lane, const c128 (&v)[EPT]) {
  if constexpr (TileMap<EPT, TV>::kPair) {
#pragma unroll
    for (int p = 0; p < EPT / 2; ++p) {
      const flt4 t = {(float)v[2 * p].x, (float)v[2 * p].y, (float)v[2 * p + 1].x, (float)v[2 * p + 1].y};
      *reinterpret_cast<flt4*>(row + 128 * p + 2 * lane) = t;
    }
  } else {
#pragma unroll
    for (int q = 0; q < EPT; ++q) st_basis(row + 64 * q + lane, v[q]);
  }
}

// acc += conj(v) * u  (re, im)
__device__ inline void cdot_acc(double& re, double& im, c128 v, c128 u) {
  re = fma(v.x, u.x, re);
  re = fma(v.y, u.y, re);
  im = fma(v.x, u.y, im);
  im = fma(-v.y, u.x, im);
}

// ---------------------------------------------------------------- dot pass
// The dot pass splits the basis rows into gridDim.y chunks of a multiple of
// 64 rows.  With whole rows per block a launch holds only as many blocks as
// tiles: too few to fill the chip on small grids, and at sizes just above a
// power of two a few more than fit at once, so the last partial round of
// blocks streams at a fraction of the bandwidth.  Chunks make the rounds many
// and the partial one small.  A block's sums per (tile, row) are the same
// whatever the chunking.
__host__ __device__ inline int dot_chunk_rows(int maxit, int chunks) {
  return 64 * ((maxit + 64 * chunks - 1) / (64 * chunks));
}
// chunks for a launch of `blocks` tile blocks: 64 rows per chunk below 512
// blocks, up to 256 rows from 1024 blocks
inline int dot_chunks(int blocks, int maxit) {
  const int rows = 64 * std::min(4, std::max(1, blocks / 256));
  return (maxit + rows - 1) / rows;
}

// Each wave owns 64*EPT consecutive unknowns; lane l handles l, l+64, ...
template <int EPT, int RPI, typename TV>
__global__ void __launch_bounds__(AWG) arn_dots_kernel(ArnBatch bt) {
  HS_ARN_BLOCK(bt);
  if (a.st->done) return;
  const int k = a.st->k;
  // rows [r_lo, r_hi) of V; the first chunk also stores Z[k], W and the
  // u^H u, u^H w partials
  const int rows = dot_chunk_rows(bt.maxit, (int)gridDim.y);  // as the launch chose the chunks
  const int r_lo = (int)blockIdx.y * rows;
  if (blockIdx.y > 0 && r_lo >= k) return;  // block-uniform
  const int r_hi = min(k, r_lo + rows);
  const bool lead = blockIdx.y == 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wave = blk * WPB + wv;
  const bool active = wave < a.nw;  // idle waves stay for the block barriers
  const int64_t N = a.N;
  const int M = a.maxit;
  using TM = TileMap<EPT, TV>;
  const int64_t base = (int64_t)wave * (64 * EPT);
  c128 u[EPT], w[EPT];
  double uu = 0.0, uwx = 0.0, uwy = 0.0;
  c128* __restrict__ Zk = a.Z + (int64_t)k * N;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int64_t e = base + TM::off(q, lane);
    if (active && e < N) {
      u[q] = a.U[e];
      w[q] = spmv_at(a.P, a.Zc, e);
      if (lead) {
        st_stream(Zk + e, a.Zc[e]);  // read again only by x = Z y
        a.W[e] = w[q];
      }
    } else {
      u[q] = {0.0, 0.0};
      w[q] = {0.0, 0.0};
    }
    uu = fma(u[q].x, u[q].x, fma(u[q].y, u[q].y, uu));
    cdot_acc(uwx, uwy, u[q], w[q]);
  }
  uu = bfly(uu);
  uwx = bfly(uwx);
  uwy = bfly(uwy);
  // Partials live in one slab per block: c128 entry 2i is s_i, 2i+1 is t_i,
  // 2M and 2M+1 are u^H u and u^H w.  Each trip reduces 4 RPI values over
  // the wave; lane l keeps the one of trip l % SPAN, so every 16 rows the
  // 64 lanes hold 64 consecutive doubles of the slab.  Every 64 rows the
  // four waves add theirs in LDS (in wave order) and wave 0 stores 2 KB.
  __shared__ double lds[WPB][256];
  __shared__ double red[WPB][3];
  double* __restrict__ slab = reinterpret_cast<double*>(a.part + (int64_t)blk * (2 * M + 2));
  if (lead) {  // block-uniform
    if (lane == 0) {
      red[wv][0] = uu;
      red[wv][1] = uwx;
      red[wv][2] = uwy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s0 = red[0][0], s1 = red[0][1], s2 = red[0][2];
      for (int q = 1; q < WPB; ++q) {
        s0 += red[q][0];
        s1 += red[q][1];
        s2 += red[q][2];
      }
      slab[4 * (int64_t)M + 0] = s0;
      slab[4 * (int64_t)M + 1] = 0.0;
      slab[4 * (int64_t)M + 2] = s1;
      slab[4 * (int64_t)M + 3] = s2;
    }
  }
  constexpr int SPAN = 64 / (4 * RPI);   // lanes per reduced value = trips per 16 rows
  const int g = lane % SPAN, idx = lane / SPAN;
  // Trip = RPI consecutive basis vectors of this wave's tile.  The next
  // trip's loads are issued before the current trip is reduced, so the
  // reduction overlaps memory latency; it is held as loaded (storage
  // precision) and converted at use.  Rows >= r_hi load row 0 instead
  // (always allocated; stored once k > 0); their sums are never stored.
  // Unknowns >= N hold zero in the basis and in u, w, so no selection is
  // needed.
  constexpr int TW = 64 * EPT;
  const TV* __restrict__ vt = static_cast<const TV*>(a.V) + (int64_t)wave * M * TW;
  auto load_trip = [&](int i, RawRow<EPT, TV> (&x)[RPI]) {
#pragma unroll
    for (int j = 0; j < RPI; ++j) x[j].load(i + j < r_hi ? vt + (int64_t)(i + j) * TW : vt, lane);
  };
  RawRow<EPT, TV> xc[RPI], xn[RPI];
  if (active) load_trip(r_lo, xc);
  for (int i0 = r_lo; i0 < r_hi; i0 += 64) {
    double keep[4] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
#pragma unroll
        for (int t = 0; t < SPAN; ++t) {
          const int i = i0 + 16 * f + t * RPI;
          if (i >= r_hi) break;  // wave-uniform
          load_trip(i + RPI, xn);
          double r[4 * RPI];
#pragma unroll
          for (int q = 0; q < 4 * RPI; ++q) r[q] = 0.0;
#pragma unroll
          for (int j = 0; j < RPI; ++j)
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
              const c128 x = xc[j].get(q);
              cdot_acc(r[4 * j + 0], r[4 * j + 1], x, u[q]);
              cdot_acc(r[4 * j + 2], r[4 * j + 3], x, w[q]);
            }
#pragma unroll
          for (int j = 0; j < RPI; ++j) xc[j] = xn[j];
          const double val = wave::sum<4 * RPI>(r, lane);
          if (g == t) keep[f] = val;
        }
      }
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) lds[wv][64 * f + lane] = keep[f];
    __syncthreads();
    if (wv == 0) {
      // lane (g, idx) of group f: row i0 + 16 f + g RPI + idx / 4, entry
      // 2 row + (idx / 2) % 2, component idx % 2 -> double 4 (i0 + 16 f) + 4 RPI g + idx
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const int ib = i0 + 16 * f;
        if (ib + g * RPI + (idx >> 2) < r_hi) {
          const int o = 64 * f + lane;
          slab[4 * (int64_t)ib + 4 * RPI * g + idx] = (lds[0][o] + lds[1][o]) + (lds[2][o] + lds[3][o]);
        }
      }
    }
    __syncthreads();
  }
}

// First level of the slab sums.  Block (x, c) takes 64 consecutive slab
// entries (one per lane; consecutive lanes read consecutive entries) and the
// c-th of FOLD_CHUNKS contiguous ranges of slabs; its four waves take
// quarters of that range and are added in order.  Result: fold[c][entry].
// The Hessenberg-column kernel adds the FOLD_CHUNKS values in order.
__global__ void __launch_bounds__(AWG) arn_fold_kernel(ArnBatch bt) {
  const ArnDev a = bt.tab[blockIdx.z];
  if (a.st->done) return;
  const int k = a.st->k, M = a.maxit;
  const int64_t ld = 2 * M + 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jb = blockIdx.x * 64;  // first entry of the block
  if (!(jb < 2 * k || jb + 63 >= 2 * M)) return;  // block-uniform: no live entry
  const int j = jb + lane;
  const bool live = j < 2 * k || j == 2 * M || j == 2 * M + 1;
  const int nb = stream_blocks(a);  // one slab per block of the dot pass
  const int per_chunk = (nb + FOLD_CHUNKS - 1) / FOLD_CHUNKS;
  const int c0 = blockIdx.y * per_chunk, c1 = min(nb, c0 + per_chunk);
  const int per_wave = (per_chunk + WPB - 1) / WPB;
  const int w0 = c0 + wv * per_wave, w1 = min(c1, w0 + per_wave);
  double x[4] = {0.0, 0.0, 0.0, 0.0}, y[4] = {0.0, 0.0, 0.0, 0.0};
  if (live) {
    const c128* __restrict__ p = a.part + j;
    int w = w0;
    for (; w + 4 <= w1; w += 4) {  // four independent chains keep loads in flight
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const c128 v = p[(int64_t)(w + q) * ld];
        x[q] += v.x;
        y[q] += v.y;
      }
    }
    for (; w < w1; ++w) {
      const c128 v = p[(int64_t)w * ld];
      x[0] += v.x;
      y[0] += v.y;
    }
  }
  __shared__ c128 acc[WPB][64];
  acc[wv][lane] = {(x[0] + x[1]) + (x[2] + x[3]), (y[0] + y[1]) + (y[2] + y[3])};
  __syncthreads();
  if (wv == 0 && live) {
    double sx = acc[0][lane].x, sy = acc[0][lane].y;
    for (int q = 1; q < WPB; ++q) {
      sx += acc[q][lane].x;
      sy += acc[q][lane].y;
    }
    a.fold[(int64_t)blockIdx.y * ld + j] = {sx, sy};
  }
}

// --------------------------------------------------------- Hessenberg column
// One block: reorthogonalisation norm, final column k-1 with its Givens
// rotation and the convergence test, first-pass entries of column k.
__global__ void __launch_bounds__(AWG) arn_column_kernel(ArnBatch bt) {
  const ArnDev a = bt.tab[blockIdx.x];
  ArnState* st = a.st;
  if (st->done) return;
  const int k = st->k, M = a.maxit;
  const int64_t ld = M + 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ double red[3][WPB];
  __shared__ int sh_done;
  {  // second level of the slab sums: the FOLD_CHUNKS partials in order
    const int64_t fl = 2 * M + 2;
    for (int j = tid; j < 2 * k + 2; j += AWG) {
      const int e = j < 2 * k ? j : 2 * M + (j - 2 * k);
      double sx = 0.0, sy = 0.0;
      for (int c = 0; c < FOLD_CHUNKS; ++c) {
        const c128 v = a.fold[(int64_t)c * fl + e];
        sx += v.x;
        sy += v.y;
      }
      const int out = e >= 2 * M ? e : ((e & 1) ? M + (e >> 1) : (e >> 1));
      a.dots[out] = {sx, sy};
    }
    __syncthreads();
  }
  double ss = 0.0, hx = 0.0, hy = 0.0;
  for (int i = tid; i < k; i += AWG) {
    const c128 s = a.dots[i], t = a.dots[M + i];
    ss = fma(s.x, s.x, fma(s.y, s.y, ss));
    cdot_acc(hx, hy, s, t);
  }
  ss = bfly(ss);
  hx = bfly(hx);
  hy = bfly(hy);
  if (lane == 0) {
    red[0][wv] = ss;
    red[1][wv] = hx;
    red[2][wv] = hy;
  }
  if (tid == 0) sh_done = 0;
  __syncthreads();
  ss = red[0][0];
  hx = red[1][0];
  hy = red[2][0];
  for (int q = 1; q < WPB; ++q) {
    ss += red[0][q];
    hx += red[1][q];
    hy += red[2][q];
  }
  const double uu = a.dots[2 * M].x;
  const c128 uw = a.dots[2 * M + 1];
  const double a2 = uu - ss;
  const double alpha = a2 > 0.0 ? sqrt(a2) : 0.0;

  if (k >= 1) {
    const double beta = st->beta;
    c128* __restrict__ col = a.R + (int64_t)(k - 1) * ld;
    for (int i = tid; i < k; i += AWG) {
      const c128 s = a.dots[i];
      col[i].x = fma(beta, s.x, col[i].x);
      col[i].y = fma(beta, s.y, col[i].y);
    }
    __syncthreads();
    if (wv == 0) {
      // previous rotations 0..k-2 in order.  The chain is wave-uniform: each
      // chunk of 64 rotation parameters (and the column entries they act on)
      // is fetched by the 64 lanes into LDS, then every lane walks the chunk
      // reading them as broadcasts, which do not depend on the chain, so
      // only the rotation arithmetic itself is serial.
      __shared__ double rc_s[64];
      __shared__ c128 rs_s[64], rb_s[64], ro_s[64];
      c128 av = col[0];
      for (int b0 = 0; b0 < k - 1; b0 += 64) {
        const int i = b0 + lane;
        const int cnt = min(64, k - 1 - b0);
        if (i < k - 1) {
          rc_s[lane] = a.cs[i];
          rs_s[lane] = a.sn[i];
          rb_s[lane] = col[i + 1];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 8
        for (int q = 0; q < cnt; ++q) {
          const double c = rc_s[q];
          const c128 sq = rs_s[q];
          const c128 bq = rb_s[q];
          // (a, b) <- (c a + s b, -conj(s) a + c b)
          const c128 na = {c * av.x + (sq.x * bq.x - sq.y * bq.y), c * av.y + (sq.x * bq.y + sq.y * bq.x)};
          const c128 nb = {c * bq.x - (sq.x * av.x + sq.y * av.y), c * bq.y - (sq.x * av.y - sq.y * av.x)};
          if (lane == 0) ro_s[q] = na;
          av = nb;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (i < k - 1) col[i] = ro_s[lane];
        // the next chunk overwrites the LDS arrays only after every lane has
        // read its output entry
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // new rotation k-1 zeroing the subdiagonal beta * alpha
      const c128 bv = {beta * alpha, 0.0};
      double c;
      c128 sr;
      const double na = sqrt(av.x * av.x + av.y * av.y);
      if (na == 0.0) {
        c = 0.0;
        sr = {1.0, 0.0};
      } else {
        const double nrm = hypot(na, sqrt(bv.x * bv.x + bv.y * bv.y));
        c = na / nrm;
        const c128 ph = {av.x / na, av.y / na};
        sr = {(ph.x * bv.x + ph.y * bv.y) / nrm, (ph.y * bv.x - ph.x * bv.y) / nrm};
      }
      const c128 rkk = {c * av.x + (sr.x * bv.x - sr.y * bv.y), c * av.y + (sr.x * bv.y + sr.y * bv.x)};
      const c128 gp = a.g[k - 1];
      const c128 gk = {-(sr.x * gp.x + sr.y * gp.y), -(sr.x * gp.y - sr.y * gp.x)};
      if (lane == 0) {
        col[k - 1] = rkk;
        col[k] = {0.0, 0.0};
        a.cs[k - 1] = c;
        a.sn[k - 1] = sr;
        a.g[k - 1] = {c * gp.x, c * gp.y};
        a.g[k] = gk;
        const double res = sqrt(gk.x * gk.x + gk.y * gk.y);
        const double rel = res / st->beta0;
        a.hist[k] = rel;
        st->relres = rel;
        st->m = k;
        int d = 0;
        if (!isfinite(res) || !isfinite(alpha) || !isfinite(beta) || !isfinite(rkk.x) || !isfinite(rkk.y))
          d = -1;
        else if (res <= st->tol_abs)
          d = 1;
        else if (k >= st->maxit)  // the iteration limit of this cycle (<= M)
          d = 3;
        st->done = d;
        sh_done = d;
      }
    }
  } else if (tid == 0) {
    a.g[0] = {st->beta0 * alpha, 0.0};
    if (!isfinite(alpha)) {
      st->done = -1;
      sh_done = -1;
    }
  }
  __syncthreads();
  // Column k is written even when the stop test has just fired: if the host's
  // true-residual check rejects the stop, it resumes with step k's update.
  if (sh_done < 0 || k >= M) return;
  if (!(alpha > 0.0)) {  // u_k in the span of V (a zero right-hand side is caught on the host)
    if (tid == 0 && sh_done == 0) {
      st->done = 2;
      st->m = k;
    }
    return;
  }
  // first-pass entries of column k
  const c128 c = {(uw.x - hx) / alpha, (uw.y - hy) / alpha};
  c128* __restrict__ colk = a.R + (int64_t)k * ld;
  for (int i = tid; i < k; i += AWG) colk[i] = a.dots[M + i];
  if (tid == 0) {
    colk[k] = c;
    st->alpha = alpha;
    st->c = c;
  }
}

// ------------------------------------------------------------- update pass
// v_k = (u_k - V s) / alpha -> V[k];  w1 = w - V t - c v_k -> U;  ||w1||^2
template <int EPT, int RPI, typename TV>
__global__ void __launch_bounds__(AWG) arn_update_kernel(ArnBatch bt) {
  HS_ARN_BLOCK(bt);
  const ArnState* st = a.st;
  if (st->done) return;
  const int k = st->k, M = a.maxit;
  const double inv = 1.0 / st->alpha;
  const c128 c = st->c;
  const int lane = threadIdx.x & 63;
  const int wave = blk * WPB + (threadIdx.x >> 6);
  if (wave >= a.nw) return;
  const int64_t N = a.N;
  using TM = TileMap<EPT, TV>;
  const int64_t base = (int64_t)wave * (64 * EPT);
  c128 av[EPT], aw[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int64_t e = base + TM::off(q, lane);
    av[q] = e < N ? a.U[e] : c128{0.0, 0.0};
    aw[q] = e < N ? a.W[e] : c128{0.0, 0.0};
  }
  constexpr int TW = 64 * EPT;  // tile-major basis, as in the dot pass
  TV* __restrict__ vt = static_cast<TV*>(a.V) + (int64_t)wave * M * TW;
  for (int i = 0; i < k; i += RPI) {
    const TV* __restrict__ vi = vt + (int64_t)i * TW;
    const int nr = min(RPI, k - i);  // wave-uniform
    if (nr == RPI) {
      c128 x[RPI][EPT];
#pragma unroll
      for (int j = 0; j < RPI; ++j) ld_row<EPT, TV>(vi + j * TW, lane, x[j]);
#pragma unroll
      for (int j = 0; j < RPI; ++j) {
        const c128 sj = a.dots[i + j], tj = a.dots[M + i + j];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          cfms(av[q], x[j][q], sj);
          cfms(aw[q], x[j][q], tj);
        }
      }
    } else {
      for (int j = 0; j < nr; ++j) {
        const c128 sj = a.dots[i + j], tj = a.dots[M + i + j];
        c128 x[EPT];
        ld_row<EPT, TV>(vi + j * TW, lane, x);
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          cfms(av[q], x[q], sj);
          cfms(aw[q], x[q], tj);
        }
      }
    }
  }
  TV* __restrict__ Vk = vt + (int64_t)k * TW;
  // v_k as stored; w1 is orthogonalised against the stored vector, so the
  // process is DCGS2 over the basis the next passes read
  c128 v[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) v[q] = to_basis({av[q].x * inv, av[q].y * inv}, Vk);
  st_row<EPT, TV>(Vk, lane, v);  // zero at unknowns >= N (av is zero there)
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int64_t e = base + TM::off(q, lane);
    if (e < N) {
      c128 w1 = aw[q];
      cfms(w1, c, v[q]);
      a.U[e] = w1;
      nrm = fma(w1.x, w1.x, fma(w1.y, w1.y, nrm));
    }
  }
  nrm = bfly(nrm);
  if (lane == 0) a.pn[wave] = nrm;
}

// beta_k = ||w1|| (every block folds the partials in the same order);
// u_{k+1} = w1 / beta_k; block 0 advances the step.
template <int EPT>
__global__ void __launch_bounds__(AWG) arn_scale_kernel(ArnBatch bt) {
  HS_ARN_BLOCK(bt);
  ArnState* st = a.st;
  if (st->done) return;
  __shared__ double red[WPB];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double s = 0.0;
  for (int q = threadIdx.x; q < a.nw; q += AWG) s += a.pn[q];
  s = bfly(s);
  if (lane == 0) red[wv] = s;
  __syncthreads();
  double tot = red[0];
  for (int q = 1; q < WPB; ++q) tot += red[q];
  const double beta = sqrt(tot);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int wave = blk * WPB + wv;
  if (wave < a.nw) {
    const int64_t e0 = (int64_t)wave * (64 * EPT) + lane;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int64_t e = e0 + 64 * q;
      if (e < a.N) {
        const c128 w = a.U[e];
        a.U[e] = {w.x * inv, w.y * inv};
      }
    }
  }
  if (blk == 0 && threadIdx.x == 0) {
    st->beta = beta;
    if (!isfinite(beta)) st->done = -1;
    st->k = st->k + 1;
  }
}

// basis vectors 0..k-1 := r in the tile-major layout (timing helper)
template <int EPT, typename TV>
__global__ void __launch_bounds__(AWG) arn_fill_basis_kernel(ArnBatch bt, const c128* __restrict__ r, int k) {
  HS_ARN_BLOCK(bt);
  constexpr int TW = 64 * EPT;
  const int lane = threadIdx.x & 63;
  const int wave = blk * WPB + (threadIdx.x >> 6);
  if (wave >= a.nw) return;
  const int64_t base = (int64_t)wave * TW;
  TV* __restrict__ vt = static_cast<TV*>(a.V) + (int64_t)wave * a.maxit * TW;
  c128 v[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int64_t e = base + TileMap<EPT, TV>::off(q, lane);
    v[q] = e < a.N ? r[e] : c128{0.0, 0.0};
  }
  for (int i = 0; i < k; ++i) st_row<EPT, TV>(vt + (int64_t)i * TW, lane, v);
}

__global__ void arn_init_kernel(ArnDev a, double beta0, double tol_abs, int limit) {
  ArnState* st = a.st;
  st->k = 0;
  st->done = 0;
  st->m = 0;
  st->maxit = limit;
  st->beta0 = beta0;
  st->tol_abs = tol_abs;
  st->beta = beta0;
  st->alpha = 1.0;
  st->c = {0.0, 0.0};
  st->relres = 1.0;
  st->pad = 0.0;
  a.hist[0] = 1.0;
}

__global__ void arn_resume_kernel(ArnDev a) { a.st->done = 0; }

__global__ void arn_set_done_kernel(ArnDev a, int code) { a.st->done = code; }

__global__ void arn_set_step_kernel(ArnDev a, int k) {
  a.st->k = k;
  a.st->done = 0;
  a.st->alpha = 1.0;
  a.st->c = {0.0, 0.0};
}

// y = R^{-1} g on the first m columns, column-oriented back substitution
__global__ void __launch_bounds__(AWG) arn_backsub_kernel(ArnDev a, int m) {
  const int64_t ld = a.maxit + 1;
  __shared__ c128 yi_s;
  for (int i = threadIdx.x; i < m; i += AWG) a.y[i] = a.g[i];
  __syncthreads();
  for (int i = m - 1; i >= 0; --i) {
    const c128* __restrict__ col = a.R + (int64_t)i * ld;
    if (threadIdx.x == 0) {
      const c128 yi = cmul(a.y[i], cinv(col[i]));
      a.y[i] = yi;
      yi_s = yi;
    }
    __syncthreads();
    const c128 yi = yi_s;
    for (int q = threadIdx.x; q < i; q += AWG) {
      c128 t = a.y[q];
      cfms(t, col[q], yi);
      a.y[q] = t;
    }
    __syncthreads();
  }
}

}  // namespace

// Built-in shape: the widest tile that still gives >= 16 waves per CU
// (4096 waves; at 1,050,625 unknowns that is 4, what the autotuner picks on
// MI355X there).
int arn_ept(int64_t N) {
  // the widest tile (at most 4 unknowns per lane: wider tiles stream slower
  // from the tile-major basis) that still gives 4096 waves
  for (int e : {4, 2})
    if ((N + 64 * e - 1) / (64 * e) >= 4096) return e;
  return 1;
}

// Launch shapes chosen per problem size (by the autotuner or by hand); the
// built-in choice otherwise.  The elements per lane fix the partition of the
// dot products, so a solve is reproducible for a fixed table.
namespace {
std::mutex g_cfg_mu;
std::map<int64_t, std::pair<int, int>> g_cfg;
}  // namespace

void arn_config(int64_t N, int* ept, int* rpi) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  const auto it = g_cfg.find(N);
  if (it != g_cfg.end()) {
    *ept = it->second.first;
    *rpi = it->second.second;
  } else {
    *ept = arn_ept(N);
    *rpi = 2;
  }
}

void arn_set_config(int64_t N, int ept, int rpi) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  if (ept == 0 && rpi == 0)
    g_cfg.erase(N);
  else
    g_cfg[N] = {ept, rpi};
}
int arn_stream_blocks(int nw) { return (nw + WPB - 1) / WPB; }
int arn_waves(int64_t N, int ept) { return (int)((N + 64 * (int64_t)ept - 1) / (64 * (int64_t)ept)); }

#define HS_ARN_EPT(KERNEL)                                                         \
  switch (b.ept) {                                                                 \
    case 8: KERNEL<8><<<b.blocks, AWG, 0, s>>>(b); break;                          \
    case 4: KERNEL<4><<<b.blocks, AWG, 0, s>>>(b); break;                          \
    case 2: KERNEL<2><<<b.blocks, AWG, 0, s>>>(b); break;                          \
    case 1: KERNEL<1><<<b.blocks, AWG, 0, s>>>(b); break;                          \
    default: throw Failure{HS_EINVAL, "unsupported elements per lane"};            \
  }                                                                                \
  HS_HIP(hipGetLastError())

#define HS_ARN_EPT_RPI_CASE(KERNEL, E, TV, GRID)                                   \
  case E:                                                                          \
    if (b.rpi == 4)                                                                \
      KERNEL<E, 4, TV><<<GRID, AWG, 0, s>>>(b);                                    \
    else                                                                           \
      KERNEL<E, 2, TV><<<GRID, AWG, 0, s>>>(b);                                    \
    break;

#define HS_ARN_EPT_RPI_T(KERNEL, TV, GRID)                                         \
  switch (b.ept) {                                                                 \
    HS_ARN_EPT_RPI_CASE(KERNEL, 8, TV, GRID)                                       \
    HS_ARN_EPT_RPI_CASE(KERNEL, 4, TV, GRID)                                       \
    HS_ARN_EPT_RPI_CASE(KERNEL, 2, TV, GRID)                                       \
    HS_ARN_EPT_RPI_CASE(KERNEL, 1, TV, GRID)                                       \
    default: throw Failure{HS_EINVAL, "unsupported elements per lane"};            \
  }

// shape and basis storage type of the two streaming passes
#define HS_ARN_EPT_RPI(KERNEL, GRID)                                                    \
  HS_REQUIRE(b.rpi == 2 || b.rpi == 4, "rows per trip must be 2 or 4");            \
  HS_REQUIRE(b.vprec == HS_C128 || b.vprec == HS_C64, "basis precision must be HS_C128 or HS_C64"); \
  if (b.vprec == HS_C64) {                                                         \
    HS_ARN_EPT_RPI_T(KERNEL, c64, GRID)                                              \
  } else {                                                                         \
    HS_ARN_EPT_RPI_T(KERNEL, c128, GRID)                                             \
  }                                                                                \
  HS_HIP(hipGetLastError())

void k_arn_init(const ArnDev& a, double beta0, double tol_abs, hipStream_t s, int limit) {
  arn_init_kernel<<<1, 1, 0, s>>>(a, beta0, tol_abs, limit > 0 ? std::min(limit, a.maxit) : a.maxit);
  HS_HIP(hipGetLastError());
}
void k_arn_dots(const ArnBatch& b, hipStream_t s) {
  HS_ARN_EPT_RPI(arn_dots_kernel, dim3(b.blocks, dot_chunks(b.blocks, b.maxit)));
}
template <typename TV>
void fill_basis(const ArnBatch& b, const c128* r, int k, hipStream_t s) {
  switch (b.ept) {
    case 8: arn_fill_basis_kernel<8, TV><<<b.blocks, AWG, 0, s>>>(b, r, k); break;
    case 4: arn_fill_basis_kernel<4, TV><<<b.blocks, AWG, 0, s>>>(b, r, k); break;
    case 2: arn_fill_basis_kernel<2, TV><<<b.blocks, AWG, 0, s>>>(b, r, k); break;
    case 1: arn_fill_basis_kernel<1, TV><<<b.blocks, AWG, 0, s>>>(b, r, k); break;
    default: throw Failure{HS_EINVAL, "unsupported elements per lane"};
  }
  HS_HIP(hipGetLastError());
}
void k_arn_fill_basis(const ArnBatch& b, const c128* r, int k, hipStream_t s) {
  if (b.vprec == HS_C64)
    fill_basis<c64>(b, r, k, s);
  else
    fill_basis<c128>(b, r, k, s);
}
void k_arn_fold(const ArnBatch& b, hipStream_t s) {
  arn_fold_kernel<<<dim3((2 * b.maxit + 2 + 63) / 64, FOLD_CHUNKS, b.count), AWG, 0, s>>>(b);
  HS_HIP(hipGetLastError());
}
void k_arn_column(const ArnBatch& b, hipStream_t s) {
  arn_column_kernel<<<b.count, AWG, 0, s>>>(b);
  HS_HIP(hipGetLastError());
}
void k_arn_update(const ArnBatch& b, hipStream_t s) { HS_ARN_EPT_RPI(arn_update_kernel, b.blocks); }
void k_arn_scale(const ArnBatch& b, hipStream_t s) { HS_ARN_EPT(arn_scale_kernel); }
void k_arn_resume(const ArnDev& a, hipStream_t s) {
  arn_resume_kernel<<<1, 1, 0, s>>>(a);
  HS_HIP(hipGetLastError());
}
void k_arn_set_done(const ArnDev& a, int code, hipStream_t s) {
  arn_set_done_kernel<<<1, 1, 0, s>>>(a, code);
  HS_HIP(hipGetLastError());
}
void k_arn_set_step(const ArnDev& a, int k, hipStream_t s) {
  arn_set_step_kernel<<<1, 1, 0, s>>>(a, k);
  HS_HIP(hipGetLastError());
}
void k_arn_backsub(const ArnDev& a, int m, hipStream_t s) {
  arn_backsub_kernel<<<1, AWG, 0, s>>>(a, m);
  HS_HIP(hipGetLastError());
}

}  // namespace hs
