// Arnoldi / modified Gram-Schmidt building blocks for flexible GMRES
// (Sec. 5: GMRES to a relative tolerance), all complex128.
//
// Reductions are deterministic: every block folds its grid-stride share in a
// fixed order (thread -> wave shuffles -> LDS), writes one partial, and the
// next kernel re-folds the KRED partials in index order before using the
// value.  No atomics, so two runs are bitwise identical.
#include "hs_internal.h"

namespace hs {

constexpr int KRED = 512;  // blocks of every reduction kernel
constexpr int KWG = 256;

namespace {

template <typename X>
__device__ inline X block_sum(X v, X* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  X s = red[0];
  for (int w = 1; w < KWG / 64; ++w) s += red[w];
  return s;
}

// Fold the KRED partials of the previous kernel: every block sums them in the
// same fixed order (strided per thread, then the block tree), so every block
// obtains the same value.
__device__ inline c128 fold(const c128* __restrict__ partial) {
  __shared__ double fx_s[KWG / 64], fy_s[KWG / 64];
  double fx = 0.0, fy = 0.0;
  for (int b = threadIdx.x; b < KRED; b += KWG) {
    fx += partial[b].x;
    fy += partial[b].y;
  }
  fx = block_sum(fx, fx_s);
  fy = block_sum(fy, fy_s);
  return {fx, fy};
}

__device__ inline double fold_re(const double* __restrict__ partial) {
  __shared__ double f_s[KWG / 64];
  double f = 0.0;
  for (int b = threadIdx.x; b < KRED; b += KWG) f += partial[b];
  return block_sum(f, f_s);
}

// partial[blk] = sum conj(a) b
__global__ void __launch_bounds__(KWG) dot_kernel(int64_t n, const c128* __restrict__ a, const c128* __restrict__ b,
                                                  c128* __restrict__ partial) {
  __shared__ double rx[KWG / 64], ry[KWG / 64];
  double sx = 0.0, sy = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * KWG + threadIdx.x; i < n; i += (int64_t)KRED * KWG) {
    const c128 u = a[i], v = b[i];
    sx += u.x * v.x + u.y * v.y;
    sy += u.x * v.y - u.y * v.x;
  }
  sx = block_sum(sx, rx);
  sy = block_sum(sy, ry);
  if (threadIdx.x == 0) partial[blockIdx.x] = {sx, sy};
}

// One modified Gram-Schmidt projection step, fused with the dot product of
// the next one:  h = fold(pprev);  w -= h vprev;  pout = sum conj(vcur) w
// (or the |w|^2 partials into pnorm when vcur == nullptr).  With z != nullptr
// the kernel first forms w = A z (the Arnoldi mat-vec) instead of reading w.
// Block 0 stores h to hout.
__global__ void __launch_bounds__(KWG) mgs_kernel(ProblemDev P, const c128* __restrict__ z, int64_t n,
                                                  c128* __restrict__ w, const c128* __restrict__ vprev,
                                                  const c128* __restrict__ pprev, c128* __restrict__ hout,
                                                  const c128* __restrict__ vcur, c128* __restrict__ pout,
                                                  double* __restrict__ pnorm) {
  __shared__ double rx[KWG / 64], ry[KWG / 64];
  c128 h = {0.0, 0.0};
  if (vprev) {
    h = fold(pprev);
    if (blockIdx.x == 0 && threadIdx.x == 0) *hout = h;
  }
  double sx = 0.0, sy = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * KWG + threadIdx.x; i < n; i += (int64_t)KRED * KWG) {
    c128 v = z ? spmv_at(P, z, i) : w[i];
    if (vprev) cfms(v, h, vprev[i]);
    if (z || vprev) w[i] = v;
    if (vcur) {
      const c128 u = vcur[i];
      sx += u.x * v.x + u.y * v.y;
      sy += u.x * v.y - u.y * v.x;
    } else {
      sx += v.x * v.x + v.y * v.y;
    }
  }
  sx = block_sum(sx, rx);
  sy = block_sum(sy, ry);
  if (threadIdx.x == 0) {
    if (vcur)
      pout[blockIdx.x] = {sx, sy};
    else
      pnorm[blockIdx.x] = sx;
  }
}

// norm^2 partials
__global__ void __launch_bounds__(KWG) norm2_kernel(int64_t n, const c128* __restrict__ a, double* __restrict__ pnorm) {
  __shared__ double rx[KWG / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * KWG + threadIdx.x; i < n; i += (int64_t)KRED * KWG) {
    const c128 u = a[i];
    s += u.x * u.x + u.y * u.y;
  }
  s = block_sum(s, rx);
  if (threadIdx.x == 0) pnorm[blockIdx.x] = s;
}

// nrm = sqrt(fold(pnorm)); out = in / nrm (unless nrm == 0); block 0 stores nrm
__global__ void __launch_bounds__(KWG) scale_kernel(int64_t n, const c128* __restrict__ in, c128* __restrict__ out,
                                                    const double* __restrict__ pnorm, double* __restrict__ nrm_out) {
  const double nrm = sqrt(fold_re(pnorm));
  if (blockIdx.x == 0 && threadIdx.x == 0) *nrm_out = nrm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * KWG + threadIdx.x; i < n; i += (int64_t)KRED * KWG) {
    const c128 u = in[i];
    out[i] = {u.x * inv, u.y * inv};
  }
}

// x = sum_{i<m} y_i Z_i (Z rows of length n, stride ld)
// x = x0 + sum_q y_q Z_q  (x0 == nullptr: zero)
__global__ void __launch_bounds__(KWG) combo_kernel(int64_t n, int m, const c128* __restrict__ y,
                                                    const c128* __restrict__ Z, int64_t ld, const c128* x0,
                                                    c128* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * KWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * KWG) {
    c128 acc = x0 ? x0[i] : c128{0.0, 0.0};
    for (int q = 0; q < m; ++q) cfma(acc, y[q], Z[(int64_t)q * ld + i]);
    x[i] = acc;
  }
}

// r = b - r  (r holds A x on entry)
__global__ void __launch_bounds__(KWG) bminus_kernel(int64_t n, const c128* __restrict__ b, c128* __restrict__ r) {
  for (int64_t i = (int64_t)blockIdx.x * KWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * KWG)
    r[i] = csub(b[i], r[i]);
}

__global__ void __launch_bounds__(KWG) fold_norm_kernel(const double* __restrict__ pnorm, double* __restrict__ out) {
  const double f = fold_re(pnorm);
  if (threadIdx.x == 0) *out = sqrt(f);
}

}  // namespace

void k_dot(int64_t n, const c128* a, const c128* b, c128* partial, hipStream_t s) {
  dot_kernel<<<KRED, KWG, 0, s>>>(n, a, b, partial);
  HS_HIP(hipGetLastError());
}
void k_mgs(const ProblemDev& P, const c128* z, int64_t n, c128* w, const c128* vprev, const c128* pprev, c128* hout,
           const c128* vcur, c128* pout, double* pnorm, hipStream_t s) {
  mgs_kernel<<<KRED, KWG, 0, s>>>(P, z, n, w, vprev, pprev, hout, vcur, pout, pnorm);
  HS_HIP(hipGetLastError());
}
void k_norm2(int64_t n, const c128* a, double* pnorm, hipStream_t s) {
  norm2_kernel<<<KRED, KWG, 0, s>>>(n, a, pnorm);
  HS_HIP(hipGetLastError());
}
void k_scale(int64_t n, const c128* in, c128* out, const double* pnorm, double* nrm_out, hipStream_t s) {
  scale_kernel<<<KRED, KWG, 0, s>>>(n, in, out, pnorm, nrm_out);
  HS_HIP(hipGetLastError());
}
void k_combo(int64_t n, int m, const c128* y, const c128* Z, int64_t ld, c128* x, hipStream_t s, const c128* x0) {
  combo_kernel<<<1024, KWG, 0, s>>>(n, m, y, Z, ld, x0, x);
  HS_HIP(hipGetLastError());
}
void k_bminus(int64_t n, const c128* b, c128* r, hipStream_t s) {
  bminus_kernel<<<1024, KWG, 0, s>>>(n, b, r);
  HS_HIP(hipGetLastError());
}
void k_fold_norm(const double* pnorm, double* out, hipStream_t s) {
  fold_norm_kernel<<<1, KWG, 0, s>>>(pnorm, out);
  HS_HIP(hipGetLastError());
}
int k_red_blocks() { return KRED; }

}  // namespace hs
