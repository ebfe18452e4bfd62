// Local subdomain factorisation and solves (Sec. 3: exact local solves with
// A_i = R_i A R_i^T, Dirichlet on the artificial boundary).
//
// With x-fastest ordering a subdomain matrix of nx x ny nodes is block
// tridiagonal: diagonal blocks D_j (one grid line, tridiagonal nx x nx) and
// diagonal couplings E_j = A[line j, line j-1], F_j = A[line j, line j+1].
// Block LU gives Schur blocks S_0 = D_0, S_j = D_j - E_j S_{j-1}^{-1} F_{j-1};
// the factor stores G_j = S_j^{-1} (dense, nx x nx), obtained by in-place
// Gauss-Jordan with partial (row) pivoting inside each Schur block.  A solve
// is then two sweeps of dense nx x nx mat-vecs:
//   forward  t_j = G_j (b_j - E_j t_{j-1})
//   backward x_j = t_j - G_j (F_j x_{j+1})
// which read every G_j twice: the same bytes as a band LU with the lean
// (2p+1) layout, but as coalesced dense mat-vecs instead of a row-by-row
// dependency chain.  One workgroup per subdomain; all subdomains in one launch.
//
// Factor layout (per grid line, TPR = 4 threads per row): row r is split into
// TPR contiguous column segments of cseg = ceil(nx/TPR); thread t = r*TPR + s
// owns segment s, and the entry (r, s*cseg + q) is stored at q*(TPR*nx) + t
// (zero where the column is past nx).  A solve step therefore issues cseg
// loads per thread, each of which is one contiguous TPR*nx-wide sweep.
// Complex64 factors are stored in pairs: entries q = 2p and 2p + 1 of thread
// t sit side by side at p*(2*TPR*nx) + 2t + (q & 1), so a solve step loads 16
// bytes per thread (one dwordx4) instead of 8; when cseg is odd the last
// segment row follows the pairs unpaired (entry (cseg-1)*TPR*nx + t, one
// 8-byte load).  Either way a line holds exactly cseg*TPR*nx entries, and a
// solve step issues loads for exactly the line's cseg segment rows: the
// solve is instantiated per segment count and each subdomain takes its own.
#include <algorithm>
#include <mutex>
#include <vector>

#include "hs_internal.h"
#include "hs_wave.h"

namespace hs {

namespace {

constexpr int WG = 256;
constexpr int TPR = 4;      // threads per row in the solve (one quad: the row sums use DPP)
constexpr int CSEG_MAX = 24; // nx <= TPR * CSEG_MAX = 96

// rows of thread segments stored per grid line (either layout)
__host__ __device__ inline int line_rows(int nx) { return (nx + TPR - 1) / TPR; }

template <typename T>
__device__ inline cplx<T> to_t(c128 v) {
  return {(T)v.x, (T)v.y};
}

// ------------------------------------------------------------ factor
// Each Schur block is inverted in place by Gauss-Jordan with partial row
// pivoting and row swaps, blocked FNB = 8 pivots at a time (the scheme of the
// coarse fronts, in LDS):
//  (1) one wave runs the panel's pivot steps on the panel columns of the rows
//      not pivoted yet, held in registers (pivot = largest modulus, lowest
//      row on ties; the pivot row swaps into place, in LDS too); Y = the
//      pivot rows' final panel values;
//  (2) YZ = Y M[C, :] from the pivot rows as they were;
//  (3) M[i][j] -= M[i][C] YZ[:, j] for the rows and columns outside the panel,
//      in 16 x 16 tiles on the matrix cores (complex64: FP32 MFMA;
//      complex128: FP64 MFMA; a complex product is four real ones and the
//      eight panel columns two k-steps of 4);
//  (4) the pivot rows take YZ (Y on the panel columns), every other row's
//      panel columns become -M[i][C] Y.
// The block then holds (P S)^{-1} for the row permutation P of the swaps, so
// G = S^{-1} = M P: G[r][c] = M[r][pos(c)], pos(c) = the final position of
// row c.  The next line's Schur update reads G through pos row by row.
constexpr int FNB = 8;

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float acc __attribute__((ext_vector_type(4)));
  static __device__ inline acc mac(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }  // of register r
  static __device__ inline float bcast(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
  }
};
template <>
struct Mfma<double> {
  typedef double acc __attribute__((ext_vector_type(4)));
  static __device__ inline acc mac(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ inline double bcast(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
  }
};

// wave-wide maximum of (value, index): larger value, then lower index.  DPP
// within rows of 16 lanes (pairs across lane bits 0, 1, the mirror inside 8,
// then bit 3), then the permlane swaps across bits 4 and 5.
template <int CTRL>
__device__ inline int dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <typename T>
__device__ inline void amax_pick(T& b, int& i, T ob, int oi) {
  if (ob > b || (ob == b && oi < i)) {
    b = ob;
    i = oi;
  }
}
__device__ inline unsigned swap_partner(unsigned v, int lane, bool across32) {
  const auto r = across32 ? __builtin_amdgcn_permlane32_swap(v, v, false, false)
                          : __builtin_amdgcn_permlane16_swap(v, v, false, false);
  const bool hi = across32 ? lane >= 32 : ((lane >> 4) & 1);
  return hi ? r[0] : r[1];
}
__device__ inline float swap_partner(float v, int lane, bool across32) {
  return __uint_as_float(swap_partner(__float_as_uint(v), lane, across32));
}
__device__ inline double swap_partner(double v, int lane, bool across32) {
  const unsigned lo = swap_partner((unsigned)__double2loint(v), lane, across32);
  const unsigned hi = swap_partner((unsigned)__double2hiint(v), lane, across32);
  return __hiloint2double((int)hi, (int)lo);
}
template <typename T>
__device__ inline void wave_argmax(T& b, int& i, int lane) {
  amax_pick(b, i, wave::dpp<wave::kDppXor1>(b), dpp_int<wave::kDppXor1>(i));
  amax_pick(b, i, wave::dpp<wave::kDppXor2>(b), dpp_int<wave::kDppXor2>(i));
  amax_pick(b, i, wave::dpp<wave::kDppHalfMirror>(b), dpp_int<wave::kDppHalfMirror>(i));
  amax_pick(b, i, wave::dpp<wave::kDppRor8>(b), dpp_int<wave::kDppRor8>(i));
  amax_pick(b, i, swap_partner(b, lane, false), (int)swap_partner((unsigned)i, lane, false));
  amax_pick(b, i, swap_partner(b, lane, true), (int)swap_partner((unsigned)i, lane, true));
}

template <typename T>
__global__ void __launch_bounds__(WG) local_factor_kernel(ProblemDev P, const SubDesc* __restrict__ desc,
                                                          cplx<T>* __restrict__ G, int* __restrict__ status,
                                                          int pair) {
  using C = cplx<T>;
  using X = Mfma<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  const SubDesc d = desc[blockIdx.x];
  const int nx = d.nx, ny = d.ny;
  const int nt = (nx + 15) >> 4, nxp = 16 * nt;
  C* M = (C*)smem;              // the block, row-major
  C* YZ = M + nx * nx;          // FNB x nxp
  C* Ys = YZ + FNB * nxp;       // FNB x FNB
  int* orig = (int*)(Ys + FNB * FNB);  // the row of S at each position
  int* pos = orig + nx;                // the position of each row of S
  __shared__ int s_sing, s_nmv;
  __shared__ int mv_to[2 * FNB], mv_from[2 * FNB];  // the rows a panel's swaps move
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = WG / 64;
  if (tid == 0) s_sing = 0;

  for (int j = 0; j < ny; ++j) {
    const int y = d.ey0 + j;
    // the line's stencil coefficients (in the YZ space, free until the first panel)
    T* cf = reinterpret_cast<T*>(YZ);  // ea, fb, diag re, diag im, west, east; nx each
    for (int q = tid; q < nx; q += WG) {
      const Row5 ra = row5(P, d.ex0 + q, y);
      cf[q] = j > 0 ? (T)ra.s : (T)0;                            // A[(q,j),(q,j-1)]
      cf[nx + q] = j > 0 ? (T)row5(P, d.ex0 + q, y - 1).n : (T)0;  // A[(q,j-1),(q,j)]
      cf[2 * nx + q] = (T)ra.d.x;
      cf[3 * nx + q] = (T)ra.d.y;
      cf[4 * nx + q] = (T)ra.w;
      cf[5 * nx + q] = (T)ra.e;
    }
    __syncthreads();
    // S_j = D_j - E_j G_{j-1} F_{j-1}, G_{j-1}[a][b] = M[a][pos(b)]: one wave
    // per row, which reads the whole row before it writes it
    for (int a = wv; a < nx; a += NW) {
      C g[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int b = lane + 64 * h;
        g[h] = (j > 0 && b < nx) ? M[a * nx + pos[b]] : C{0, 0};
      }
      const T ea = cf[a];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int b = lane + 64 * h;
        if (b >= nx) continue;
        const T fb = cf[nx + b];
        C v = {-ea * fb * g[h].x, -ea * fb * g[h].y};
        if (b == a) {
          v.x += cf[2 * nx + a];
          v.y += cf[3 * nx + a];
        } else if (b == a - 1) {
          v.x += cf[4 * nx + a];
        } else if (b == a + 1) {
          v.x += cf[5 * nx + a];
        }
        M[a * nx + b] = v;
      }
    }
    for (int q = tid; q < nx; q += WG) orig[q] = q;
    __syncthreads();
    for (int k0 = 0; k0 < nx; k0 += FNB) {
      const int nbp = min(FNB, nx - k0);
      // (1) the panel, on wave 0: positions lane and lane + 64
      if (wv == 0) {
        const int r0 = lane, r1 = lane + 64;
        int src0 = r0, src1 = r1;  // the position whose row moves to r0, r1
        C p0[FNB], p1[FNB];
#pragma unroll
        for (int c = 0; c < FNB; ++c) {
          p0[c] = (r0 >= k0 && r0 < nx && c < nbp) ? M[r0 * nx + k0 + c] : C{0, 0};
          p1[c] = (r1 >= k0 && r1 < nx && c < nbp) ? M[r1 * nx + k0 + c] : C{0, 0};
        }
#pragma unroll
        for (int s = 0; s < FNB; ++s) {  // unrolled: the panel column s is a register index
          if (s >= nbp) break;
          const int k = k0 + s;
          C e0 = p0[0], e1 = p1[0];
#pragma unroll
          for (int c = 1; c < FNB; ++c)
            if (c == s) {
              e0 = p0[c];
              e1 = p1[c];
            }
          T best = (T)-1;
          int bi = 0x7fffffff;
          if (r0 >= k && r0 < nx) {
            const T m = cabs2(e0);
            if (m > best) { best = m; bi = r0; }
          }
          if (r1 >= k && r1 < nx) {
            const T m = cabs2(e1);
            if (m > best || (m == best && r1 < bi)) { best = m; bi = r1; }
          }
          wave_argmax(best, bi, lane);
          if (!(best > (T)0) && lane == 0) s_sing = 1;
          if (bi >= nx) bi = k;  // every candidate was NaN: keep the row in place
          const int p = __builtin_amdgcn_readfirstlane(bi);
          // rows p and k trade places: panel registers and the whole rows in LDS
          C pr[FNB], pk[FNB];
#pragma unroll
          for (int c = 0; c < FNB; ++c) {
            const C vp = p >= 64 ? p1[c] : p0[c];
            const C vk = k >= 64 ? p1[c] : p0[c];
            pr[c] = {X::bcast(vp.x, p & 63), X::bcast(vp.y, p & 63)};
            pk[c] = {X::bcast(vk.x, k & 63), X::bcast(vk.y, k & 63)};
          }
          if (p != k) {  // in LDS the rows move once the panel is done (src)
#pragma unroll
            for (int c = 0; c < FNB; ++c) {
              if (r0 == k) p0[c] = pr[c];
              if (r1 == k) p1[c] = pr[c];
              if (r0 == p) p0[c] = pk[c];
              if (r1 == p) p1[c] = pk[c];
            }
            const int sp = __builtin_amdgcn_readlane(p >= 64 ? src1 : src0, p & 63);
            const int sk = __builtin_amdgcn_readlane(k >= 64 ? src1 : src0, k & 63);
            if (r0 == k) src0 = sp;
            if (r1 == k) src1 = sp;
            if (r0 == p) src0 = sk;
            if (r1 == p) src1 = sk;
          }
          C piv = pr[0];
#pragma unroll
          for (int c = 1; c < FNB; ++c)
            if (c == s) piv = pr[c];
          if (!(cabs2(piv) > (T)0)) piv = {(T)1, (T)0};
          const C ip = cinv(piv);
#pragma unroll
          for (int c = 0; c < FNB; ++c) pr[c] = (c == s) ? ip : cmul(pr[c], ip);
          // eliminate column s from the panel's other rows (not the earlier panels')
          auto step = [&](C (&pv)[FNB], int r) {
            if (r < k0 || r >= nx) return;
            if (r == k) {
#pragma unroll
              for (int c = 0; c < FNB; ++c) pv[c] = pr[c];
              return;
            }
            C fct = pv[0];
#pragma unroll
            for (int c = 1; c < FNB; ++c)
              if (c == s) fct = pv[c];
#pragma unroll
            for (int c = 0; c < FNB; ++c) {
              if (c == s)
                pv[c] = {-(fct.x * ip.x - fct.y * ip.y), -(fct.x * ip.y + fct.y * ip.x)};
              else
                cfms(pv[c], fct, pr[c]);
            }
          };
          step(p0, r0);
          step(p1, r1);
        }
        // Y: the pivot rows' final panel values
        if (r0 >= k0 && r0 < k0 + nbp)
#pragma unroll
          for (int c = 0; c < FNB; ++c) Ys[(r0 - k0) * FNB + c] = p0[c];
        if (r1 >= k0 && r1 < k0 + nbp)
#pragma unroll
          for (int c = 0; c < FNB; ++c) Ys[(r1 - k0) * FNB + c] = p1[c];
        // the moved rows (at most two per pivot), listed in lane order
        const unsigned long long m0 = __ballot(r0 < nx && src0 != r0), m1 = __ballot(r1 < nx && src1 != r1);
        const int n0 = __popcll(m0);
        if (r0 < nx && src0 != r0) {
          const int at = __popcll(m0 & ((1ull << lane) - 1));
          mv_to[at] = r0;
          mv_from[at] = src0;
        }
        if (r1 < nx && src1 != r1) {
          const int at = n0 + __popcll(m1 & ((1ull << lane) - 1));
          mv_to[at] = r1;
          mv_from[at] = src1;
        }
        if (lane == 0) s_nmv = n0 + __popcll(m1);
      }
      __syncthreads();
      {  // the swaps in LDS: every moved row is read before any is written
        constexpr int MV = (2 * FNB * TPR * CSEG_MAX + WG - 1) / WG;
        const int nm = s_nmv, ne = nm * nx;
        C tmp[MV];
        int og = 0;
#pragma unroll
        for (int t = 0; t < MV; ++t) {
          const int e = tid + t * WG;
          if (e < ne) {
            const int m = e / nx, c = e - m * nx;
            tmp[t] = M[mv_from[m] * nx + c];
          }
        }
        if (tid < nm) og = orig[mv_from[tid]];
        __syncthreads();
#pragma unroll
        for (int t = 0; t < MV; ++t) {
          const int e = tid + t * WG;
          if (e < ne) {
            const int m = e / nx, c = e - m * nx;
            M[mv_to[m] * nx + c] = tmp[t];
          }
        }
        if (tid < nm) orig[mv_to[tid]] = og;
      }
      __syncthreads();
      // (2) YZ = Y M[C, :], zero past the block and past the panel's pivots
      for (int q = tid; q < FNB * nxp; q += WG) {
        const int c = q / nxp, jj = q - c * nxp;
        C acc = {0, 0};
        if (c < nbp && jj < nx)
          for (int cc = 0; cc < nbp; ++cc) cfma(acc, Ys[c * FNB + cc], M[(k0 + cc) * nx + jj]);
        YZ[q] = acc;
      }
      __syncthreads();
      // (3) M -= M[:, C] YZ outside the panel's rows and columns, on the matrix cores
      for (int tile = wv; tile < nt * nt; tile += NW) {
        const int ti = tile / nt, tj = tile - ti * nt;
        typename X::acc cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < FNB / 4; ++ks) {
          const int i = 16 * ti + (lane & 15), kk = 4 * ks + (lane >> 4);
          const C av = (i < nx && kk < nbp) ? M[i * nx + k0 + kk] : C{0, 0};
          const C bv = YZ[kk * nxp + 16 * tj + (lane & 15)];
          cre = X::mac(av.x, bv.x, cre);
          cre = X::mac(-av.y, bv.y, cre);
          cim = X::mac(av.x, bv.y, cim);
          cim = X::mac(av.y, bv.x, cim);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * ti + X::row(lane, r), jc = 16 * tj + (lane & 15);
          const bool in_panel = (i >= k0 && i < k0 + nbp) || (jc >= k0 && jc < k0 + nbp);
          if (i < nx && jc < nx && !in_panel) {
            C v = M[i * nx + jc];
            v.x -= cre[r];
            v.y -= cim[r];
            M[i * nx + jc] = v;
          }
        }
      }
      __syncthreads();
      // (4) the pivot rows take YZ and Y; the other rows' panel columns become -M[i][C] Y
      for (int q = tid; q < nbp * nx; q += WG) {  // the pivot rows, entry by entry
        const int s = q / nx, jc = q - s * nx;
        M[(k0 + s) * nx + jc] = (jc >= k0 && jc < k0 + nbp) ? Ys[s * FNB + (jc - k0)] : YZ[s * nxp + jc];
      }
      for (int i = tid; i < nx; i += WG) {  // the other rows, one thread each
        if (i >= k0 && i < k0 + nbp) continue;
        C a[FNB];
#pragma unroll
        for (int c = 0; c < FNB; ++c) a[c] = c < nbp ? M[i * nx + k0 + c] : C{0, 0};
#pragma unroll
        for (int c = 0; c < FNB; ++c) {
          if (c >= nbp) break;
          C acc = {0, 0};
#pragma unroll
          for (int cc = 0; cc < FNB; ++cc)
            if (cc < nbp) cfma(acc, a[cc], Ys[cc * FNB + c]);
          M[i * nx + k0 + c] = {-acc.x, -acc.y};
        }
      }
      __syncthreads();
    }
    for (int q = tid; q < nx; q += WG) pos[orig[q]] = q;
    __syncthreads();
    // G[r][c] = M[r][pos(c)], stored in the thread-segment layout
    const int cseg = line_rows(nx), T4 = TPR * nx;
    const int npair = pair ? cseg / 2 : 0;  // paired segment rows come first
    C* Gj = G + d.gofs + (int64_t)j * cseg * T4;
    for (int q = tid; q < cseg * T4; q += WG) {
      int qq, t;
      if (q < npair * 2 * T4) {
        const int p = q / (2 * T4), rem = q - p * (2 * T4);
        t = rem >> 1;
        qq = 2 * p + (rem & 1);
      } else {  // unpaired rows (the odd last one of a paired line)
        qq = q / T4;
        t = q - qq * T4;
      }
      const int r = t / TPR, c = (t % TPR) * cseg + qq;
      Gj[q] = (c < nx) ? M[r * nx + pos[c]] : C{0, 0};
    }
    __syncthreads();
  }
  if (tid == 0 && s_sing) status[blockIdx.x] = 1;
}

// ------------------------------------------------------------- solve
// Visit order of the grid lines: forward 0..ny-1, then backward ny-2..0.
__device__ inline int line_of(int k, int ny) { return k < ny ? k : 2 * ny - 2 - k; }

// Loads are unconditional (idle threads read a valid lane's address) and
// their count is the compile-time segment count CS, so the compiler can count
// the outstanding loads and keep the prefetched lines in flight.
template <typename T, int CS>
__device__ inline void load_line(cplx<T> (&buf)[CS], const cplx<T>* __restrict__ Gl, int T4, int tc) {
  if constexpr (sizeof(T) == 4) {   // paired complex64 layout: one 16-byte load per two entries
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4* G4 = (const f4*)Gl;
#pragma unroll
    for (int p = 0; p < CS / 2; ++p) {
      const f4 v = G4[p * T4 + tc];
      buf[2 * p] = {v.x, v.y};
      buf[2 * p + 1] = {v.z, v.w};
    }
    if constexpr (CS % 2 == 1) buf[CS - 1] = Gl[(CS - 1) * T4 + tc];  // the unpaired last row
  } else {
#pragma unroll
    for (int q = 0; q < CS; ++q) buf[q] = Gl[q * T4 + tc];
  }
}

// one step: out_r = sum_c G_j[r][c] y[c] for the thread's segment, reduced
// over the TPR threads of the row (DPP within the quad); factor entries are widened
// from the storage type TS to the arithmetic type TC
template <typename TS, typename TC, int CS>
__device__ inline cplx<TC> seg_matvec(const cplx<TS> (&buf)[CS], const cplx<TC>* y, int s) {
  cplx<TC> acc = {0, 0};
#pragma unroll
  for (int q = 0; q < CS; ++q) cfma(acc, cplx<TC>{(TC)buf[q].x, (TC)buf[q].y}, y[s * CS + q]);
  // the TPR = 4 threads of a row are one quad: DPP quad permutations
  acc.x += wave::dpp<wave::kDppXor1>(acc.x);
  acc.y += wave::dpp<wave::kDppXor1>(acc.y);
  acc.x += wave::dpp<wave::kDppXor2>(acc.x);
  acc.y += wave::dpp<wave::kDppXor2>(acc.y);
  return acc;
}

// TS: storage type of the factors (what is streamed from HBM); T: arithmetic
// type of the sweeps, the gathered right-hand side and the local solution.
// One workgroup solves one subdomain: gather, forward and backward sweeps,
// scatter into the local-solution array.
template <typename TS, typename T, int DEPTH, int CSEG>
__device__ inline void local_solve_one(const SubDesc& d, const ProblemDev& P, const cplx<TS>* __restrict__ G,
                                       const c128* __restrict__ r, cplx<T>* __restrict__ sol, unsigned char* smem) {
  using C = cplx<T>;
  using CS = cplx<TS>;
  const int nx = d.nx, ny = d.ny;
  const int cseg = CSEG, T4 = TPR * nx;
  const int64_t LS = (int64_t)CSEG * T4;   // factor entries per grid line
  C* X = (C*)smem;                          // ny * nx: b, then t, then x
  C* yb = X + nx * ny;                      // two padded input vectors
  const int ylen = TPR * cseg;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int t = tid, row = t / TPR, sg = t % TPR;
  const bool act = t < T4;
  const int tc = act ? t : T4 - 1;
  const int ntot = nx * ny;
  for (int q = tid; q < ntot; q += nth) {
    const int jj = q / nx, a = q - jj * nx;
    const int64_t gl = (int64_t)(d.ey0 + jj - P.lo) * P.nu + (d.ex0 + a - P.lo);
    X[q] = to_t<T>(r[gl]);
  }
  for (int q = tid; q < 2 * ylen; q += nth) yb[q] = {0, 0};
  __syncthreads();
  for (int a = tid; a < nx; a += nth) yb[a] = X[a];   // y_0 = b_0
  const CS* Gs = G + d.gofs;
  const int nsteps = 2 * ny - 1;
  auto line_ptr = [&](int k) { return Gs + (int64_t)line_of(k < nsteps ? k : nsteps - 1, ny) * LS; };
  CS bA[CSEG], bB[CSEG], bC[CSEG];
  load_line<TS, CSEG>(bA, line_ptr(0), T4, tc);
  if (DEPTH >= 2) load_line<TS, CSEG>(bB, line_ptr(1), T4, tc);
  __syncthreads();
  auto step = [&](int k, const CS (&cur)[CSEG], CS (&pf)[CSEG]) {
    load_line<TS, CSEG>(pf, line_ptr(k + DEPTH), T4, tc);   // prefetch DEPTH lines ahead
    const C* y = yb + (k & 1) * ylen;
    C* yn = yb + ((k + 1) & 1) * ylen;
    const int j = line_of(k, ny);
    C out = {0, 0};
    if (act) out = seg_matvec<TS, T, CSEG>(cur, y, sg);
    if (act && sg == 0) {
      const int x = d.ex0 + row;
      const C val = (k < ny) ? out : csub(X[j * nx + row], out);  // t_j, or x_j = t_j - G_j F_j x_{j+1}
      if (k + 1 < nsteps) {
        const int jn = line_of(k + 1, ny);
        C nv;
        if (k + 1 < ny) {                           // y_{j+1} = b_{j+1} - E_{j+1} t_j
          const T e = (T)row5(P, x, d.ey0 + jn).s;
          const C b = X[jn * nx + row];
          nv = {b.x - e * val.x, b.y - e * val.y};
        } else {                                    // F_{jn} x_{jn+1}
          const T f = (T)row5(P, x, d.ey0 + jn).n;
          nv = {f * val.x, f * val.y};
        }
        yn[row] = nv;
      }
      X[j * nx + row] = val;
    }
    __syncthreads();
  };
  int k = 0;
  if constexpr (DEPTH >= 2) {
    for (; k + 2 < nsteps; k += 3) {
      step(k, bA, bC);
      step(k + 1, bB, bA);
      step(k + 2, bC, bB);
    }
    if (k < nsteps) step(k, bA, bC);
    if (k + 1 < nsteps) step(k + 1, bB, bA);
  } else {
    for (; k + 1 < nsteps; k += 2) {
      step(k, bA, bB);
      step(k + 1, bB, bA);
    }
    if (k < nsteps) step(k, bA, bB);
  }
  C* out = sol + d.sofs;
  for (int q = tid; q < ntot; q += nth) out[q] = X[q];
}

// The solve instantiated for the subdomain's segment count (wave-uniform),
// one of CS..HI.  A kernel holds the counts of one class range: with all
// eighteen inlined into one kernel the register allocation degrades (spills),
// with six it matches a single instantiation.
template <typename TS, typename T, int DEPTH, int CS, int HI>
__device__ inline void local_solve_sub(const SubDesc& d, const ProblemDev& P, const cplx<TS>* __restrict__ G,
                                       const c128* __restrict__ r, cplx<T>* __restrict__ sol, unsigned char* smem) {
  if constexpr (CS <= HI) {
    if (line_rows(d.nx) == CS)
      local_solve_one<TS, T, DEPTH, CS>(d, P, G, r, sol, smem);
    else
      local_solve_sub<TS, T, DEPTH, CS + 1, HI>(d, P, G, r, sol, smem);
  }
}

// segment-count ranges of the solve kernels; a launch's subdomains are
// grouped into classes, each within one range (local_classes)
constexpr int kRangeLo[] = {1, 4, 7, 9, 13, 19};
constexpr int kRangeHi[] = {6, 9, 12, 14, 18, 24};
constexpr int kRanges = 6;
static_assert(kRangeHi[kRanges - 1] == CSEG_MAX, "the ranges cover every segment count");

// Persistent launch: workgroup b takes subdomains b, b + gridDim.x, ... of
// desc[0, nsub) in order (all with segment counts in [LO, HI]).
// tab != nullptr: a batch; each subdomain names its instance, whose
// operator, factors, local solutions and vector offset come from tab.  A
// grid smaller than the subdomain count leaves CU slots to the coarse
// sweeps that run concurrently on another stream.
template <typename TS, typename T, int DEPTH, int LO, int HI>
__global__ void __launch_bounds__(TPR * TPR * CSEG_MAX) local_solve_kernel(ProblemDev P, const SubDesc* __restrict__ desc, int nsub,
                                                          const cplx<TS>* __restrict__ G,
                                                          const c128* __restrict__ r, cplx<T>* __restrict__ sol,
                                                          const LocalArgs* __restrict__ tab,
                                                          const ArnState* __restrict__ st) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int sd = blockIdx.x; sd < nsub; sd += gridDim.x) {
    const SubDesc d = desc[sd];
    if (tab && inst_idle(st, d.inst)) continue;  // workgroup-uniform: no barrier is skipped by part of it
    if (tab) {
      const LocalArgs& L = tab[d.inst];
      local_solve_sub<TS, T, DEPTH, LO, HI>(d, L.P, (const cplx<TS>*)L.G, L.rhs ? L.rhs : r + L.voff,
                                            (cplx<T>*)L.sol, smem);
    } else {
      local_solve_sub<TS, T, DEPTH, LO, HI>(d, P, G, r, sol, smem);
    }
    __syncthreads();  // the next subdomain reuses the LDS
  }
}

// kernel of (storage, arithmetic) types and range q
template <typename TS, typename T, int DEPTH>
const void* solve_kernel_of(int q) {
  switch (q) {
    case 0: return (const void*)local_solve_kernel<TS, T, DEPTH, kRangeLo[0], kRangeHi[0]>;
    case 1: return (const void*)local_solve_kernel<TS, T, DEPTH, kRangeLo[1], kRangeHi[1]>;
    case 2: return (const void*)local_solve_kernel<TS, T, DEPTH, kRangeLo[2], kRangeHi[2]>;
    case 3: return (const void*)local_solve_kernel<TS, T, DEPTH, kRangeLo[3], kRangeHi[3]>;
    case 4: return (const void*)local_solve_kernel<TS, T, DEPTH, kRangeLo[4], kRangeHi[4]>;
    default: return (const void*)local_solve_kernel<TS, T, DEPTH, kRangeLo[5], kRangeHi[5]>;
  }
}

template <typename TS, typename T, int DEPTH>
void launch_solve_classes(const LocalLaunch& L, const ProblemDev& P, const void* G, const c128* r, void* sol,
                          const LocalArgs* tab, size_t lds, int threads, int grid, hipStream_t s,
                          const ArnState* stt = nullptr) {
  for (const LocalClass& c : L.cls) {
    const int g = (grid > 0 && grid < c.count) ? grid : c.count;
    const SubDesc* desc = L.desc + c.first;
    const cplx<TS>* Gt = (const cplx<TS>*)G;
    cplx<T>* sol_t = (cplx<T>*)sol;
    switch (c.range) {
      case 0:
        local_solve_kernel<TS, T, DEPTH, kRangeLo[0], kRangeHi[0]><<<g, threads, lds, s>>>(P, desc, c.count, Gt, r, sol_t, tab, stt);
        break;
      case 1:
        local_solve_kernel<TS, T, DEPTH, kRangeLo[1], kRangeHi[1]><<<g, threads, lds, s>>>(P, desc, c.count, Gt, r, sol_t, tab, stt);
        break;
      case 2:
        local_solve_kernel<TS, T, DEPTH, kRangeLo[2], kRangeHi[2]><<<g, threads, lds, s>>>(P, desc, c.count, Gt, r, sol_t, tab, stt);
        break;
      case 3:
        local_solve_kernel<TS, T, DEPTH, kRangeLo[3], kRangeHi[3]><<<g, threads, lds, s>>>(P, desc, c.count, Gt, r, sol_t, tab, stt);
        break;
      case 4:
        local_solve_kernel<TS, T, DEPTH, kRangeLo[4], kRangeHi[4]><<<g, threads, lds, s>>>(P, desc, c.count, Gt, r, sol_t, tab, stt);
        break;
      default:
        local_solve_kernel<TS, T, DEPTH, kRangeLo[5], kRangeHi[5]><<<g, threads, lds, s>>>(P, desc, c.count, Gt, r, sol_t, tab, stt);
    }
    HS_HIP(hipGetLastError());
  }
}

template <typename T>
__global__ void to_c128_kernel(int64_t n, const cplx<T>* __restrict__ in, c128* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = {(double)in[i].x, (double)in[i].y};
}

__global__ void round_c64_kernel(int64_t n, const c128* __restrict__ in, c64* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = {(float)in[i].x, (float)in[i].y};
}

template <typename T>
size_t factor_lds(int nx) {
  const int nxp = 16 * ((nx + 15) / 16);
  return (size_t)(nx * nx + FNB * nxp + FNB * FNB) * sizeof(cplx<T>) + 2 * nx * sizeof(int) + 64;
}
template <typename T>
size_t solve_lds(int nx, int ny) {
  const int ylen = TPR * ((nx + TPR - 1) / TPR);
  return (size_t)(nx * ny + 2 * ylen) * sizeof(cplx<T>) + 64;
}

}  // namespace

size_t local_factor_lds_bytes(int prec, int nx) {
  return prec == HS_C64 ? factor_lds<float>(nx) : factor_lds<double>(nx);
}
size_t local_solve_lds_bytes(int prec, int nx, int ny) {
  return prec == HS_C64 ? solve_lds<float>(nx, ny) : solve_lds<double>(nx, ny);
}

void launch_local_factor(const ProblemDev& P, int prec, int nsub, const SubDesc* desc, void* G, int* status,
                         size_t lds, bool pair, hipStream_t s) {
  {  // the kernel's dynamic-LDS limit is only ever raised (set-ups on several host threads)
    static std::mutex mu;
    static size_t raised[2] = {0, 0};
    std::lock_guard<std::mutex> lk(mu);
    const int p = prec == HS_C64 ? 0 : 1;
    if (lds > raised[p]) {
      const void* fn = p == 0 ? (const void*)local_factor_kernel<float> : (const void*)local_factor_kernel<double>;
      HS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      raised[p] = lds;
    }
  }
  if (prec == HS_C64)
    local_factor_kernel<float><<<nsub, WG, lds, s>>>(P, desc, (c64*)G, status, pair ? 1 : 0);
  else
    local_factor_kernel<double><<<nsub, WG, lds, s>>>(P, desc, (c128*)G, status, pair ? 1 : 0);
  HS_HIP(hipGetLastError());
}

int local_solve_threads(int max_nx) { return ((TPR * max_nx + 63) / 64) * 64; }
int64_t local_line_entries(int nx) { return (int64_t)line_rows(nx) * TPR * nx; }
// padding after the last line so that unconditional prefetch loads stay in bounds
int64_t local_factor_pad() { return (int64_t)CSEG_MAX * TPR * TPR * CSEG_MAX; }

// Raise the dynamic-LDS limit of the solve kernels once, at set-up, so that a
// launch enqueues stream work only (it may sit inside a captured graph).  The
// limit only grows, so handles built earlier keep working.
// gprec: factor storage; cprec: arithmetic and local solution.
void prepare_local_solve(int gprec, int cprec, size_t lds) {
  static std::mutex mu;  // set-ups on several host threads
  std::lock_guard<std::mutex> lk(mu);
  static size_t raised[3] = {0, 0, 0};
  const int p = gprec == HS_C128 ? 1 : (cprec == HS_C64 ? 0 : 2);
  if (lds <= raised[p]) return;
  for (int q = 0; q < kRanges; ++q) {
    const void* fn = p == 0 ? solve_kernel_of<float, float, 2>(q)
                            : (p == 1 ? solve_kernel_of<double, double, 1>(q) : solve_kernel_of<float, double, 2>(q));
    HS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  }
  raised[p] = lds;
}

std::vector<LocalClass> local_classes(std::vector<SubDesc>& desc) {
  // each distinct segment count, smallest first, joins the open class if
  // its range holds it, else opens a class in the range that reaches
  // furthest above it
  std::vector<int> range_of_count(CSEG_MAX + 1, -1);
  std::vector<int> counts;
  for (const SubDesc& d : desc) counts.push_back(line_rows(d.nx));
  std::vector<int> distinct = counts;
  std::sort(distinct.begin(), distinct.end());
  distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
  int open = -1;
  for (int c : distinct) {
    if (c < 1 || c > CSEG_MAX) throw Failure{HS_EINVAL, "subdomain line longer than the local solve supports"};
    if (open < 0 || c > kRangeHi[open]) {
      open = -1;
      for (int q = 0; q < kRanges; ++q)
        if (kRangeLo[q] <= c && c <= kRangeHi[q] && (open < 0 || kRangeHi[q] > kRangeHi[open])) open = q;
    }
    range_of_count[c] = open;
  }
  // stable: the caller's order (largest first, repeats interleaved) holds
  // within a class
  std::vector<int> idx(desc.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    return range_of_count[counts[a]] < range_of_count[counts[b]];
  });
  std::vector<SubDesc> sorted;
  std::vector<LocalClass> cls;
  for (int i : idx) {
    const int q = range_of_count[counts[i]];
    if (cls.empty() || cls.back().range != q) cls.push_back({(int)sorted.size(), 0, q});
    ++cls.back().count;
    sorted.push_back(desc[i]);
  }
  desc.swap(sorted);
  return cls;
}

void launch_local_solve(const LocalLaunch& L, const ProblemDev& P, int gprec, int cprec, const void* G,
                        const c128* r, void* sol, size_t lds, int threads, hipStream_t s, int grid) {
  if (gprec == HS_C128)
    launch_solve_classes<double, double, 1>(L, P, G, r, sol, nullptr, lds, threads, grid, s);
  else if (cprec == HS_C64)
    launch_solve_classes<float, float, 2>(L, P, G, r, sol, nullptr, lds, threads, grid, s);
  else
    launch_solve_classes<float, double, 2>(L, P, G, r, sol, nullptr, lds, threads, grid, s);
}

void launch_local_solve_batch(const LocalLaunch& L, int gprec, int cprec, const LocalArgs* tab, const c128* r,
                              size_t lds, int threads, int grid, hipStream_t s, const ArnState* st) {
  const ProblemDev P0{};
  if (gprec == HS_C128)
    launch_solve_classes<double, double, 1>(L, P0, nullptr, r, nullptr, tab, lds, threads, grid, s, st);
  else if (cprec == HS_C64)
    launch_solve_classes<float, float, 2>(L, P0, nullptr, r, nullptr, tab, lds, threads, grid, s, st);
  else
    launch_solve_classes<float, double, 2>(L, P0, nullptr, r, nullptr, tab, lds, threads, grid, s, st);
}

void launch_round_c64(int64_t count, const c128* in, c64* out, hipStream_t s) {
  round_c64_kernel<<<(int)((count + 255) / 256), 256, 0, s>>>(count, in, out);
  HS_HIP(hipGetLastError());
}

void launch_local_to_c128(int prec, int64_t count, const void* sol, c128* out, hipStream_t s) {
  const int blocks = (int)((count + 255) / 256);
  if (prec == HS_C64)
    to_c128_kernel<float><<<blocks, 256, 0, s>>>(count, (const c64*)sol, out);
  else
    to_c128_kernel<double><<<blocks, 256, 0, s>>>(count, (const c128*)sol, out);
  HS_HIP(hipGetLastError());
}

}  // namespace hs
