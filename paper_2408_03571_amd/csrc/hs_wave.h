// Wave-level sums without the LDS crossbar (gfx950): DPP within rows of 16
// lanes and the permlane swaps across rows.  __shfl_xor / __shfl_down go
// through ds_bpermute, one LDS round trip per 32 bits.
#pragma once

#include <hip/hip_runtime.h>

namespace hs {
namespace wave {

template <int CTRL>
__device__ inline double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppRor8 = 0x128;       // row_ror:8, lane l <- l ^ 8 within 16
constexpr int kDppHalfMirror = 0x141; // lane l <- 7 - l within 8

// v_permlane32_swap: lanes 32..63 of x trade places with lanes 0..31 of y.
// Afterwards x + y holds, in lane l, the sum over lanes l and l ^ 32 of x
// (l < 32) or of y (l >= 32): one halving step with no select.  With x = y
// every lane holds the sum over l and l ^ 32, lower lane first.
__device__ inline double halve32(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
// v_permlane16_swap: odd rows of x trade places with even rows of y; the
// same halving across lane bit 4.
__device__ inline double halve16(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// Wave sums of NV = 4, 8 or 16 values per lane by recursive halving (each
// step pairs lanes across one bit, keeps half of the values and adds the
// partner's copy of them).  Afterwards every lane of the group of 64/NV
// lanes l with l / (64/NV) == j holds the sum of value j.  Every NV follows
// one tree, lane bits 5, 4, 3, then the pairs (l, 7-l), then bits 0 and 1,
// so a sum does not depend on NV.
template <int NV>
__device__ inline double sum(double (&v)[NV], int lane) {
  static_assert(NV == 4 || NV == 8 || NV == 16, "4, 8 or 16 values");
#pragma unroll
  for (int q = 0; q < NV / 2; ++q) v[q] = halve32(v[q], v[q + NV / 2]);
#pragma unroll
  for (int q = 0; q < NV / 4; ++q) v[q] = halve16(v[q], v[q + NV / 4]);
  double r;
  if constexpr (NV == 4) {
    r = v[0] + dpp<kDppRor8>(v[0]);
    r += dpp<kDppHalfMirror>(r);
  } else {
#pragma unroll
    for (int q = 0; q < NV / 8; ++q) {
      const bool hi = lane & 8;
      const double keep = hi ? v[q + NV / 8] : v[q];
      const double send = hi ? v[q] : v[q + NV / 8];
      v[q] = keep + dpp<kDppRor8>(send);
    }
    if constexpr (NV == 16) {
      const bool hi = lane & 4;  // partner 7 - l has the other bit 2
      const double keep = hi ? v[1] : v[0];
      const double send = hi ? v[0] : v[1];
      r = keep + dpp<kDppHalfMirror>(send);
    } else {
      r = v[0];
      r += dpp<kDppHalfMirror>(r);
    }
  }
  r += dpp<kDppXor1>(r);
  r += dpp<kDppXor2>(r);
  return r;
}

}  // namespace wave
}  // namespace hs
