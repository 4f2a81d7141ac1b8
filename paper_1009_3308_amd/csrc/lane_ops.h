// Cross-lane sums of a wavefront in registers (gfx950): the butterfly that the
// recurrence-based Legendre analyses use to add sixteen values over the 64
// latitude lanes of a wave without LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace nse {

constexpr int kButterfly = 16;  // values summed per lane

// Cross-lane moves of doubles in registers (no LDS): the gfx950 lane-half swaps
// and DPP row mirrors / quad permutations, applied to both 32-bit halves.
__device__ inline double lane_swap_sum32(double a, double b) {
  // v_permlane32_swap: lanes 32..63 of a trade places with lanes 0..31 of b; the
  // sum of the two results is a[l] + a[l ^ 32] in the lower half and
  // b[l] + b[l ^ 32] in the upper half
  const unsigned long long ai = __double_as_longlong(a), bi = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ai, (unsigned)bi, false, false);
  const auto hi =
      __builtin_amdgcn_permlane32_swap((unsigned)(ai >> 32), (unsigned)(bi >> 32), false, false);
  const double a2 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double b2 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return a2 + b2;
}
__device__ inline double lane_swap_sum16(double a, double b) {
  // v_permlane16_swap: odd 16-lane rows of a trade places with even rows of b
  const unsigned long long ai = __double_as_longlong(a), bi = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ai, (unsigned)bi, false, false);
  const auto hi =
      __builtin_amdgcn_permlane16_swap((unsigned)(ai >> 32), (unsigned)(bi >> 32), false, false);
  const double a2 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double b2 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return a2 + b2;
}
template <int CTRL>
__device__ inline double lane_dpp(double v) {
  const unsigned long long i = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)i, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(i >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
constexpr int kDppRowMirror = 0x140;      // lane i of a 16-lane row reads lane 15 - i
constexpr int kDppRowHalfMirror = 0x141;  // lane i of an 8-lane half row reads lane 7 - i
constexpr int kDppQuadXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppQuadXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]

// Single-precision forms of the same moves (one 32-bit register each).
__device__ inline float lane_swap_sum32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline float lane_swap_sum16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int CTRL>
__device__ inline float lane_dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 64 lanes of x[j], j < 16, by halving exchanges: partners differ
// in lane bit 5 (swap), 4 (swap), 3 (row mirror, lane ^ 15), 2 (half-row
// mirror, lane ^ 7), the lane keeping the half of the index set its own bit
// selects; then plain sums over lane ^ 2 and lane ^ 1. On return x[0] holds the
// sum for j = 8 b5 + 4 b4 + 2 b3 + b2 of the lane. T is double or float.
template <typename T>
__device__ inline void lane_butterfly16(T (&xr)[kButterfly], T (&xi)[kButterfly], int lane) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    xr[i] = lane_swap_sum32(xr[i], xr[i + 8]);
    xi[i] = lane_swap_sum32(xi[i], xi[i + 8]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    xr[i] = lane_swap_sum16(xr[i], xr[i + 4]);
    xi[i] = lane_swap_sum16(xi[i], xi[i + 4]);
  }
  {
    const bool hi = (lane & 8) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const T kr = hi ? xr[i + 2] : xr[i], ki = hi ? xi[i + 2] : xi[i];
      const T sr = hi ? xr[i] : xr[i + 2], si = hi ? xi[i] : xi[i + 2];
      xr[i] = kr + lane_dpp<kDppRowMirror>(sr);
      xi[i] = ki + lane_dpp<kDppRowMirror>(si);
    }
  }
  {
    const bool hi = (lane & 4) != 0;
    const T kr = hi ? xr[1] : xr[0], ki = hi ? xi[1] : xi[0];
    const T sr = hi ? xr[0] : xr[1], si = hi ? xi[0] : xi[1];
    xr[0] = kr + lane_dpp<kDppRowHalfMirror>(sr);
    xi[0] = ki + lane_dpp<kDppRowHalfMirror>(si);
  }
  xr[0] += lane_dpp<kDppQuadXor2>(xr[0]);
  xi[0] += lane_dpp<kDppQuadXor2>(xi[0]);
  xr[0] += lane_dpp<kDppQuadXor1>(xr[0]);
  xi[0] += lane_dpp<kDppQuadXor1>(xi[0]);
}

// Maximum over the 64 lanes of four non-negative doubles (NaN kept), with the
// exchanges of lane_butterfly16: after the two lane-half swaps row r (lanes
// 16 r .. 16 r + 15) holds partial maxima of v[r]; the row mirror, half-row
// mirror and the two quad permutations complete each row. On return lane 16 r
// holds the maximum of v[r].
__device__ inline double lane_nanmax(double a, double b) { return (a != a || a > b) ? a : b; }
__device__ inline double lane_swap_max(double a, double b, bool rows16) {
  const unsigned long long ai = __double_as_longlong(a), bi = __double_as_longlong(b);
  unsigned lo0, lo1, hi0, hi1;
  if (rows16) {
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ai, (unsigned)bi, false, false);
    const auto hi =
        __builtin_amdgcn_permlane16_swap((unsigned)(ai >> 32), (unsigned)(bi >> 32), false, false);
    lo0 = lo[0], lo1 = lo[1], hi0 = hi[0], hi1 = hi[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ai, (unsigned)bi, false, false);
    const auto hi =
        __builtin_amdgcn_permlane32_swap((unsigned)(ai >> 32), (unsigned)(bi >> 32), false, false);
    lo0 = lo[0], lo1 = lo[1], hi0 = hi[0], hi1 = hi[1];
  }
  const double a2 = __longlong_as_double((long long)(((unsigned long long)hi0 << 32) | lo0));
  const double b2 = __longlong_as_double((long long)(((unsigned long long)hi1 << 32) | lo1));
  return lane_nanmax(a2, b2);
}
__device__ inline double lane_max4(const double (&v)[4]) {
  const double w0 = lane_swap_max(v[0], v[2], false);  // lanes 0..31: v[0], 32..63: v[2]
  const double w1 = lane_swap_max(v[1], v[3], false);
  double u = lane_swap_max(w0, w1, true);               // row r: v[r]
  u = lane_nanmax(u, lane_dpp<kDppRowMirror>(u));
  u = lane_nanmax(u, lane_dpp<kDppRowHalfMirror>(u));
  u = lane_nanmax(u, lane_dpp<kDppQuadXor2>(u));
  u = lane_nanmax(u, lane_dpp<kDppQuadXor1>(u));
  return u;
}

}  // namespace nse
