// Split-bf16 Legendre contractions on MFMA (the synthesis and analysis of
// Section 4.2 with bf16 products and FP32 accumulation).
//
// The tables are the FP64 recurrence values rounded to FP32 (half the bytes of
// the FP64 pass). Each operand x is split into three bf16 pieces
// x ~ x0 + x1 + x2 (each the rounded remainder of the previous ones), and the
// six products xi*yj with i + j <= 2 (relative weight >= 2^-16) run on
// v_mfma_f32_16x16x32_bf16, accumulating in FP32 over blocks of 32 terms; the
// block sums are added in FP64. The Legendre recurrences, the coefficient
// panels, the quadrature weights, the FFTs, the grid products and the time-step
// update stay in FP64.
//
// Synthesis: per (order m, 64-latitude tile) a workgroup of four waves; wave w
// computes C[16 latitudes][16 columns] = sum_k T1[m][k][lat] B[k][col] over the
// whole degree range, with columns 0-7 the even-degree and 8-15 the odd-degree
// panel values (4 fields x re/im). B is the same for the four waves and is
// split once per workgroup into LDS in operand order (only the four degrees of
// each column's parity; the rest of the operand is zero). The northern value is
// E + O and the mirrored southern value E - O.
// Analysis: per (order m, 64-degree tile) four waves; wave w computes
// C[4 used rows][16 degrees] = sum_p A[row][p] T2[m][p][k] with rows We.re,
// We.im, Wo.re, Wo.im (the ring spectra folded over latitude pairs, split once
// per workgroup into LDS; only the four live rows are stored), then the
// epilogue of spectral_ops.h.
// The table operand of the next block is loaded while the current one is
// multiplied.
//
// MFMA operand layouts (checked on gfx950): for 16x16x32 bf16, lane l supplies
// row l%16 of A and column l%16 of B for K = 8*(l/16) .. +7, and receives C rows
// 4*(l/16) .. +3 of column l%16.
#include "spectral_ops.h"

namespace nse {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kLpWaves = 4;
constexpr int kLpThreads = 64 * kLpWaves;

// x ~ h0 + h1 + h2 with h0 = bf16(x), h1 = bf16(x - h0), h2 = bf16(x - h0 - h1).
// For a double x the remainders are formed exactly in FP64.
__device__ __forceinline__ void split3(double x, __bf16& h0, __bf16& h1, __bf16& h2) {
  h0 = (__bf16)(float)x;
  const double r1 = x - (double)(float)h0;
  h1 = (__bf16)(float)r1;
  const double r2 = r1 - (double)(float)h1;
  h2 = (__bf16)(float)r2;
}
// For a float x the remainders x - h0 and x - h0 - h1 are exact in FP32.
__device__ __forceinline__ void split3f(float x, __bf16& h0, __bf16& h1, __bf16& h2) {
  h0 = (__bf16)x;
  const float r1 = x - (float)h0;
  h1 = (__bf16)r1;
  h2 = (__bf16)(r1 - (float)h1);
}

__device__ __forceinline__ floatx4 mfma_bf16x3(const bf16x8& a0, const bf16x8& a1,
                                               const bf16x8& a2, const bf16x8& b0,
                                               const bf16x8& b1, const bf16x8& b2) {
  floatx4 c = {0.f, 0.f, 0.f, 0.f};
  // smallest terms first
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, c, 0, 0, 0);
  return c;
}

// bf16x8 with the four given values at positions par, par+2, par+4, par+6 and
// zeros elsewhere.
__device__ __forceinline__ bf16x8 interleave(bf16x4 v, int par) {
  const __bf16 z = (__bf16)0.0f;
  bf16x8 r;
  if (par == 0) {
    r[0] = v[0]; r[1] = z; r[2] = v[1]; r[3] = z; r[4] = v[2]; r[5] = z; r[6] = v[3]; r[7] = z;
  } else {
    r[0] = z; r[1] = v[0]; r[2] = z; r[3] = v[1]; r[4] = z; r[5] = v[2]; r[6] = z; r[7] = v[3];
  }
  return r;
}

}  // namespace

// LDS: the split panel [block][piece][64 lanes] with only the four degrees of
// the lane's parity stored (bf16x4; the other four of the operand are zero),
// reused for the 4 x 256 FP64 partial results at the end.
size_t synthesis_lp_lds_bytes(int N) {
  const int nblk = (N + 2 + 31) / 32;
  size_t split = (size_t)nblk * 3 * 64 * sizeof(bf16x4);
  const size_t cst = sizeof(double) * kLpWaves * 256;
  return split > cst ? split : cst;
}

// LDS of the split-panel kernel: alpha coefficients and the four panels.
size_t split_panel_lp_lds_bytes(int N) { return sizeof(double2) * (size_t)(5 * N + 11); }

// The split B operand of the synthesis for one (order m, member), computed
// once per step and shared by every latitude tile: the four coefficient panels
// of the order are built in LDS (spectral_ops.h), then each 32-degree block is
// split into three bf16 pieces in operand order: lane column c = l%16 holds
// (parity c >> 3, field (c & 7) >> 1, re/im c & 1) for K = 8*(l/16) .. +7, of
// which only the four degrees of the column's parity are stored (bf16x4).
__global__ __launch_bounds__(kLpThreads) void k_split_panel_lp(GroupView g, SynthInput in,
                                                               int mode) {
  if (gate_closed(g)) return;  // an ended attempt of a device-controlled run
  const int N = g.N;
  const int m = blockIdx.x, b = blockIdx.y;
  const int L = N + 2 - m;
  const int nblk = (L + 31) / 32;
  extern __shared__ double2 sh[];
  double2* a = sh;              // [N + 3]
  double2* pan = sh + (N + 3);  // [L][4]
  load_order(a, g, in, b, m, L);
  __syncthreads();
  build_panel<4>(pan, a, N, m, L, mode, in.coriolis, in.stream != 0);
  __syncthreads();
  bf16x4* out = reinterpret_cast<bf16x4*>(g.lps + (int64_t)b * g.lpsoff[N + 1] + g.lpsoff[m]);
  for (int it = threadIdx.x; it < nblk * 64; it += blockDim.x) {
    const int kb = it >> 6, l = it & 63;
    const int c = l & 15, q = l >> 4;
    const int par = c >> 3, fld = (c & 7) >> 1, cmp = c & 1;
    bf16x4 h[3];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int k = kb * 32 + 8 * q + 2 * jj + par;  // the degrees of this column's parity
      double v = 0.0;
      if (k < L) {
        const double2 P = pan[4 * k + fld];
        v = cmp ? P.y : P.x;
      }
      __bf16 h0, h1, h2;
      split3(v, h0, h1, h2);
      h[0][jj] = h0;
      h[1][jj] = h1;
      h[2][jj] = h2;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) out[(kb * 3 + i) * 64 + l] = h[i];
  }
}

__global__ __launch_bounds__(kLpThreads) void k_synthesis_lp(GroupView g, SynthInput in, int mode) {
  if (gate_closed(g)) return;  // an ended attempt of a device-controlled run
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (nh + 63) / 64;
  const int m = blockIdx.x / ntile;
  const int tile = blockIdx.x - m * ntile;
  const int b = blockIdx.y;
  const int L = N + 2 - m;
  const int nblk = (L + 31) / 32;
  extern __shared__ double2 sh[];
  bf16x4* bsplit = reinterpret_cast<bf16x4*>(sh);  // [nblk][3][64]
  double* cst = reinterpret_cast<double*>(sh);     // reused: [wave][16][16]
  // the order's split panel (k_split_panel_lp), copied into LDS
  const bf16x4* src =
      reinterpret_cast<const bf16x4*>(g.lps + (int64_t)b * g.lpsoff[N + 1] + g.lpsoff[m]);
  for (int it = threadIdx.x; it < nblk * 3 * 64; it += blockDim.x) bsplit[it] = src[it];
  __syncthreads();
  const int mypar = (threadIdx.x & 15) >> 3;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, q = lane >> 4;
  const int prow = tile * 64 + wave * 16 + r16;  // latitude row supplied to A
  const bool row_ok = prow < nh;
  const float* T = g.T1f + t1_order_offset(N, m, nh) + prow;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  float tn[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 8 * q + j;
    tn[j] = (row_ok && k < L) ? T[(int64_t)k * nh] : 0.f;
  }
  for (int kb = 0; kb < nblk; ++kb) {
    float tc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) tc[j] = tn[j];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = (kb + 1) * 32 + 8 * q + j;
      tn[j] = (row_ok && k < L) ? T[(int64_t)k * nh] : 0.f;
    }
    bf16x8 a0, a1, a2;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      __bf16 h0, h1, h2;
      split3f(tc[j], h0, h1, h2);
      a0[j] = h0;
      a1[j] = h1;
      a2[j] = h2;
    }
    const bf16x4* B = bsplit + kb * 3 * 64 + lane;
    const floatx4 cc = mfma_bf16x3(a0, a1, a2, interleave(B[0], mypar), interleave(B[64], mypar),
                                   interleave(B[128], mypar));
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += (double)cc[i];
  }
  __syncthreads();  // the split panel is no longer needed: reuse it
  // C rows 4q+i (latitudes of this wave), column r16
#pragma unroll
  for (int i = 0; i < 4; ++i) cst[(wave * 16 + 4 * q + i) * 16 + r16] = acc[i];
  __syncthreads();
  // one (field, latitude) per thread: E = columns 2f, 2f+1; O = columns 8+2f, 9+2f
  const int f = threadIdx.x >> 6;
  const int latl = threadIdx.x & 63;
  const int p = tile * 64 + latl;
  const int nf = (mode == SYNTH_NONLINEAR) ? 4 : 3;
  if (f >= nf || p >= nh) return;
  const double* row = cst + latl * 16;
  const double er = row[2 * f], ei = row[2 * f + 1], orr = row[8 + 2 * f], oi = row[9 + 2 * f];
  double2* out = g.F + ((int64_t)(b * 4 + f) * (N + 1) + m) * nlat;
  out[p] = make_double2(er + orr, ei + oi);
  const int ps = nlat - 1 - p;
  if (ps != p) out[ps] = make_double2(er - orr, ei - oi);
}

// LDS: folded spectra We, Wo [2][nh], then the split A operand
// [block][piece][4 K-slices][4 live rows] (rows 4..15 of A are zero).
size_t analysis_lp_lds_bytes(int nh) {
  const int nblk = (nh + 31) / 32;
  return 2 * sizeof(double2) * (size_t)nh + (size_t)nblk * 3 * 16 * sizeof(bf16x8);
}

__global__ __launch_bounds__(kLpThreads) void k_analysis_lp(GroupView g, AnalOutput out) {
  if (gate_closed(g)) return;  // an ended attempt of a device-controlled run
  const int N = g.N, nh = g.nh;
  const int ntile = (N + 1 + 63) / 64;
  const int item = xcd_item(blockIdx.x, 4 * ntile);
  const int m = item / ntile;
  const int tile = item - m * ntile;
  if (m > N || tile * 64 > N - m) return;  // uniform across the workgroup
  const int b = blockIdx.y;
  const int nblk = (nh + 31) / 32;
  extern __shared__ double2 wsh[];  // We [nh], Wo [nh], then the split A operand
  bf16x8* asplit = reinterpret_cast<bf16x8*>(wsh + 2 * nh);  // [nblk][3][16]
  const double2* Wb = g.W + ((int64_t)b * (N + 1) + m) * g.nlat;
  for (int p = threadIdx.x; p < nh; p += blockDim.x) {
    const double2 qn = Wb[p];
    const double2 qs = Wb[g.nlat - 1 - p];
    wsh[p] = make_double2(qn.x + qs.x, qn.y + qs.y);
    wsh[nh + p] = make_double2(qn.x - qs.x, qn.y - qs.y);
  }
  __syncthreads();
  // A operand of every 32-latitude block, split once: lane row r = l%16 holds
  // We.re, We.im, Wo.re, Wo.im for r < 4 (zero otherwise), K = 8*(l/16) .. +7
  for (int it = threadIdx.x; it < nblk * 16; it += blockDim.x) {
    const int pb = it >> 4, r = it & 3, q = (it >> 2) & 3;
    bf16x8 h[3];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int p = pb * 32 + 8 * q + j;
      double v = 0.0;
      if (p < nh) {
        const double2 w = wsh[((r >> 1) ? nh : 0) + p];
        v = (r & 1) ? w.y : w.x;
      }
      __bf16 h0, h1, h2;
      split3(v, h0, h1, h2);
      h[0][j] = h0;
      h[1][j] = h1;
      h[2][j] = h2;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) asplit[(pb * 3 + i) * 16 + q * 4 + r] = h[i];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, q = lane >> 4;
  const int kcol = tile * 64 + wave * 16 + r16;  // degree offset of this lane's B column
  const bool col_ok = m + kcol <= N;
  // rows p of this 64-degree tile, contiguous; this lane's degree column
  const float* T = g.T2f + g.t2off[m] + (int64_t)tile * nh * kTile + wave * 16 + r16;
  bf16x8 zero8;
#pragma unroll
  for (int j = 0; j < 8; ++j) zero8[j] = (__bf16)0.0f;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  float tn[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int p = 8 * q + j;
    tn[j] = (col_ok && p < nh) ? T[(int64_t)p * kTile] : 0.f;
  }
  for (int pb = 0; pb < nblk; ++pb) {
    float tc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) tc[j] = tn[j];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int p = (pb + 1) * 32 + 8 * q + j;
      tn[j] = (col_ok && p < nh) ? T[(int64_t)p * kTile] : 0.f;
    }
    bf16x8 b0, b1, b2;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      __bf16 h0, h1, h2;
      split3f(tc[j], h0, h1, h2);
      b0[j] = h0;
      b1[j] = h1;
      b2[j] = h2;
    }
    bf16x8 a0 = zero8, a1 = zero8, a2 = zero8;
    if (r16 < 4) {
      const bf16x8* A = asplit + pb * 3 * 16 + q * 4 + r16;
      a0 = A[0];
      a1 = A[16];
      a2 = A[32];
    }
    const floatx4 cc = mfma_bf16x3(a0, a1, a2, b0, b1, b2);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += (double)cc[i];
  }
  // lanes 0..15 hold rows 0..3 (We.re, We.im, Wo.re, Wo.im) of degree kcol
  if (q != 0 || !col_ok) return;
  const bool odd = kcol & 1;
  finish_degree(g, out, b, m, kcol, odd ? acc[2] : acc[0], odd ? acc[3] : acc[1]);
}

hipError_t launch_synthesis_lp(const GroupView& g, const SynthInput& in, int mode, int prec,
                               hipStream_t s) {
  if (prec != NSE_PREC_BF16X3) return hipErrorInvalidValue;
  if (!g.lps) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_split_panel_lp, dim3(g.N + 1, g.nb), dim3(kLpThreads),
                     split_panel_lp_lds_bytes(g.N), s, g, in, mode);
  const int ntile = (g.nh + 63) / 64;
  dim3 grid((g.N + 1) * ntile, g.nb);
  hipLaunchKernelGGL(k_synthesis_lp, grid, dim3(kLpThreads), synthesis_lp_lds_bytes(g.N), s, g,
                     in, mode);
  return hipGetLastError();
}

hipError_t launch_analysis_lp(const GroupView& g, const AnalOutput& out, int prec, hipStream_t s) {
  if (prec != NSE_PREC_BF16X3) return hipErrorInvalidValue;
  const int ntile = (g.N + 1 + 63) / 64;
  dim3 grid(xcd_grid((g.N + 1) * ntile, 4 * ntile), g.nb);
  hipLaunchKernelGGL(k_analysis_lp, grid, dim3(kLpThreads), analysis_lp_lds_bytes(g.nh), s, g,
                     out);
  return hipGetLastError();
}

}  // namespace nse
