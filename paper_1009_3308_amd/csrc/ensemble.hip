// Member-batched Legendre contractions for truncation groups with several
// members (an ensemble of flows that share N and the grid): the same sums as
// the synthesis and analysis of Section 4.2, with the table entries of one
// (order, tile) reused by a block of B members as the columns of an FP64
// matrix product on MFMA (v_mfma_f64_16x16x4f64). One table pass then serves
// B members instead of one, which turns the HBM-bound per-member sums into
// a compute-bound product.
//
// Synthesis, per (order m, tile of 64 northern latitudes, member block):
//   E[lat][c] = sum_{k even} T1[m][k][lat] P[k][c],  O = same over odd k,
// with the columns c = (member, field, re/im) of the coefficient panels
// (8 per member; the panels are those of spectral_ops.h, built here for a
// chunk of 32 degrees at a time into LDS); F(north) = E + O, F(south) = E - O.
// Wave w owns latitudes 16w..16w+15 of the tile: its A operand is a 16 x 4
// block of the table (four even or four odd degrees), its B operand a 4 x 16
// block of the panel chunk.
// Analysis, per (order m, tile of 64 degrees, member block):
//   s[k][c] = sum_p T2[m][k][p] Wf[p][c],  Wf = We (k even) or Wo (k odd),
// with the columns c = (member, re/im) of the ring spectra folded over
// latitude pairs, staged 64 latitudes at a time into LDS. Wave w owns degrees
// 32(w%2)..+31 of the tile (16 even rows and 16 odd rows) and half of each
// latitude chunk; the two halves meet in LDS and the epilogue of
// spectral_ops.h finishes each (member, degree).
//
// FP64 MFMA operand layout (checked on gfx950): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and receives D[l/16 + 4r][l%16], r = 0..3.
#include "spectral_ops.h"

namespace nse {

typedef double doublex4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kMbThreads = 256;
constexpr int kChunk = 32;  // panel degrees per LDS chunk (a multiple of 8)

__device__ __forceinline__ doublex4 mfma64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Predictor coefficient alpha[m + kk] of member b (zero outside l = 1..N,
// real at m = 0).
__device__ __forceinline__ double2 coef_at(const GroupView& g, const SynthInput& in, int b,
                                           int m, int kk) {
  const int N = g.N, ll = m + kk;
  double2 v = make_double2(0.0, 0.0);
  if (kk < 0 || ll < 1 || ll > N) return v;
  const int64_t slot = g.off[b] + coeff_offset(N, m) + kk;
#pragma unroll
  for (int i = 0; i < kMaxSources; ++i) {
    if (i < in.nsrc) {
      const double2 x = in.src[i][slot];
      v.x += in.coef[i] * x.x;
      v.y += in.coef[i] * x.y;
    }
  }
  if (m == 0) v.y = 0.0;
  return v;
}

// The four panel values of member b at k = l - m (nonlinear mode), as in
// build_panel: i m psi, S psi, S zeta_a, i m zeta_a.
__device__ __forceinline__ void panel4(const GroupView& g, const SynthInput& in, int b, int m,
                                       int k, double2 v[4]) {
  const int N = g.N, l = m + k;
  const double dl = (double)l, dm = (double)m;
  double2 ps[3], zs[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int kk = k - 1 + d, ll = m + kk;
    const double2 a = coef_at(g, in, b, m, kk);
    ps[d] = zs[d] = make_double2(0.0, 0.0);
    if (kk >= 0 && ll >= 1 && ll <= N) {
      const double lam = (double)ll * (ll + 1);
      const double sq = sqrt(lam), r = 1.0 / sq;
      ps[d] = make_double2(a.x * r, a.y * r);
      zs[d] = make_double2(a.x * sq, a.y * sq);
      if (m == 0 && ll == 1) zs[d].x += in.coriolis;
    }
  }
  const double e_l = (l > m) ? sqrt((dl * dl - dm * dm) / (4.0 * dl * dl - 1.0)) : 0.0;
  const double e_l1 = sqrt(((dl + 1) * (dl + 1) - dm * dm) / (4.0 * (dl + 1) * (dl + 1) - 1.0));
  const double cm = (dl - 1.0) * e_l, cp = (dl + 2.0) * e_l1;
  v[0] = make_double2(-dm * ps[1].y, dm * ps[1].x);
  v[1] = make_double2(cm * ps[0].x - cp * ps[2].x, cm * ps[0].y - cp * ps[2].y);
  v[2] = make_double2(cm * zs[0].x - cp * zs[2].x, cm * zs[0].y - cp * zs[2].y);
  v[3] = make_double2(-dm * zs[1].y, dm * zs[1].x);
}

template <int B>
__global__ __launch_bounds__(kMbThreads) void k_synthesis_mb(GroupView g, SynthInput in) {
  constexpr int NC = 8 * B;                // live columns per parity
  constexpr int NCB = (NC + 15) / 16;      // 16-column blocks
  constexpr int W = NCB * 16;              // LDS row width
  __shared__ double pan[kChunk][W];
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (nh + 63) / 64;
  const int m = blockIdx.x / ntile;
  const int tile = blockIdx.x - m * ntile;
  const int b0 = blockIdx.y * B;
  const int L = N + 2 - m;  // degrees m .. N+1
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int arow = lane & 15, kq = lane >> 4;
  const int lat = tile * 64 + wave * 16 + arow;  // this lane's A-operand latitude
  const bool lat_ok = lat < nh;
  const double* T = g.T1 + t1_order_offset(N, m, nh) + lat;

  doublex4 accE[NCB], accO[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) accE[c] = accO[c] = doublex4{0.0, 0.0, 0.0, 0.0};
  if (NC < W) {  // columns past the last member stay zero
    for (int i = threadIdx.x; i < kChunk * (W - NC); i += kMbThreads)
      pan[i / (W - NC)][NC + i % (W - NC)] = 0.0;
  }

  for (int kc = 0; kc < L; kc += kChunk) {
    for (int i = threadIdx.x; i < kChunk * B; i += kMbThreads) {
      const int kk = i / B, bb = i - kk * B;
      const int k = kc + kk, b = b0 + bb;
      double2 v[4] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0),
                      make_double2(0.0, 0.0)};
      if (k < L && b < g.nb) panel4(g, in, b, m, k, v);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        pan[kk][bb * 8 + 2 * f] = v[f].x;
        pan[kk][bb * 8 + 2 * f + 1] = v[f].y;
      }
    }
    __syncthreads();
    const int kend = min(kChunk, L - kc);
    for (int k8 = 0; k8 < kend; k8 += 8) {
      const int kE = kc + k8 + 2 * kq, kO = kE + 1;
      const double aE = (lat_ok && kE < L) ? T[(int64_t)kE * nh] : 0.0;
      const double aO = (lat_ok && kO < L) ? T[(int64_t)kO * nh] : 0.0;
      const double* pE = &pan[k8 + 2 * kq][arow];
      const double* pO = &pan[k8 + 2 * kq + 1][arow];
#pragma unroll
      for (int c = 0; c < NCB; ++c) {
        accE[c] = mfma64(aE, pE[16 * c], accE[c]);
        accO[c] = mfma64(aO, pO[16 * c], accO[c]);
      }
    }
    __syncthreads();
  }

  // lane holds rows (latitudes) kq + 4r of its wave's 16, column arow of each block
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    const int col = 16 * c + arow;
    if (col >= NC) continue;
    const int bb = col >> 3, f = (col & 7) >> 1, ri = col & 1;
    const int b = b0 + bb;
    if (b >= g.nb) continue;
    double* out = reinterpret_cast<double*>(g.F + ((int64_t)(b * 4 + f) * (N + 1) + m) * nlat);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = tile * 64 + wave * 16 + kq + 4 * r;
      if (p >= nh) continue;
      const double e = accE[c][r], o = accO[c][r];
      out[2 * p + ri] = e + o;
      const int ps = nlat - 1 - p;
      if (ps != p) out[2 * ps + ri] = e - o;
    }
  }
}

template <int B>
__global__ __launch_bounds__(kMbThreads) void k_analysis_mb(GroupView g, AnalOutput out) {
  static_assert(2 * B <= 16, "one 16-column block: (member, re/im)");
  __shared__ double wf[2][64][16];  // folded ring spectra of a 64-latitude chunk: [parity][p][col]
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (N + 2 + 63) / 64;  // tiles of T2 (degrees m .. N+1)
  const int m = blockIdx.x / ntile;
  const int tile = blockIdx.x - m * ntile;
  const int Lk = N + 1 - m;  // degrees m .. N
  if (tile * 64 >= Lk) return;  // uniform across the workgroup
  const int b0 = blockIdx.y * B;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = wave & 1, q = wave >> 1;
  const int arow = lane & 15, kq = lane >> 4;
  const double* T = g.T2 + g.t2off[m] + (int64_t)tile * nh * kTile + 32 * h + 2 * arow;

  for (int i = threadIdx.x; i < 2 * 64 * 16; i += kMbThreads) (&wf[0][0][0])[i] = 0.0;
  __syncthreads();
  doublex4 accE = {0.0, 0.0, 0.0, 0.0}, accO = {0.0, 0.0, 0.0, 0.0};
  for (int pc = 0; pc < nh; pc += 64) {
    for (int i = threadIdx.x; i < 64 * B; i += kMbThreads) {
      const int pp = i / B, bb = i - pp * B;
      const int p = pc + pp, b = b0 + bb;
      double2 we = make_double2(0.0, 0.0), wo = we;
      if (p < nh && b < g.nb) {
        const double2* Wb = g.W + (int64_t)b * nlat * (N + 1) + m;
        const double2 wn = Wb[(int64_t)p * (N + 1)];
        const double2 ws = Wb[(int64_t)(nlat - 1 - p) * (N + 1)];
        we = make_double2(wn.x + ws.x, wn.y + ws.y);
        wo = make_double2(wn.x - ws.x, wn.y - ws.y);
      }
      wf[0][pp][2 * bb] = we.x;
      wf[0][pp][2 * bb + 1] = we.y;
      wf[1][pp][2 * bb] = wo.x;
      wf[1][pp][2 * bb + 1] = wo.y;
    }
    __syncthreads();
#pragma unroll 4
    for (int p4 = 0; p4 < 32; p4 += 4) {
      const int pp = 32 * q + p4 + kq;
      const int p = pc + pp;
      double2 a = make_double2(0.0, 0.0);
      if (p < nh) a = *reinterpret_cast<const double2*>(T + (int64_t)p * kTile);
      accE = mfma64(a.x, wf[0][pp][arow], accE);
      accO = mfma64(a.y, wf[1][pp][arow], accO);
    }
    __syncthreads();
  }
  // the two latitude halves meet in LDS: red[q][local degree][col]
  double* red = &wf[0][0][0];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = kq + 4 * r;  // row of the 16 even (or odd) degrees of this wave
    red[(q * 64 + 32 * h + 2 * row) * 16 + arow] = accE[r];
    red[(q * 64 + 32 * h + 2 * row + 1) * 16 + arow] = accO[r];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * B; i += kMbThreads) {
    const int kl = i / B, bb = i - kl * B;
    const int k = tile * 64 + kl, b = b0 + bb;
    if (k >= Lk || b >= g.nb) continue;
    const double sx = red[kl * 16 + 2 * bb] + red[(64 + kl) * 16 + 2 * bb];
    const double sy = red[kl * 16 + 2 * bb + 1] + red[(64 + kl) * 16 + 2 * bb + 1];
    finish_degree(g, out, b, m, k, sx, sy);
  }
}

}  // namespace

hipError_t launch_synthesis_mb(const GroupView& g, const SynthInput& in, int B, hipStream_t s) {
  const int ntile = (g.nh + 63) / 64;
  dim3 grid((g.N + 1) * ntile, (g.nb + B - 1) / B);
  switch (B) {
    case 2: hipLaunchKernelGGL(k_synthesis_mb<2>, grid, dim3(kMbThreads), 0, s, g, in); break;
    case 4: hipLaunchKernelGGL(k_synthesis_mb<4>, grid, dim3(kMbThreads), 0, s, g, in); break;
    case 8: hipLaunchKernelGGL(k_synthesis_mb<8>, grid, dim3(kMbThreads), 0, s, g, in); break;
    case 16: hipLaunchKernelGGL(k_synthesis_mb<16>, grid, dim3(kMbThreads), 0, s, g, in); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_analysis_mb(const GroupView& g, const AnalOutput& out, int B, hipStream_t s) {
  const int ntile = (g.N + 2 + 63) / 64;
  dim3 grid((g.N + 1) * ntile, (g.nb + B - 1) / B);
  switch (B) {
    case 2: hipLaunchKernelGGL(k_analysis_mb<2>, grid, dim3(kMbThreads), 0, s, g, out); break;
    case 4: hipLaunchKernelGGL(k_analysis_mb<4>, grid, dim3(kMbThreads), 0, s, g, out); break;
    case 8: hipLaunchKernelGGL(k_analysis_mb<8>, grid, dim3(kMbThreads), 0, s, g, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nse
