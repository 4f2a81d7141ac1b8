// Quadrature analysis and the time-step update.
//
// Analysis (Section 3, eqs. (disc_ip), (disc_vec_orth_proj); Section 4.2):
//   n[l,m] = lambda_l^(-1/2) sum_p Pbar[l,m](mu_p) (We_m(p) or Wo_m(p)),
// where the ring kernel has already applied the longitude DFT and the weights
// (2 pi / M) w_p, and the rings of each latitude pair are folded here into
// We = Q(p) + Q(p') (for l-m even) and Wo = Q(p) - Q(p') (odd), using
// Pbar[l,m](-mu) = (-1)^(l+m) Pbar[l,m](mu), so the sum runs over northern
// latitudes only. This is
// (u . Grad(zeta + 2 Omega cos theta), Y[l,m])_M lambda^(-1/2)
// = (B(u,u) + C u, Z[l,m])_M (eqs. (app1_weak_form), (short_nonlin1), (C)).
//
// Step update (eq. (ode_disc) with the Stokes term of eq. (stok_eig) implicit):
//   alpha_new = (h (f - n) - sum_{j>=1} c_j hist[j-1]) / (c_0 + h nu lambda_l),
// then either stored as the next fixed-point iterate or written to hist[0]
// after rotating hist[j] <- hist[j-1].
//
// Workgroups of four waves per (order m, tile of 64 degrees, member): one
// thread per degree l (coalesced reads of T2[m][p][l-m] across the wavefront),
// each wave summing a quarter of the northern latitudes, partial sums added
// through LDS. Orders are taken in XCD-local chunks of four neighbouring m so
// that the strided reads of W[lat][m] share L2 lines.
#include "nse_internal.h"

namespace nse {

constexpr int kAnalWaves = 4;
constexpr int kAnalThreads = 64 * kAnalWaves;

size_t analysis_lds_bytes(int nh) {
  return 2 * sizeof(double2) * (size_t)nh + sizeof(double) * 2 * kAnalThreads;
}

__global__ __launch_bounds__(kAnalThreads) void k_analysis(GroupView g, AnalOutput out) {
  const int N = g.N, nh = g.nh;
  const int ntile = (N + 1 + 63) / 64;
  const int item = xcd_item(blockIdx.x, 4 * ntile);
  const int m = item / ntile;
  const int tile = item - m * ntile;
  if (m > N || tile * 64 > N - m) return;  // uniform across the workgroup
  const int b = blockIdx.y;
  const int L = N + 2 - m;  // row length of T2 for this order
  extern __shared__ double2 wsh[];  // [2][nh] then [2][kAnalThreads] doubles
  double* red = reinterpret_cast<double*>(wsh + 2 * nh);
  // fold the ring spectra of each latitude pair: We = Q(p) + Q(p'), Wo = Q(p) - Q(p')
  const double2* Wb = g.W + (int64_t)b * g.nlat * (N + 1) + m;
  for (int p = threadIdx.x; p < nh; p += blockDim.x) {
    const double2 qn = Wb[(int64_t)p * (N + 1)];
    const double2 qs = Wb[(int64_t)(g.nlat - 1 - p) * (N + 1)];
    wsh[p] = make_double2(qn.x + qs.x, qn.y + qs.y);
    wsh[nh + p] = make_double2(qn.x - qs.x, qn.y - qs.y);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int k = tile * 64 + lane;
  const int l = m + k;
  const int pq = (nh + kAnalWaves - 1) / kAnalWaves;
  const int p0 = wave * pq;
  const int p1 = min(nh, p0 + pq);
  double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
  if (l <= N) {
    const double2* Ws = wsh + ((k & 1) ? nh : 0);
    const double* t = g.T2 + table_offset(N, m, nh) + k;
    int p = p0;
#pragma unroll 4
    for (; p + 1 < p1; p += 2) {
      const double t0 = t[(int64_t)p * L];
      const double t1 = t[(int64_t)(p + 1) * L];
      const double2 w0 = Ws[p], w1 = Ws[p + 1];
      ax = fma(t0, w0.x, ax);
      ay = fma(t0, w0.y, ay);
      bx = fma(t1, w1.x, bx);
      by = fma(t1, w1.y, by);
    }
    if (p < p1) {
      const double t0 = t[(int64_t)p * L];
      const double2 w0 = Ws[p];
      ax = fma(t0, w0.x, ax);
      ay = fma(t0, w0.y, ay);
    }
  }
  red[threadIdx.x] = ax + bx;
  red[kAnalThreads + threadIdx.x] = ay + by;
  __syncthreads();
  if (wave != 0 || l > N) return;
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int w = 0; w < kAnalWaves; ++w) {
    sx += red[w * 64 + lane];
    sy += red[kAnalThreads + w * 64 + lane];
  }
  const double lam = (double)l * (l + 1);
  double2 n = make_double2(0.0, 0.0);
  if (l >= 1) {
    const double r = 1.0 / sqrt(lam);
    n = make_double2(sx * r, m == 0 ? 0.0 : sy * r);
  }
  const int64_t slot = g.off[b] + coeff_offset(N, m) + k;
  if (out.mode == ANAL_NONLINEAR) {
    out.n_out[slot] = n;
    return;
  }
  // time-step update
  double2 rhs = make_double2(0.0, 0.0);
  if (out.forcing) {
    const double2 f = out.forcing[slot];
    rhs = make_double2(out.h * f.x, out.h * f.y);
  }
  rhs.x -= out.h * n.x;
  rhs.y -= out.h * n.y;
  double2 old[kMaxStepCoef];
#pragma unroll
  for (int j = 0; j < kMaxStepCoef; ++j) old[j] = make_double2(0.0, 0.0);
  const int nold = out.depth;
#pragma unroll
  for (int j = 0; j < kMaxStepCoef - 1; ++j)
    if (j < nold) old[j] = out.hist[(int64_t)j * out.state_count + slot];
#pragma unroll
  for (int j = 1; j < kMaxStepCoef; ++j) {
    if (j < out.ncoef) {
      rhs.x -= out.c[j] * old[j - 1].x;
      rhs.y -= out.c[j] * old[j - 1].y;
    }
  }
  const double denom = out.c[0] + out.h * g.nu[b] * lam;
  double2 a = make_double2(rhs.x / denom, rhs.y / denom);
  if (l == 0) a = make_double2(0.0, 0.0);
  if (m == 0) a.y = 0.0;
  if (out.nonfinite && !(isfinite(a.x) && isfinite(a.y))) *out.nonfinite = 1;
  if (out.mode == ANAL_STEP_ITER) {
    out.iter[slot] = a;
    return;
  }
#pragma unroll
  for (int j = kMaxStepCoef - 1; j >= 1; --j)
    if (j < nold) out.hist[(int64_t)j * out.state_count + slot] = old[j - 1];
  out.hist[slot] = a;
}

hipError_t launch_analysis(const GroupView& g, const AnalOutput& out, hipStream_t s) {
  dim3 block(kAnalThreads);
  const int ntile = (g.N + 1 + 63) / 64;
  dim3 grid(xcd_grid((g.N + 1) * ntile, 4 * ntile), g.nb);
  hipLaunchKernelGGL(k_analysis, grid, block, analysis_lds_bytes(g.nh), s, g, out);
  return hipGetLastError();
}

}  // namespace nse
