// Quadrature analysis and the time-step update.
//
// Analysis (Section 3, eqs. (disc_ip), (disc_vec_orth_proj); Section 4.2):
//   n[l,m] = lambda_l^(-1/2) sum_p Pbar[l,m](mu_p) (We_m(p) or Wo_m(p)),
// where the ring kernel has already applied the longitude DFT, the weights
// (2 pi / M) w_p and the north/south folding (We for l-m even, Wo for odd),
// so the sum runs over northern latitudes only. This is
// (u . Grad(zeta + 2 Omega cos theta), Y[l,m])_M lambda^(-1/2)
// = (B(u,u) + C u, Z[l,m])_M (eqs. (app1_weak_form), (short_nonlin1), (C)).
//
// Step update (eq. (ode_disc) with the Stokes term of eq. (stok_eig) implicit):
//   alpha_new = (h (f - n) - sum_{j>=1} c_j hist[j-1]) / (c_0 + h nu lambda_l),
// then either stored as the next fixed-point iterate or written to hist[0]
// after rotating hist[j] <- hist[j-1].
//
// One thread per degree l (coalesced reads of T2[m][p][l-m] across the
// wavefront); workgroups over (order m, block of degrees, member).
#include "nse_internal.h"

namespace nse {

constexpr int kAnalThreads = 64;

__global__ __launch_bounds__(kAnalThreads) void k_analysis(GroupView g, AnalOutput out) {
  const int m = blockIdx.x;
  const int b = blockIdx.z;
  const int N = g.N, nh = g.nh;
  const int L = N + 2 - m;  // row length of T2 for this order
  extern __shared__ double2 wsh[];  // [2][nh]
  const double2* Wm = g.W + ((int64_t)b * (N + 1) + m) * 2 * nh;
  for (int i = threadIdx.x; i < 2 * nh; i += blockDim.x) wsh[i] = Wm[i];
  __syncthreads();

  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  const int l = m + k;
  if (l > N) return;
  const double2* Ws = wsh + ((k & 1) ? nh : 0);
  const double* t = g.T2 + table_offset(N, m, nh) + k;
  double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
  int p = 0;
#pragma unroll 4
  for (; p + 1 < nh; p += 2) {
    const double t0 = t[(int64_t)p * L];
    const double t1 = t[(int64_t)(p + 1) * L];
    const double2 w0 = Ws[p], w1 = Ws[p + 1];
    ax = fma(t0, w0.x, ax);
    ay = fma(t0, w0.y, ay);
    bx = fma(t1, w1.x, bx);
    by = fma(t1, w1.y, by);
  }
  if (p < nh) {
    const double t0 = t[(int64_t)p * L];
    const double2 w0 = Ws[p];
    ax = fma(t0, w0.x, ax);
    ay = fma(t0, w0.y, ay);
  }
  const double lam = (double)l * (l + 1);
  double2 n = make_double2(0.0, 0.0);
  if (l >= 1) {
    const double r = 1.0 / sqrt(lam);
    n = make_double2((ax + bx) * r, m == 0 ? 0.0 : (ay + by) * r);
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
  dim3 grid(g.N + 1, (g.N + 1 + kAnalThreads - 1) / kAnalThreads, g.nb);
  const size_t lds = 2 * sizeof(double2) * (size_t)g.nh;
  hipLaunchKernelGGL(k_analysis, grid, block, lds, s, g, out);
  return hipGetLastError();
}

}  // namespace nse
