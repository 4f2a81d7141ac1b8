// Normalised associated Legendre functions Pbar[l,m](mu_p) on the northern
// Gauss-Legendre nodes (Section 2, eq. (sph_har), with the Condon-Shortley
// phase and int_{-1}^{1} Pbar^2 dmu = 1 / (2 pi)), computed once per group in
// FP64 on the GPU and stored twice (layouts in nse_internal.h):
//   T1[m][k][p]             (latitude fastest: read by the synthesis),
//   T2[m][deg tile][p][64]  (degree fastest: read by the analysis),
// for l = m .. N+1 (k = l - m; the sin(theta) d/dtheta fields reach degree N+1).
// The southern hemisphere follows from Pbar[l,m](-mu) = (-1)^(l+m) Pbar[l,m](mu).
#include "nse_internal.h"

namespace nse {

// One thread per (m, p). Recurrences:
//   Pbar[m,m]   = -sqrt((2k+1)/(2k)) sin(theta) Pbar[m-1,m-1],  Pbar[0,0] = 1/sqrt(4 pi),
//   Pbar[l,m]   = a(l,m) (mu Pbar[l-1,m] - Pbar[l-2,m] / a(l-1,m)),
//   a(l,m)      = sqrt((4 l^2 - 1) / (l^2 - m^2)).
// Values that leave the double range near the poles flush to zero.
__global__ void k_legendre_table(GroupView g, double* T1, double* T2, float* T1f, float* T2f) {
  const int m = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.nh || m > g.N) return;
  const int N = g.N, nh = g.nh;
  const int L = N + 2 - m;  // degrees m .. N+1
  const double x = g.mu[p];
  const double s = sqrt((1.0 - x) * (1.0 + x));
  double pmm = 0.28209479177387814347;  // 1 / sqrt(4 pi)
  for (int k = 1; k <= m; ++k) pmm *= -sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
  const int64_t b1 = t1_order_offset(N, m, nh) + p;
  const int64_t b2 = g.t2off[m] + (int64_t)p * kTile;
  double prev2 = 0.0, prev1 = pmm;
  double a_prev = 0.0;
  for (int k = 0; k < L; ++k) {
    const int l = m + k;
    double v;
    if (k == 0) {
      v = pmm;
    } else {
      const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
      v = (k == 1) ? a * x * prev1 : a * (x * prev1 - prev2 / a_prev);
      a_prev = a;
      prev2 = prev1;
      prev1 = v;
    }
    const int64_t i1 = b1 + (int64_t)k * nh;
    const int64_t i2 = b2 + (int64_t)(k / kTile) * nh * kTile + (k % kTile);
    T1[i1] = v;
    T2[i2] = v;
    if (T1f) {
      T1f[i1] = (float)v;
      T2f[i2] = (float)v;
    }
  }
}

hipError_t launch_legendre_table(const GroupView& g, double* T1, double* T2, float* T1f,
                                 float* T2f, hipStream_t s) {
  dim3 block(64);
  dim3 grid((g.nh + 63) / 64, g.N + 1);
  hipLaunchKernelGGL(k_legendre_table, grid, block, 0, s, g, T1, T2, T1f, T2f);
  return hipGetLastError();
}

}  // namespace nse
