// Diagnostics of the experiments (Section 5.3): the energy spectrum E(L)
// (eq. (energy)), the band-limited input and the diagonal solve of the
// approximate inertial manifold (eq. (eq:p-p)). All elementwise over the
// coefficients; the nonlinear term in between comes from the hot path.
#include "nse_internal.h"

namespace nse {

namespace {

// E[b][L] = |alpha[L,0]|^2 + 2 sum_{m=1}^{L} |alpha[L,m]|^2 (the stored m > 0
// coefficient stands for m and -m); one thread per degree.
__global__ __launch_bounds__(256) void k_energy_spectrum(GroupView g, const double2* alpha,
                                                         double* E) {
  const int N = g.N, b = blockIdx.y;
  const int L = blockIdx.x * blockDim.x + threadIdx.x;
  if (L > N) return;
  const int64_t base = g.off[b];
  double e = 0.0;
  for (int m = 0; m <= L; ++m) {
    const double2 a = alpha[base + coeff_offset(N, m) + (L - m)];
    e += (m == 0 ? 1.0 : 2.0) * (a.x * a.x + a.y * a.y);
  }
  E[(int64_t)b * (N + 1) + L] = e;
}

// dst (truncation g.N) = the coefficients of degree 1..lmax of src (stored at
// truncation n_src), zero elsewhere.
__global__ __launch_bounds__(256) void k_band_input(GroupView g, const double2* src, int n_src,
                                                    int lmax, double2* dst) {
  const int N = g.N;
  const int m = blockIdx.x, b = blockIdx.z;
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  if (k > N - m) return;
  const int l = m + k;
  double2 v = make_double2(0.0, 0.0);
  if (l >= 1 && l <= lmax && l <= n_src) v = src[coeff_offset(n_src, m) + k];
  if (m == 0) v.y = 0.0;
  dst[g.off[b] + coeff_offset(N, m) + k] = v;
}

// phi[l,m] = (f - n)[l,m] / (nu lambda_l - 2 i Omega m / lambda_l) for l > N1,
// zero for l <= N1: the diagonal (nu A + C)^(-1) on Z[l,m] ((stok_eig),
// (Coriolis_ZLm)) of the band N1 < l <= N.
__global__ __launch_bounds__(256) void k_inertial_manifold(GroupView g, const double2* n,
                                                           const double2* f, int N1, double omega,
                                                           double2* phi) {
  const int N = g.N;
  const int m = blockIdx.x, b = blockIdx.z;
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  if (k > N - m) return;
  const int l = m + k;
  const int64_t s = g.off[b] + coeff_offset(N, m) + k;
  double2 out = make_double2(0.0, 0.0);
  if (l > N1 && l >= 1) {
    const double lam = (double)l * (l + 1);
    const double2 nn = n[s];
    double2 r = f ? f[s] : make_double2(0.0, 0.0);
    r = make_double2(r.x - nn.x, r.y - nn.y);
    const double dr = g.nu[b] * lam, di = -2.0 * omega * m / lam;
    const double den = dr * dr + di * di;
    out = make_double2((r.x * dr + r.y * di) / den, (r.y * dr - r.x * di) / den);
    if (m == 0) out.y = 0.0;
  }
  phi[s] = out;
}

}  // namespace

hipError_t launch_energy_spectrum(const GroupView& g, const double2* alpha, double* E,
                                  hipStream_t s) {
  dim3 grid((g.N + 1 + 255) / 256, g.nb);
  hipLaunchKernelGGL(k_energy_spectrum, grid, dim3(256), 0, s, g, alpha, E);
  return hipGetLastError();
}

hipError_t launch_band_input(const GroupView& g, const double2* src, int n_src, int lmax,
                             double2* dst, hipStream_t s) {
  dim3 grid(g.N + 1, (g.N + 1 + 255) / 256, g.nb);
  hipLaunchKernelGGL(k_band_input, grid, dim3(256), 0, s, g, src, n_src, lmax, dst);
  return hipGetLastError();
}

hipError_t launch_inertial_manifold(const GroupView& g, const double2* n, const double2* f,
                                    int N1, double omega, double2* phi, hipStream_t s) {
  dim3 grid(g.N + 1, (g.N + 1 + 255) / 256, g.nb);
  hipLaunchKernelGGL(k_inertial_manifold, grid, dim3(256), 0, s, g, n, f, N1, omega, phi);
  return hipGetLastError();
}

}  // namespace nse
