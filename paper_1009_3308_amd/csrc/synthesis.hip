// Legendre synthesis: for every order m and latitude, the Fourier coefficients
// of the grid fields needed by the nonlinear term (Section 4.2: direct Legendre
// sums in latitude, one contraction per azimuthal order m).
//
// With psi = sum lambda^(-1/2) alpha Y (u = Curl psi) and the absolute
// vorticity zeta_a = sum lambda^(1/2) alpha Y + 2 Omega cos(theta)
// (eqs. (stok_eig), (eq:vort), (C)), the four fields are
//   f0 = d psi / d phi            coefficients  i m psi[l]
//   f1 = sin(theta) d psi/dtheta  coefficients  (l-1) e(l) psi[l-1] - (l+2) e(l+1) psi[l+1]
//   f2 = sin(theta) d zeta_a/dtheta   (same recurrence on zeta_a)
//   f3 = d zeta_a / d phi         coefficients  i m zeta_a[l]
// with e(l) = sqrt((l^2 - m^2) / (4 l^2 - 1)), from the identity
//   sin(theta) dPbar[l,m]/dtheta = l e(l+1) Pbar[l+1,m] - (l+1) e(l) Pbar[l-1,m];
// f1 and f2 reach degree N+1. The grid product is then
//   u . Grad zeta_a = (f0 f2 - f1 f3) / sin^2(theta).
// For the grid-output mode the fields are f0 = d psi/d phi, f1 = sin(theta)
// d psi/d theta and f2 = zeta (no rotation term), f3 = 0.
//
// One workgroup per (order m, block of northern latitudes, member). The
// panel of coefficients for this m is built in LDS, then each thread streams
// its latitude column of T1[m][l-m][p] (coalesced across the wavefront) and
// accumulates even (l-m even) and odd parts separately, giving both the
// northern value E + O and the mirrored southern value E - O.
#include "nse_internal.h"

namespace nse {

constexpr int kSynthThreads = 128;

__global__ __launch_bounds__(kSynthThreads) void k_synthesis(GroupView g, SynthInput in,
                                                              int mode) {
  const int m = blockIdx.x;
  const int b = blockIdx.z;
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int L = N + 2 - m;  // degrees m .. N+1
  extern __shared__ double2 sh[];
  double2* a = sh;          // [L + 1] state coefficients alpha[l], l = m..N (0 beyond)
  double2* pan = sh + (L + 1);  // [L][4]

  const int64_t base = g.off[b] + coeff_offset(N, m);
  for (int k = threadIdx.x; k < L + 1; k += blockDim.x) {
    const int l = m + k;
    double2 v = make_double2(0.0, 0.0);
    if (l >= 1 && l <= N) {
#pragma unroll
      for (int i = 0; i < kMaxSources; ++i) {
        if (i < in.nsrc) {
          const double2 x = in.src[i][base + k];
          v.x += in.coef[i] * x.x;
          v.y += in.coef[i] * x.y;
        }
      }
      if (m == 0) v.y = 0.0;
    }
    a[k] = v;
  }
  __syncthreads();

  const double dm = (double)m;
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    const int l = m + k;
    const double dl = (double)l;
    // psi and zeta_a at degrees l-1, l, l+1 (zero outside m..N)
    auto psi_at = [&](int kk) -> double2 {
      const int ll = m + kk;
      if (kk < 0 || ll < 1 || ll > N) return make_double2(0.0, 0.0);
      const double r = 1.0 / sqrt((double)ll * (ll + 1));
      return make_double2(a[kk].x * r, a[kk].y * r);
    };
    auto zeta_at = [&](int kk) -> double2 {
      const int ll = m + kk;
      if (kk < 0 || ll < 1 || ll > N) return make_double2(0.0, 0.0);
      const double r = sqrt((double)ll * (ll + 1));
      double2 z = make_double2(a[kk].x * r, a[kk].y * r);
      if (mode == SYNTH_NONLINEAR && m == 0 && ll == 1) z.x += in.coriolis;
      return z;
    };
    const double e_l = (l > m) ? sqrt((dl * dl - dm * dm) / (4.0 * dl * dl - 1.0)) : 0.0;
    const double e_l1 = sqrt(((dl + 1) * (dl + 1) - dm * dm) / (4.0 * (dl + 1) * (dl + 1) - 1.0));
    const double cm = (dl - 1.0) * e_l, cp = (dl + 2.0) * e_l1;
    const double2 pm = psi_at(k - 1), p0 = psi_at(k), pp = psi_at(k + 1);
    const double2 zm = zeta_at(k - 1), z0 = zeta_at(k), zp = zeta_at(k + 1);
    double2 f0 = make_double2(-dm * p0.y, dm * p0.x);                 // i m psi
    double2 f1 = make_double2(cm * pm.x - cp * pp.x, cm * pm.y - cp * pp.y);
    double2 f2, f3;
    if (mode == SYNTH_NONLINEAR) {
      f2 = make_double2(cm * zm.x - cp * zp.x, cm * zm.y - cp * zp.y);
      f3 = make_double2(-dm * z0.y, dm * z0.x);                       // i m zeta_a
    } else {
      f2 = z0;
      f3 = make_double2(0.0, 0.0);
    }
    pan[4 * k + 0] = f0;
    pan[4 * k + 1] = f1;
    pan[4 * k + 2] = f2;
    pan[4 * k + 3] = f3;
  }
  __syncthreads();

  const int p = blockIdx.y * blockDim.x + threadIdx.x;
  if (p >= nh) return;
  const double* t = g.T1 + table_offset(N, m, nh) + p;
  double2 e[4], o[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    e[f] = make_double2(0.0, 0.0);
    o[f] = make_double2(0.0, 0.0);
  }
  int k = 0;
#pragma unroll 2
  for (; k + 1 < L; k += 2) {
    const double t0 = t[(int64_t)k * nh];
    const double t1 = t[(int64_t)(k + 1) * nh];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double2 A = pan[4 * k + f];
      const double2 B = pan[4 * (k + 1) + f];
      e[f].x = fma(t0, A.x, e[f].x);
      e[f].y = fma(t0, A.y, e[f].y);
      o[f].x = fma(t1, B.x, o[f].x);
      o[f].y = fma(t1, B.y, o[f].y);
    }
  }
  if (k < L) {
    const double t0 = t[(int64_t)k * nh];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double2 A = pan[4 * k + f];
      e[f].x = fma(t0, A.x, e[f].x);
      e[f].y = fma(t0, A.y, e[f].y);
    }
  }
  const int ps = nlat - 1 - p;
  const int nf = (mode == SYNTH_NONLINEAR) ? 4 : 3;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    if (f >= nf) break;
    double2* out = g.F + ((int64_t)(b * 4 + f) * nlat) * (N + 1) + m;
    out[(int64_t)p * (N + 1)] = make_double2(e[f].x + o[f].x, e[f].y + o[f].y);
    if (ps != p)
      out[(int64_t)ps * (N + 1)] = make_double2(e[f].x - o[f].x, e[f].y - o[f].y);
  }
}

hipError_t launch_synthesis(const GroupView& g, const SynthInput& in, int mode, hipStream_t s) {
  dim3 block(kSynthThreads);
  dim3 grid(g.N + 1, (g.nh + kSynthThreads - 1) / kSynthThreads, g.nb);
  const size_t lds = sizeof(double2) * (size_t)((g.N + 3) + 4 * (g.N + 2));
  hipLaunchKernelGGL(k_synthesis, grid, block, lds, s, g, in, mode);
  return hipGetLastError();
}

}  // namespace nse
