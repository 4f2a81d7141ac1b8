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
// One workgroup of four waves per (order m, tile of 64 northern latitudes,
// member). The panel of coefficients for this m is built in LDS; each wave
// then streams a quarter of the degree range of its latitude column of
// T1[m][l-m][p] (coalesced across the wavefront), accumulating even (l-m even)
// and odd parts separately, and the four partial sums are added through LDS.
// Each latitude yields the northern value E + O and the mirrored southern value
// E - O. Output F[b][f][m][lat] is written latitude-contiguous.
#include "nse_internal.h"

namespace nse {

constexpr int kSynthWaves = 4;
constexpr int kSynthThreads = 64 * kSynthWaves;
constexpr int kRed = 16;  // partial sums per lane: 4 fields x (E, O) x (re, im)

__host__ __device__ inline int synth_pan_slots(int N) {
  // panel [L][4] double2, reused afterwards for the cross-wave reduction
  const int pan = 4 * (N + 2);
  const int red = kSynthWaves * kRed * 64 / 2;
  return pan > red ? pan : red;
}

size_t synthesis_lds_bytes(int N) {
  return sizeof(double2) * (size_t)((N + 3) + synth_pan_slots(N));
}

__global__ __launch_bounds__(kSynthThreads) void k_synthesis(GroupView g, SynthInput in,
                                                              int mode) {
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (nh + 63) / 64;
  const int m = blockIdx.x / ntile;
  const int tile = blockIdx.x - m * ntile;
  const int b = blockIdx.y;
  const int L = N + 2 - m;  // degrees m .. N+1
  extern __shared__ double2 sh[];
  double2* a = sh;              // [L + 1] state coefficients alpha[l], l = m..N (0 beyond)
  double2* pan = sh + (N + 3);  // [L][4]

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
    // psi and zeta_a at degrees l-1, l, l+1 (zero outside 1..N)
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

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int p = tile * 64 + lane;
  // even-length quarter of the degree range for this wave
  const int chunk = ((L + 2 * kSynthWaves - 1) / (2 * kSynthWaves)) * 2;
  const int k0 = wave * chunk;
  const int k1 = min(L, k0 + chunk);
  double acc[kRed];
#pragma unroll
  for (int i = 0; i < kRed; ++i) acc[i] = 0.0;
  if (p < nh && k0 < k1) {
    const double* t = g.T1 + table_offset(N, m, nh) + p;
    int k = k0;
#pragma unroll 4
    for (; k + 1 < k1; k += 2) {
      const double t0 = t[(int64_t)k * nh];
      const double t1 = t[(int64_t)(k + 1) * nh];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const double2 A = pan[4 * k + f];
        const double2 B = pan[4 * (k + 1) + f];
        acc[4 * f + 0] = fma(t0, A.x, acc[4 * f + 0]);
        acc[4 * f + 1] = fma(t0, A.y, acc[4 * f + 1]);
        acc[4 * f + 2] = fma(t1, B.x, acc[4 * f + 2]);
        acc[4 * f + 3] = fma(t1, B.y, acc[4 * f + 3]);
      }
    }
    if (k < k1) {
      const double t0 = t[(int64_t)k * nh];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const double2 A = pan[4 * k + f];
        acc[4 * f + 0] = fma(t0, A.x, acc[4 * f + 0]);
        acc[4 * f + 1] = fma(t0, A.y, acc[4 * f + 1]);
      }
    }
  }
  __syncthreads();  // panel no longer needed: reuse it for the reduction
  double* red = reinterpret_cast<double*>(pan);  // [wave][kRed][64]
#pragma unroll
  for (int i = 0; i < kRed; ++i) red[(wave * kRed + i) * 64 + lane] = acc[i];
  __syncthreads();
  // wave f finishes field f for its 64 latitudes
  const int f = wave;
  const int nf = (mode == SYNTH_NONLINEAR) ? 4 : 3;
  if (f >= nf || p >= nh) return;
  double er = 0.0, ei = 0.0, orr = 0.0, oi = 0.0;
#pragma unroll
  for (int w = 0; w < kSynthWaves; ++w) {
    er += red[(w * kRed + 4 * f + 0) * 64 + lane];
    ei += red[(w * kRed + 4 * f + 1) * 64 + lane];
    orr += red[(w * kRed + 4 * f + 2) * 64 + lane];
    oi += red[(w * kRed + 4 * f + 3) * 64 + lane];
  }
  double2* out = g.F + ((int64_t)(b * 4 + f) * (N + 1) + m) * nlat;
  out[p] = make_double2(er + orr, ei + oi);
  const int ps = nlat - 1 - p;
  if (ps != p) out[ps] = make_double2(er - orr, ei - oi);
}

hipError_t launch_synthesis(const GroupView& g, const SynthInput& in, int mode, hipStream_t s) {
  dim3 block(kSynthThreads);
  const int ntile = (g.nh + 63) / 64;
  dim3 grid((g.N + 1) * ntile, g.nb);
  hipLaunchKernelGGL(k_synthesis, grid, block, synthesis_lds_bytes(g.N), s, g, in, mode);
  return hipGetLastError();
}

}  // namespace nse
