// Spectral-side pieces shared by the FP64 and reduced-precision contraction
// kernels: the per-order input and coefficient panels of the synthesis, and
// the per-degree epilogue of the analysis (post-scaling and time step).
#pragma once

#include "ndf_device.h"
#include "nse_internal.h"

namespace nse {

// alpha[l, m] for l = m..N into a[k], k = l - m (sum of the input sources,
// e.g. the extrapolated predictor); zero for l = 0 and for k up to L, where
// L = N + 2 - m is the number of degrees the panels reach (m..N+1).
__device__ inline void load_order(double2* a, const GroupView& g, const SynthInput& in, int b,
                                  int m, int L) {
  const int N = g.N;
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
}

// The four coefficient panels of order m (value of field f at k = l - m < L):
// with psi = lambda^(-1/2) alpha and the absolute vorticity zeta_a =
// lambda^(1/2) alpha (+ 2 Omega sqrt(4 pi / 3) at (1, 0)),
//   f0 = i m psi,  f1 = sin(theta) dpsi/dtheta,  f2 = sin(theta) dzeta_a/dtheta,  f3 = i m zeta_a,
// where sin(theta) d/dtheta acts on the coefficients by
//   (l-1) e(l) c[l-1] - (l+2) e(l+1) c[l+1],  e(l) = sqrt((l^2 - m^2) / (4 l^2 - 1)),
// from sin(theta) dPbar[l,m]/dtheta = l e(l+1) Pbar[l+1,m] - (l+1) e(l) Pbar[l-1,m].
// Grid-output mode: f0 = i m psi, f1 = sin(theta) dpsi/dtheta, f2 = zeta, f3 = 0.
// a[] holds alpha[m + k] for k = 0..L (zero outside 1..N), see load_order.
__device__ inline double2 panel_value(const double2* a, int N, int m, int k, int f, int mode,
                                      double coriolis) {
  const int l = m + k;
  const double dl = (double)l, dm = (double)m;
  // scale of psi (s = -1) or zeta_a (s = +1) at offset kk
  auto coef = [&](int kk, bool zeta) -> double2 {
    const int ll = m + kk;
    if (kk < 0 || ll < 1 || ll > N) return make_double2(0.0, 0.0);
    const double lam = (double)ll * (ll + 1);
    const double r = zeta ? sqrt(lam) : 1.0 / sqrt(lam);
    double2 z = make_double2(a[kk].x * r, a[kk].y * r);
    if (zeta && mode != SYNTH_GRID && m == 0 && ll == 1) z.x += coriolis;
    return z;
  };
  if (f == 0 || (f == 3 && mode != SYNTH_GRID)) {
    const double2 c = coef(k, f == 3);
    return make_double2(-dm * c.y, dm * c.x);  // i m c
  }
  if (f == 3) return make_double2(0.0, 0.0);
  if (f == 2 && mode == SYNTH_GRID) return coef(k, true);
  const bool zeta = (f == 2);
  const double e_l = (l > m) ? sqrt((dl * dl - dm * dm) / (4.0 * dl * dl - 1.0)) : 0.0;
  const double e_l1 = sqrt(((dl + 1) * (dl + 1) - dm * dm) / (4.0 * (dl + 1) * (dl + 1) - 1.0));
  const double cm = (dl - 1.0) * e_l, cp = (dl + 2.0) * e_l1;
  const double2 lo = coef(k - 1, zeta), hi = coef(k + 1, zeta);
  return make_double2(cm * lo.x - cp * hi.x, cm * lo.y - cp * hi.y);
}

// All four panels of order m into pan[NF k + f], k < L (one degree per thread,
// the neighbouring coefficients shared by the four fields). With `stream` set,
// the grid-output mode puts the stream function -lambda^(-1/2) alpha (Psi_N of
// eq. (eq:vort_app)) in f2 instead of the vorticity.
template <int NF = 4>
__device__ inline void build_panel(double2* pan, const double2* a, int N, int m, int L, int mode,
                                   double coriolis, bool stream = false) {
  const double dm = (double)m;
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    const int l = m + k;
    const double dl = (double)l;
    double2 ps[3], zs[3];  // psi and zeta_a at k-1, k, k+1
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int kk = k - 1 + d, ll = m + kk;
      ps[d] = zs[d] = make_double2(0.0, 0.0);
      if (kk >= 0 && ll >= 1 && ll <= N) {
        const double lam = (double)ll * (ll + 1);
        const double sq = sqrt(lam), r = 1.0 / sq;
        ps[d] = make_double2(a[kk].x * r, a[kk].y * r);
        zs[d] = make_double2(a[kk].x * sq, a[kk].y * sq);
        if (mode != SYNTH_GRID && m == 0 && ll == 1) zs[d].x += coriolis;
      }
    }
    const double e_l = (l > m) ? sqrt((dl * dl - dm * dm) / (4.0 * dl * dl - 1.0)) : 0.0;
    const double e_l1 = sqrt(((dl + 1) * (dl + 1) - dm * dm) / (4.0 * (dl + 1) * (dl + 1) - 1.0));
    const double cm = (dl - 1.0) * e_l, cp = (dl + 2.0) * e_l1;
    pan[NF * k + 0] = make_double2(-dm * ps[1].y, dm * ps[1].x);
    pan[NF * k + 1] = make_double2(cm * ps[0].x - cp * ps[2].x, cm * ps[0].y - cp * ps[2].y);
    if (mode != SYNTH_GRID) {
      pan[NF * k + 2] = make_double2(cm * zs[0].x - cp * zs[2].x, cm * zs[0].y - cp * zs[2].y);
      pan[NF * k + 3] = make_double2(-dm * zs[1].y, dm * zs[1].x);
    } else {
      pan[NF * k + 2] = stream ? make_double2(-ps[1].x, -ps[1].y) : zs[1];
      pan[NF * k + 3] = make_double2(0.0, 0.0);
    }
  }
}

// Degree l = m + k of the analysis: s = sum_p Pbar[l,m](mu_p) (We or Wo).
// n[l,m] = lambda_l^(-1/2) s (zero at l = 0, real at m = 0); then either
// stored (nonlinear mode) or used in the NDF step
//   alpha_new = (h (f - n) - sum_{j>=1} c_j hist[j-1]) / (c_0 + h nu lambda_l),
// written as the next fixed-point iterate or, on the last sweep, to hist[0]
// after rotating hist[j] <- hist[j-1] (eq. (ode_disc), eq. (stok_eig)).
// Inputs of the step update of degree l = m + k, in[0] = f[l,m] (zero without
// forcing) and in[1 + j] = hist[j][l,m] for j < depth; nothing in the nonlinear
// mode. Kernels can request them early and keep them until finish_degree_from.
constexpr int kDegreeInputs = kMaxStepCoef;  // forcing + up to kMaxStepCoef - 1 history slots
// ANAL_NDF: in[0] = f, in[1] = D[0], in[2] = y0, in[3] = psi, in[4] = dprev,
// in[5] = D[order] (order > 1), in[6] = D[order + 1] (order < kmax).
// NDF: the kernel instance serves ANAL_NDF (the mode's inputs are compiled
// into that instance only).
template <bool NDF = false>
__device__ inline void load_degree_inputs(const GroupView& g, const AnalOutput& out, int b, int m,
                                          int k, double2* in) {
  if (out.mode == ANAL_NONLINEAR) return;
  const int64_t slot = g.off[b] + coeff_offset(g.N, m) + k;
  if (NDF && out.mode == ANAL_NDF) {
    const double2 z = make_double2(0.0, 0.0);
    const int64_t S = out.state_count;
    const NdfCtl& c = *out.ctl;
    const int q = c.k;
    in[0] = out.forcing ? out.forcing[slot] : z;
    in[2] = out.y0[slot];
    in[3] = out.psi[slot];
    in[4] = (out.dprev && c.sweep != 0) ? out.dprev[slot] : z;  // none on a first sweep
    if (c.prep_in_analysis && (c.prep_accept || c.prep_transform)) {
      // the attempt opened in this slot: its update of the differences, which
      // the synthesis only used for the predictor, is applied here (each
      // element by one thread)
      double2 D[kNdfDepth];
      prepared_differences(out.D, S, out.ddepth, prepare_params(c, out.dacc), slot, D);
      in[1] = D[0];
      in[5] = in[6] = z;
#pragma unroll
      for (int j = 0; j < kNdfDepth; ++j) {
        if (j < out.ddepth) out.Dw[(int64_t)j * S + slot] = D[j];
        if (j == q && q > 1) in[5] = D[j];
        if (j == q + 1 && q < out.kmax) in[6] = D[j];
      }
      return;
    }
    in[1] = out.D[slot];
    in[5] = q > 1 ? out.D[(int64_t)q * S + slot] : z;
    in[6] = q < out.kmax ? out.D[(int64_t)(q + 1) * S + slot] : z;
    return;
  }
  in[0] = out.forcing ? out.forcing[slot] : make_double2(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < kMaxStepCoef - 1; ++j)
    in[1 + j] = (j < out.depth) ? out.hist[(int64_t)j * out.state_count + slot]
                                : make_double2(0.0, 0.0);
}

template <bool NDF = false>
__device__ inline void finish_degree_from(const GroupView& g, const AnalOutput& out, int b, int m,
                                          int k, double sx, double sy, const double2* in,
                                          double* nv = nullptr);

__device__ inline void finish_degree(const GroupView& g, const AnalOutput& out, int b, int m,
                                     int k, double sx, double sy) {
  double2 in[kDegreeInputs];
  load_degree_inputs(g, out, b, m, k, in);
  finish_degree_from(g, out, b, m, k, sx, sy, in);
}

// As finish_degree, with the step-update inputs already loaded (load_degree_inputs).
// NDF (out.mode == ANAL_NDF): nv receives the coefficient's four weighted norm
// terms (squares).
template <bool NDF>
__device__ inline void finish_degree_from(const GroupView& g, const AnalOutput& out, int b, int m,
                                          int k, double sx, double sy, const double2* in,
                                          double* nv) {
  const int l = m + k;
  const double lam = (double)l * (l + 1);
  double2 n = make_double2(0.0, 0.0);
  if (l >= 1) {
    const double r = 1.0 / sqrt(lam);
    n = make_double2(sx * r, m == 0 ? 0.0 : sy * r);
  }
  const int64_t slot = g.off[b] + coeff_offset(g.N, m) + k;
  if (out.mode == ANAL_NONLINEAR) {
    out.n_out[slot] = n;
    return;
  }
  if constexpr (NDF) {
    // the corrector of k_ndf_correct, with n in registers
    const NdfCtl& c = *out.ctl;
    const int q = c.k;
    const double h = c.h, fs = c.fscale;
    const double Lam = g.nu[b] * lam;
    const double2 f = make_double2(fs * in[0].x, fs * in[0].y);
    const double2 D0 = in[1], y0 = in[2], ps = in[3], dp = in[4];
    const double hL = h * Lam;
    const double den = ndf_alpha(q) + hL;
    double2 d = make_double2((h * (f.x - n.x) - hL * y0.x - ps.x) / den,
                             (h * (f.y - n.y) - hL * y0.y - ps.y) / den);
    if (l == 0) d = make_double2(0.0, 0.0);
    if (m == 0) d.y = 0.0;
    const double2 y = make_double2(y0.x + d.x, y0.y + d.y);
    out.dout[slot] = d;
    out.yout[slot] = y;
    const double wt2 = fmax(fmax(D0.x * D0.x + D0.y * D0.y, y.x * y.x + y.y * y.y), out.thr2);
    const double2 e0 = make_double2(d.x - dp.x, d.y - dp.y);
    nv[0] = (e0.x * e0.x + e0.y * e0.y) / wt2;
    nv[1] = (d.x * d.x + d.y * d.y) / wt2;
    const double2 e2 = make_double2(in[5].x + d.x, in[5].y + d.y);
    const double2 e3 = make_double2(d.x - in[6].x, d.y - in[6].y);
    nv[2] = q > 1 ? (e2.x * e2.x + e2.y * e2.y) / wt2 : 0.0;
    nv[3] = q < out.kmax ? (e3.x * e3.x + e3.y * e3.y) / wt2 : 0.0;
    return;
  }
  const double2 f = in[0];
  double2 rhs = make_double2(out.h * f.x, out.h * f.y);
  rhs.x -= out.h * n.x;
  rhs.y -= out.h * n.y;
  double2 old[kMaxStepCoef];
#pragma unroll
  for (int j = 0; j < kMaxStepCoef; ++j) old[j] = make_double2(0.0, 0.0);
  const int nold = out.depth;
#pragma unroll
  for (int j = 0; j < kMaxStepCoef - 1; ++j)
    if (j < nold) old[j] = in[1 + j];
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
  if (out.shift) {
    out.hist[slot - out.state_count] = a;
    return;
  }
#pragma unroll
  for (int j = kMaxStepCoef - 1; j >= 1; --j)
    if (j < nold) out.hist[(int64_t)j * out.state_count + slot] = old[j - 1];
  out.hist[slot] = a;
}

}  // namespace nse
