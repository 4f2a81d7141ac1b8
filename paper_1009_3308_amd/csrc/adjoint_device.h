// Device pieces of the adjoint of the spectral prologue and of one NDF_p step
// (eq. (ode_disc) transposed): the predictor cotangent alpha_bar from the panel
// cotangents, and the update of one coefficient's history cotangents.
#pragma once

#include "nse_internal.h"

namespace nse {

// alpha_bar at degree l = m + k of member b from the panel cotangents of
// order m (P = Pbar[b][m][k][f]): the panels are f0 = i m psi, f1 = S psi,
// f2 = S zeta_a, f3 = i m zeta_a with psi = lambda^(-1/2) alpha,
// zeta_a = lambda^(1/2) alpha and S c[k] = cm(k) c[k-1] - cp(k) c[k+1],
// cm(k) = (l-1) e(l), cp(k) = (l+2) e(l+1), so
//   psi_bar[j]  = -i m f0_bar[j] + cm(j+1) f1_bar[j+1] - cp(j-1) f1_bar[j-1],
//   zeta_bar[j] = -i m f3_bar[j] + cm(j+1) f2_bar[j+1] - cp(j-1) f2_bar[j-1],
//   alpha_bar[j] = lambda^(-1/2) (psi_bar[j] + lambda zeta_bar[j]),
// zero at l = 0 and real at m = 0; cm(j+1) = l e(l+1) and cp(j-1) = (l+1) e(l)
// come from the group's table rec_p, lambda^(-1/2) from rec_g.
__device__ inline double2 alpha_bar_at(const GroupView& g, const double2* P, int m, int k) {
  const int N = g.N, L = N + 2 - m, l = m + k;
  if (l < 1) return make_double2(0.0, 0.0);
  const double dm = (double)m;
  const int64_t sl = rec_slot(N, l, m);
  const double2 cc = g.rec_p[sl];  // (cm(k+1), cp(k-1))
  const double rs = g.rec_g[sl].y;  // lambda^(-1/2)
  double2 psib = make_double2(dm * P[4 * k + 0].y, -dm * P[4 * k + 0].x);  // -i m f0_bar
  double2 zetb = make_double2(dm * P[4 * k + 3].y, -dm * P[4 * k + 3].x);  // -i m f3_bar
  if (k + 1 < L) {
    psib.x = fma(cc.x, P[4 * (k + 1) + 1].x, psib.x);
    psib.y = fma(cc.x, P[4 * (k + 1) + 1].y, psib.y);
    zetb.x = fma(cc.x, P[4 * (k + 1) + 2].x, zetb.x);
    zetb.y = fma(cc.x, P[4 * (k + 1) + 2].y, zetb.y);
  }
  if (k >= 1) {
    psib.x = fma(-cc.y, P[4 * (k - 1) + 1].x, psib.x);
    psib.y = fma(-cc.y, P[4 * (k - 1) + 1].y, psib.y);
    zetb.x = fma(-cc.y, P[4 * (k - 1) + 2].x, zetb.x);
    zetb.y = fma(-cc.y, P[4 * (k - 1) + 2].y, zetb.y);
  }
  const double lam = (double)l * (l + 1);
  return make_double2(rs * fma(lam, zetb.x, psib.x), m == 0 ? 0.0 : rs * fma(lam, zetb.y, psib.y));
}

// The history update of StepAdjointArgs at degree l = m + k (k <= N - m) of
// member b, from the panel cotangents in g.Pbar, stored to a.hout (in place
// when a.hout == a.hin: the rows are read before any is written).
__device__ inline void step_adjoint_store(const GroupView& g, const StepAdjointArgs& a, int b,
                                          int m, int k) {
  const int N = g.N, l = m + k;
  const double2* P = g.Pbar + ((int64_t)b * (N + 1) + m) * (N + 2) * 4;  // [k][f]
  const int64_t S = a.state_count, slot = g.off[b] + coeff_offset(N, m) + k;
  const double2 ab = alpha_bar_at(g, P, m, k);
  const double lam = (double)l * (l + 1);
  const double q = 1.0 / fma(a.h * g.nu[b], lam, a.c[0]);
  double2 r = a.hin[slot];
  r = make_double2(r.x * q, r.y * q);  // r = hin[0] / (c_0 + h nu lambda)
  if (l == 0) r = make_double2(0.0, 0.0);
  if (m == 0) r.y = 0.0;
  double2 h[kMaxStepCoef];
#pragma unroll
  for (int j = 0; j < kMaxStepCoef; ++j)
    h[j] = j + 1 < a.depth ? a.hin[(int64_t)(j + 1) * S + slot] : make_double2(0.0, 0.0);
  // row j = hin[j+1] - c_{j+1} r + pi_j alpha_bar (terms past depth, ncoef, npi absent)
#pragma unroll
  for (int j = 0; j < kMaxStepCoef; ++j) {
    double2 v = h[j];
    if (j + 1 < a.ncoef) {
      v.x = fma(-a.c[j + 1], r.x, v.x);
      v.y = fma(-a.c[j + 1], r.y, v.y);
    }
    if (j < a.npi) {
      v.x = fma(a.pi[j], ab.x, v.x);
      v.y = fma(a.pi[j], ab.y, v.y);
    }
    if (j < a.depth) a.hout[(int64_t)j * S + slot] = v;
  }
}

}  // namespace nse
