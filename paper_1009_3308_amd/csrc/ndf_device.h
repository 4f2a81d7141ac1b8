// Device pieces of the adaptive NDF integrator (Section 4.2, eq. (ode_disc) in
// backward differences at a quasi-constant step) shared by the sweep-slot step
// kernel (ndf_adaptive.hip), the synthesis that takes over its work in a
// single-group context (synthesis.hip) and the analysis epilogue that then
// updates the differences (spectral_ops.h): the update of one element's
// differences when an attempt opens, its predictor, and thread 0's controller
// step of a sweep slot.
#pragma once

#include "ndf_control.h"

namespace nse {

// The control block, copied through LDS in 8-byte words.
constexpr int kCtlWords = sizeof(NdfCtl) / sizeof(unsigned long long);
static_assert(sizeof(NdfCtl) % sizeof(unsigned long long) == 0, "8-byte words");

struct PrepareParams {
  int accept, k_acc, transform, k, predict;
  const double2* dacc;
  const double (*R)[kNdfMaxOrder + 1];
};

__device__ inline PrepareParams prepare_params(const NdfCtl& c, const double2* const dsel[2]) {
  return PrepareParams{c.prep_accept, c.prep_k_acc,         c.prep_transform, c.prep_k,
                       c.prep_predict, dsel[c.prep_dsel], c.prepR};
}

// The differences D[0..depth) of state slot s after the accepted-step update
// (with the correction dacc of an order-k_acc step) and the rescaling to a new
// step, in registers.
__device__ inline void prepared_differences(const double2* Dg, int64_t S, int depth,
                                            const PrepareParams& pp, int64_t s,
                                            double2 (&D)[kNdfDepth]) {
  const int k = pp.k;
#pragma unroll
  for (int j = 0; j < kNdfDepth; ++j)
    D[j] = (j < depth) ? Dg[(int64_t)j * S + s] : make_double2(0.0, 0.0);
  if (pp.accept) {
    // nabla^{k+1} y_{n+1} = d, nabla^{k+2} y_{n+1} = d - nabla^{k+1} y_n,
    // nabla^j y_{n+1} = nabla^j y_n + nabla^{j+1} y_{n+1}
    const int ka = pp.k_acc;
    const double2 d = pp.dacc[s];
#pragma unroll
    for (int j = 0; j < kNdfDepth; ++j)
      if (j == ka + 2) D[j] = make_double2(d.x - D[j - 1].x, d.y - D[j - 1].y);
#pragma unroll
    for (int j = 0; j < kNdfDepth; ++j)
      if (j == ka + 1) D[j] = d;
#pragma unroll
    for (int j = kNdfDepth - 2; j >= 0; --j)
      if (j <= ka) D[j] = make_double2(D[j].x + D[j + 1].x, D[j].y + D[j + 1].y);
  }
  if (pp.transform) {
#pragma unroll
    for (int j = 0; j < kNdfDepth; ++j) {
      double2 v = make_double2(0.0, 0.0);
      if (j <= k) {
#pragma unroll
        for (int i = 0; i <= kNdfMaxOrder; ++i)
          if (i >= j && i <= k) {
            v.x += pp.R[j][i] * D[i].x;
            v.y += pp.R[j][i] * D[i].y;
          }
      }
      D[j] = v;  // rows are computed from D[i >= j] before D[j] is replaced
    }
  }
}

// The predictor y0 = sum_{j<=k} D[j] and psi = sum_{1<=j<=k} gamma_j D[j].
__device__ inline void ndf_predictor(const double2 (&D)[kNdfDepth], int k, const double* gam,
                                     double2& y, double2& p) {
  y = D[0];
  p = make_double2(0.0, 0.0);
#pragma unroll
  for (int j = 1; j <= kNdfMaxOrder; ++j)
    if (j <= k) {
      y.x += D[j].x;
      y.y += D[j].y;
      p.x += gam[j] * D[j].x;
      p.y += gam[j] * D[j].y;
    }
}

// Prepare of state slot s: the updated differences stored (when they change),
// y0 and psi stored, and ycopy (if given) receiving y0 (the first iterate of a
// device-controlled attempt).
__device__ inline void prepare_element(const NdfArgs& a, const PrepareParams& pp, int64_t s,
                                       double2* ycopy) {
  double2 D[kNdfDepth];
  prepared_differences(a.D, a.S, a.depth, pp, s, D);
  if (pp.accept || pp.transform) {
#pragma unroll
    for (int j = 0; j < kNdfDepth; ++j)
      if (j < a.depth) a.D[(int64_t)j * a.S + s] = D[j];
  }
  if (pp.predict) {
    double2 y, p;
    ndf_predictor(D, pp.k, a.gam, y, p);
    a.y0[s] = y;
    a.psi[s] = p;
    if (ycopy) ycopy[s] = y;
  }
}

// Thread 0's controller step at the start of sweep slot st.sel on the control
// block sc (in LDS) and the previous sweep's four squared norm maxima: a
// freshly opened first attempt is prepared; a running attempt goes through the
// controller, which on the attempt's end records it (into the log when
// write_log) and opens the next. Returns whether the slot prepares an attempt.
// Every workgroup that runs it on the same inputs reaches the same result.
__device__ inline int ndf_slot_decide(NdfCtl& sc, const double norm[4], const NdfStepArgs& st,
                                      bool write_log) {
  int p = 0;
  if (sc.fresh) {
    sc.fresh = 0;
    p = sc.running;
  } else if (sc.running) {
    double row[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) row[q] = sqrt(norm[q]);
    const int r = ndf_decide(sc, row, st.sched, 1 - st.sel);
    if (r == NDF_ENDED) {
      if (write_log) st.log[(sc.nlog - 1) % kNdfLogCap] = sc.rec;
      p = sc.running;
    }
  }
  return p;
}

}  // namespace nse
