// Step and order control of the adaptive NDF integrator (Section 4.2: the NDF_p
// formulas of eq. (ode_disc), p = 1..5, with the step chosen by comparing the
// error estimates of neighbouring orders, as in the ODE suite the section
// follows). The controller is written once, for host and device: the host runs
// it when a forcing callback has to be called at every time level, a kernel
// after each corrector sweep otherwise, so that the host never waits between
// sweeps.
#pragma once

#include "nse_internal.h"

namespace nse {

constexpr int kMaxNewton = 8;
constexpr int kNdfLogCap = 4096;  // device ring buffer of attempt records
// Device-controlled runs keep each sweep's four norm maxima in kNdfSpread
// copies, one 64-byte line each, so that the atomic maxima of many workgroups
// do not queue on one address; the deciding kernel reduces the copies.
constexpr int kNdfSpread = 64;
constexpr int kNdfSpreadStride = 8;  // 64-bit words per copy
constexpr int kNdfSpreadRow = kNdfSpread * kNdfSpreadStride;  // words per sweep

// kappa_p of the NDF_p formulas (Section 4.2, after eq. (ode_disc)).
__host__ __device__ inline double ndf_kappa(int k) {
  switch (k) {
    case 1: return -0.1850;
    case 2: return -1.0 / 9.0;
    case 3: return -0.0823;
    case 4: return -0.0415;
    default: return 0.0;
  }
}
__host__ __device__ inline double ndf_gamma(int k) {
  double g = 0.0;
  for (int j = 1; j <= k; ++j) g += 1.0 / j;
  return g;
}
// (1 - kappa_k) gamma_k and kappa_k gamma_k + 1/(k+1)
__host__ __device__ inline double ndf_alpha(int k) { return (1.0 - ndf_kappa(k)) * ndf_gamma(k); }
__host__ __device__ inline double ndf_error_constant(int k) {
  return ndf_kappa(k) * ndf_gamma(k) + 1.0 / (k + 1);
}
__host__ __device__ inline double ndf_binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}
__host__ __device__ inline bool ndf_finite(double x) { return x - x == 0.0; }

// Rescaling of backward differences from spacing h to rho h, order k:
// D_new[j] = sum_i R[j][i] D[i]. The interpolant through y_n .. y_{n-k} is
// p(t_n + s h) = sum_i c_i(s) D[i], c_i(s) = prod_{t<i} (s + t) / (t + 1)
// (Newton's backward form); the new differences are
// nabla'^j = sum_{q<=j} (-1)^q C(j, q) p(t_n - q rho h).
// The loops run to the largest order with guards, so that they unroll into
// straight-line code with constant reciprocals and binomials (one thread runs
// this on the device).
__host__ __device__ inline void step_change(int k, double rho,
                                            double R[kNdfMaxOrder + 1][kNdfMaxOrder + 1]) {
  constexpr int K = kNdfMaxOrder;
  double c[K + 1][K + 1];  // c[q][i] = c_i(-q rho)
#pragma unroll
  for (int q = 0; q <= K; ++q) {
    const double s = -q * rho;
    c[q][0] = 1.0;
#pragma unroll
    for (int i = 1; i <= K; ++i) c[q][i] = c[q][i - 1] * (s + (i - 1)) * (1.0 / i);
  }
#pragma unroll
  for (int j = 0; j <= K; ++j)
#pragma unroll
    for (int i = 0; i <= K; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q <= j; ++q)
        acc += ((q & 1) ? -1.0 : 1.0) * ndf_binom(j, q) * c[q][i];
      R[j][i] = (j <= k && i >= j && i <= k) ? acc : 0.0;
    }
}

// Forcing scale s(t) evaluated on the device (nse_forcing_schedule).
__host__ __device__ inline double schedule_scale(const nse_forcing_schedule& f, double t) {
  if (t <= f.t_on) return f.before;
  return f.amp * cos(f.omega * t + f.phase) * exp(-f.decay * (t - f.t_on));
}

// Controller state. On a device-controlled run it lives in device memory and
// is copied to the host between batches of attempts.
struct NdfCtl {
  // parameters
  double rtol, hmax, t_end;  // hmax = +inf when unbounded
  int kmax, K;               // largest order, corrector sweeps per attempt
  int device;                // 1: the attempt sequence runs gated on the device
  // state
  double t, h;
  int k, nconst, nfail, last;
  // pending work of the next k_ndf_prepare: the accepted correction (buffer
  // pend_dsel of an order-pend_k step), then a rescaling of D[0..pend_tk]
  int pend_accept, pend_k, pend_dsel, pend_transform, pend_tk;
  double R[kNdfMaxOrder + 1][kNdfMaxOrder + 1];
  // the running attempt
  int sweep;
  double dd1, dd_prev;
  double fscale;  // s(t + h)
  // device-controlled runs: a captured sequence of sweep slots, each a step
  // kernel (controller on the previous sweep's norms, and the prepare of a newly
  // opened attempt) and the chain with the corrector; the chain runs while
  // `running` (an attempt is open)
  int running;
  int fresh;   // the host opened the attempt: the next step kernel only prepares
  int done;    // t reached t_end
  int status;  // NDF_OK or the NDF_FAIL_* that stopped the run
  int prep_accept, prep_k_acc, prep_dsel, prep_transform, prep_k, prep_predict;
  // 1: this slot's prepare left the update of the differences to the analysis
  // epilogue (the synthesis did the step kernel's work), 0: already applied
  int prep_in_analysis, pad0;
  double prepR[kNdfMaxOrder + 1][kNdfMaxOrder + 1];
  // counters
  long long accepted, error_failures, newton_failures, evaluations, nlog;
  nse_adaptive_record rec;  // the attempt that ended last
};

enum { NDF_OK = 0, NDF_FAIL_CORRECTOR = 1, NDF_FAIL_ESTIMATE = 2, NDF_FAIL_UNDERFLOW = 3 };
enum { NDF_GO = 0, NDF_STOP = 1 };              // ndf_begin_attempt
enum { NDF_CONTINUE = 0, NDF_ENDED = 1 };       // ndf_after_sweep (or an NDF_FAIL_*, negated)

// Changes h (and rescales D[0..k] at the next prepare), composing with a
// rescaling that is still pending.
__host__ __device__ inline void ndf_rescale(NdfCtl& c, double h_new) {
  // loops to the largest order with guards: constant indices, registers only
  constexpr int K = kNdfMaxOrder;
  double R[K + 1][K + 1];
  step_change(c.k, h_new / c.h, R);
  if (c.pend_transform) {
    double P[K + 1][K + 1];
#pragma unroll
    for (int j = 0; j <= K; ++j)
#pragma unroll
      for (int i = 0; i <= K; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t <= K; ++t)
          if (t <= c.k) acc += R[j][t] * c.R[t][i];
        P[j][i] = (j <= c.k && i <= c.k) ? acc : 0.0;
      }
#pragma unroll
    for (int j = 0; j <= K; ++j)
#pragma unroll
      for (int i = 0; i <= K; ++i) c.R[j][i] = P[j][i];
  } else {
#pragma unroll
    for (int j = 0; j <= K; ++j)
#pragma unroll
      for (int i = 0; i <= K; ++i) c.R[j][i] = R[j][i];
  }
  c.pend_transform = 1;
  c.pend_tk = c.k;
  c.h = h_new;
  c.nconst = 0;
}

// Step size of the next attempt: at most hmax, and a step ending within 10 % of
// t_end ends there. NDF_STOP once t_end is reached; NDF_FAIL_UNDERFLOW (negated)
// when h falls below 16 eps |t|.
__host__ __device__ inline int ndf_begin_attempt(NdfCtl& c) {
  if (!(c.t < c.t_end)) return NDF_STOP;
  double h_new = c.h < c.hmax ? c.h : c.hmax;
  int last = 0;
  if (c.t + 1.1 * h_new >= c.t_end) {
    h_new = c.t_end - c.t;
    last = 1;
  }
  if (h_new != c.h) ndf_rescale(c, h_new);
  if (c.h <= 16.0 * 2.220446049250313e-16 * fabs(c.t)) return -NDF_FAIL_UNDERFLOW;
  c.last = last;
  c.sweep = 0;
  return NDF_GO;
}

__host__ __device__ inline double ndf_ratio(double e, double cst, int q, double rtol) {
  const double r = cst * pow(e / rtol, 1.0 / (q + 1));
  return 1.0 / (r > 0.1 ? r : 0.1);
}

__host__ __device__ inline void ndf_record(NdfCtl& c, double err, int sweeps, int outcome) {
  c.rec.t = c.t;
  c.rec.h = c.h;
  c.rec.err = err;
  c.rec.order = c.k;
  c.rec.sweeps = sweeps;
  c.rec.outcome = outcome;
  c.rec.reserved = 0;
  c.nlog++;
}

// After corrector sweep c.sweep + 1 with the square roots of its four norms
// (row: [0] d - dprev, [1] d, [2] D[k] + d, [3] d - D[k+1]): the Newton test
// from the second sweep on (rho = ratio of successive correction norms;
// rho >= 0.9 fails, rho / (1 - rho) ||d - dprev|| <= 0.1 rtol converges), then
// at the end of the attempt the error test and the step and order control.
// NDF_CONTINUE: run another sweep; NDF_ENDED: c.rec holds the attempt;
// -NDF_FAIL_*: a non-finite norm.
__host__ __device__ inline int ndf_after_sweep(NdfCtl& c, const double row[4]) {
  const int i = ++c.sweep;
  c.evaluations++;
  const int K = c.K, k = c.k;
  const double h = c.h, rtol = c.rtol;
  bool converged = false;
  if (K == 1) {
    if (!ndf_finite(row[0])) return -NDF_FAIL_CORRECTOR;
    converged = true;
  } else if (i == 1) {
    c.dd1 = row[0];
    return NDF_CONTINUE;
  } else {
    if (i == 2) {
      c.dd_prev = c.dd1;
      if (!ndf_finite(c.dd_prev)) return -NDF_FAIL_CORRECTOR;
    }
    const double dd = row[0];
    if (!ndf_finite(dd)) return -NDF_FAIL_CORRECTOR;
    if (dd == 0.0) {
      converged = true;
    } else {
      const double rho = c.dd_prev > 0.0 ? dd / c.dd_prev : INFINITY;
      if (rho < 0.9) {
        if (rho / (1.0 - rho) * dd <= 0.1 * rtol) {
          converged = true;
        } else {
          c.dd_prev = dd;
          if (i < K) return NDF_CONTINUE;
        }
      }
    }
  }
  if (!converged) {
    c.newton_failures++;
    ndf_record(c, __builtin_nan(""), i, NSE_ATTEMPT_NEWTON_FAIL);
    ndf_rescale(c, 0.3 * h);
    return NDF_ENDED;
  }
  if (!ndf_finite(row[1]) || !ndf_finite(row[2]) || !ndf_finite(row[3]))
    return -NDF_FAIL_ESTIMATE;
  const double err = ndf_error_constant(k) * row[1];
  if (err > rtol) {
    c.error_failures++;
    ndf_record(c, err, i, NSE_ATTEMPT_ERROR_FAIL);
    ++c.nfail;
    double ratio;
    if (c.nfail == 1) {
      ratio = 0.833 * pow(rtol / err, 1.0 / (k + 1));
      if (ratio < 0.1) ratio = 0.1;
      if (k > 1) {
        const double ekm1 = ndf_error_constant(k - 1) * row[2];
        double rkm1 = 1.0;
        if (ekm1 > 0.0) {
          rkm1 = 0.769 * pow(rtol / ekm1, 1.0 / k);
          if (rkm1 < 0.1) rkm1 = 0.1;
          if (rkm1 > 1.0) rkm1 = 1.0;
        }
        if (rkm1 > ratio) {
          ratio = rkm1;
          c.k = k - 1;
        }
      }
    } else {
      ratio = 0.5;
      if (c.nfail >= 3) c.k = 1;
    }
    ndf_rescale(c, ratio * h);
    return NDF_ENDED;
  }
  // accepted
  ndf_record(c, err, i, NSE_ATTEMPT_ACCEPTED);
  c.accepted++;
  c.nfail = 0;
  c.pend_accept = 1;
  c.pend_k = k;
  c.pend_dsel = (i - 1) & 1;
  c.t = c.last ? c.t_end : c.t + h;
  c.nconst++;
  if (c.nconst >= k + 2) {
    double r = ndf_ratio(err, 1.2, k, rtol);
    int knew = k;
    if (k > 1) {
      const double rm = ndf_ratio(ndf_error_constant(k - 1) * row[2], 1.3, k - 1, rtol);
      if (rm > r) {
        r = rm;
        knew = k - 1;
      }
    }
    if (k < c.kmax) {
      const double rp = ndf_ratio(ndf_error_constant(k + 1) * row[3], 1.4, k + 1, rtol);
      if (rp > r) {
        r = rp;
        knew = k + 1;
      }
    }
    if (r > 1.0) {
      c.k = knew;
      const double hn = r * h;
      ndf_rescale(c, hn < c.hmax ? hn : c.hmax);
    }
  }
  return NDF_ENDED;
}

// max that keeps a NaN operand (fmax would drop it)
__host__ __device__ inline double nanmax(double a, double b) { return (a != a || a > b) ? a : b; }

// Parameters of the next k_ndf_prepare from the pending work (predict: the
// predictor of order k follows).
__host__ __device__ inline void ndf_take_prepare(NdfCtl& c, int predict) {
  c.prep_accept = c.pend_accept;
  c.prep_k_acc = c.pend_k;
  c.prep_dsel = c.pend_dsel;
  c.prep_transform = c.pend_transform;
  c.prep_k = predict ? c.k : (c.pend_transform ? c.pend_tk : c.k);
  c.prep_predict = predict;
#pragma unroll
  for (int j = 0; j <= kNdfMaxOrder; ++j)
#pragma unroll
    for (int i = 0; i <= kNdfMaxOrder; ++i) c.prepR[j][i] = c.R[j][i];
  c.pend_accept = c.pend_transform = 0;
}

// Opens the next attempt of a device-controlled run (host before the first
// one, the step kernel after each): its step size, forcing scale and prepare
// snapshot; or the end of the run (done, or the failure in status).
__host__ __device__ inline void ndf_open_attempt(NdfCtl& c, const nse_forcing_schedule& sched) {
  c.running = 0;
  const int r = ndf_begin_attempt(c);
  if (r == NDF_STOP) {
    c.done = 1;
  } else if (r < 0) {
    c.status = -r;
  } else {
    c.fscale = schedule_scale(sched, c.t + c.h);
    ndf_take_prepare(c, 1);
    c.running = 1;
  }
}

// Controller of a device-controlled run after a sweep whose correction went to
// buffer `dsel_last`: another sweep, or the attempt's end (record in c.rec)
// and the next attempt opened. Returns NDF_CONTINUE, NDF_ENDED or -NDF_FAIL_*.
__host__ __device__ inline int ndf_decide(NdfCtl& c, const double row[4],
                                          const nse_forcing_schedule& sched, int dsel_last) {
  const int r = ndf_after_sweep(c, row);
  if (r == NDF_CONTINUE) return r;
  if (r < 0) {
    c.running = 0;
    c.status = -r;
    return r;
  }
  if (c.pend_accept) c.pend_dsel = dsel_last;
  ndf_open_attempt(c, sched);
  return NDF_ENDED;
}

// The step kernel of sweep slot j (buffer parity sel = j % 2): reads the
// controller state from ctl_in, writes it to ctl_out, reduces the norms of the
// previous slot (spread_in), clears this slot's norms (spread_clear).
struct NdfStepArgs {
  const NdfCtl* ctl_in;
  NdfCtl* ctl_out;
  const unsigned long long* spread_in;
  unsigned long long* spread_clear;
  int sel;
  nse_adaptive_record* log;
  nse_forcing_schedule sched;
};
hipError_t launch_ndf_step(const NdfArgs& a, const NdfStepArgs& st, hipStream_t s);
// The synthesis of sweep slot st.sel with the step kernel's work in its
// prologue, for one group whose nonlinear synthesis is the FP64 kernel with one
// latitude per lane and whose launch is resident at once (synthesis_takes_step):
// every workgroup runs the controller step; the workgroup of order 0, tile 0,
// member 0 writes the control block, the log and the cleared norm row; when an
// attempt opens every workgroup forms its order's predictor from the updated
// differences without storing them (the first latitude tile stores y0, psi and
// the iterate) and the analysis epilogue stores the differences. Not gated.
bool synthesis_takes_step(const GroupView& g);
hipError_t launch_synthesis_step(const GroupView& g, const SynthInput& in, const NdfArgs& a,
                                 const NdfStepArgs& st, hipStream_t s);

}  // namespace nse
