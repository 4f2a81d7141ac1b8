// Device side of the adaptive NDF integrator (Section 4.2, eq. (ode_disc) with
// orders 1..5, written in backward differences at a quasi-constant step).
// k_ndf_prepare and k_ndf_correct are elementwise over the state; the nonlinear
// term between them comes from the synthesis / ring / analysis chain. On a
// device-controlled run k_ndf_decide runs the controller of ndf_control.h
// after each sweep and opens the next attempt.
#include "ndf_control.h"

namespace nse {

namespace {

__device__ inline double2 zero2() { return make_double2(0.0, 0.0); }
__device__ inline double abs2(double2 z) { return z.x * z.x + z.y * z.y; }

// The control block in LDS: copied in by the whole workgroup, worked on by
// thread 0, copied back.
constexpr int kCtlWords = sizeof(NdfCtl) / sizeof(unsigned long long);
static_assert(sizeof(NdfCtl) % sizeof(unsigned long long) == 0, "8-byte words");

__device__ inline void ctl_load(NdfCtl* sc, const NdfCtl* c) {
  const unsigned long long* src = reinterpret_cast<const unsigned long long*>(c);
  unsigned long long* dst = reinterpret_cast<unsigned long long*>(sc);
  for (int i = threadIdx.x; i < kCtlWords; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}
__device__ inline void ctl_store(NdfCtl* c, const NdfCtl* sc) {
  __syncthreads();
  const unsigned long long* src = reinterpret_cast<const unsigned long long*>(sc);
  unsigned long long* dst = reinterpret_cast<unsigned long long*>(c);
  for (int i = threadIdx.x; i < kCtlWords; i += blockDim.x) dst[i] = src[i];
}

// Runs the controller after sweep slot `slot` (ndf_decide) if that slot ran:
// the norms of the sweep, the next slot's gate or the attempt's record (to the
// log ring) and the opening of the next attempt.
__global__ __launch_bounds__(64) void k_ndf_decide(NdfCtl* c, const unsigned long long* spread_row,
                                                   int slot, nse_adaptive_record* log,
                                                   nse_forcing_schedule sched) {
  static_assert(kNdfSpread == 64, "one copy per lane");
  if (__hip_atomic_load(&c->gates[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  __shared__ NdfCtl sc;
  // the sweep's norms: the maximum over the spread copies (lane t: copy t)
  double v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    v[q] = __longlong_as_double((long long)spread_row[threadIdx.x * kNdfSpreadStride + q]);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] = nanmax(v[q], __shfl_xor(v[q], o, 64));
  ctl_load(&sc, c);
  if (threadIdx.x == 0) {
    double row[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) row[q] = sqrt(v[q]);
    if (ndf_decide(sc, slot, row, sched) == NDF_ENDED) log[(sc.nlog - 1) % kNdfLogCap] = sc.rec;
  }
  ctl_store(c, &sc);
}

// Accepted-step update of the differences, rescaling to a new step and the
// predictor of the next attempt, one state slot per thread.
__global__ __launch_bounds__(256) void k_ndf_prepare(NdfArgs a) {
  const NdfCtl* ctl = a.ctl;
  if (ctl && __hip_atomic_load(&ctl->open, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    return;
  if (blockIdx.x == 0 && (int)threadIdx.x < a.nnorms) a.norms[threadIdx.x] = 0ull;
  if (blockIdx.x == 0 && a.done && (int)threadIdx.x < a.nnorms / 4) a.done[threadIdx.x] = 0u;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a.spread)
    for (int64_t w = s; w < a.spread_words; w += (int64_t)gridDim.x * blockDim.x) a.spread[w] = 0ull;
  if (s >= a.S) return;
  const int accept = ctl ? ctl->prep_accept : a.accept;
  const int transform = ctl ? ctl->prep_transform : a.transform;
  const int predict = ctl ? ctl->prep_predict : a.predict;
  const int k = ctl ? ctl->prep_k : a.k;
  const auto R = ctl ? ctl->prepR : a.R;
  double2 D[kNdfDepth];
#pragma unroll
  for (int j = 0; j < kNdfDepth; ++j) D[j] = (j < a.depth) ? a.D[(int64_t)j * a.S + s] : zero2();
  if (accept) {
    // nabla^{k+1} y_{n+1} = d, nabla^{k+2} y_{n+1} = d - nabla^{k+1} y_n,
    // nabla^j y_{n+1} = nabla^j y_n + nabla^{j+1} y_{n+1}
    const int ka = ctl ? ctl->prep_k_acc : a.k_acc;
    const double2 d = ctl ? a.dsel[ctl->prep_dsel][s] : a.dacc[s];
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
  if (transform) {
#pragma unroll
    for (int j = 0; j < kNdfDepth; ++j) {
      double2 v = zero2();
      if (j <= k) {
#pragma unroll
        for (int i = 0; i <= kNdfMaxOrder; ++i)
          if (i >= j && i <= k) {
            v.x += R[j][i] * D[i].x;
            v.y += R[j][i] * D[i].y;
          }
      }
      D[j] = v;  // rows are computed from D[i >= j] before D[j] is replaced
    }
  }
  if (accept || transform) {
#pragma unroll
    for (int j = 0; j < kNdfDepth; ++j)
      if (j < a.depth) a.D[(int64_t)j * a.S + s] = D[j];
  }
  if (predict) {
    double2 y = D[0], p = zero2();
#pragma unroll
    for (int j = 1; j <= kNdfMaxOrder; ++j)
      if (j <= k) {
        y.x += D[j].x;
        y.y += D[j].y;
        p.x += a.gam[j] * D[j].x;
        p.y += a.gam[j] * D[j].y;
      }
    a.y0[s] = y;
    a.psi[s] = p;
  }
}

// Max over the block of four non-negative values, then one atomic per value.
// Non-negative IEEE doubles order like their bit patterns, and a NaN sorts
// above +inf, so a non-finite norm reaches the host.
__device__ inline void block_max4(double v[4], unsigned long long* out) {
  __shared__ double part[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] = nanmax(v[q], __shfl_xor(v[q], o, 64));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
    for (int q = 0; q < 4; ++q) part[wave][q] = v[q];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int q = threadIdx.x;
    double r = part[0][q];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = nanmax(r, part[w][q]);
    unsigned long long bits = (unsigned long long)__double_as_longlong(r);
    if (r != r) bits = 0x7ff8000000000000ull;  // one positive NaN pattern
    atomicMax(out + q, bits);
    __threadfence();
  }
}

// The last workgroup of a publishing launch copies the four norms of the sweep
// to host memory and then the sequence word, which the host polls.
__device__ inline void publish_norms(const NdfArgs& a) {
  __syncthreads();  // this workgroup's atomics are complete
  if (threadIdx.x != 0) return;
  __threadfence();
  const unsigned nblocks = gridDim.x * gridDim.y * gridDim.z;
  if (atomicAdd(a.done + a.sweep, 1u) != nblocks - 1) return;
  __threadfence();
  volatile unsigned long long* pub = a.pub;
#pragma unroll
  for (int q = 0; q < 4; ++q) pub[4 * a.sweep + q] = atomicAdd(a.nrow + q, 0ull);
  __threadfence_system();
  pub[a.nnorms] = a.seq;
  __threadfence_system();
}

// One corrector sweep (or F(t0, y0) in NDF_RHS mode) for the members of a group:
// block (m, degree chunk, member). The four weighted norms use
// wt = max(|y_n|, |y_i|, atol/rtol) per complex coefficient (squared here).
__global__ __launch_bounds__(256) void k_ndf_correct(GroupView g, NdfArgs a) {
  const NdfCtl* ctl = a.ctl;
  if (ctl &&
      __hip_atomic_load(&ctl->gates[a.sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    return;
  const int ak_k = ctl ? ctl->k : a.k;
  const double h = ctl ? ctl->h : a.h;
  const double fscale = ctl ? ctl->fscale : a.fscale;
  const int N = g.N;
  const int m = blockIdx.x, b = blockIdx.z;
  const int kk = blockIdx.y * blockDim.x + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (kk <= N - m) {
    const int l = m + kk;
    const int64_t s = g.off[b] + coeff_offset(N, m) + kk;
    const double Lam = g.nu[b] * ((double)l * (l + 1));
    const double2 n = a.n[s];
    double2 f = a.f ? a.f[s] : zero2();
    f = make_double2(fscale * f.x, fscale * f.y);
    const double2 D0 = a.D[s];
    if (a.mode == NDF_RHS) {
      double2 F = make_double2(f.x - Lam * D0.x - n.x, f.y - Lam * D0.y - n.y);
      if (l == 0) F = zero2();
      if (m == 0) F.y = 0.0;
      a.dout[s] = F;
      v[0] = abs2(F) / fmax(abs2(D0), a.thr2);
    } else {
      const double2 y0 = a.y0[s], ps = a.psi[s];
      const double hL = h * Lam;
      const double den = (ctl ? ndf_alpha(ak_k) : a.ak) + hL;
      double2 d = make_double2((h * (f.x - n.x) - hL * y0.x - ps.x) / den,
                               (h * (f.y - n.y) - hL * y0.y - ps.y) / den);
      if (l == 0) d = zero2();
      if (m == 0) d.y = 0.0;
      const double2 y = make_double2(y0.x + d.x, y0.y + d.y);
      const double2 dp = a.dprev ? a.dprev[s] : zero2();
      a.dout[s] = d;
      a.yout[s] = y;
      const double wt2 = fmax(fmax(abs2(D0), abs2(y)), a.thr2);
      v[0] = abs2(make_double2(d.x - dp.x, d.y - dp.y)) / wt2;
      v[1] = abs2(d) / wt2;
      if (ak_k > 1) {
        const double2 Dk = a.D[(int64_t)ak_k * a.S + s];
        v[2] = abs2(make_double2(Dk.x + d.x, Dk.y + d.y)) / wt2;
      }
      if (ak_k < a.kmax) {
        const double2 Dk1 = a.D[(int64_t)(ak_k + 1) * a.S + s];
        v[3] = abs2(make_double2(d.x - Dk1.x, d.y - Dk1.y)) / wt2;
      }
    }
  }
  block_max4(v, ctl ? a.nrow + (blockIdx.x % kNdfSpread) * kNdfSpreadStride : a.nrow);
  if (!ctl && a.publish) publish_norms(a);
}

}  // namespace

hipError_t launch_ndf_prepare(const NdfArgs& a, hipStream_t s) {
  const int64_t blocks = (a.S + 255) / 256;
  hipLaunchKernelGGL(k_ndf_prepare, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ndf_decide(NdfCtl* c, const unsigned long long* spread_row, int slot,
                             nse_adaptive_record* log, const nse_forcing_schedule& sched,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_ndf_decide, dim3(1), dim3(64), 0, s, c, spread_row, slot, log, sched);
  return hipGetLastError();
}

hipError_t launch_ndf_correct(const GroupView& g, const NdfArgs& a, hipStream_t s) {
  dim3 grid(g.N + 1, (g.N + 1 + 255) / 256, g.nb);
  hipLaunchKernelGGL(k_ndf_correct, grid, dim3(256), 0, s, g, a);
  return hipGetLastError();
}

}  // namespace nse
