// Device side of the adaptive NDF integrator (Section 4.2, eq. (ode_disc) with
// orders 1..5, written in backward differences at a quasi-constant step).
// k_ndf_prepare and k_ndf_correct are elementwise over the state; the nonlinear
// term between them comes from the synthesis / ring / analysis chain. On a
// device-controlled run k_ndf_step opens every sweep slot: the controller of
// ndf_control.h on the previous sweep's norms and, when an attempt has just
// been opened, its prepare.
#include "lane_ops.h"
#include "ndf_device.h"

namespace nse {

namespace {

__device__ inline double2 zero2() { return make_double2(0.0, 0.0); }
__device__ inline double abs2(double2 z) { return z.x * z.x + z.y * z.y; }

// Host-controlled prepare (its parameters in the arguments); clears the sweep norms.
__global__ __launch_bounds__(256) void k_ndf_prepare(NdfArgs a) {
  if (blockIdx.x == 0 && (int)threadIdx.x < a.nnorms) a.norms[threadIdx.x] = 0ull;
  if (blockIdx.x == 0 && a.done && (int)threadIdx.x < a.nnorms / 4) a.done[threadIdx.x] = 0u;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.S) return;
  PrepareParams pp{a.accept, a.k_acc, a.transform, a.k, a.predict, a.dacc, a.R};
  prepare_element(a, pp, s, nullptr);
}

// Opens sweep slot `sel` of a device-controlled run. Every workgroup copies the
// controller state and reduces the previous sweep's norm copies, thread 0 runs
// the controller (the same inputs give every workgroup the same result), and
// when an attempt has just been opened every workgroup prepares its share of the
// state; workgroup 0 writes the new state and the attempt record.
__global__ __launch_bounds__(256) void k_ndf_step(NdfArgs a, NdfStepArgs st) {
  static_assert(kNdfSpread == 64, "one copy per lane of wave 0");
  __shared__ NdfCtl sc;
  __shared__ int prep;
  __shared__ double norm[4];
  const unsigned long long* src = reinterpret_cast<const unsigned long long*>(st.ctl_in);
  unsigned long long* dst = reinterpret_cast<unsigned long long*>(&sc);
  unsigned long long w[(kCtlWords + 255) / 256];
#pragma unroll
  for (int i = 0; i < (kCtlWords + 255) / 256; ++i) {
    const int j = threadIdx.x + 256 * i;
    if (j < kCtlWords) w[i] = src[j];
  }
  if (threadIdx.x < 64) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      v[q] = __longlong_as_double((long long)st.spread_in[threadIdx.x * kNdfSpreadStride + q]);
    const double mx = lane_max4(v);  // lane 16 q: the maximum of v[q]
    if ((threadIdx.x & 15) == 0) norm[threadIdx.x >> 4] = mx;
  }
#pragma unroll
  for (int i = 0; i < (kCtlWords + 255) / 256; ++i) {
    const int j = threadIdx.x + 256 * i;
    if (j < kCtlWords) dst[j] = w[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    prep = ndf_slot_decide(sc, norm, st, blockIdx.x == 0);
    sc.prep_in_analysis = 0;  // this kernel applies the whole prepare
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t s0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t w2 = s0; w2 < a.spread_words; w2 += stride) st.spread_clear[w2] = 0ull;
  if (prep) {
    const PrepareParams pp = prepare_params(sc, a.dsel);
    for (int64_t s = s0; s < a.S; s += stride) prepare_element(a, pp, s, a.yout);
  }
  if (blockIdx.x == 0) {
    const unsigned long long* from = reinterpret_cast<const unsigned long long*>(&sc);
    unsigned long long* to = reinterpret_cast<unsigned long long*>(st.ctl_out);
    for (int j = threadIdx.x; j < kCtlWords; j += blockDim.x) to[j] = from[j];
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
  if (ctl && __hip_atomic_load(&ctl->running, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
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
      // device-controlled: no previous correction on an attempt's first sweep
      const double2 dp = (a.dprev && !(ctl && ctl->sweep == 0)) ? a.dprev[s] : zero2();
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

hipError_t launch_ndf_step(const NdfArgs& a, const NdfStepArgs& st, hipStream_t s) {
  const int64_t blocks = (a.S + 255) / 256;
  hipLaunchKernelGGL(k_ndf_step, dim3((unsigned)blocks), dim3(256), 0, s, a, st);
  return hipGetLastError();
}

hipError_t launch_ndf_correct(const GroupView& g, const NdfArgs& a, hipStream_t s) {
  dim3 grid(g.N + 1, (g.N + 1 + 255) / 256, g.nb);
  hipLaunchKernelGGL(k_ndf_correct, grid, dim3(256), 0, s, g, a);
  return hipGetLastError();
}

}  // namespace nse
