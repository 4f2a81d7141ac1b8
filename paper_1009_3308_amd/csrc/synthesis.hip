// Legendre synthesis: for every order m and latitude, the Fourier coefficients
// of the grid fields needed by the nonlinear term (Section 4.2: direct Legendre
// sums in latitude, one contraction per azimuthal order m). The four fields and
// their coefficient panels are described in spectral_ops.h; the grid product is
//   u . Grad zeta_a = (f0 f2 - f1 f3) / sin^2(theta).
//
// One workgroup of four waves per (order m, tile of 64 northern latitudes,
// member). The panel of coefficients for this m is built in LDS; each wave
// then streams a quarter of the degree range of its latitude column of
// T1[m][l-m][p] (coalesced across the wavefront), accumulating even (l-m even)
// and odd parts separately, and the four partial sums are added through LDS.
// Each latitude yields the northern value E + O and the mirrored southern value
// E - O. Output F[b][f][m][lat] is written latitude-contiguous.
#include "spectral_ops.h"

namespace nse {

constexpr int kSynthWaves = 4;
constexpr int kSynthThreads = 64 * kSynthWaves;
constexpr int kBatch = 8;  // table rows per load batch (even)

// NF fields: per lane 4 NF partial sums (NF fields x (E, O) x (re, im)).
// The panel [L][NF] double2 is reused afterwards for the cross-wave reduction.
__host__ __device__ inline int synth_pan_slots(int N, int NF) {
  const int pan = NF * (N + 2);
  const int red = kSynthWaves * 4 * NF * 64 / 2;
  return pan > red ? pan : red;
}

size_t synthesis_lds_bytes(int N, int NF) {
  return sizeof(double2) * (size_t)((N + 3) + synth_pan_slots(N, NF));
}

// TT: element type of the table and of the products and accumulation (double
// for NSE_PREC_FP64, float for NSE_PREC_FP32); the cross-wave sums are FP64.
// NF: 4 (nonlinear and grid modes) or 5 (adjoint mode).
template <typename TT, int NF>
__global__ __launch_bounds__(kSynthThreads) void k_synthesis(GroupView g, SynthInput in,
                                                              int mode) {
  constexpr int kRed = 4 * NF;
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (nh + 63) / 64;
  const int m = blockIdx.x / ntile;
  const int tile = blockIdx.x - m * ntile;
  const int b = blockIdx.y;
  const int L = N + 2 - m;  // degrees m .. N+1
  extern __shared__ double2 sh[];
  double2* a = sh;              // [L + 1] state coefficients alpha[l], l = m..N (0 beyond)
  double2* pan = sh + (N + 3);  // [L][NF]

  load_order(a, g, in, b, m, L);
  __syncthreads();
  build_panel<NF>(pan, a, N, m, L, mode, in.coriolis, in.stream != 0);
  if (NF == 5) {
    // fifth field: lambda^(-1/2) n_bar, l = max(m, 1)..N, real at m = 0 (n_bar formed
    // here from hbar_out[0] inside the step adjoint)
    const double2* nb = in.adj + g.off[b] + coeff_offset(N, m);
    for (int k = threadIdx.x; k < L; k += blockDim.x) {
      const int l = m + k;
      double2 v = make_double2(0.0, 0.0);
      if (l >= 1 && l <= N) {
        const double lam = (double)l * (l + 1);
        double r = 1.0 / sqrt(lam);
        if (in.adj_step) r *= -in.adj_h / (in.adj_c0 + in.adj_h * g.nu[b] * lam);
        v = make_double2(nb[k].x * r, m == 0 ? 0.0 : nb[k].y * r);
      }
      pan[NF * k + 4] = v;
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int p = tile * 64 + lane;
  // even-length quarter of the degree range for this wave
  const int chunk = ((L + 2 * kSynthWaves - 1) / (2 * kSynthWaves)) * 2;
  const int k0 = wave * chunk;
  const int k1 = min(L, k0 + chunk);
  TT acc[kRed];
#pragma unroll
  for (int i = 0; i < kRed; ++i) acc[i] = TT(0);
  if (p < nh && k0 < k1) {
    const TT* t = synthesis_table<TT>(g) + t1_order_offset(N, m, nh) + p;
    // batches of kBatch degrees; the next batch's table loads are issued before
    // the current batch's FMAs so that 2 kBatch loads are in flight
    TT tn[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) tn[u] = (k0 + u < k1) ? t[(int64_t)(k0 + u) * nh] : TT(0);
    for (int kb = k0; kb < k1; kb += kBatch) {
      TT tc[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) tc[u] = tn[u];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int k = kb + kBatch + u;
        tn[u] = (k < k1) ? t[(int64_t)k * nh] : TT(0);
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int k = kb + u;
        if (k < k1) {
          const int par = (u & 1) * 2;  // kb and k0 are even: parity of k is that of u
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            const double2 A = pan[NF * k + f];
            acc[4 * f + par + 0] = fma(tc[u], (TT)A.x, acc[4 * f + par + 0]);
            acc[4 * f + par + 1] = fma(tc[u], (TT)A.y, acc[4 * f + par + 1]);
          }
        }
      }
    }
  }
  __syncthreads();  // panel no longer needed: reuse it for the reduction
  double* red = reinterpret_cast<double*>(pan);  // [wave][kRed][64]
#pragma unroll
  for (int i = 0; i < kRed; ++i) red[(wave * kRed + i) * 64 + lane] = (double)acc[i];
  __syncthreads();
  // wave w finishes fields w, w+4, ... for its 64 latitudes
  const int nf = (mode == SYNTH_GRID) ? 3 : NF;
  if (p >= nh) return;
  double2* Fout = (NF == 5) ? g.Fa : g.F;
  for (int f = wave; f < nf; f += kSynthWaves) {
    double er = 0.0, ei = 0.0, orr = 0.0, oi = 0.0;
#pragma unroll
    for (int w = 0; w < kSynthWaves; ++w) {
      er += red[(w * kRed + 4 * f + 0) * 64 + lane];
      ei += red[(w * kRed + 4 * f + 1) * 64 + lane];
      orr += red[(w * kRed + 4 * f + 2) * 64 + lane];
      oi += red[(w * kRed + 4 * f + 3) * 64 + lane];
    }
    double2* out = Fout + ((int64_t)(b * NF + f) * (N + 1) + m) * nlat;
    out[p] = make_double2(er + orr, ei + oi);
    const int ps = nlat - 1 - p;
    if (ps != p) out[ps] = make_double2(er - orr, ei - oi);
  }
}

hipError_t launch_synthesis(const GroupView& g, const SynthInput& in, int mode, hipStream_t s) {
  dim3 block(kSynthThreads);
  const int ntile = (g.nh + 63) / 64;
  dim3 grid((g.N + 1) * ntile, g.nb);
  if (mode == SYNTH_ADJ)
    hipLaunchKernelGGL((k_synthesis<double, 5>), grid, block, synthesis_lds_bytes(g.N, 5), s, g,
                       in, mode);
  else if (g.precision == NSE_PREC_FP32)
    hipLaunchKernelGGL((k_synthesis<float, 4>), grid, block, synthesis_lds_bytes(g.N, 4), s, g,
                       in, mode);
  else
    hipLaunchKernelGGL((k_synthesis<double, 4>), grid, block, synthesis_lds_bytes(g.N, 4), s, g,
                       in, mode);
  return hipGetLastError();
}

}  // namespace nse
