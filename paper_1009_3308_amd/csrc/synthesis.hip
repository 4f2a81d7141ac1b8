// Legendre synthesis: for every order m and latitude, the Fourier coefficients
// of the grid fields needed by the nonlinear term (Section 4.2: direct Legendre
// sums in latitude, one contraction per azimuthal order m). The four fields and
// their coefficient panels are described in spectral_ops.h; the grid product is
//   u . Grad zeta_a = (f0 f2 - f1 f3) / sin^2(theta).
//
// One workgroup of four waves per (order m, tile of northern latitudes,
// member). The panel of coefficients for this m is built in LDS; each wave
// then takes a quarter of the degree range, accumulating even (l-m even) and
// odd parts separately, and the four partial sums are added through LDS. Each
// latitude yields the northern value E + O and the mirrored southern value
// E - O. Output F[b][f][m][lat] is written latitude-contiguous.
//
// The Legendre values come from T1[m][l-m][p] in two ways. FP32 streams the
// column of the table (coalesced across the wavefront). FP64 (nonlinear, grid
// and the adjoint's five-field mode) reads only two table rows per wave and
// continues the three-term recurrence in registers (OTF below): the table is no
// longer streamed and the loop is bound by the LDS reads of the panel, which is
// why the lanes of the four-field modes take one to three latitudes each.
#include "spectral_ops.h"

namespace nse {

constexpr int kSynthWaves = 4;
constexpr int kSynthThreads = 64 * kSynthWaves;
constexpr int kBatch = 8;  // table rows per load batch (even)
constexpr int kOtfBatch = 4;  // degrees per recurrence batch (even)

// NF fields: per lane 4 NF partial sums (NF fields x (E, O) x (re, im)).
// The panel [L][NF] double2 is reused afterwards for the cross-wave reduction.
__host__ __device__ inline int synth_pan_slots(int N, int NF) {
  const int pan = NF * (N + 2 + kOtfBatch);  // panel rows plus the padding a batch may read
  const int red = kSynthWaves * 4 * NF * 64 / 2;
  return pan > red ? pan : red;
}

// LDS: coefficients, panel (reused for the reduction) and, with OTF, the
// recurrence coefficients of the order.
size_t synthesis_lds_bytes(int N, int NF, bool otf) {
  return sizeof(double2) *
         (size_t)((N + 3) + synth_pan_slots(N, NF) + (otf ? N + 2 + kOtfBatch : 0));
}
size_t synthesis_lds_bytes(int N, int NF) { return synthesis_lds_bytes(N, NF, false); }

// TT: element type of the table and of the products and accumulation (double
// for NSE_PREC_FP64, float for NSE_PREC_FP32); the cross-wave sums are FP64.
// NF: 4 (nonlinear and grid modes) or 5 (adjoint mode).
// OTF (FP64 only): the Legendre values are not streamed from T1 but continued
// in registers by the three-term recurrence of eq. (sph_har),
//   Pbar[l,m] = a(l,m) mu Pbar[l-1,m] - (a(l,m) / a(l-1,m)) Pbar[l-2,m],
//   a(l,m) = sqrt((4 l^2 - 1) / (l^2 - m^2)),
// from two table rows at the start of each wave's degree range (seeds), with
// the coefficient pairs of the order in LDS. The table traffic drops from the
// whole T1 to two rows per wave.
// R (OTF only): latitudes per lane (tiles of 64 R latitudes, lane l taking
// l, l + 64, ...): every panel value read from LDS then serves R latitudes,
// which is what bounds the OTF loop (the LDS, shared by the four SIMDs).
template <typename TT, int NF, bool OTF = false, int R = 1>
__global__ __launch_bounds__(kSynthThreads) void k_synthesis(GroupView g, SynthInput in,
                                                              int mode) {
  constexpr int kRed = 4 * NF;
  constexpr int kB = (R == 1) ? kOtfBatch : 2;  // degrees per recurrence batch
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (nh + 64 * R - 1) / (64 * R);
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
  double2* rc = pan + synth_pan_slots(N, NF);  // OTF: [L] (a(l,m), a(l,m) / a(l-1,m))
  if (OTF) {
    for (int k = threadIdx.x; k < L + kOtfBatch; k += blockDim.x) {
      const int l = m + k;
      double2 c = make_double2(0.0, 0.0);
      if (k >= 2 && k < L) {
        const double dl = (double)l, dm = (double)m;
        const double al = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - dm * dm));
        const double al1 = sqrt((4.0 * (dl - 1.0) * (dl - 1.0) - 1.0) /
                                ((dl - 1.0) * (dl - 1.0) - dm * dm));
        c = make_double2(al, al / al1);
      }
      rc[k] = c;
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int pbase = tile * 64 * R + lane;  // latitude of slot r: pbase + 64 r
  // even-length quarter of the degree range for this wave
  const int chunk = ((L + 2 * kSynthWaves - 1) / (2 * kSynthWaves)) * 2;
  const int k0 = wave * chunk;
  const int k1 = min(L, k0 + chunk);
  TT acc[R][kRed];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < kRed; ++i) acc[r][i] = TT(0);
  if (OTF && k0 < k1) {
    // seeds: the table rows k0 and k0 + 1 (k0 even), then the recurrence
    const double* t = g.T1 + t1_order_offset(N, m, nh);
    double P2[R], P1[R], x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int p = pbase + 64 * r;
      P2[r] = P1[r] = x[r] = 0.0;
      if (p < nh) {
        P2[r] = t[(int64_t)k0 * nh + p];
        if (k0 + 1 < k1) P1[r] = t[(int64_t)(k0 + 1) * nh + p];
        x[r] = g.mu[p];
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double2 A0 = pan[NF * k0 + f];
      const double2 A1 = (k0 + 1 < k1) ? pan[NF * (k0 + 1) + f] : make_double2(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc[r][4 * f + 0] = fma((TT)P2[r], (TT)A0.x, acc[r][4 * f + 0]);
        acc[r][4 * f + 1] = fma((TT)P2[r], (TT)A0.y, acc[r][4 * f + 1]);
        acc[r][4 * f + 2] = fma((TT)P1[r], (TT)A1.x, acc[r][4 * f + 2]);
        acc[r][4 * f + 3] = fma((TT)P1[r], (TT)A1.y, acc[r][4 * f + 3]);
      }
    }
    // batches of kB degrees: the batch's coefficient pairs and panel entries are
    // read from LDS first, then the recurrence runs through the batch for every
    // latitude of the lane and the products are accumulated (entries past k1
    // are padding and are not accumulated)
    for (int kb = k0 + 2; kb < k1; kb += kB) {
      double2 c[kB], A[kB][NF];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        c[u] = rc[kb + u];
#pragma unroll
        for (int f = 0; f < NF; ++f) A[u][f] = pan[NF * (kb + u) + f];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double v[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          v[u] = fma(c[u].x * x[r], P1[r], -c[u].y * P2[r]);
          P2[r] = P1[r];
          P1[r] = v[u];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          if (kb + u < k1) {
            const int par = (u & 1) * 2;  // kb is even
#pragma unroll
            for (int f = 0; f < NF; ++f) {
              acc[r][4 * f + par + 0] = fma((TT)v[u], (TT)A[u][f].x, acc[r][4 * f + par + 0]);
              acc[r][4 * f + par + 1] = fma((TT)v[u], (TT)A[u][f].y, acc[r][4 * f + par + 1]);
            }
          }
        }
      }
    }
  }
  if (!OTF && pbase < nh && k0 < k1) {
    const int p = pbase;
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
            acc[0][4 * f + par + 0] = fma(tc[u], (TT)A.x, acc[0][4 * f + par + 0]);
            acc[0][4 * f + par + 1] = fma(tc[u], (TT)A.y, acc[0][4 * f + par + 1]);
          }
        }
      }
    }
  }
  // cross-wave sums, one latitude slot at a time through the (no longer needed)
  // panel; wave w finishes fields w, w+4, ... of its 64 latitudes
  double* red = reinterpret_cast<double*>(pan);  // [wave][kRed][64]
  const int nf = (mode == SYNTH_GRID) ? 3 : NF;
  double2* Fout = (NF == 5) ? g.Fa : g.F;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRed; ++i) red[(wave * kRed + i) * 64 + lane] = (double)acc[r][i];
    __syncthreads();
    const int p = pbase + 64 * r;
    if (p < nh) {
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
  }
}

hipError_t launch_synthesis(const GroupView& g, const SynthInput& in, int mode, hipStream_t s) {
  dim3 block(kSynthThreads);
  const int ntile = (g.nh + 63) / 64;
  dim3 grid((g.N + 1) * ntile, g.nb);
  if (mode == SYNTH_ADJ)
    hipLaunchKernelGGL((k_synthesis<double, 5, true>), grid, block,
                       synthesis_lds_bytes(g.N, 5, true), s, g, in, mode);
  else if (g.precision == NSE_PREC_FP32)
    hipLaunchKernelGGL((k_synthesis<float, 4>), grid, block, synthesis_lds_bytes(g.N, 4), s, g,
                       in, mode);
  else if (g.nh >= 384 && g.nh % 192 == 0) {
    // large grids: three latitudes per lane (measured best at nh = 384; at
    // nh <= 192 one latitude per lane is faster, the grid having too few tiles)
    dim3 grid3((g.N + 1) * (g.nh / 192), g.nb);
    hipLaunchKernelGGL((k_synthesis<double, 4, true, 3>), grid3, block,
                       synthesis_lds_bytes(g.N, 4, true), s, g, in, mode);
  } else if (g.nh >= 256) {
    dim3 grid2((g.N + 1) * ((g.nh + 127) / 128), g.nb);
    hipLaunchKernelGGL((k_synthesis<double, 4, true, 2>), grid2, block,
                       synthesis_lds_bytes(g.N, 4, true), s, g, in, mode);
  } else {
    hipLaunchKernelGGL((k_synthesis<double, 4, true>), grid, block,
                       synthesis_lds_bytes(g.N, 4, true), s, g, in, mode);
  }
  return hipGetLastError();
}

}  // namespace nse
