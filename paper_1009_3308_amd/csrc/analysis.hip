// Quadrature analysis and the time-step update.
//
// Analysis (Section 3, eqs. (disc_ip), (disc_vec_orth_proj); Section 4.2):
//   n[l,m] = lambda_l^(-1/2) sum_p Pbar[l,m](mu_p) (We_m(p) or Wo_m(p)),
// where the ring kernel has already applied the longitude DFT and the weights
// (2 pi / M) w_p, and the rings of each latitude pair are folded here into
// We = Q(p) + Q(p') (for l-m even) and Wo = Q(p) - Q(p') (odd), using
// Pbar[l,m](-mu) = (-1)^(l+m) Pbar[l,m](mu), so the sum runs over northern
// latitudes only. This is
// (u . Grad(zeta + 2 Omega cos theta), Y[l,m])_M lambda^(-1/2)
// = (B(u,u) + C u, Z[l,m])_M (eqs. (app1_weak_form), (short_nonlin1), (C)).
//
// Step update (eq. (ode_disc) with the Stokes term of eq. (stok_eig) implicit):
//   alpha_new = (h (f - n) - sum_{j>=1} c_j hist[j-1]) / (c_0 + h nu lambda_l),
// then either stored as the next fixed-point iterate or written to hist[0]
// after rotating hist[j] <- hist[j-1].
//
// Workgroups of NW waves per (order m, tile of 16 NW degrees, member). Orders
// are taken in XCD-local chunks of four neighbouring m. The ring spectra
// W[m][lat] of an order are contiguous, so the fold's loads are coalesced; the
// step update's inputs (forcing, history) of the tile's degrees are requested
// with them and wait in LDS, so the epilogue issues no load.
// With three or more latitudes per lane three waves per workgroup balance the
// CUs best: the waves of a launch are dealt out a workgroup at a time, and with
// four (or two) waves the most loaded CUs held a larger share of them (T511:
// 27.0 us against 30.9 and 28.1). With fewer latitudes per lane (N = 100 on
// 160 x 320) four waves are faster (4.7 against 5.0 us; 4.8 against 5.9 us with
// the corrector sweep of a device-controlled run).
#include "lane_ops.h"
#include "spectral_ops.h"

namespace nse {

// waves per workgroup for R latitudes per lane
__host__ __device__ constexpr int anal_waves(int R) { return R >= 3 ? 3 : 4; }
// The Legendre values are continued in registers (OTF) rather than streamed
// from a table. Wave w owns the degrees 16 w .. 16 w + 15 of the tile and its lanes are
// latitudes, lane l taking p = l + 64 r for r < R (R = ceil(nh / 64)). Each lane
// starts the recurrence of eq. (sph_har),
//   Pbar[l,m] = a(l,m) mu Pbar[l-1,m] - (a(l,m) / a(l-1,m)) Pbar[l-2,m],
// from the T1 rows of the wave's own first two degrees (coalesced across the
// lanes), and multiplies each value by its own latitude's folded spectrum
// (We for even l-m, Wo for odd) held in registers; the sixteen complex sums are
// then formed across the 64 lanes by a butterfly of register exchanges, which
// leaves degree 8 b5 + 4 b4 + 2 b3 + b2 of the wave's block (b = lane bits) in
// every lane with b1 = b0 = 0. The table traffic drops to two rows per wave.
// TT: type of the products and sums (double for NSE_PREC_FP64; float for
// NSE_PREC_FP32, where the recurrence, the weighted fold and the epilogue stay
// FP64 and each Legendre value and folded spectrum is rounded to FP32 before
// the FP32 products; the lane sums are FP32).
namespace {

constexpr int kOtfDeg = kButterfly;  // degrees per wave

template <typename TT, int R, bool NDF>
__global__ __launch_bounds__(64 * anal_waves(R)) void k_analysis_otf(GroupView g, AnalOutput out) {
  constexpr int kAnalWaves = anal_waves(R);
  constexpr int kAnalThreads = 64 * kAnalWaves;
  constexpr int kAnalTile = kAnalWaves * kButterfly;  // degrees per workgroup
  const int N = g.N, nh = g.nh;
  const int ntile = (N + 1 + kAnalTile - 1) / kAnalTile;
  const int item = xcd_item(blockIdx.x, 4 * ntile);
  const int m = item / ntile;
  const int tile = item - m * ntile;
  if (m > N || tile * kAnalTile > N - m) return;  // uniform across the workgroup
  const int b = blockIdx.y;
  // We [nh], Wo [nh], rc [kAnalTile], step inputs [kAnalTile][kDegreeInputs]
  extern __shared__ double2 wsh[];
  double2* rc = wsh + 2 * nh;
  double2* pre = rc + kAnalTile;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int kt = tile * kAnalTile;  // first degree offset k = l - m of the tile

  const int j0 = wave * kOtfDeg;        // the wave's first degree within the tile
  const bool active = kt + j0 <= N - m;  // some degree of this wave is analysed
  // seeds first, their latency overlapping the prologue: the wave's first two
  // degrees, two coalesced rows of T1 (it holds k = 0 .. N + 1 - m)
  double x[R], P1[R], P2[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = P1[r] = P2[r] = 0.0;
  if (active) {
    const double* t = g.T1 + t1_order_offset(N, m, nh) + (int64_t)(kt + j0) * nh;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int p = lane + 64 * r;
      if (p < nh) {
        P2[r] = t[p];
        P1[r] = t[nh + p];
        x[r] = g.mu[p];
      }
    }
  }
  // fold the ring spectra of each latitude pair: We = Q(p) + Q(p'), Wo = Q(p) - Q(p');
  // all of the thread's pairs (p = t + i kAnalThreads; nh <= kMaxM / 4 = 384)
  // are requested before the coefficient pairs are computed, so that their
  // square roots and the LDS writes wait for one memory round trip
  constexpr int kFold = (kMaxM / 4 + kAnalThreads - 1) / kAnalThreads;  // pairs per thread
  const double2* Wb = g.W + ((int64_t)b * (N + 1) + m) * g.nlat;
  double2 qn[kFold], qs[kFold];
#pragma unroll
  for (int i = 0; i < kFold; ++i) {
    const int p = threadIdx.x + i * kAnalThreads;
    qn[i] = qs[i] = make_double2(0.0, 0.0);
    if (p < nh) {
      qn[i] = Wb[p];
      qs[i] = Wb[g.nlat - 1 - p];
    }
  }
  // the step update's inputs of degree kt + t (t < kAnalTile), kept until the epilogue
  double2 din[kDegreeInputs];
  const bool dthread = (int)threadIdx.x < kAnalTile && kt + (int)threadIdx.x <= N - m;
  if (dthread) load_degree_inputs<NDF>(g, out, b, m, kt + threadIdx.x, din);
  // recurrence pairs of the tile's degrees (k >= 2 of the order, from the
  // group's coefficient table; zero past degree N+1, whose values are not used)
  if ((int)threadIdx.x < kAnalTile) {
    const int k = kt + threadIdx.x;
    rc[threadIdx.x] = (k >= 2 && k <= N + 1 - m) ? g.rec_a[rec_slot(N, m + k, m)]
                                                 : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int i = 0; i < kFold; ++i) {
    const int p = threadIdx.x + i * kAnalThreads;
    if (p < nh) {
      wsh[p] = make_double2(qn[i].x + qs[i].x, qn[i].y + qs[i].y);
      wsh[nh + p] = make_double2(qn[i].x - qs[i].x, qn[i].y - qs[i].y);
    }
  }
  if (dthread && out.mode != ANAL_NONLINEAR) {
#pragma unroll
    for (int i = 0; i < kDegreeInputs; ++i) pre[threadIdx.x * kDegreeInputs + i] = din[i];
  }
  // an ended attempt of a device-controlled run: checked once the loads are in
  // flight (nothing is stored before this barrier), so the flag costs no wait
  if (gate_closed(g)) return;
  __syncthreads();
  if (!active) return;
  TT Wer[R], Wei[R], Wor[R], Woi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = lane + 64 * r;
    Wer[r] = Wei[r] = Wor[r] = Woi[r] = TT(0);
    if (p < nh) {
      const double2 we = wsh[p], wo = wsh[nh + p];
      Wer[r] = (TT)we.x;
      Wei[r] = (TT)we.y;
      Wor[r] = (TT)wo.x;
      Woi[r] = (TT)wo.y;
    }
  }
  // P2 = Pbar at j0, P1 at j0 + 1 (j0 is even: even, odd)
  TT sr[kOtfDeg], si[kOtfDeg];
#pragma unroll
  for (int i = 0; i < kOtfDeg; ++i) sr[i] = si[i] = TT(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    sr[0] = fma((TT)P2[r], Wer[r], sr[0]);
    si[0] = fma((TT)P2[r], Wei[r], si[0]);
    sr[1] = fma((TT)P1[r], Wor[r], sr[1]);
    si[1] = fma((TT)P1[r], Woi[r], si[1]);
  }
#pragma unroll
  for (int i = 2; i < kOtfDeg; ++i) {
    const double2 c = rc[j0 + i];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double v = fma(c.x * x[r], P1[r], -c.y * P2[r]);
      P2[r] = P1[r];
      P1[r] = v;
      const TT vt = (TT)v;
      sr[i] = fma(vt, (i & 1) ? Wor[r] : Wer[r], sr[i]);
      si[i] = fma(vt, (i & 1) ? Woi[r] : Wei[r], si[i]);
    }
  }
  lane_butterfly16(sr, si, lane);
  if constexpr (!NDF) {
    if ((lane & 3) != 0) return;
  }
  const int j = 8 * ((lane >> 5) & 1) + 4 * ((lane >> 4) & 1) + 2 * ((lane >> 3) & 1) +
                ((lane >> 2) & 1);
  const int k = kt + j0 + j;
  if constexpr (NDF) {
    // every lane stays for the wave's norm maxima
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if ((lane & 3) == 0 && k <= N - m)
      finish_degree_from<true>(g, out, b, m, k, (double)sr[0], (double)si[0],
                               pre + (k - kt) * kDegreeInputs, v);
    const int copy = ((blockIdx.y * gridDim.x + blockIdx.x) * kAnalWaves + wave) % kNdfSpread;
    const double mx = lane_max4(v);  // lane 16 q: the wave's maximum of v[q]
    if ((lane & 15) == 0) {
      unsigned long long bits = (unsigned long long)__double_as_longlong(mx);
      if (mx != mx) bits = 0x7ff8000000000000ull;  // one positive NaN pattern
      atomicMax(out.nrow + copy * kNdfSpreadStride + (lane >> 4), bits);
    }
  } else {
    if (k > N - m) return;
    finish_degree_from(g, out, b, m, k, (double)sr[0], (double)si[0],
                       pre + (k - kt) * kDegreeInputs);
  }
}

}  // namespace

size_t analysis_otf_lds_bytes(int nh) {
  const int tile = anal_waves((nh + 63) / 64) * kButterfly;
  return sizeof(double2) * (size_t)(2 * nh + tile * (1 + kDegreeInputs));
}

template <typename TT, bool NDF>
hipError_t launch_analysis_otf(dim3 grid, dim3 block, size_t lds, hipStream_t s,
                               const GroupView& g, const AnalOutput& out) {
  switch ((g.nh + 63) / 64) {
    case 1: hipLaunchKernelGGL((k_analysis_otf<TT, 1, NDF>), grid, block, lds, s, g, out); break;
    case 2: hipLaunchKernelGGL((k_analysis_otf<TT, 2, NDF>), grid, block, lds, s, g, out); break;
    case 3: hipLaunchKernelGGL((k_analysis_otf<TT, 3, NDF>), grid, block, lds, s, g, out); break;
    case 4: hipLaunchKernelGGL((k_analysis_otf<TT, 4, NDF>), grid, block, lds, s, g, out); break;
    case 5: hipLaunchKernelGGL((k_analysis_otf<TT, 5, NDF>), grid, block, lds, s, g, out); break;
    default: hipLaunchKernelGGL((k_analysis_otf<TT, 6, NDF>), grid, block, lds, s, g, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_analysis(const GroupView& g, const AnalOutput& out, hipStream_t s) {
  const int nw = anal_waves((g.nh + 63) / 64);
  dim3 block(64 * nw);
  const int tile = nw * kButterfly;
  const int ntile = (g.N + 1 + tile - 1) / tile;
  dim3 grid(xcd_grid((g.N + 1) * ntile, 4 * ntile), g.nb);
  const size_t lds = analysis_otf_lds_bytes(g.nh);
  const bool ndf = out.mode == ANAL_NDF;
  if (g.precision == NSE_PREC_FP32)
    return ndf ? launch_analysis_otf<float, true>(grid, block, lds, s, g, out)
               : launch_analysis_otf<float, false>(grid, block, lds, s, g, out);
  return ndf ? launch_analysis_otf<double, true>(grid, block, lds, s, g, out)
             : launch_analysis_otf<double, false>(grid, block, lds, s, g, out);
}

}  // namespace nse
