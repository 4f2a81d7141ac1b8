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
// The Legendre values are not streamed from the table T1[m][l-m][p]: each wave
// reads two table rows at the start of its degree range and continues the
// three-term recurrence in FP64 registers, so the loop is bound by the LDS reads
// of the panel, which is why the lanes of the four-field modes take one to three
// latitudes each.
#include <type_traits>

#include "lane_ops.h"
#include "spectral_ops.h"

namespace nse {

constexpr int kSynthWaves = 4;
constexpr int kSynthThreads = 64 * kSynthWaves;
constexpr int kOtfBatch = 4;  // degrees per recurrence batch (even)
// panel entries each thread rounds to FP32 (four fields: N + 2 + kOtfBatch
// degrees; launch_synthesis rejects larger N)
constexpr int kPanelConvPerThread = 10;
// recurrence pairs each thread stages (N + 2 + kOtfBatch entries at most; the
// LDS bound of the kernels keeps N below 680)
constexpr int kRcPerThread = 3;

// NF fields: per lane 4 NF partial sums (NF fields x (E, O) x (re, im)).
// The panel [L][NF] double2 is reused afterwards for the cross-wave reduction.
__host__ __device__ inline int synth_pan_slots(int N, int NF) {
  const int pan = NF * (N + 2 + kOtfBatch);  // panel rows plus the padding a batch may read
  const int red = kSynthWaves * 4 * NF * 64 / 2;
  return pan > red ? pan : red;
}

// LDS: coefficients, panel (reused for the reduction) and the recurrence
// coefficients of the order.
size_t synthesis_lds_bytes(int N, int NF) {
  return sizeof(double2) * (size_t)((N + 3) + synth_pan_slots(N, NF) + N + 2 + kOtfBatch);
}

// TT: type of the products and of the per-wave accumulation (double for
// NSE_PREC_FP64; float for NSE_PREC_FP32, where the panel is rounded to FP32 once
// and each Legendre value before its products); the recurrence and the
// cross-wave sums are FP64 in both.
// NF: 4 (nonlinear and grid modes) or 5 (adjoint mode).
// The Legendre values are continued in registers by the three-term recurrence of
// eq. (sph_har),
//   Pbar[l,m] = a(l,m) mu Pbar[l-1,m] - (a(l,m) / a(l-1,m)) Pbar[l-2,m],
//   a(l,m) = sqrt((4 l^2 - 1) / (l^2 - m^2)),
// from two table rows at the start of each wave's degree range (seeds), with
// the coefficient pairs of the order in LDS. The table traffic drops from the
// whole T1 to two rows per wave.
// R: latitudes per lane (tiles of 64 R latitudes, lane l taking l, l + 64, ...):
// every panel value read from LDS then serves R latitudes, which is what bounds
// the loop (the LDS, shared by the four SIMDs).
template <typename TT, int NF, int R = 1>
__global__ __launch_bounds__(kSynthThreads) void k_synthesis(GroupView g, SynthInput in,
                                                              int mode) {
  constexpr int kRed = 4 * NF;
  constexpr int kB = (R == 1) ? kOtfBatch : 2;  // degrees per recurrence batch
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (nh + 64 * R - 1) / (64 * R);
  // the tiles of one order run on one XCD and share its L2 for the order's
  // input states and coefficients
  const int item = xcd_item(blockIdx.x, ntile);
  const int m = item / ntile;
  const int tile = item - m * ntile;
  if (m > N) return;  // uniform across the workgroup
  const int b = blockIdx.y;
  const int L = N + 2 - m;  // degrees m .. N+1
  extern __shared__ double2 sh[];
  double2* a = sh;              // [L + 1] state coefficients alpha[l], l = m..N (0 beyond)
  double2* pan = sh + (N + 3);  // [L][NF]

  // recurrence pairs of the order (k = 2 .. L-1, from the group's table),
  // requested with the input states so that one memory round trip covers both
  double2 rcv[kRcPerThread];
#pragma unroll
  for (int i = 0; i < kRcPerThread; ++i) {
    const int k = threadIdx.x + i * kSynthThreads;
    rcv[i] = (k >= 2 && k < L) ? g.rec_a[rec_slot(N, m + k, m)] : make_double2(0.0, 0.0);
  }
  load_order(a, g, in, b, m, L);
  // an ended attempt of a device-controlled run: checked once the loads are in
  // flight (nothing is stored before this barrier), so the flag costs no wait
  if (gate_closed(g)) return;
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
  double2* rc = pan + synth_pan_slots(N, NF);  // [L + kOtfBatch] (a(l,m), a(l,m) / a(l-1,m))
#pragma unroll
  for (int i = 0; i < kRcPerThread; ++i) {
    const int k = threadIdx.x + i * kSynthThreads;
    if (k < L + kOtfBatch) rc[k] = rcv[i];
  }
  __syncthreads();
  // FP32 products read the panel as float2, rounded once per entry and written
  // in place over the front of the FP64 panel (every entry is read into
  // registers before any is overwritten); the padding entries become zero
  using TT2 = typename std::conditional<std::is_same<TT, float>::value, float2, double2>::type;
  if (std::is_same<TT, float>::value) {
    constexpr int kPer = kPanelConvPerThread;
    const int npan = NF * (L + kOtfBatch);
    double2 v[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = threadIdx.x + i * kSynthThreads;
      v[i] = (e < NF * L) ? pan[e] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    float2* pf = reinterpret_cast<float2*>(pan);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = threadIdx.x + i * kSynthThreads;
      if (e < npan) pf[e] = make_float2((float)v[i].x, (float)v[i].y);
    }
    __syncthreads();
  }
  const TT2* pt = reinterpret_cast<const TT2*>(pan);

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
  if (k0 < k1) {
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
      const TT2 A0 = pt[NF * k0 + f];
      TT2 A1 = pt[NF * k0 + f];
      if (k0 + 1 < k1) A1 = pt[NF * (k0 + 1) + f];
      else A1.x = A1.y = TT(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc[r][4 * f + 0] = fma((TT)P2[r], A0.x, acc[r][4 * f + 0]);
        acc[r][4 * f + 1] = fma((TT)P2[r], A0.y, acc[r][4 * f + 1]);
        acc[r][4 * f + 2] = fma((TT)P1[r], A1.x, acc[r][4 * f + 2]);
        acc[r][4 * f + 3] = fma((TT)P1[r], A1.y, acc[r][4 * f + 3]);
      }
    }
    // batches of kB degrees: the batch's coefficient pairs and panel entries are
    // read from LDS first, then the recurrence runs through the batch for every
    // latitude of the lane and the products are accumulated (entries past k1
    // are padding and are not accumulated)
    for (int kb = k0 + 2; kb < k1; kb += kB) {
      double2 c[kB];
      TT2 A[kB][NF];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        c[u] = rc[kb + u];
#pragma unroll
        for (int f = 0; f < NF; ++f) A[u][f] = pt[NF * (kb + u) + f];
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
            const TT vt = (TT)v[u];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
              acc[r][4 * f + par + 0] = fma(vt, A[u][f].x, acc[r][4 * f + par + 0]);
              acc[r][4 * f + par + 1] = fma(vt, A[u][f].y, acc[r][4 * f + par + 1]);
            }
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

// FP64 nonlinear-mode synthesis with the colatitude derivatives taken on the
// Legendre side. With D[l] = sin(theta) dPbar[l,m]/dtheta, which the derivative
// relation above and the recurrence turn into
//   D[l] = l mu Pbar[l,m] - (2l+1) e(l) Pbar[l-1,m],
// the four fields are
//   f0 = i m sum psi[l] Pbar,  f1 = sum psi[l] D,  f2 = sum zeta_a[l] D,  f3 = i m sum zeta_a[l] Pbar
// over l = m..N, with zeta_a[l] = lambda_l psi[l] plus the Coriolis fold at
// (1, 0), which only f2 sees (f3 carries the factor m = 0 there). Per degree the
// loop reads psi[l], zeta_a[l] and two coefficient pairs from LDS, four reads
// where the panel form needs five, and D[l] has the parity opposite to Pbar[l,m] under
// mu -> -mu, so its terms go to the other half of the even/odd split. Tiles,
// latitudes per lane (R) and the cross-wave sums are those of k_synthesis.
// STEP: the synthesis of a device-controlled sweep slot that also does the
// slot's controller step (as k_ndf_step): the control block and the previous
// sweep's norms are read first and thread 0 of every workgroup runs the
// controller (the same inputs give every workgroup the same result); when an
// attempt opens, each workgroup forms its order's predictor from the updated
// differences as its input, the first latitude tile stores y0, psi and the
// iterate, and the analysis epilogue of the slot stores the differences (the
// tiles of an order all read the old ones here).
// NF = 5 (SYNTH_ADJ, the adjoint's synthesis): a fifth field
// f4 = sum lambda^(-1/2) n_bar[l] Pbar (Pbar terms, zero at l = 0, real at m = 0,
// times -h / (c_0 + h nu lambda) inside the step adjoint) written with the four
// forward fields to Fa.
template <int R, int NF, bool STEP>
__device__ __forceinline__ void synthesis_adv_body(const GroupView& g, const SynthInput& in,
                                                   const NdfArgs* na, const NdfStepArgs* ns) {
  static_assert(NF == 4 || NF == 5, "four fields, or five in the adjoint mode");
  static_assert(!STEP || NF == 4, "the controller step rides on the nonlinear synthesis");
  constexpr int kRed = 4 * NF;
  constexpr int kB = (R == 1) ? kOtfBatch : 2;  // degrees per recurrence batch
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (nh + 64 * R - 1) / (64 * R);
  // the tiles of one order run on one XCD and share its L2 for the order's
  // input states and coefficients
  const int item = xcd_item(blockIdx.x, ntile);
  const int m = item / ntile;
  const int tile = item - m * ntile;
  if (m > N) return;  // uniform across the workgroup
  const int b = blockIdx.y;
  const int K = N + 1 - m;  // degrees m .. N
  extern __shared__ double2 sh[];
  double2* psi = sh;                        // [K + kOtfBatch] psi[l] = lambda^(-1/2) alpha[l]
  double2* za = psi + (N + 1 + kOtfBatch);  // [K + kOtfBatch] zeta_a[l] = lambda_l psi[l]
  double2* rc = za + (N + 1 + kOtfBatch);   // [K + kOtfBatch] (a(l,m), a(l,m) / a(l-1,m))
  double2* dc = rc + (N + 1 + kOtfBatch);   // [K + kOtfBatch] ((2l+1) e(l), l)
  double2* n5 = dc + (N + 1 + kOtfBatch);   // NF = 5: [K + kOtfBatch] lambda^(-1/2) n_bar[l]

  const int lane = threadIdx.x & 63;
  // the wave index is uniform across the wave, so the degree bounds are scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pbase = tile * 64 * R + lane;  // latitude of slot r: pbase + 64 r
  // Degree ranges of whole batches: wave 0 takes degree 0 and the degrees
  // 1 .. chunk, wave w > 0 the degrees 1 + w chunk .. (w + 1) chunk, chunk a
  // multiple of kB, so no batch straddles two waves; past K the batch reads the
  // zero padding (its recurrence coefficients and coefficients are zero, so
  // those degrees add nothing) and the loop needs no per-degree guard.
  const int chunk = kB * ((K + kSynthWaves * kB - 1) / (kSynthWaves * kB));
  const int k0 = (wave == 0) ? 0 : 1 + wave * chunk;  // first degree of the wave
  const int kbs = (wave == 0) ? 1 : k0;                // first degree of its batches (odd)
  const int k1 = min(K, 1 + (wave + 1) * chunk);
  // The prologue's latencies overlap: the seed rows, the input states and the
  // order's recurrence coefficients (computed once per group, rec_slot) are
  // requested together, and psi and zeta_a are formed from the states directly,
  // so one barrier precedes the loop.
  // seeds: wave 0 Pbar at degree 0 (table row 0); wave w > 0 Pbar at k0 - 1 and
  // k0 - 2 (rows k0 - 1 and k0 - 2), the batches continuing from them
  double P1[R], P2[R], x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) P1[r] = P2[r] = x[r] = 0.0;
  if (k0 < k1) {
    const double* t = g.T1 + t1_order_offset(N, m, nh);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int p = pbase + 64 * r;
      if (p < nh) {
        if (wave == 0) {
          P1[r] = t[p];
        } else {
          P1[r] = t[(int64_t)(k0 - 1) * nh + p];
          P2[r] = t[(int64_t)(k0 - 2) * nh + p];
        }
        x[r] = g.mu[p];
      }
    }
  }
  const int64_t base = g.off[b] + coeff_offset(N, m);
  const int64_t rbase = rec_slot(N, m, m);
  // STEP: one degree per thread (N + 1 + kOtfBatch <= kSynthThreads), its
  // iterate and coefficients requested before the controller step
  double2 y1 = make_double2(0.0, 0.0), c1 = y1, e1 = y1;
  if constexpr (STEP) {
    const int k = threadIdx.x, l = m + k;
    if (k < K && l >= 1) y1 = in.src[0][base + k];
    if (k < K) {
      c1 = g.rec_a[rbase + k];
      e1 = g.rec_g[rbase + k];
    }
  }
  int prep = 0;
  NdfCtl* sc = nullptr;
  if constexpr (STEP) {
    // the control block after the coefficient arrays and the cross-wave buffer
    const int arrays = NF * (N + 1 + kOtfBatch), red = kSynthWaves * kRed * 64 / 2;
    sc = reinterpret_cast<NdfCtl*>(sh + (arrays > red ? arrays : red));
    double* norm = reinterpret_cast<double*>(sc + 1);
    int* prepf = reinterpret_cast<int*>(norm + 4);
    const unsigned long long* cw = reinterpret_cast<const unsigned long long*>(ns->ctl_in);
    constexpr int KW = (kCtlWords + kSynthThreads - 1) / kSynthThreads;
    unsigned long long w[KW];
#pragma unroll
    for (int i = 0; i < KW; ++i) {
      const int j = threadIdx.x + kSynthThreads * i;
      if (j < kCtlWords) w[i] = cw[j];
    }
    if (threadIdx.x < kNdfSpread) {
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        v[q] = __longlong_as_double((long long)ns->spread_in[threadIdx.x * kNdfSpreadStride + q]);
      const double mx = lane_max4(v);  // lane 16 q: the maximum of v[q]
      if ((threadIdx.x & 15) == 0) norm[threadIdx.x >> 4] = mx;
    }
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(sc);
#pragma unroll
    for (int i = 0; i < KW; ++i) {
      const int j = threadIdx.x + kSynthThreads * i;
      if (j < kCtlWords) dst[j] = w[i];
    }
    __syncthreads();
    const bool first = blockIdx.x == 0 && blockIdx.y == 0;  // order 0, tile 0, member 0
    if (threadIdx.x == 0) {
      *prepf = ndf_slot_decide(*sc, norm, *ns, first);
      sc->prep_in_analysis = *prepf;
    }
    __syncthreads();
    if (first) {
      const unsigned long long* from = reinterpret_cast<const unsigned long long*>(sc);
      unsigned long long* to = reinterpret_cast<unsigned long long*>(ns->ctl_out);
      for (int j = threadIdx.x; j < kCtlWords; j += blockDim.x) to[j] = from[j];
      for (int64_t j = threadIdx.x; j < na->spread_words; j += blockDim.x) ns->spread_clear[j] = 0ull;
    }
    if (!sc->running) return;  // no attempt open: the slot does nothing (uniform)
    prep = *prepf;
  }
  for (int k = threadIdx.x; k < K + kOtfBatch; k += blockDim.x) {
    const int l = m + k;
    // input state alpha[l] = sum_i coef_i src_i[l] (l = 1..N; real at m = 0)
    double2 src[kMaxSources];
    double2 c = make_double2(0.0, 0.0), e = c;
    if constexpr (STEP) {
#pragma unroll
      for (int i = 0; i < kMaxSources; ++i) src[i] = i == 0 ? y1 : make_double2(0.0, 0.0);
      c = c1;
      e = e1;
    } else {
#pragma unroll
      for (int i = 0; i < kMaxSources; ++i) {
        src[i] = make_double2(0.0, 0.0);
        if (i < in.nsrc && k < K && l >= 1) src[i] = in.src[i][base + k];
      }
      if (k < K) {
        c = g.rec_a[rbase + k];
        e = g.rec_g[rbase + k];
      }
    }
    double2 v = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < kMaxSources; ++i) {
      if (i < in.nsrc) {
        v.x += in.coef[i] * src[i].x;
        v.y += in.coef[i] * src[i].y;
      }
    }
    if constexpr (STEP) {
      if (prep && k < K) {
        const PrepareParams pp = prepare_params(*sc, na->dsel);
        if (pp.predict) {
          const int64_t s = base + k;
          double2 D[kNdfDepth], y, p;
          prepared_differences(na->D, na->S, na->depth, pp, s, D);
          ndf_predictor(D, pp.k, na->gam, y, p);
          if (tile == 0) {
            na->y0[s] = y;
            na->psi[s] = p;
            na->yout[s] = y;
          }
          if (l >= 1) v = y;
        }
      }
    }
    if (m == 0) v.y = 0.0;
    const double dl = (double)l;
    const double lam = (k < K) ? dl * (dl + 1.0) : 0.0;
    const double2 ps = make_double2(v.x * e.y, v.y * e.y);
    psi[k] = ps;
    za[k] = make_double2(lam * ps.x, lam * ps.y);
    rc[k] = c;
    dc[k] = make_double2(e.x, (k < K) ? dl : 0.0);
    if constexpr (NF == 5) {
      // fifth field: lambda^(-1/2) n_bar, l = max(m, 1)..N, real at m = 0
      double2 w = make_double2(0.0, 0.0);
      if (k < K && l >= 1) {
        const double2 nb = in.adj[base + k];
        double r = e.y;
        if (in.adj_step) r *= -in.adj_h / (in.adj_c0 + in.adj_h * g.nu[b] * lam);
        w = make_double2(nb.x * r, m == 0 ? 0.0 : nb.y * r);
      }
      n5[k] = w;
    }
  }
  // an ended attempt of a device-controlled run: checked once the loads are in
  // flight (nothing is stored before this barrier), so the flag costs no wait
  if (!STEP && gate_closed(g)) return;
  __syncthreads();

  // acc[r][4 f + 2 q + c]: field f, q = 0 even / 1 odd part, c = 0 re / 1 im
  double acc[R][kRed];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < kRed; ++i) acc[r][i] = 0.0;
  double XP1[R];  // mu Pbar at the newest degree
#pragma unroll
  for (int r = 0; r < R; ++r) XP1[r] = x[r] * P1[r];
  if (k0 < k1) {
    if (wave == 0) {
      // degree 0 (even): Pbar terms to the even part, D terms to the odd part
      const double2 ps = psi[0], zz = za[0], d = dc[0];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (NF == 5) {
          const double2 w = n5[0];
          acc[r][16] = fma(P1[r], w.x, acc[r][16]);
          acc[r][17] = fma(P1[r], w.y, acc[r][17]);
        }
        const double D = fma(d.y, XP1[r], -d.x * P2[r]);
        acc[r][0] = fma(P1[r], ps.x, acc[r][0]);
        acc[r][1] = fma(P1[r], ps.y, acc[r][1]);
        acc[r][6] = fma(D, ps.x, acc[r][6]);
        acc[r][7] = fma(D, ps.y, acc[r][7]);
        acc[r][10] = fma(D, zz.x, acc[r][10]);
        acc[r][11] = fma(D, zz.y, acc[r][11]);
        acc[r][12] = fma(P1[r], zz.x, acc[r][12]);
        acc[r][13] = fma(P1[r], zz.y, acc[r][13]);
      }
    }
    if (m == 0 && wave == 0 && k1 > 1) {
      // Coriolis fold: zeta_a[1,0] += coriolis, seen by f2 through D[1]
      // (degree 1 is odd, so D[1] is even); Pbar[1,0] = a(1,0) mu Pbar[0,0]
      const double2 c = rc[1], d = dc[1];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double p1 = c.x * x[r] * P1[r];
        const double D = fma(x[r], p1, -d.x * P1[r]);
        acc[r][8] = fma(in.coriolis, D, acc[r][8]);
      }
    }
    // degrees kbs .. k1 - 1 in batches of kB (kb odd: degree kb + u is odd for
    // even u)
    for (int kb = kbs; kb < k1; kb += kB) {
      double2 c[kB], ps[kB], zz[kB], d[kB], w5[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        c[u] = rc[kb + u];
        ps[u] = psi[kb + u];
        zz[u] = za[kb + u];
        d[u] = dc[kb + u];
        if constexpr (NF == 5) w5[u] = n5[kb + u];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          // mu Pbar[l] serves both this degree's D and the next recurrence step
          const double v = fma(c[u].x, XP1[r], -c[u].y * P2[r]);
          const double xv = x[r] * v;
          P2[r] = P1[r];
          P1[r] = v;
          XP1[r] = xv;
          const int qp = 2 * ((u + 1) & 1);  // part of the Pbar terms
          const int qd = 2 - qp;             // part of the D terms
          const double D = fma(d[u].y, xv, -d[u].x * P2[r]);
          acc[r][0 + qp] = fma(v, ps[u].x, acc[r][0 + qp]);
          acc[r][1 + qp] = fma(v, ps[u].y, acc[r][1 + qp]);
          acc[r][4 + qd] = fma(D, ps[u].x, acc[r][4 + qd]);
          acc[r][5 + qd] = fma(D, ps[u].y, acc[r][5 + qd]);
          acc[r][8 + qd] = fma(D, zz[u].x, acc[r][8 + qd]);
          acc[r][9 + qd] = fma(D, zz[u].y, acc[r][9 + qd]);
          acc[r][12 + qp] = fma(v, zz[u].x, acc[r][12 + qp]);
          acc[r][13 + qp] = fma(v, zz[u].y, acc[r][13 + qp]);
          if constexpr (NF == 5) {
            acc[r][16 + qp] = fma(v, w5[u].x, acc[r][16 + qp]);
            acc[r][17 + qp] = fma(v, w5[u].y, acc[r][17 + qp]);
          }
        }
      }
    }
  }
  // cross-wave sums through LDS (the coefficient arrays are no longer needed);
  // wave w finishes field w of its latitudes; f0 and f3 take the factor i m
  const double dm = (double)m;
  double* red = reinterpret_cast<double*>(sh);  // [wave][kRed][64]
#pragma unroll
  for (int r = 0; r < R; ++r) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRed; ++i) red[(wave * kRed + i) * 64 + lane] = acc[r][i];
    __syncthreads();
    const int p = pbase + 64 * r;
    for (int f = wave; f < NF && p < nh; f += kSynthWaves) {
      double er = 0.0, ei = 0.0, orr = 0.0, oi = 0.0;
#pragma unroll
      for (int w = 0; w < kSynthWaves; ++w) {
        er += red[(w * kRed + 4 * f + 0) * 64 + lane];
        ei += red[(w * kRed + 4 * f + 1) * 64 + lane];
        orr += red[(w * kRed + 4 * f + 2) * 64 + lane];
        oi += red[(w * kRed + 4 * f + 3) * 64 + lane];
      }
      double2 vn = make_double2(er + orr, ei + oi), vs = make_double2(er - orr, ei - oi);
      if (f == 0 || f == 3) {
        vn = make_double2(-dm * vn.y, dm * vn.x);
        vs = make_double2(-dm * vs.y, dm * vs.x);
      }
      double2* out = (NF == 5 ? g.Fa : g.F) + ((int64_t)(b * NF + f) * (N + 1) + m) * nlat;
      out[p] = vn;
      const int psouth = nlat - 1 - p;
      if (psouth != p) out[psouth] = vs;
    }
  }
}

template <int R, int NF>
__global__ __launch_bounds__(kSynthThreads) void k_synthesis_adv(GroupView g, SynthInput in) {
  synthesis_adv_body<R, NF, false>(g, in, nullptr, nullptr);
}

__global__ __launch_bounds__(kSynthThreads) void k_synthesis_adv_step(GroupView g, SynthInput in,
                                                                      NdfArgs a, NdfStepArgs st) {
  synthesis_adv_body<1, 4, true>(g, in, &a, &st);
}

size_t synthesis_adv_lds_bytes(int N, int nf) {
  const int arrays = nf * (N + 1 + kOtfBatch);
  const int red = kSynthWaves * 4 * nf * 64 / 2;
  return sizeof(double2) * (size_t)(arrays > red ? arrays : red);
}

// Four-field recurrence synthesis with TT products: one to three latitudes per
// lane by grid size (measured best: R = 3 at nh = 384, R = 1 at nh <= 192, where
// the grid has too few tiles for more).
template <typename TT>
hipError_t launch_synthesis_otf4(const GroupView& g, const SynthInput& in, int mode,
                                 hipStream_t s) {
  dim3 block(kSynthThreads);
  const size_t lds = synthesis_lds_bytes(g.N, 4);
  if (g.nh >= 384 && g.nh % 192 == 0) {
    const int nt = g.nh / 192;
    dim3 grid3(xcd_grid((g.N + 1) * nt, nt), g.nb);
    hipLaunchKernelGGL((k_synthesis<TT, 4, 3>), grid3, block, lds, s, g, in, mode);
  } else if (g.nh >= 256) {
    const int nt = (g.nh + 127) / 128;
    dim3 grid2(xcd_grid((g.N + 1) * nt, nt), g.nb);
    hipLaunchKernelGGL((k_synthesis<TT, 4, 2>), grid2, block, lds, s, g, in, mode);
  } else {
    const int nt = (g.nh + 63) / 64;
    dim3 grid(xcd_grid((g.N + 1) * nt, nt), g.nb);
    hipLaunchKernelGGL((k_synthesis<TT, 4>), grid, block, lds, s, g, in, mode);
  }
  return hipGetLastError();
}

hipError_t launch_synthesis(const GroupView& g, const SynthInput& in, int mode, hipStream_t s) {
  dim3 block(kSynthThreads);
  const int ntile = (g.nh + 63) / 64;
  dim3 grid(xcd_grid((g.N + 1) * ntile, ntile), g.nb);
  if (mode == SYNTH_ADJ && g.nh < 256) {
    // the derivative form with the fifth field (T255 adjoint: 14.5 us with the
    // panel form, 12.0 us; 78 VGPRs against 144)
    hipLaunchKernelGGL((k_synthesis_adv<1, 5>), grid, block, synthesis_adv_lds_bytes(g.N, 5), s,
                       g, in);
  } else if (mode == SYNTH_ADJ)
    hipLaunchKernelGGL((k_synthesis<double, 5>), grid, block,
                       synthesis_lds_bytes(g.N, 5), s, g, in, mode);
  else if (g.precision == NSE_PREC_FP32) {
    if (4 * (g.N + 2 + kOtfBatch) > kPanelConvPerThread * kSynthThreads) return hipErrorInvalidValue;
    return launch_synthesis_otf4<float>(g, in, mode, s);
  } else if (mode == SYNTH_NONLINEAR && g.nh < 256) {
    // one latitude per lane: the loop is bound by the LDS reads, and the
    // derivative-on-Legendre form reads three values per degree instead of five
    // (T255: 14.2 -> 13.8 us); with two or three latitudes per lane the panel
    // form's fewer FMAs per latitude win (T511: 38.6 us against 44.4 us)
    hipLaunchKernelGGL((k_synthesis_adv<1, 4>), grid, block, synthesis_adv_lds_bytes(g.N, 4), s, g,
                       in);
  } else {
    return launch_synthesis_otf4<double>(g, in, mode, s);
  }
  return hipGetLastError();
}

// The controller step needs about 240 VGPRs (two waves per SIMD): taken into
// the synthesis only while the launch stays resident at once (two four-wave
// workgroups per CU).
bool synthesis_takes_step(const GroupView& g) {
  const int ntile = (g.nh + 63) / 64;
  return g.precision == NSE_PREC_FP64 && g.mb_synth < 2 && g.nh < 256 &&
         g.N + 1 + kOtfBatch <= kSynthThreads && (int64_t)(g.N + 1) * ntile * g.nb <= 512;
}

hipError_t launch_synthesis_step(const GroupView& g, const SynthInput& in, const NdfArgs& a,
                                 const NdfStepArgs& st, hipStream_t s) {
  if (!synthesis_takes_step(g)) return hipErrorInvalidValue;
  const int ntile = (g.nh + 63) / 64;
  dim3 grid(xcd_grid((g.N + 1) * ntile, ntile), g.nb);
  const size_t lds = synthesis_adv_lds_bytes(g.N, 4) + sizeof(NdfCtl) + 6 * sizeof(double);
  hipLaunchKernelGGL(k_synthesis_adv_step, grid, dim3(kSynthThreads), lds, s, g, in, a, st);
  return hipGetLastError();
}

}  // namespace nse
