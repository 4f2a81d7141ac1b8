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
// Workgroups of four waves per (order m, tile of 64 degrees, member): one
// thread per degree l (coalesced reads of T2[m][p][l-m] across the wavefront),
// each wave summing a quarter of the northern latitudes, partial sums added
// through LDS. Orders are taken in XCD-local chunks of four neighbouring m so
// that the strided reads of W[lat][m] share L2 lines.
#include "lane_ops.h"
#include "spectral_ops.h"

namespace nse {

constexpr int kAnalWaves = 4;
constexpr int kAnalThreads = 64 * kAnalWaves;
constexpr int kBatch = 8;  // table rows per load batch

size_t analysis_lds_bytes(int nh) {
  return 2 * sizeof(double2) * (size_t)nh + sizeof(double) * 2 * kAnalThreads;
}

// TT: element type of the table and of the products and accumulation (double
// for NSE_PREC_FP64, float for NSE_PREC_FP32); the cross-wave sums are FP64.
template <typename TT>
__global__ __launch_bounds__(kAnalThreads) void k_analysis(GroupView g, AnalOutput out) {
  const int N = g.N, nh = g.nh;
  const int ntile = (N + 1 + 63) / 64;
  const int item = xcd_item(blockIdx.x, 4 * ntile);
  const int m = item / ntile;
  const int tile = item - m * ntile;
  if (m > N || tile * 64 > N - m) return;  // uniform across the workgroup
  const int b = blockIdx.y;
  extern __shared__ double2 wsh[];  // [2][nh] then [2][kAnalThreads] doubles
  double* red = reinterpret_cast<double*>(wsh + 2 * nh);
  // fold the ring spectra of each latitude pair: We = Q(p) + Q(p'), Wo = Q(p) - Q(p')
  const double2* Wb = g.W + (int64_t)b * g.nlat * (N + 1) + m;
  for (int p = threadIdx.x; p < nh; p += blockDim.x) {
    const double2 qn = Wb[(int64_t)p * (N + 1)];
    const double2 qs = Wb[(int64_t)(g.nlat - 1 - p) * (N + 1)];
    wsh[p] = make_double2(qn.x + qs.x, qn.y + qs.y);
    wsh[nh + p] = make_double2(qn.x - qs.x, qn.y - qs.y);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int k = tile * 64 + lane;
  const int l = m + k;
  const int pq = (nh + kAnalWaves - 1) / kAnalWaves;
  const int p0 = wave * pq;
  const int p1 = min(nh, p0 + pq);
  TT ax = TT(0), ay = TT(0), bx = TT(0), by = TT(0);
  if (l <= N) {
    const double2* Ws = wsh + ((k & 1) ? nh : 0);
    // this degree tile's block of the table: rows p of 64 degrees, contiguous
    const TT* t = analysis_table<TT>(g) + g.t2off[m] + (int64_t)tile * nh * kTile + lane;
    // batches of kBatch latitudes; the next batch's table loads are issued
    // before the current batch's FMAs
    TT tn[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) tn[u] = (p0 + u < p1) ? t[(int64_t)(p0 + u) * kTile] : TT(0);
    for (int pb = p0; pb < p1; pb += kBatch) {
      TT tc[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) tc[u] = tn[u];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int p = pb + kBatch + u;
        tn[u] = (p < p1) ? t[(int64_t)p * kTile] : TT(0);
      }
#pragma unroll
      for (int u = 0; u < kBatch; u += 2) {
        const int p = pb + u;
        if (p < p1) {
          const double2 w0 = Ws[p];
          ax = fma(tc[u], (TT)w0.x, ax);
          ay = fma(tc[u], (TT)w0.y, ay);
        }
        if (p + 1 < p1) {
          const double2 w1 = Ws[p + 1];
          bx = fma(tc[u + 1], (TT)w1.x, bx);
          by = fma(tc[u + 1], (TT)w1.y, by);
        }
      }
    }
  }
  red[threadIdx.x] = (double)ax + (double)bx;
  red[kAnalThreads + threadIdx.x] = (double)ay + (double)by;
  __syncthreads();
  if (wave != 0 || l > N) return;
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int w = 0; w < kAnalWaves; ++w) {
    sx += red[w * 64 + lane];
    sy += red[kAnalThreads + w * 64 + lane];
  }
  finish_degree(g, out, b, m, k, sx, sy);
}

// FP64 analysis with the Legendre values continued in registers (OTF): the
// same sums, the loop transposed. Workgroup (m, tile of 64 degrees, member) as
// above; wave w owns the degrees 16 w .. 16 w + 15 of the tile and its lanes are
// latitudes, lane l taking p = l + 64 r for r < R (R = ceil(nh / 64)). Each lane
// starts the recurrence of eq. (sph_har),
//   Pbar[l,m] = a(l,m) mu Pbar[l-1,m] - (a(l,m) / a(l-1,m)) Pbar[l-2,m],
// from the T1 rows of the wave's own first two degrees (coalesced across the
// lanes), and multiplies each value by its own latitude's folded spectrum
// (We for even l-m, Wo for odd) held in registers; the sixteen complex sums are
// then formed across the 64 lanes by a butterfly of register exchanges, which
// leaves degree 8 b5 + 4 b4 + 2 b3 + b2 of the wave's block (b = lane bits) in
// every lane with b1 = b0 = 0. The table traffic drops to two rows per wave.
namespace {

constexpr int kOtfDeg = kButterfly;  // degrees per wave

template <int R>
__global__ __launch_bounds__(kAnalThreads) void k_analysis_otf(GroupView g, AnalOutput out) {
  const int N = g.N, nh = g.nh;
  const int ntile = (N + 1 + 63) / 64;
  const int item = xcd_item(blockIdx.x, 4 * ntile);
  const int m = item / ntile;
  const int tile = item - m * ntile;
  if (m > N || tile * 64 > N - m) return;  // uniform across the workgroup
  const int b = blockIdx.y;
  extern __shared__ double2 wsh[];  // We [nh], Wo [nh], rc [64]
  double2* rc = wsh + 2 * nh;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int kt = tile * 64;  // first degree offset k = l - m of the tile

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
  // the thread's first pair is requested before the coefficient pairs are
  // computed, so that their square roots overlap its latency
  const double2* Wb = g.W + (int64_t)b * g.nlat * (N + 1) + m;
  double2 qn = make_double2(0.0, 0.0), qs = qn;
  if ((int)threadIdx.x < nh) {
    qn = Wb[(int64_t)threadIdx.x * (N + 1)];
    qs = Wb[(int64_t)(g.nlat - 1 - (int)threadIdx.x) * (N + 1)];
  }
  // recurrence pairs of the tile's degrees (k >= 2 of the order)
  if (threadIdx.x < 64) {
    const int k = kt + threadIdx.x;
    double2 c = make_double2(0.0, 0.0);
    if (k >= 2) {
      const double dl = (double)(m + k), dm = (double)m;
      const double al = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - dm * dm));
      const double al1 =
          sqrt((4.0 * (dl - 1.0) * (dl - 1.0) - 1.0) / ((dl - 1.0) * (dl - 1.0) - dm * dm));
      c = make_double2(al, al / al1);
    }
    rc[threadIdx.x] = c;
  }
  for (int p = threadIdx.x; p < nh; p += blockDim.x) {
    if (p != (int)threadIdx.x) {
      qn = Wb[(int64_t)p * (N + 1)];
      qs = Wb[(int64_t)(g.nlat - 1 - p) * (N + 1)];
    }
    wsh[p] = make_double2(qn.x + qs.x, qn.y + qs.y);
    wsh[nh + p] = make_double2(qn.x - qs.x, qn.y - qs.y);
  }
  __syncthreads();
  if (!active) return;
  double2 We[R], Wo[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = lane + 64 * r;
    We[r] = Wo[r] = make_double2(0.0, 0.0);
    if (p < nh) {
      We[r] = wsh[p];
      Wo[r] = wsh[nh + p];
    }
  }
  // P2 = Pbar at j0, P1 at j0 + 1 (j0 is even: even, odd)
  double sr[kOtfDeg], si[kOtfDeg];
#pragma unroll
  for (int i = 0; i < kOtfDeg; ++i) sr[i] = si[i] = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    sr[0] = fma(P2[r], We[r].x, sr[0]);
    si[0] = fma(P2[r], We[r].y, si[0]);
    sr[1] = fma(P1[r], Wo[r].x, sr[1]);
    si[1] = fma(P1[r], Wo[r].y, si[1]);
  }
#pragma unroll
  for (int i = 2; i < kOtfDeg; ++i) {
    const double2 c = rc[j0 + i];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double v = fma(c.x * x[r], P1[r], -c.y * P2[r]);
      P2[r] = P1[r];
      P1[r] = v;
      const double2 w = (i & 1) ? Wo[r] : We[r];
      sr[i] = fma(v, w.x, sr[i]);
      si[i] = fma(v, w.y, si[i]);
    }
  }
  lane_butterfly16(sr, si, lane);
  if ((lane & 3) != 0) return;
  const int j = 8 * ((lane >> 5) & 1) + 4 * ((lane >> 4) & 1) + 2 * ((lane >> 3) & 1) +
                ((lane >> 2) & 1);
  const int k = kt + j0 + j;
  if (k > N - m) return;
  finish_degree(g, out, b, m, k, sr[0], si[0]);
}

}  // namespace

size_t analysis_otf_lds_bytes(int nh) { return sizeof(double2) * (size_t)(2 * nh + 64); }

hipError_t launch_analysis(const GroupView& g, const AnalOutput& out, hipStream_t s) {
  dim3 block(kAnalThreads);
  const int ntile = (g.N + 1 + 63) / 64;
  dim3 grid(xcd_grid((g.N + 1) * ntile, 4 * ntile), g.nb);
  if (g.precision == NSE_PREC_FP32) {
    hipLaunchKernelGGL(k_analysis<float>, grid, block, analysis_lds_bytes(g.nh), s, g, out);
    return hipGetLastError();
  }
  const size_t lds = analysis_otf_lds_bytes(g.nh);
  switch ((g.nh + 63) / 64) {
    case 1: hipLaunchKernelGGL(k_analysis_otf<1>, grid, block, lds, s, g, out); break;
    case 2: hipLaunchKernelGGL(k_analysis_otf<2>, grid, block, lds, s, g, out); break;
    case 3: hipLaunchKernelGGL(k_analysis_otf<3>, grid, block, lds, s, g, out); break;
    case 4: hipLaunchKernelGGL(k_analysis_otf<4>, grid, block, lds, s, g, out); break;
    case 5: hipLaunchKernelGGL(k_analysis_otf<5>, grid, block, lds, s, g, out); break;
    default: hipLaunchKernelGGL(k_analysis_otf<6>, grid, block, lds, s, g, out); break;
  }
  return hipGetLastError();
}

}  // namespace nse
