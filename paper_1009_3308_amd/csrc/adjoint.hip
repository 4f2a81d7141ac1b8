// Adjoint (vector-Jacobian product on the stored real doubles) of the
// synthesis and of the spectral prologue of the nonlinear term, and the
// element-wise parts of the adjoint of one NDF_p step (eq. (ode_disc)).
//
// Synthesis^T: the synthesis computes G_f(m, lat) = sum_k Pbar[m+k, m](mu_lat)
// P_f(m, k) for the four panel fields (complex-linear with real coefficients),
// so its transpose is the unweighted Legendre analysis
//   Pbar_f(m, k) = sum_lat Pbar[m+k, m](mu_lat) Gbar_f(lat, m),   k < N+2-m,
// folded over latitude pairs (the equator ring of an odd rule counted once).
// Prologue^T: the panels are f0 = i m psi, f1 = S psi, f2 = S zeta_a,
// f3 = i m zeta_a with psi = lambda^(-1/2) alpha, zeta_a = lambda^(1/2) alpha
// (+ constant) and S c[k] = cm(k) c[k-1] - cp(k) c[k+1], cm(k) = (l-1) e(l),
// cp(k) = (l+2) e(l+1), l = m + k; so
//   psi_bar[j]  = -i m f0_bar[j] + cm(j+1) f1_bar[j+1] - cp(j-1) f1_bar[j-1],
//   zeta_bar[j] = -i m f3_bar[j] + cm(j+1) f2_bar[j+1] - cp(j-1) f2_bar[j-1],
//   alpha_bar[j] = lambda^(-1/2) psi_bar[j] + lambda^(1/2) zeta_bar[j],
// zero at l = 0 and real at m = 0 (those inputs are fixed to zero).
#include "adjoint_device.h"
#include "lane_ops.h"
#include "spectral_ops.h"

namespace nse {

constexpr int kAdjWaves = 4;
constexpr int kAdjThreads = 64 * kAdjWaves;
constexpr int kAdjBatch = 8;  // table rows per load batch

size_t synthesis_adjoint_lds_bytes(int nh) {
  // folded cotangents [4 fields][2 parities][nh], reused for the cross-wave sums
  const size_t fold = sizeof(double2) * 8 * (size_t)nh;
  const size_t red = sizeof(double) * 8 * kAdjThreads;
  return fold > red ? fold : red;
}

// One workgroup of four waves per (order m, tile of 64 degrees k < N+2-m,
// member); one thread per degree, each wave summing a quarter of the northern
// latitudes of T2[m][tile][p][64]. The cotangents of one order, Fbar[b][f][m][:],
// are contiguous over latitude, so the fold reads them coalesced; orders are
// taken in XCD-local chunks of four neighbouring m.
__global__ __launch_bounds__(kAdjThreads) void k_synthesis_adjoint(GroupView g) {
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (N + 2 + 63) / 64;
  const int item = xcd_item(blockIdx.x, 4 * ntile);
  const int m = item / ntile;
  const int tile = item - m * ntile;
  const int L = N + 2 - m;
  if (m > N || tile * 64 >= L) return;  // uniform across the workgroup
  const int b = blockIdx.y;
  extern __shared__ double2 fsh[];  // [f][parity][nh]
  const int64_t fstride = (int64_t)(N + 1) * nlat;
  const double2* Gb = g.Fbar + (int64_t)b * 4 * fstride + (int64_t)m * nlat;  // Fbar[b][f][m][lat]
  for (int i = threadIdx.x; i < 4 * nh; i += blockDim.x) {
    const int f = i / nh, p = i - f * nh;
    const int ps = nlat - 1 - p;
    const double2 gn = Gb[f * fstride + p];
    double2 we = gn, wo = make_double2(0.0, 0.0);
    if (ps != p) {
      const double2 gs = Gb[f * fstride + ps];
      we = make_double2(gn.x + gs.x, gn.y + gs.y);
      wo = make_double2(gn.x - gs.x, gn.y - gs.y);
    }
    fsh[(2 * f) * nh + p] = we;
    fsh[(2 * f + 1) * nh + p] = wo;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = tile * 64 + lane;
  const int pq = (nh + kAdjWaves - 1) / kAdjWaves;
  const int p0 = wave * pq, p1 = min(nh, p0 + pq);
  double acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0.0;
  if (k < L) {
    const int par = k & 1;
    const double* t = g.T2 + g.t2off[m] + (int64_t)tile * nh * kTile + lane;
    // batches of kAdjBatch latitudes; the next batch's table loads are issued
    // before the current batch's FMAs
    double tn[kAdjBatch];
#pragma unroll
    for (int u = 0; u < kAdjBatch; ++u) tn[u] = (p0 + u < p1) ? t[(int64_t)(p0 + u) * kTile] : 0.0;
    for (int pb = p0; pb < p1; pb += kAdjBatch) {
      double tc[kAdjBatch];
#pragma unroll
      for (int u = 0; u < kAdjBatch; ++u) tc[u] = tn[u];
#pragma unroll
      for (int u = 0; u < kAdjBatch; ++u) {
        const int p = pb + kAdjBatch + u;
        tn[u] = (p < p1) ? t[(int64_t)p * kTile] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kAdjBatch; ++u) {
        const int p = pb + u;
        if (p < p1) {
#pragma unroll
          for (int f = 0; f < 4; ++f) {
            const double2 w = fsh[(2 * f + par) * nh + p];
            acc[2 * f + 0] = fma(tc[u], w.x, acc[2 * f + 0]);
            acc[2 * f + 1] = fma(tc[u], w.y, acc[2 * f + 1]);
          }
        }
      }
    }
  }
  __syncthreads();  // the folded cotangents are no longer needed
  double* red = reinterpret_cast<double*>(fsh);  // [8][kAdjThreads]
#pragma unroll
  for (int i = 0; i < 8; ++i) red[i * kAdjThreads + threadIdx.x] = acc[i];
  __syncthreads();
  if (wave != 0 || k >= L) return;
  double2* out = g.Pbar + (((int64_t)b * (N + 1) + m) * (N + 2) + k) * 4;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int w = 0; w < kAdjWaves; ++w) {
      sx += red[(2 * f) * kAdjThreads + w * 64 + lane];
      sy += red[(2 * f + 1) * kAdjThreads + w * 64 + lane];
    }
    out[f] = make_double2(sx, sy);
  }
}

// One workgroup per (order m, member); one thread per degree l = m..N.
__global__ __launch_bounds__(256) void k_prep_adjoint(GroupView g, double2* alpha_bar) {
  const int N = g.N;
  const int m = blockIdx.x, b = blockIdx.y;
  const double2* P = g.Pbar + ((int64_t)b * (N + 1) + m) * (N + 2) * 4;  // [k][f]
  for (int k = threadIdx.x; k <= N - m; k += blockDim.x)
    alpha_bar[g.off[b] + coeff_offset(N, m) + k] = alpha_bar_at(g, P, m, k);
}

// The same sums with the Legendre values continued in registers instead of
// streamed from T2 (grids with nh <= 64 R, R <= 3 latitudes per lane). As in the
// recurrence analysis of the forward path, wave w of the (m, 64-degree tile)
// workgroup owns the degrees 16 w .. 16 w + 15 of the tile and its lanes are
// latitudes; each lane seeds the recurrence of eq. (sph_har) from the T1 rows of
// the wave's first two degrees and keeps the sixteen values of each of its
// latitudes in registers. Then, field by field, it multiplies them by its
// latitudes' folded cotangents (even or odd part by the parity of k) and the
// sixteen complex sums are formed across the lanes by the register butterfly,
// which leaves degree 8 b5 + 4 b4 + 2 b3 + b2 of the wave's block (b = lane bits)
// in the lanes with b1 = b0 = 0.
template <int R>
__global__ __launch_bounds__(kAdjThreads) void k_synthesis_adjoint_otf(GroupView g) {
  constexpr int kDeg = kButterfly;  // degrees per wave
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (N + 2 + 63) / 64;
  const int item = xcd_item(blockIdx.x, 4 * ntile);
  const int m = item / ntile;
  const int tile = item - m * ntile;
  const int L = N + 2 - m;  // k < L; T1 holds the rows k = 0 .. L - 1 of order m
  if (m > N || tile * 64 >= L) return;  // uniform across the workgroup
  const int b = blockIdx.y;
  extern __shared__ double2 fsh[];  // [f][parity][nh], then the tile's recurrence pairs [64]
  double2* rc = fsh + 8 * nh;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kt = tile * 64;
  const int j0 = wave * kDeg;
  const bool active = kt + j0 < L;
  // seeds first, their latency overlapping the fold
  double x[R], P1[R], P2[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = P1[r] = P2[r] = 0.0;
  if (active) {
    const double* t = g.T1 + t1_order_offset(N, m, nh) + (int64_t)(kt + j0) * nh;
    const bool second = kt + j0 + 1 < L;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int p = lane + 64 * r;
      if (p < nh) {
        P2[r] = t[p];
        if (second) P1[r] = t[nh + p];
        x[r] = g.mu[p];
      }
    }
  }
  // the cotangents of the four fields at every latitude pair (4 nh <= 256 R items,
  // R per thread), all requested before the first LDS write
  const int64_t fstride = (int64_t)(N + 1) * nlat;
  const double2* Gb = g.Fbar + (int64_t)b * 4 * fstride + (int64_t)m * nlat;  // Fbar[b][f][m][lat]
  double2 gn[R], gs[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int idx = threadIdx.x + i * kAdjThreads;
    gn[i] = gs[i] = make_double2(0.0, 0.0);
    if (idx < 4 * nh) {
      const int f = idx / nh, p = idx - f * nh;
      const int ps = nlat - 1 - p;
      gn[i] = Gb[f * fstride + p];
      if (ps != p) gs[i] = Gb[f * fstride + ps];
    }
  }
  // recurrence pairs (a(l,m), a(l,m) / a(l-1,m)) of the tile's degrees k = 2 .. L - 1;
  // zero elsewhere, so the values past the order's last degree stay zero
  if (threadIdx.x < 64) {
    const int k = kt + threadIdx.x;
    rc[threadIdx.x] = (k >= 2 && k < L) ? g.rec_a[rec_slot(N, m + k, m)] : make_double2(0.0, 0.0);
  }
  // fold: We = G(p) + G(p'), Wo = G(p) - G(p') (the equator ring of an odd rule,
  // its own mirror, counted once: gs = 0)
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int idx = threadIdx.x + i * kAdjThreads;
    if (idx < 4 * nh) {
      const int f = idx / nh, p = idx - f * nh;
      fsh[(2 * f) * nh + p] = make_double2(gn[i].x + gs[i].x, gn[i].y + gs[i].y);
      fsh[(2 * f + 1) * nh + p] = make_double2(gn[i].x - gs[i].x, gn[i].y - gs[i].y);
    }
  }
  __syncthreads();
  if (!active) return;
  double v[kDeg][R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    v[0][r] = P2[r];
    v[1][r] = P1[r];
  }
#pragma unroll
  for (int i = 2; i < kDeg; ++i) {
    const double2 c = rc[j0 + i];
#pragma unroll
    for (int r = 0; r < R; ++r) v[i][r] = fma(c.x * x[r], v[i - 1][r], -c.y * v[i - 2][r]);
  }
  const int j = 8 * ((lane >> 5) & 1) + 4 * ((lane >> 4) & 1) + 2 * ((lane >> 3) & 1) +
                ((lane >> 2) & 1);
  const int k = kt + j0 + j;
  double2* out = g.Pbar + (((int64_t)b * (N + 1) + m) * (N + 2) + k) * 4;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double sr[kDeg], si[kDeg];
#pragma unroll
    for (int i = 0; i < kDeg; ++i) sr[i] = si[i] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int p = lane + 64 * r;
      double2 we = make_double2(0.0, 0.0), wo = we;
      if (p < nh) {
        we = fsh[(2 * f) * nh + p];
        wo = fsh[(2 * f + 1) * nh + p];
      }
#pragma unroll
      for (int i = 0; i < kDeg; ++i) {
        const double2 w = (i & 1) ? wo : we;  // kt and j0 are even: the parity of k is that of i
        sr[i] = fma(v[i][r], w.x, sr[i]);
        si[i] = fma(v[i][r], w.y, si[i]);
      }
    }
    lane_butterfly16(sr, si, lane);
    if ((lane & 3) == 0 && k < L) out[f] = make_double2(sr[0], si[0]);
  }
}

size_t synthesis_adjoint_otf_lds_bytes(int nh) { return sizeof(double2) * (size_t)(8 * nh + 64); }

hipError_t launch_synthesis_adjoint(const GroupView& g, hipStream_t s) {
  const int ntile = (g.N + 2 + 63) / 64;
  dim3 grid(xcd_grid((g.N + 1) * ntile, 4 * ntile), g.nb);
  const size_t lds = synthesis_adjoint_otf_lds_bytes(g.nh);
  switch ((g.nh + 63) / 64) {
    case 1: hipLaunchKernelGGL(k_synthesis_adjoint_otf<1>, grid, dim3(kAdjThreads), lds, s, g); break;
    case 2: hipLaunchKernelGGL(k_synthesis_adjoint_otf<2>, grid, dim3(kAdjThreads), lds, s, g); break;
    case 3: hipLaunchKernelGGL(k_synthesis_adjoint_otf<3>, grid, dim3(kAdjThreads), lds, s, g); break;
    default:
      hipLaunchKernelGGL(k_synthesis_adjoint, grid, dim3(kAdjThreads),
                         synthesis_adjoint_lds_bytes(g.nh), s, g);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_prep_adjoint(const GroupView& g, double2* alpha_bar, hipStream_t s) {
  dim3 grid(g.N + 1, g.nb);
  hipLaunchKernelGGL(k_prep_adjoint, grid, dim3(256), 0, s, g, alpha_bar);
  return hipGetLastError();
}

// The history update that ends the adjoint of one step (StepAdjointArgs), one
// thread per (order m, degree k), in place over hist_bar (each thread reads its
// coefficient's cotangents before it writes them). The cotangent of the
// nonlinear term, n_bar = -h r, was formed inside the five-field synthesis
// from the same hbar_out[0].
__global__ __launch_bounds__(256) void k_prep_step_adjoint(GroupView g, StepAdjointArgs a) {
  const int N = g.N;
  const int m = blockIdx.x, b = blockIdx.z;
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  if (k > N - m) return;
  step_adjoint_store(g, a, b, m, k);
}

hipError_t launch_prep_step_adjoint(const GroupView& g, const StepAdjointArgs& a, hipStream_t s) {
  dim3 grid(g.N + 1, (g.N + 1 + 255) / 256, g.nb);
  hipLaunchKernelGGL(k_prep_step_adjoint, grid, dim3(256), 0, s, g, a);
  return hipGetLastError();
}

}  // namespace nse
