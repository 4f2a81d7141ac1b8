// Member-batched Legendre contractions for truncation groups with several
// members (an ensemble of flows that share N and the grid): the same sums as
// the synthesis and analysis of Section 4.2, with the table entries of one
// (order, tile) reused by a block of B members as the columns of an FP64
// matrix product on MFMA (v_mfma_f64_16x16x4f64). One table pass then serves
// B members instead of one, which turns the HBM-bound per-member sums into
// a compute-bound product.
//
// Synthesis, per (order m, tile of 64 northern latitudes, member block):
//   E[lat][c] = sum_{k even} T1[m][k][lat] P[k][c],  O = same over odd k,
// with the columns c = (member, field, re/im) of the coefficient panels
// (8 per member; the panels are those of spectral_ops.h, computed first for
// every member by a small kernel into a panel buffer whose rows follow T1);
// F(north) = E + O, F(south) = E - O. Both operands of an MFMA come straight
// from global memory into registers (the table from HBM, the panels from L2),
// the next two MFMA steps' operands being loaded while the current ones are
// multiplied; no LDS and no barriers.
// Wave w owns latitudes 16w..16w+15 of the tile: its A operand is a 16 x 4
// block of the table (four even or four odd degrees), its B operand a 4 x 16
// block of the panels.
// Analysis, per (order m, tile of 64 degrees, member block):
//   s[k][c] = sum_p T2[m][k][p] Wf[p][c],  Wf = We (k even) or Wo (k odd),
// with the columns c = (member, re/im) of the ring spectra folded over
// latitude pairs, staged 64 latitudes at a time into LDS (the next chunk's ring
// spectra and table operands are loaded during the current chunk's products). Wave w owns degrees
// 32(w%2)..+31 of the tile (16 even rows and 16 odd rows) and half of each
// latitude chunk; the two halves meet in LDS and the epilogue of
// spectral_ops.h finishes each (member, degree).
//
// FP64 MFMA operand layout (checked on gfx950): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and receives D[l/16 + 4r][l%16], r = 0..3.
#include "spectral_ops.h"

namespace nse {

typedef double doublex4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kMbThreads = 256;
constexpr int kMaxAl = kMaxM / 2 + 4;  // predictor coefficients of one order (N + 4 at most)

__device__ __forceinline__ doublex4 mfma64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Panel values of one degree from the predictor coefficients a[k-1], a[k],
// a[k+1] (already summed over the sources), as in build_panel.
__device__ __forceinline__ void panel4(const double2 a[3], int N, int m, int k, double coriolis,
                                       double v[8]) {
  const int l = m + k;
  const double dl = (double)l, dm = (double)m;
  double2 ps[3], zs[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ll = l - 1 + d;
    ps[d] = zs[d] = make_double2(0.0, 0.0);
    if (ll >= m && ll >= 1 && ll <= N) {
      const double lam = (double)ll * (ll + 1);
      const double sq = sqrt(lam), r = 1.0 / sq;
      ps[d] = make_double2(a[d].x * r, a[d].y * r);
      zs[d] = make_double2(a[d].x * sq, a[d].y * sq);
      if (m == 0 && ll == 1) zs[d].x += coriolis;
    }
  }
  const double e_l = (l > m) ? sqrt((dl * dl - dm * dm) / (4.0 * dl * dl - 1.0)) : 0.0;
  const double e_l1 = sqrt(((dl + 1) * (dl + 1) - dm * dm) / (4.0 * (dl + 1) * (dl + 1) - 1.0));
  const double cm = (dl - 1.0) * e_l, cp = (dl + 2.0) * e_l1;
  v[0] = -dm * ps[1].y;
  v[1] = dm * ps[1].x;
  v[2] = cm * ps[0].x - cp * ps[2].x;
  v[3] = cm * ps[0].y - cp * ps[2].y;
  v[4] = cm * zs[0].x - cp * zs[2].x;
  v[5] = cm * zs[0].y - cp * zs[2].y;
  v[6] = -dm * zs[1].y;
  v[7] = dm * zs[1].x;
}

// Panels of every member of the group for one order m, written to
// Pmb[m][k][b][8] (rows k < L = N+2-m in the row order of T1; members past the
// group are written as zeros): one workgroup per (m, member).
__global__ __launch_bounds__(kMbThreads) void k_panel_mb(GroupView g, SynthInput in) {
  __shared__ double2 al[kMaxAl];
  const int N = g.N;
  const int m = blockIdx.x, b = blockIdx.y;
  const int L = N + 2 - m;
  double* P = g.Pmb + (t1_order_offset(N, m, 1) * g.nbp + b) * 8;
  if (b >= g.nb) {
    for (int k = threadIdx.x; k < L; k += kMbThreads) {
      double* row = P + (int64_t)k * g.nbp * 8;
#pragma unroll
      for (int f = 0; f < 8; ++f) row[f] = 0.0;
    }
    return;
  }
  const int64_t base = g.off[b] + coeff_offset(N, m);
  for (int kk = threadIdx.x; kk < L + 2; kk += kMbThreads) {  // al[kk] = alpha[m + kk - 1]
    const int k = kk - 1, ll = m + k;
    double2 v = make_double2(0.0, 0.0);
    if (k >= 0 && ll >= 1 && ll <= N) {
#pragma unroll
      for (int s = 0; s < kMaxSources; ++s) {
        if (s < in.nsrc) {
          const double2 x = in.src[s][base + k];
          v.x += in.coef[s] * x.x;
          v.y += in.coef[s] * x.y;
        }
      }
      if (m == 0) v.y = 0.0;
    }
    al[kk] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < L; k += kMbThreads) {
    const double2 a3[3] = {al[k], al[k + 1], al[k + 2]};
    double v[8];
    panel4(a3, N, m, k, in.coriolis, v);
    double* row = P + (int64_t)k * g.nbp * 8;
#pragma unroll
    for (int f = 0; f < 8; ++f) row[f] = v[f];
  }
}

// Work items (order m, member block, latitude tile) are taken in XCD-local
// chunks of one order, so the blocks and tiles of an order share an L2.
template <int B>
__global__ __launch_bounds__(kMbThreads) void k_synthesis_mb(GroupView g) {
  constexpr int NC = 8 * B;                // live columns per parity
  constexpr int NCB = (NC + 15) / 16;      // 16-column blocks
  constexpr int NJ = 2;                    // MFMA steps (8 degrees each) per pipeline stage
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (nh + 63) / 64;
  const int nblk = (g.nb + B - 1) / B;
  const int item = xcd_item(blockIdx.x, ntile * nblk);
  const int m = item / (ntile * nblk);
  if (m > N) return;
  const int rest = item - m * ntile * nblk;
  const int blk = rest / ntile, tile = rest - blk * ntile;
  const int L = N + 2 - m;  // degrees m .. N+1
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int arow = lane & 15, kq = lane >> 4;
  const int lat = tile * 64 + wave * 16 + arow;  // this lane's A-operand latitude
  const bool lat_ok = lat < nh;
  const double* T = g.T1 + t1_order_offset(N, m, nh) + lat;
  const int64_t pstride = (int64_t)g.nbp * 8;
  const double* P = g.Pmb + t1_order_offset(N, m, 1) * pstride + blk * B * 8 + arow;

  doublex4 accE[NCB], accO[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) accE[c] = accO[c] = doublex4{0.0, 0.0, 0.0, 0.0};
  // operands of one stage: degrees kc + 8 j + 2 kq (even) and +1 (odd)
  double aE[NJ], aO[NJ], bE[NJ][NCB], bO[NJ][NCB];
  double nE[NJ], nO[NJ], cE[NJ][NCB], cO[NJ][NCB];
  auto load = [&](int kc, double* xE, double* xO, double (*yE)[NCB], double (*yO)[NCB]) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int kE = kc + 8 * j + 2 * kq, kO = kE + 1;
      xE[j] = (lat_ok && kE < L) ? T[(int64_t)kE * nh] : 0.0;
      xO[j] = (lat_ok && kO < L) ? T[(int64_t)kO * nh] : 0.0;
#pragma unroll
      for (int c = 0; c < NCB; ++c) {
        const bool live = 16 * c + arow < NC;
        yE[j][c] = (live && kE < L) ? P[(int64_t)kE * pstride + 16 * c] : 0.0;
        yO[j][c] = (live && kO < L) ? P[(int64_t)kO * pstride + 16 * c] : 0.0;
      }
    }
  };
  load(0, aE, aO, bE, bO);
  for (int kc = 0; kc < L; kc += 8 * NJ) {
    const bool more = kc + 8 * NJ < L;
    if (more) load(kc + 8 * NJ, nE, nO, cE, cO);  // in flight during this stage's products
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
      for (int c = 0; c < NCB; ++c) {
        accE[c] = mfma64(aE[j], bE[j][c], accE[c]);
        accO[c] = mfma64(aO[j], bO[j][c], accO[c]);
      }
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        aE[j] = nE[j];
        aO[j] = nO[j];
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
          bE[j][c] = cE[j][c];
          bO[j][c] = cO[j][c];
        }
      }
    }
  }

  // lane holds rows (latitudes) kq + 4r of its wave's 16, column arow of each block
  const int b0 = blk * B;
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    const int col = 16 * c + arow;
    if (col >= NC) continue;
    const int bb = col >> 3, f = (col & 7) >> 1, ri = col & 1;
    const int b = b0 + bb;
    if (b >= g.nb) continue;
    double* out = reinterpret_cast<double*>(g.F + ((int64_t)(b * 4 + f) * (N + 1) + m) * nlat);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = tile * 64 + wave * 16 + kq + 4 * r;
      if (p >= nh) continue;
      const double e = accE[c][r], o = accO[c][r];
      out[2 * p + ri] = e + o;
      const int ps = nlat - 1 - p;
      if (ps != p) out[2 * ps + ri] = e - o;
    }
  }
}

template <int B>
__global__ __launch_bounds__(kMbThreads) void k_analysis_mb(GroupView g, AnalOutput out) {
  static_assert(2 * B <= 16, "one 16-column block: (member, re/im)");
  constexpr int NW = (64 * B + kMbThreads - 1) / kMbThreads;  // fold items per thread
  __shared__ double wf[2][64][16];  // folded ring spectra of a 64-latitude chunk: [parity][p][col]
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (N + 2 + 63) / 64;  // tiles of T2 (degrees m .. N+1)
  const int m = blockIdx.x / ntile;
  const int tile = blockIdx.x - m * ntile;
  const int Lk = N + 1 - m;  // degrees m .. N
  if (tile * 64 >= Lk) return;  // uniform across the workgroup
  const int b0 = blockIdx.y * B;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = wave & 1, q = wave >> 1;
  const int arow = lane & 15, kq = lane >> 4;
  const double* T = g.T2 + g.t2off[m] + (int64_t)tile * nh * kTile + 32 * h + 2 * arow;

  // ring spectra of latitude p and its mirror for this thread's fold items
  double2 wn[NW], ws[NW];
  auto load_w = [&](int pc) {
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int i = threadIdx.x + j * kMbThreads;
      const int pp = i / B, bb = i - pp * B;
      const int p = pc + pp, b = b0 + bb;
      wn[j] = ws[j] = make_double2(0.0, 0.0);
      if (i < 64 * B && p < nh && b < g.nb) {
        const double2* Wb = g.W + (int64_t)b * nlat * (N + 1) + m;
        wn[j] = Wb[(int64_t)p * (N + 1)];
        ws[j] = Wb[(int64_t)(nlat - 1 - p) * (N + 1)];
      }
    }
  };
  // table operands (even, odd degree) of this wave's eight MFMA steps of a chunk
  auto load_t = [&](int pc, double2* a) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int p = pc + 32 * q + 4 * j + kq;
      a[j] = (p < nh) ? *reinterpret_cast<const double2*>(T + (int64_t)p * kTile)
                      : make_double2(0.0, 0.0);
    }
  };

  for (int i = threadIdx.x; i < 2 * 64 * 16; i += kMbThreads) (&wf[0][0][0])[i] = 0.0;
  double2 a[8], an[8];
  load_w(0);
  load_t(0, a);
  __syncthreads();
  doublex4 accE = {0.0, 0.0, 0.0, 0.0}, accO = {0.0, 0.0, 0.0, 0.0};
  for (int pc = 0; pc < nh; pc += 64) {
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int i = threadIdx.x + j * kMbThreads;
      if (i < 64 * B) {
        const int pp = i / B, bb = i - pp * B;
        wf[0][pp][2 * bb] = wn[j].x + ws[j].x;
        wf[0][pp][2 * bb + 1] = wn[j].y + ws[j].y;
        wf[1][pp][2 * bb] = wn[j].x - ws[j].x;
        wf[1][pp][2 * bb + 1] = wn[j].y - ws[j].y;
      }
    }
    __syncthreads();
    const bool more = pc + 64 < nh;
    if (more) {  // next chunk's loads are in flight during this chunk's products
      load_w(pc + 64);
      load_t(pc + 64, an);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int pp = 32 * q + 4 * j + kq;
      accE = mfma64(a[j].x, wf[0][pp][arow], accE);
      accO = mfma64(a[j].y, wf[1][pp][arow], accO);
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = an[j];
    }
    __syncthreads();
  }
  // the two latitude halves meet in LDS: red[q][local degree][col]
  double* red = &wf[0][0][0];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = kq + 4 * r;  // row of the 16 even (or odd) degrees of this wave
    red[(q * 64 + 32 * h + 2 * row) * 16 + arow] = accE[r];
    red[(q * 64 + 32 * h + 2 * row + 1) * 16 + arow] = accO[r];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * B; i += kMbThreads) {
    const int kl = i / B, bb = i - kl * B;
    const int k = tile * 64 + kl, b = b0 + bb;
    if (k >= Lk || b >= g.nb) continue;
    const double sx = red[kl * 16 + 2 * bb] + red[(64 + kl) * 16 + 2 * bb];
    const double sy = red[kl * 16 + 2 * bb + 1] + red[(64 + kl) * 16 + 2 * bb + 1];
    finish_degree(g, out, b, m, k, sx, sy);
  }
}

}  // namespace

hipError_t launch_synthesis_mb(const GroupView& g, const SynthInput& in, int B, hipStream_t s) {
  if (!g.Pmb) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_panel_mb, dim3(g.N + 1, g.nbp), dim3(kMbThreads), 0, s, g, in);
  const int ntile = (g.nh + 63) / 64;
  const int per_m = ntile * ((g.nb + B - 1) / B);
  dim3 grid(xcd_grid((g.N + 1) * per_m, per_m));
  switch (B) {
    case 2: hipLaunchKernelGGL(k_synthesis_mb<2>, grid, dim3(kMbThreads), 0, s, g); break;
    case 4: hipLaunchKernelGGL(k_synthesis_mb<4>, grid, dim3(kMbThreads), 0, s, g); break;
    case 8: hipLaunchKernelGGL(k_synthesis_mb<8>, grid, dim3(kMbThreads), 0, s, g); break;
    case 16: hipLaunchKernelGGL(k_synthesis_mb<16>, grid, dim3(kMbThreads), 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_analysis_mb(const GroupView& g, const AnalOutput& out, int B, hipStream_t s) {
  const int ntile = (g.N + 2 + 63) / 64;
  dim3 grid((g.N + 1) * ntile, (g.nb + B - 1) / B);
  switch (B) {
    case 2: hipLaunchKernelGGL(k_analysis_mb<2>, grid, dim3(kMbThreads), 0, s, g, out); break;
    case 4: hipLaunchKernelGGL(k_analysis_mb<4>, grid, dim3(kMbThreads), 0, s, g, out); break;
    case 8: hipLaunchKernelGGL(k_analysis_mb<8>, grid, dim3(kMbThreads), 0, s, g, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nse
