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
// Two waves per tile, each owning 32 latitudes (two 16-row blocks): its A
// operands are 16 x 4 blocks of the table (four even or four odd degrees), its
// B operand a 4 x 16 block of the panels, shared by the two row blocks.
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

__device__ __forceinline__ doublex4 mfma64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Panels of every member of the group for one order m, written to
// Pmb[m][k][b][8] (rows k < L = N+2-m in the row order of T1; members past the
// group are written as zeros): one workgroup per (m, chunk of pm members),
// the members' predictor coefficients staged in LDS, the pm members of one
// degree written as one contiguous row piece (pm = 8, or 4 when the staging of
// eight members would not fit 64 KiB).
int panel_members(int N) { return (size_t)10 * (N + 4) * sizeof(double2) <= 65536 ? 8 : 4; }

__global__ __launch_bounds__(kMbThreads) void k_panel_mb(GroupView g, SynthInput in, int pm) {
  extern __shared__ double2 al_dyn[];  // [pm][N + 4]
  const int N = g.N;
  const int m = blockIdx.x, b0 = blockIdx.y * pm;
  const int L = N + 2 - m;
  auto al = [&](int bb, int kk) -> double2& { return al_dyn[bb * (N + 4) + kk]; };
  // per-degree coefficients shared by the members: (sqrt(lambda), 1/sqrt(lambda))
  // at l = m + kk - 1 and (cm, cp) at k = kk
  double2* sq = al_dyn + pm * (N + 4);  // [L + 2]
  double2* cc = sq + (N + 4);           // [L]
  for (int kk = threadIdx.x; kk < L + 2; kk += kMbThreads) {
    const int ll = m + kk - 1;
    double2 v = make_double2(0.0, 0.0);
    if (ll >= m && ll >= 1 && ll <= N) {
      const double q = sqrt((double)ll * (ll + 1));
      v = make_double2(q, 1.0 / q);
    }
    sq[kk] = v;
    if (kk < L) {
      const double dl = (double)(m + kk), dm = (double)m;
      const double e_l = (kk > 0) ? sqrt((dl * dl - dm * dm) / (4.0 * dl * dl - 1.0)) : 0.0;
      const double e_l1 = sqrt(((dl + 1) * (dl + 1) - dm * dm) / (4.0 * (dl + 1) * (dl + 1) - 1.0));
      cc[kk] = make_double2((dl - 1.0) * e_l, (dl + 2.0) * e_l1);
    }
  }
  const int64_t base = coeff_offset(N, m);
  for (int i = threadIdx.x; i < pm * (L + 2); i += kMbThreads) {
    const int bb = i / (L + 2), kk = i - bb * (L + 2);  // al(bb, kk) = alpha[m + kk - 1]
    const int k = kk - 1, ll = m + k, b = b0 + bb;
    double2 v = make_double2(0.0, 0.0);
    if (b < g.nb && k >= 0 && ll >= 1 && ll <= N) {
      const int64_t slot = g.off[b] + base + k;
#pragma unroll
      for (int s = 0; s < kMaxSources; ++s) {
        if (s < in.nsrc) {
          const double2 x = in.src[s][slot];
          v.x += in.coef[s] * x.x;
          v.y += in.coef[s] * x.y;
        }
      }
      if (m == 0) v.y = 0.0;
    }
    al(bb, kk) = v;
  }
  __syncthreads();
  double* P = g.Pmb + (t1_order_offset(N, m, 1) * g.nbp + b0) * 8;
  for (int i = threadIdx.x; i < pm * L; i += kMbThreads) {
    const int k = i / pm, bb = i - k * pm;
    double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (b0 + bb < g.nb) {
      double2 ps[3], zs[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double2 a = al(bb, k + d), q = sq[k + d];
        ps[d] = make_double2(a.x * q.y, a.y * q.y);
        zs[d] = make_double2(a.x * q.x, a.y * q.x);
        if (m == 0 && m + k - 1 + d == 1) zs[d].x += in.coriolis;
      }
      const double2 c = cc[k];
      const double dm = (double)m;
      v[0] = -dm * ps[1].y;
      v[1] = dm * ps[1].x;
      v[2] = c.x * ps[0].x - c.y * ps[2].x;
      v[3] = c.x * ps[0].y - c.y * ps[2].y;
      v[4] = c.x * zs[0].x - c.y * zs[2].x;
      v[5] = c.x * zs[0].y - c.y * zs[2].y;
      v[6] = -dm * zs[1].y;
      v[7] = dm * zs[1].x;
    }
    double2* row = reinterpret_cast<double2*>(P + ((int64_t)k * g.nbp + bb) * 8);
#pragma unroll
    for (int f = 0; f < 4; ++f) row[f] = make_double2(v[2 * f], v[2 * f + 1]);
  }
}

// Work items (order m, member block, latitude tile) are taken in XCD-local
// chunks of one order, so the blocks and tiles of an order share an L2.
// Two waves per 64-latitude tile, each owning two 16-latitude row blocks, so
// that every panel operand loaded feeds two MFMAs.
constexpr int kSynMbThreads = 128;

template <int B>
__global__ __launch_bounds__(kSynMbThreads) void k_synthesis_mb(GroupView g) {
  static_assert(B >= 2, "16 or more panel columns");
  constexpr int NC = 8 * B;                // columns per parity
  constexpr int NCB = NC / 16;             // 16-column blocks
  constexpr int NJ = B >= 8 ? 1 : 2;       // MFMA steps (8 degrees each) per pipeline stage
  constexpr int RB = 2;                    // 16-latitude row blocks per wave
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
  const int lat0 = tile * 64 + wave * 32 + arow;  // this lane's A-operand latitude, row block 0
  if (tile * 64 + wave * 32 >= nh) return;        // uniform across the wave; no barriers below
  bool lat_ok[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) lat_ok[rb] = lat0 + 16 * rb < nh;
  const double* T = g.T1 + t1_order_offset(N, m, nh) + lat0;
  const int64_t pstride = (int64_t)g.nbp * 8;
  const double* P = g.Pmb + t1_order_offset(N, m, 1) * pstride + blk * B * 8 + arow;

  doublex4 accE[RB][NCB], accO[RB][NCB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int c = 0; c < NCB; ++c) accE[rb][c] = accO[rb][c] = doublex4{0.0, 0.0, 0.0, 0.0};
  // operands of one stage: degrees kc + 8 j + 2 kq (even) and +1 (odd)
  double aE[NJ][RB], aO[NJ][RB], bE[NJ][NCB], bO[NJ][NCB];
  double nE[NJ][RB], nO[NJ][RB], cE[NJ][NCB], cO[NJ][NCB];
  auto load = [&](int kc, double (*xE)[RB], double (*xO)[RB], double (*yE)[NCB],
                  double (*yO)[NCB]) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int kE = kc + 8 * j + 2 * kq, kO = kE + 1;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        xE[j][rb] = (lat_ok[rb] && kE < L) ? T[(int64_t)kE * nh + 16 * rb] : 0.0;
        xO[j][rb] = (lat_ok[rb] && kO < L) ? T[(int64_t)kO * nh + 16 * rb] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < NCB; ++c) {
        yE[j][c] = (kE < L) ? P[(int64_t)kE * pstride + 16 * c] : 0.0;
        yO[j][c] = (kO < L) ? P[(int64_t)kO * pstride + 16 * c] : 0.0;
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
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          accE[rb][c] = mfma64(aE[j][rb], bE[j][c], accE[rb][c]);
          accO[rb][c] = mfma64(aO[j][rb], bO[j][c], accO[rb][c]);
        }
      }
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          aE[j][rb] = nE[j][rb];
          aO[j][rb] = nO[j][rb];
        }
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
          bE[j][c] = cE[j][c];
          bO[j][c] = cO[j][c];
        }
      }
    }
  }

  // lane holds rows (latitudes) kq + 4r of each row block, column arow of each column block
  const int b0 = blk * B;
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    const int col = 16 * c + arow;
    const int bb = col >> 3, f = (col & 7) >> 1, ri = col & 1;
    const int b = b0 + bb;
    if (b >= g.nb) continue;
    double* out = reinterpret_cast<double*>(g.F + ((int64_t)(b * 4 + f) * (N + 1) + m) * nlat);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = tile * 64 + wave * 32 + 16 * rb + kq + 4 * r;
        if (p >= nh) continue;
        const double e = accE[rb][c][r], o = accO[rb][c][r];
        out[2 * p + ri] = e + o;
        const int ps = nlat - 1 - p;
        if (ps != p) out[2 * ps + ri] = e - o;
      }
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
  const int nblk = (g.nb + B - 1) / B;
  // items (m, member block, tile) in XCD-local chunks of eight orders: the eight
  // orders of one 128-byte line of W[b][lat][m] share that XCD's L2
  const int per_m = nblk * ntile;
  const int item = xcd_item_snake(blockIdx.x, 8 * per_m);
  const int m = item / per_m;
  if (m > N) return;
  const int rest = item - m * per_m;
  const int blk = rest / ntile, tile = rest - blk * ntile;
  const int Lk = N + 1 - m;  // degrees m .. N
  if (tile * 64 >= Lk) return;  // uniform across the workgroup
  const int b0 = blk * B;
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
  const int pm = panel_members(g.N);
  hipLaunchKernelGGL(k_panel_mb, dim3(g.N + 1, g.nbp / pm), dim3(kMbThreads),
                     sizeof(double2) * (pm + 2) * (g.N + 4), s, g, in, pm);
  const int ntile = (g.nh + 63) / 64;
  const int per_m = ntile * ((g.nb + B - 1) / B);
  dim3 grid(xcd_grid((g.N + 1) * per_m, per_m));
  switch (B) {
    case 2: hipLaunchKernelGGL(k_synthesis_mb<2>, grid, dim3(kSynMbThreads), 0, s, g); break;
    case 4: hipLaunchKernelGGL(k_synthesis_mb<4>, grid, dim3(kSynMbThreads), 0, s, g); break;
    case 8: hipLaunchKernelGGL(k_synthesis_mb<8>, grid, dim3(kSynMbThreads), 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_analysis_mb(const GroupView& g, const AnalOutput& out, int B, hipStream_t s) {
  const int ntile = (g.N + 2 + 63) / 64;
  const int per_m = ntile * ((g.nb + B - 1) / B);
  dim3 grid(xcd_grid((g.N + 1) * per_m, 8 * per_m));
  switch (B) {
    case 2: hipLaunchKernelGGL(k_analysis_mb<2>, grid, dim3(kMbThreads), 0, s, g, out); break;
    case 4: hipLaunchKernelGGL(k_analysis_mb<4>, grid, dim3(kMbThreads), 0, s, g, out); break;
    case 8: hipLaunchKernelGGL(k_analysis_mb<8>, grid, dim3(kMbThreads), 0, s, g, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nse
