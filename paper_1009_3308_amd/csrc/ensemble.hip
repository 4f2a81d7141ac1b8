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
// (8 per member; the panels of spectral_ops.h, built in LDS 32 degrees at a
// time from the members' predictor coefficients); F(north) = E + O,
// F(south) = E - O. Wave w owns latitudes 16w..16w+15 of the tile: its A
// operand is a 16 x 4 block of the table (four even or four odd degrees), its
// B operand a 4 x 16 block of the panel chunk in LDS.
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

template <int B>
__global__ __launch_bounds__(kMbThreads) void k_analysis_mb(GroupView g, AnalOutput out) {
  if (gate_closed(g)) return;  // an ended attempt of a device-controlled run
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
        const double2* Wb = g.W + ((int64_t)b * (N + 1) + m) * nlat;
        wn[j] = Wb[p];
        ws[j] = Wb[nlat - 1 - p];
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

// Member-batched synthesis with the panels built in LDS: per (order m,
// 64-latitude tile, block of B members) four waves of 16 latitudes. The
// per-degree coefficients of order m (lambda^(+-1/2), cm, cp) are computed
// once per workgroup; the degree range is taken in chunks of 32: the members'
// predictor coefficients of a chunk are staged in LDS, the chunk's panels
// (8 columns per member) are built in LDS, and each wave multiplies its table
// rows by them on MFMA. The predictor coefficients and table operands of the
// next chunk are loaded while the current chunk is multiplied.
constexpr int kChunkS = 32;

template <int B>
__global__ __launch_bounds__(kMbThreads) void k_synthesis_mb(GroupView g, SynthInput in) {
  if (gate_closed(g)) return;  // an ended attempt of a device-controlled run
  constexpr int NC = 8 * B;            // panel columns per parity
  constexpr int NCB = NC / 16;         // 16-column blocks
  constexpr int WP = NC + 2;           // LDS row stride (doubles), padded against bank conflicts
  constexpr int NA = B * (kChunkS + 2);                        // predictor items per chunk
  constexpr int NAT = (NA + kMbThreads - 1) / kMbThreads;      // per thread
  extern __shared__ double lds_s[];
  const int N = g.N, nh = g.nh, nlat = g.nlat;
  const int ntile = (nh + 63) / 64;
  const int nblk = (g.nb + B - 1) / B;
  const int item = xcd_item(blockIdx.x, ntile * nblk);
  const int m = item / (ntile * nblk);
  if (m > N) return;  // uniform across the workgroup
  const int rest = item - m * ntile * nblk;
  const int blk = rest / ntile, tile = rest - blk * ntile;
  const int b0 = blk * B;
  const int L = N + 2 - m;
  double* pan = lds_s;                                        // [kChunkS][WP]
  double2* al = reinterpret_cast<double2*>(pan + kChunkS * WP);  // [B][kChunkS + 2]
  double2* sq = al + NA;                                      // [N + 4]: (sqrt lam, 1/sqrt lam) at m+kk-1
  double2* cc = sq + (N + 4);                                 // [N + 2]: (cm, cp) at k
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int arow = lane & 15, kq = lane >> 4;
  const int lat = tile * 64 + wave * 16 + arow;
  const bool lat_ok = lat < nh;
  const double* T = g.T1 + t1_order_offset(N, m, nh) + (lat_ok ? lat : 0);
  const int64_t base0 = coeff_offset(N, m);
  const double dm = (double)m;

  for (int kk = threadIdx.x; kk < L + 2; kk += kMbThreads) {
    const int ll = m + kk - 1;
    double2 v = make_double2(0.0, 0.0);
    if (kk >= 1 && ll >= 1 && ll <= N) {
      const double q = sqrt((double)ll * (ll + 1));
      v = make_double2(q, 1.0 / q);
    }
    sq[kk] = v;
    if (kk < L) {
      const double dl = (double)(m + kk);
      const double e_l = (kk > 0) ? sqrt((dl * dl - dm * dm) / (4.0 * dl * dl - 1.0)) : 0.0;
      const double e_l1 = sqrt(((dl + 1) * (dl + 1) - dm * dm) / (4.0 * (dl + 1) * (dl + 1) - 1.0));
      cc[kk] = make_double2((dl - 1.0) * e_l, (dl + 2.0) * e_l1);
    }
  }
  if (NC < WP) {  // padding columns are never read; nothing to clear
  }

  // predictor coefficients of the chunk starting at kc (degrees kc-1 .. kc+kChunkS)
  double2 ra[NAT];
  auto load_alpha = [&](int kc) {
#pragma unroll
    for (int j = 0; j < NAT; ++j) {
      const int i = threadIdx.x + j * kMbThreads;
      const int bb = i / (kChunkS + 2), kk = i - bb * (kChunkS + 2);
      const int k = kc - 1 + kk, b = b0 + bb, ll = m + k;
      double2 v = make_double2(0.0, 0.0);
      if (i < NA && b < g.nb && k >= 0 && ll >= 1 && ll <= N) {
        const int64_t slot = g.off[b] + base0 + k;
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
      ra[j] = v;
    }
  };
  // table operands of a chunk: four MFMA steps of degrees kc + 8 j + 2 kq (+1)
  double aE[4], aO[4], nE[4], nO[4];
  auto load_t = [&](int kc, double* xE, double* xO) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kE = kc + 8 * j + 2 * kq, kO = kE + 1;
      xE[j] = (lat_ok && kE < L) ? T[(int64_t)kE * nh] : 0.0;
      xO[j] = (lat_ok && kO < L) ? T[(int64_t)kO * nh] : 0.0;
    }
  };
  load_alpha(0);
  load_t(0, aE, aO);

  doublex4 accE[NCB], accO[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) accE[c] = accO[c] = doublex4{0.0, 0.0, 0.0, 0.0};

  for (int kc = 0; kc < L; kc += kChunkS) {
    __syncthreads();  // previous chunk's products done: al and pan are free
#pragma unroll
    for (int j = 0; j < NAT; ++j) {
      const int i = threadIdx.x + j * kMbThreads;
      if (i < NA) al[i] = ra[j];
    }
    __syncthreads();
    // panels of the chunk: item (kk, bb)
    for (int i = threadIdx.x; i < kChunkS * B; i += kMbThreads) {
      const int kk = i / B, bb = i - kk * B;
      const int k = kc + kk;
      double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (k < L && b0 + bb < g.nb) {
        double2 ps[3], zs[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double2 a = al[bb * (kChunkS + 2) + kk + d], q = sq[k + d];
          ps[d] = make_double2(a.x * q.y, a.y * q.y);
          zs[d] = make_double2(a.x * q.x, a.y * q.x);
          if (m == 0 && k - 1 + d == 1) zs[d].x += in.coriolis;
        }
        const double2 c = cc[k];
        v[0] = -dm * ps[1].y;
        v[1] = dm * ps[1].x;
        v[2] = c.x * ps[0].x - c.y * ps[2].x;
        v[3] = c.x * ps[0].y - c.y * ps[2].y;
        v[4] = c.x * zs[0].x - c.y * zs[2].x;
        v[5] = c.x * zs[0].y - c.y * zs[2].y;
        v[6] = -dm * zs[1].y;
        v[7] = dm * zs[1].x;
      }
#pragma unroll
      for (int f = 0; f < 8; ++f) pan[kk * WP + bb * 8 + f] = v[f];
    }
    const bool more = kc + kChunkS < L;
    if (more) {  // next chunk's loads are in flight during this chunk's products
      load_alpha(kc + kChunkS);
      load_t(kc + kChunkS, nE, nO);
    }
    __syncthreads();
    const int kend = min(kChunkS, L - kc);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (8 * j < kend) {
        const double* pE = pan + (8 * j + 2 * kq) * WP + arow;
        const double* pO = pE + WP;
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
          accE[c] = mfma64(aE[j], pE[16 * c], accE[c]);
          accO[c] = mfma64(aO[j], pO[16 * c], accO[c]);
        }
      }
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        aE[j] = nE[j];
        aO[j] = nO[j];
      }
    }
  }

  // lane holds rows (latitudes) kq + 4r of its wave's 16, column arow of each block
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    const int col = 16 * c + arow;
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

size_t synthesis_mb_lds_bytes(int N, int B) {
  return sizeof(double) * (size_t)kChunkS * (8 * B + 2) +
         sizeof(double2) * ((size_t)B * (kChunkS + 2) + (size_t)(N + 4) + (size_t)(N + 2));
}

}  // namespace

hipError_t launch_synthesis_mb(const GroupView& g, const SynthInput& in, int B, hipStream_t s) {
  const int ntile = (g.nh + 63) / 64;
  const int per_m = ntile * ((g.nb + B - 1) / B);
  dim3 grid(xcd_grid((g.N + 1) * per_m, per_m));
  const size_t lds = synthesis_mb_lds_bytes(g.N, B);
  switch (B) {
    case 2: hipLaunchKernelGGL(k_synthesis_mb<2>, grid, dim3(kMbThreads), lds, s, g, in); break;
    case 4: hipLaunchKernelGGL(k_synthesis_mb<4>, grid, dim3(kMbThreads), lds, s, g, in); break;
    case 8: hipLaunchKernelGGL(k_synthesis_mb<8>, grid, dim3(kMbThreads), lds, s, g, in); break;
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
