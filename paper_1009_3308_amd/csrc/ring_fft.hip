// Longitude transforms and the grid product (Section 4.2: FFT in the
// azimuthal direction at the M equispaced longitudes of eq. (quadrule)).
//
// One workgroup per latitude ring. Two real fields share one complex FFT: for
// fields a, b with Fourier coefficients G^a_m, G^b_m, m = 0..N, the length-M
// sequence
//   x_m = G^a_m + i G^b_m,  x_{M-m} = conj(G^a_m) + i conj(G^b_m)
// has the inverse DFT g^a_j + i g^b_j. The pairs are (f0, f1), the two
// components of the stream-function gradient, and (f2, f3), the two of the
// absolute-vorticity gradient, so that the advection term is the real part of
// one product:
//   q = (f0 f2 - f1 f3) / sin^2(theta) = Re[(f0 + i f1)(f2 + i f3)] / sin^2(theta)
//     = u . Grad(zeta + 2 Omega cos theta).
// A transform's rounding error is relative to the larger of its two fields;
// the vorticity gradient is larger than the stream-function gradient by about
// the degree squared for a spectrum with weight at high degree, so each
// transform holds two fields of one kind.
// One forward FFT of q gives its spectrum Q_m; the quadrature factor
// (2 pi / M) w_p of eq. (quadrule) is applied and Q_m, m = 0..N, is written for
// the ring (W[m][lat], latitude fastest); the analysis folds the two rings of
// each latitude pair.
//
// The FFT is a mixed-radix (8, 4, 2, 5, 3) Stockham transform done in place in
// LDS: each stage reads R values at stride M/R into registers, applies
// twiddles from a half table exp(-2 pi i e / M), e < M/2 (an LDS copy, or the
// global table through L1 where the LDS is better spent on more rings per CU),
// performs a radix-R butterfly and writes back in autosort order after a
// barrier. The two inverse transforms run in the same stages. With the odd
// radices last, the stage strides are powers of two and the index arithmetic
// is shifts.
#include <type_traits>

#include "nse_internal.h"

namespace nse {

namespace {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// s * i * a for s = +-1
__device__ __forceinline__ double2 cmul_si(double2 a, double s) { return make_double2(-s * a.y, s * a.x); }

// cos/sin of 2 pi / 3, 2 pi / 5 and 4 pi / 5 in closed form:
// sqrt(3)/2, (sqrt(5)-1)/4, -(sqrt(5)+1)/4, sqrt(10+2 sqrt(5))/4, sqrt(10-2 sqrt(5))/4.
constexpr double kS3 = 0.86602540378443864676;
constexpr double kC1 = 0.30901699437494742410;
constexpr double kC2 = -0.80901699437494742410;
constexpr double kS1 = 0.95105651629515357212;
constexpr double kS2 = 0.58778525229247312917;

// DFT of length R with kernel exp(s 2 pi i j k / R), in place.
template <int R>
__device__ __forceinline__ void butterfly(double2* v, double s) {
  if constexpr (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const double2 t = cadd(v[1], v[2]);
    const double2 d = cmul_si(csub(v[1], v[2]), s * kS3);
    const double2 c = make_double2(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
    v[0] = cadd(v[0], t);
    v[1] = cadd(c, d);
    v[2] = csub(c, d);
  } else if constexpr (R == 4) {
    const double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const double2 b0 = cadd(v[1], v[3]), b1 = cmul_si(csub(v[1], v[3]), s);
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
  } else if constexpr (R == 5) {
    const double2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const double2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    const double2 x0 = v[0];
    const double2 c1 = make_double2(x0.x + kC1 * t1.x + kC2 * t2.x, x0.y + kC1 * t1.y + kC2 * t2.y);
    const double2 c2 = make_double2(x0.x + kC2 * t1.x + kC1 * t2.x, x0.y + kC2 * t1.y + kC1 * t2.y);
    const double2 s1 = cmul_si(make_double2(kS1 * d1.x + kS2 * d2.x, kS1 * d1.y + kS2 * d2.y), s);
    const double2 s2 = cmul_si(make_double2(kS2 * d1.x - kS1 * d2.x, kS2 * d1.y - kS1 * d2.y), s);
    v[0] = cadd(x0, cadd(t1, t2));
    v[1] = cadd(c1, s1);
    v[4] = csub(c1, s1);
    v[2] = cadd(c2, s2);
    v[3] = csub(c2, s2);
  } else if constexpr (R == 8) {
    // radix 8 from two radix-4 transforms of the even and odd samples
    double2 e[4] = {v[0], v[2], v[4], v[6]};
    double2 o[4] = {v[1], v[3], v[5], v[7]};
    butterfly<4>(e, s);
    butterfly<4>(o, s);
    constexpr double h = 0.70710678118654752440;  // 1 / sqrt(2)
    const double2 o1 = make_double2(h * (o[1].x - s * o[1].y), h * (o[1].y + s * o[1].x));
    const double2 o2 = cmul_si(o[2], s);
    const double2 o3 = make_double2(h * (-o[3].x - s * o[3].y), h * (-o[3].y + s * o[3].x));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
}

// LDS rows are padded by one slot every 16 complex values so that the strided
// accesses of the Stockham stages spread over the LDS banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }
__host__ __device__ inline int padded_len(int M) { return M + (M >> 4) + 1; }

// exp(-2 pi i e / M) from the half table tw[0 .. M/2) in LDS.
__device__ __forceinline__ double2 twiddle(const double2* tw, int e, int half) {
  if (e < half) return tw[e];
  const double2 t = tw[e - half];
  return make_double2(-t.x, -t.y);
}

// q = j / Ns, k = j mod Ns (shifts when Ns is a power of two).
__device__ __forceinline__ void split(int j, int Ns, int lg, int& q, int& k) {
  if (lg >= 0) {
    q = j >> lg;
    k = j & (Ns - 1);
  } else {
    q = j / Ns;
    k = j - q * Ns;
  }
}

// In-place Stockham stage of radix R on NA arrays in LDS (NA = 1 or 2): every
// thread first reads, twiddles and transforms all butterflies it owns into
// registers, then (after a barrier) writes them in autosort order.
// sign = -1 forward (exp(-2 pi i jk/M)), +1 inverse.
template <int R, int NA, int MAXM, int NT>
__device__ __forceinline__ void stage(double2* x0, double2* x1, int M, int Ns, int lg,
                                      const double2* tw, double sign) {
  constexpr int MAXB = ((MAXM / R) * NA + NT - 1) / NT;
  const int span = M / R;
  const int step = M / (Ns * R);
  const int total = span * NA;
  const int half = M >> 1;
  double2 v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int t = threadIdx.x + c * NT;
    dst[c] = -1;
    if (t < total) {
      const int a = (NA == 1) ? 0 : (t >= span ? 1 : 0);
      const int j = t - a * span;
      const double2* x = a ? x1 : x0;
#pragma unroll
      for (int r = 0; r < R; ++r) v[c][r] = x[pad(j + r * span)];
      int q, k;
      split(j, Ns, lg, q, k);
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double2 w = twiddle(tw, r * k * step, half);
          w.y *= -sign;  // the table holds exp(-2 pi i e / M); forward uses it as is
          v[c][r] = cmul(v[c][r], w);
        }
      }
      butterfly<R>(v[c], sign);
      dst[c] = (a << 24) | (q * Ns * R + k);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    if (dst[c] >= 0) {
      double2* x = (dst[c] >> 24) ? x1 : x0;
      const int idx = dst[c] & 0xffffff;
#pragma unroll
      for (int r = 0; r < R; ++r) x[pad(idx + r * Ns)] = v[c][r];
    }
  }
  __syncthreads();
}

// Full in-place transform of one or two LDS arrays.
template <int NA, int MAXM, int NT>
__device__ void fft(double2* x0, double2* x1, const FftPlan& plan, int M, const double2* tw,
                    double sign) {
  int Ns = 1;
  for (int st = 0; st < plan.nstages; ++st) {
    const int R = plan.radix[st];
    const int lg = plan.ns_log2[st];
    switch (R) {
      case 2: stage<2, NA, MAXM, NT>(x0, x1, M, Ns, lg, tw, sign); break;
      case 3: stage<3, NA, MAXM, NT>(x0, x1, M, Ns, lg, tw, sign); break;
      case 4: stage<4, NA, MAXM, NT>(x0, x1, M, Ns, lg, tw, sign); break;
      case 5: stage<5, NA, MAXM, NT>(x0, x1, M, Ns, lg, tw, sign); break;
      default: stage<8, NA, MAXM, NT>(x0, x1, M, Ns, lg, tw, sign); break;
    }
    Ns *= R;
  }
}

// Compile-time plans for M = 3 * 2^k, the default grid of every truncation
// (M = 3(N+1) for N = 2^j - 1): radix-8 stages (radix 4 where the power of
// two needs it), radix 3 last, so every stride before the last stage is a
// power of two. With M, the radices, the strides and the direction known at
// compile time, the index arithmetic of a stage folds into constants.
template <int M> struct CtPlan { static constexpr int n = 0; static constexpr int r[1] = {0}; };
template <> struct CtPlan<48> { static constexpr int n = 3; static constexpr int r[3] = {4, 4, 3}; };
template <> struct CtPlan<96> { static constexpr int n = 3; static constexpr int r[3] = {8, 4, 3}; };
template <> struct CtPlan<192> { static constexpr int n = 3; static constexpr int r[3] = {8, 8, 3}; };
template <> struct CtPlan<384> { static constexpr int n = 4; static constexpr int r[4] = {8, 4, 4, 3}; };
template <> struct CtPlan<768> { static constexpr int n = 4; static constexpr int r[4] = {8, 8, 4, 3}; };
template <> struct CtPlan<1536> { static constexpr int n = 4; static constexpr int r[4] = {8, 8, 8, 3}; };
// M = 320 (N = 100 on 160 x 320, the grid of the paper's Example 2): radix 5
// last, so the product and the forward store run as separate passes
template <> struct CtPlan<320> { static constexpr int n = 3; static constexpr int r[3] = {8, 8, 5}; };
// plans whose last stage is radix 3 at stride M/3 (fused product and store)
template <int M> constexpr bool ct_fused() { return CtPlan<M>::n > 0 && CtPlan<M>::r[CtPlan<M>::n - 1] == 3; }

constexpr int ct_log2(int x) { return x <= 1 ? 0 : 1 + ct_log2(x / 2); }

// exp(SGN 2 pi i e / M) for 0 <= e < M from the half table tw[0 .. M/2) of
// exp(-2 pi i e / M).
template <int M, int SGN>
__device__ __forceinline__ double2 tw_at(const double2* tw, int e) {
  constexpr int half = M / 2;
  double2 w = tw[e < half ? e : e - half];
  if (e >= half) w = make_double2(-w.x, -w.y);
  if (SGN > 0) w.y = -w.y;
  return w;
}

// The twiddles w[r] = exp(SGN 2 pi i r e / M), r = 1 .. R-1, of one butterfly
// (R e < R M / R = M): radix 4 and 8 read w, w^2 (and w^4) from the table and
// form the other powers by products (at most two roundings more than a table
// entry), which takes three of the seven table reads of a radix-8 butterfly.
template <int R, int M, int SGN>
__device__ __forceinline__ void stage_twiddles(double2* w, const double2* tw, int e) {
  if constexpr (R == 4 || R == 8) {
    w[1] = tw_at<M, SGN>(tw, e);
    w[2] = tw_at<M, SGN>(tw, 2 * e);
    w[3] = cmul(w[1], w[2]);
    if constexpr (R == 8) {
      w[4] = tw_at<M, SGN>(tw, 4 * e);
      w[5] = cmul(w[1], w[4]);
      w[6] = cmul(w[2], w[4]);
      w[7] = cmul(w[3], w[4]);
    }
  } else {
#pragma unroll
    for (int r = 1; r < R; ++r) w[r] = tw_at<M, SGN>(tw, r * e);
  }
}

// One Stockham stage of radix R at stride NS (a power of two) on NA arrays of
// length M (x1 = x0 + padded_len(M) when NA = 2); SGN = -1 forward, +1 inverse.
template <int R, int NS, int M, int NA, int NT, int SGN>
__device__ __forceinline__ void stage_ct(double2* x0, const double2* tw) {
  constexpr int span = M / R, total = span * NA, MAXB = (total + NT - 1) / NT;
  constexpr int step = M / (NS * R), lg = ct_log2(NS);
  constexpr int PL = M + (M >> 4) + 1;
  double2 v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int t = threadIdx.x + c * NT;
    dst[c] = -1;
    if (total % NT == 0 || t < total) {
      const int a = (NA == 1) ? 0 : (t >= span ? 1 : 0);
      const int j = t - a * span;
      const double2* x = x0 + a * PL;
#pragma unroll
      for (int r = 0; r < R; ++r) v[c][r] = x[pad(j + r * span)];
      const int k = j & (NS - 1), q = j >> lg;
      if constexpr (NS > 1) {
        double2 w[R];
        stage_twiddles<R, M, SGN>(w, tw, k * step);
#pragma unroll
        for (int r = 1; r < R; ++r) v[c][r] = cmul(v[c][r], w[r]);
      }
      butterfly<R>(v[c], (double)SGN);
      dst[c] = a * PL + q * NS * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    if (dst[c] >= 0) {
      const int base = dst[c] >= PL ? PL : 0;
      const int idx = dst[c] - base;
#pragma unroll
      for (int r = 0; r < R; ++r) x0[base + pad(idx + r * NS)] = v[c][r];
    }
  }
  __syncthreads();
}

template <int M, int S, int NS, int NA, int NT, int SGN>
__device__ __forceinline__ void stages_ct(double2* x0, const double2* tw) {
  if constexpr (S < CtPlan<M>::n) {
    constexpr int R = CtPlan<M>::r[S];
    stage_ct<R, NS, M, NA, NT, SGN>(x0, tw);
    stages_ct<M, S + 1, NS * R, NA, NT, SGN>(x0, tw);
  }
}

// Inverse transforms of the two LDS arrays x0 = f0 + i f1 and x1 = f2 + i f3 (x1 =
// x0 + padded_len(M)) for a compile-time plan whose last stage is radix 3 at
// stride M/3, fused with the grid product: every stage before the last as in
// stages_ct; in the last, thread j computes butterfly j of both arrays, whose
// outputs are the grid values at j, j + M/3 and j + 2M/3 (the positions it
// read), forms q = Re(x0 x1) / sin^2 there and writes q in place to x0, so the
// write-back of the last stage, the separate product pass and two barriers go.
template <int M, int S, int NS, int NT>
__device__ __forceinline__ void fft_ct_inverse_product(double2* x0, const double2* tw,
                                                       double inv_sin2) {
  constexpr int n = CtPlan<M>::n;
  if constexpr (S < n - 1) {
    constexpr int R = CtPlan<M>::r[S];
    stage_ct<R, NS, M, 2, NT, 1>(x0, tw);
    fft_ct_inverse_product<M, S + 1, NS * R, NT>(x0, tw, inv_sin2);
  } else {
    static_assert(CtPlan<M>::r[n - 1] == 3 && NS * 3 == M, "last stage: radix 3 at stride M/3");
    constexpr int PL = M + (M >> 4) + 1, MAXB = (NS + NT - 1) / NT;
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int j = threadIdx.x + b * NT;  // butterfly j (q = 0, k = j at stride NS = M/3)
      if (NS % NT == 0 || j < NS) {
        double2 v[2][3];
        const double2 w1 = tw_at<M, 1>(tw, j);  // inverse twiddles of butterfly j
        const double2 w2 = cmul(w1, w1);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
          for (int r = 0; r < 3; ++r) v[a][r] = x0[a * PL + pad(j + r * NS)];
          v[a][1] = cmul(v[a][1], w1);
          v[a][2] = cmul(v[a][2], w2);
          butterfly<3>(v[a], 1.0);
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
          x0[pad(j + r * NS)] =
              make_double2((v[0][r].x * v[1][r].x - v[0][r].y * v[1][r].y) * inv_sin2, 0.0);
      }
    }
    __syncthreads();
  }
}

// Forward transform of one LDS array for a compile-time plan whose last stage
// is radix 3 at stride M/3: every stage before it as in stages_ct, then the
// last stage computes only its butterflies' first outputs, X_m for m < M/3
// (they hold every m <= N since 3N + 2 <= M), and stores c X_m for m <= N
// straight to out[m * ostride], without the LDS write-back and its barriers.
template <int M, int S, int NS, int NT>
__device__ __forceinline__ void fft_ct_forward_store(double2* x0, const double2* tw, double c,
                                                     double2* __restrict__ out, int64_t ostride,
                                                     int N) {
  constexpr int n = CtPlan<M>::n;
  if constexpr (S < n - 1) {
    constexpr int R = CtPlan<M>::r[S];
    stage_ct<R, NS, M, 1, NT, -1>(x0, tw);
    fft_ct_forward_store<M, S + 1, NS * R, NT>(x0, tw, c, out, ostride, N);
  } else {
    static_assert(CtPlan<M>::r[n - 1] == 3 && NS * 3 == M, "last stage: radix 3 at stride M/3");
    constexpr int MAXB = (NS + NT - 1) / NT;
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int j = threadIdx.x + b * NT;  // butterfly j = k (q = 0 at stride NS = M/3)
      if (j <= N) {
        double2 v0 = x0[pad(j)], v1 = x0[pad(j + NS)], v2 = x0[pad(j + 2 * NS)];
        if (j != 0) {
          const double2 w1 = tw_at<M, -1>(tw, j);  // j < M / 3
          v1 = cmul(v1, w1);
          v2 = cmul(v2, cmul(w1, w1));
        }
        // first output of the radix-3 butterfly: v0 + (v1 + v2)
        const double2 t = cadd(v1, v2);
        out[(int64_t)j * ostride] = make_double2(c * (v0.x + t.x), c * (v0.y + t.y));
      }
    }
  }
}

// Transform of one or two LDS arrays (x1 must be x0 + padded_len(M) when
// NA = 2): the compile-time plan when CM > 0, else the runtime plan.
template <int NA, int MAXM, int NT, int CM>
__device__ __forceinline__ void fft_any(double2* x0, double2* x1, const FftPlan& plan, int M,
                                        const double2* tw, double sign) {
  if constexpr (CM > 0) {
    if (sign > 0)
      stages_ct<CM, 0, 1, NA, NT, 1>(x0, tw);
    else
      stages_ct<CM, 0, 1, NA, NT, -1>(x0, tw);
  } else {
    fft<NA, MAXM, NT>(x0, x1, plan, M, tw, sign);
  }
}

// The ring's inputs for the forward kernel: the twiddle half table into tw and
// the spectra of two field pairs into x0 = (Fa0, Fb0) and x1 = (Fa1, Fb1): for a
// pair (a, b), x_m = G^a_m + i G^b_m, x_{M-m} = conj(G^a_m) + i conj(G^b_m) and
// zero elsewhere, G[m] read from F[f][m][lat] (stride nlat between orders).
// Every global load is issued before the first LDS write
// (one memory round trip for the ring instead of one per array); thread t
// loads order m = t mod (N+1) of pair t / (N+1). Since 3N + 2 <= M <= MAXM,
// 2 (N+1) <= 2 (MAXM / 3 + 1) <= KI NT.
template <int MAXM, int NT, bool COPYTW = true>
__device__ void load_ring(double2* x0, double2* x1, double2* tw, const double2* __restrict__ gtw,
                          const double2* __restrict__ Fa0, const double2* __restrict__ Fb0,
                          const double2* __restrict__ Fa1, const double2* __restrict__ Fb1,
                          int lat, int N, int M, int nlat) {
  constexpr int KI = (2 * (MAXM / 3 + 1) + NT - 1) / NT;
  constexpr int KT = (MAXM / 2 + NT - 1) / NT;
  const int n1 = N + 1;
  double2 ga[KI], gb[KI], t[KT];
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int idx = threadIdx.x + i * NT;
    ga[i] = gb[i] = make_double2(0.0, 0.0);
    if (idx < 2 * n1) {
      const bool second = idx >= n1;
      const int64_t off = (int64_t)(idx - (second ? n1 : 0)) * nlat + lat;
      ga[i] = (second ? Fa1 : Fa0)[off];
      gb[i] = (second ? Fb1 : Fb0)[off];
    }
  }
#pragma unroll
  for (int i = 0; i < KT; ++i) {
    const int j = threadIdx.x + i * NT;
    if (COPYTW && j < M / 2) t[i] = gtw[j];
  }
#pragma unroll
  for (int i = 0; i < KT; ++i) {
    const int j = threadIdx.x + i * NT;
    if (COPYTW && j < M / 2) tw[j] = t[i];
  }
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int idx = threadIdx.x + i * NT;
    if (idx < 2 * n1) {
      const bool second = idx >= n1;
      const int m = idx - (second ? n1 : 0);
      double2* x = second ? x1 : x0;
      if (m == 0) {
        x[0] = make_double2(ga[i].x, gb[i].x);
      } else {
        x[pad(m)] = make_double2(ga[i].x - gb[i].y, ga[i].y + gb[i].x);       // ga + i gb
        x[pad(M - m)] = make_double2(ga[i].x + gb[i].y, -ga[i].y + gb[i].x);  // conj(ga) + i conj(gb)
      }
    }
  }
  for (int j = N + 1 + threadIdx.x; j < M - N; j += NT) {
    x0[pad(j)] = make_double2(0.0, 0.0);
    x1[pad(j)] = make_double2(0.0, 0.0);
  }
}

// ---------------------------------------------------------------------------
// Nonlinear-mode ring kernel for M = 3 S, S = 128, 256 (the default grids of
// N = 127 and 255). With k = k1 + 3 k2 and n = S n1 + n2 (k1, n1 < 3;
// k2, n2 < S) the length-M transforms split into three S-point transforms and
// one radix-3 pass:
//   inverse: Y_k1 = IDFT_S(X[k1 + 3 .]),  x[S n1 + n2] = sum_k1 e^{2 pi i k1 n1/3} e^{2 pi i k1 n2/M} Y_k1[n2];
//   forward: Z_k1[n2] = e^{-2 pi i k1 n2/M} sum_n1 q[S n1 + n2] e^{-2 pi i k1 n1/3},  Q[k1 + 3 k2] = DFT_S(Z_k1)[k2].
// Each S-point transform belongs to one wave, which runs its Stockham stages
// on its own LDS row: a wave's LDS accesses complete in program order, so the
// stages need no workgroup barrier. The radix-3 passes of both directions and
// the grid product meet in one pass (thread n2 holds the three grid points
// S n1 + n2 of both paired fields), so the ring needs three workgroup barriers
// (after the loads, after the six inverse transforms, after the fused pass)
// where the radix-8/4/3 plan over the whole ring took about ten.
template <int S> struct WavePlan { static constexpr int n = 0; static constexpr int r[1] = {0}; };
template <> struct WavePlan<128> { static constexpr int n = 4; static constexpr int r[4] = {2, 4, 4, 4}; };
template <> struct WavePlan<256> { static constexpr int n = 4; static constexpr int r[4] = {4, 4, 4, 4}; };

__host__ __device__ constexpr int wave_row(int S) { return S + (S >> 4) + 1; }

// exp(-2 pi i e / M), e < M, from the half table tw[0 .. M/2).
template <int M>
__device__ __forceinline__ double2 tw_full(const double2* tw, int e) {
  constexpr int half = M / 2;
  if (e < half) return tw[e];
  const double2 t = tw[e - half];
  return make_double2(-t.x, -t.y);
}

// One Stockham stage of radix R at stride NS over the S points of a wave's LDS
// row x (in place: every lane reads its butterflies, then writes them); the
// twiddles of length S are those of length M = 3 S at three times the index.
// With STORE (the last forward stage, NS R = S) the outputs k2 = j + r NS go
// to out[(k1 + 3 k2) * ostride] (scaled by c) for k1 + 3 k2 <= N instead.
template <int R, int NS, int S, int SGN, bool STORE>
__device__ __forceinline__ void wave_stage(double2* x, const double2* tw, int lane, double c,
                                           double2* __restrict__ out, int64_t ostride, int k1,
                                           int N) {
  constexpr int M = 3 * S, span = S / R, MAXB = (span + 63) / 64;
  constexpr int step = S / (NS * R), lg = ct_log2(NS);
  double2 v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = lane + 64 * b;
    dst[b] = -1;
    if (span % 64 == 0 || j < span) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = x[pad(j + r * span)];
      const int k = j & (NS - 1), q = j >> lg;
      if constexpr (NS > 1) {
        // length-S twiddles: those of length M = 3 S at three times the index
        double2 w[R];
        stage_twiddles<R, M, SGN>(w, tw, 3 * k * step);
#pragma unroll
        for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], w[r]);
      }
      butterfly<R>(v[b], (double)SGN);
      dst[b] = q * NS * R + k;
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    if (dst[b] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (STORE) {
          const int m = k1 + 3 * (dst[b] + r * NS);
          if (m <= N) out[(int64_t)m * ostride] = make_double2(c * v[b][r].x, c * v[b][r].y);
        } else {
          x[pad(dst[b] + r * NS)] = v[b][r];
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
}

template <int S, int ST, int NS, int SGN, bool STORE_LAST>
__device__ __forceinline__ void wave_fft(double2* x, const double2* tw, int lane, double c,
                                         double2* __restrict__ out, int64_t ostride, int k1,
                                         int N) {
  if constexpr (ST < WavePlan<S>::n) {
    constexpr int R = WavePlan<S>::r[ST];
    constexpr bool last = ST + 1 == WavePlan<S>::n;
    wave_stage<R, NS, S, SGN, STORE_LAST && last>(x, tw, lane, c, out, ostride, k1, N);
    wave_fft<S, ST + 1, NS * R, SGN, STORE_LAST>(x, tw, lane, c, out, ostride, k1, N);
  }
}

// Workgroup of NR neighbouring rings, NT / NR >= max(S, 384) threads per ring:
// waves 6 r .. 6 r + 5 hold the inverse transforms Y_{a,k1} of ring r (a = 0:
// f0 + i f1, a = 1: f2 + i f3) on LDS rows 6 r + 3 a + k1, threads
// r NT / NR + n2 (n2 < S) the fused pass of ring r, waves 3 r .. 3 r + 2 its
// forward transforms. With NR = 2 the loads of the two rings' spectra pair up
// on the same cache lines (lanes 2 j and 2 j + 1 read the two latitudes of one
// order): T255 ring 8.2 -> 7.6 us, the launch's 192 workgroups leaving 64 CUs
// idle while the others hold the two rings that the busiest CUs held before.
// TWL: the twiddle half table copied to LDS (after the rows) instead of read
// from the global table through L1: the better choice when many members'
// rings share the CUs (throughput), the global table when one member's rings
// are latency-bound.
template <int S, int NT, bool TWL, int NR>
__global__ __launch_bounds__(NT) void k_ring_nl(GroupView g) {
  constexpr int M = 3 * S, PS = wave_row(S), RT = NT / NR;
  static_assert(RT >= S && RT >= 384, "threads per ring");
  const int N = g.N, nlat = g.nlat;
  const int lat0 = NR * xcd_item(blockIdx.x, 8 / NR);  // XCD chunks of 8 latitudes
  if (lat0 >= nlat) return;
  const int b = blockIdx.y;
  extern __shared__ double2 lds[];
  double2* twl = lds + 6 * NR * PS;
  const double2* tw = TWL ? twl : g.tw;
  if constexpr (TWL) {
    for (int j = threadIdx.x; j < M / 2; j += NT) twl[j] = g.tw[j];  // ordered by the first barrier
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t fstride = (int64_t)(N + 1) * nlat;
  const double2* F0 = g.F + (int64_t)b * 4 * fstride + lat0;

  // loads: every spectrum value once (thread t: ring rr = t mod NR, order
  // m = t' mod (N+1) of pair a = t' / (N+1), t' = t / NR, both fields of the
  // pair), all requested before the first LDS write; X_a[m] = G^f_m + i G^f'_m
  // goes to row 3a + m mod 3 of its ring at m / 3 and X_a[M - m] =
  // conj(G^f_m) + i conj(G^f'_m) to row 3a + (M - m) mod 3 at (M - m) / 3
  constexpr int KI = (2 * (S + 1) + RT - 1) / RT;  // N + 1 <= M / 3 + 1 = S + 1
  const int n1 = N + 1;
  const int rr = threadIdx.x % NR, tt = threadIdx.x / NR;
  const bool rvalid = lat0 + rr < nlat;  // an odd last ring pair holds one ring
  double2 ga[KI], gb[KI];
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int idx = tt + i * RT;
    ga[i] = gb[i] = make_double2(0.0, 0.0);
    if (idx < 2 * n1 && rvalid) {
      const int a = idx >= n1 ? 1 : 0, m = idx - a * n1;
      const double2* Fa = F0 + (int64_t)(2 * a) * fstride + (int64_t)m * nlat + rr;
      ga[i] = Fa[0];
      gb[i] = Fa[fstride];
    }
  }
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int idx = tt + i * RT;
    if (idx < 2 * n1) {
      const int a = idx >= n1 ? 1 : 0, m = idx - a * n1;
      double2* rows = lds + (6 * rr + 3 * a) * PS;
      if (m == 0) {
        rows[0] = make_double2(ga[i].x, gb[i].x);
      } else {
        rows[(m % 3) * PS + pad(m / 3)] = make_double2(ga[i].x - gb[i].y, ga[i].y + gb[i].x);
        const int k = M - m;
        rows[(k % 3) * PS + pad(k / 3)] = make_double2(ga[i].x + gb[i].y, gb[i].x - ga[i].y);
      }
    }
  }
  // the zero band N < k < M - N of both arrays of every ring
  const int zb = M - 2 * N - 1;
  for (int t = threadIdx.x; t < NR * 2 * zb; t += NT) {
    const int r = t / (2 * zb), u = t - r * 2 * zb;
    const int a = u >= zb ? 1 : 0;
    const int k = N + 1 + u - a * zb;
    lds[(6 * r + 3 * a + k % 3) * PS + pad(k / 3)] = make_double2(0.0, 0.0);
  }
  // an ended attempt of a device-controlled run: checked once the loads are in
  // flight (nothing is stored before this barrier), so the flag costs no wait
  if (gate_closed(g)) return;
  __syncthreads();
  if (wave < 6 * NR) wave_fft<S, 0, 1, 1, false>(lds + wave * PS, tw, lane, 0.0, nullptr, 0, 0, 0);
  __syncthreads();
  // fused pass of ring r at n2: inverse twiddles and radix 3 of both pairs, the
  // grid product at S n1 + n2, forward radix 3 and twiddles
  {
    const int r = threadIdx.x / RT, n2 = threadIdx.x - r * RT;
    const int lat = lat0 + r;
    if (n2 < S && lat < nlat) {
      const int p = lat < g.nh ? lat : nlat - 1 - lat;  // northern node of the ring
      const double x = g.mu[p];
      const double inv_sin2 = 1.0 / ((1.0 - x) * (1.0 + x));
      double2* rows = lds + 6 * r * PS;
      const double2 w1 = tw_full<M>(tw, n2), w2 = cmul(w1, w1);
      double2 y[2][3];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) y[a][k1] = rows[(3 * a + k1) * PS + pad(n2)];
        y[a][1] = cmul(y[a][1], make_double2(w1.x, -w1.y));
        y[a][2] = cmul(y[a][2], make_double2(w2.x, -w2.y));
        butterfly<3>(y[a], 1.0);
      }
      double2 z[3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
        z[j] = make_double2((y[0][j].x * y[1][j].x - y[0][j].y * y[1][j].y) * inv_sin2, 0.0);
      butterfly<3>(z, -1.0);
      z[1] = cmul(z[1], w1);
      z[2] = cmul(z[2], w2);
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) rows[k1 * PS + pad(n2)] = z[k1];
    }
  }
  __syncthreads();
  if (wave < 3 * NR) {
    const int r = wave / 3, k1 = wave - 3 * r;
    const int lat = lat0 + r;
    if (lat < nlat) {
      const int p = lat < g.nh ? lat : nlat - 1 - lat;
      // quadrature factor (2 pi / M) w_p; the equator ring of an odd rule is its
      // own mirror and is folded twice by the analysis
      const double c = (6.283185307179586477 / M) * g.w[p] * (2 * p + 1 == nlat ? 0.5 : 1.0);
      double2* Wl = g.W + (int64_t)b * (N + 1) * nlat + lat;  // W[b][m][lat]
      wave_fft<S, 0, 1, -1, true>(lds + (6 * r + k1) * PS, tw, lane, c, Wl, nlat, k1, N);
    }
  }
}

// Adjoint of the ring step on the same split transforms (M = 3 S; the
// operation is that of k_ring_adj below): nine inverse S-point transforms
// (rows 3a + k1: a = 0, 1 the forward pairs f0 + i f1 and f2 + i f3, a = 2 the
// real field of spectrum Qbar / 2), one fused pass at n2 (inverse radix 3 of
// the three arrays, the cotangents gbar at S n1 + n2, forward radix 3 of
// gbar0 + i gbar1 and gbar2 + i gbar3), six forward S-point transforms into
// rows 0..5, and the unpacking of the two real transforms of each array.
// Waves take the rows in turn, so any NT / NR >= max(S, 384) covers them. With
// NR = 2 the workgroup holds two neighbouring rings (ring r on rows 9 r .. 9 r + 8,
// 78.6 KB of LDS at S = 256), and the loads of Fa and the stores of Fbar pair up
// on the same 32 bytes (lanes 2 j and 2 j + 1 take the two latitudes of one
// order): the T255 backward pass 1.8% shorter than with one ring per workgroup.
template <int S, int NT, int NR>
__global__ __launch_bounds__(NT) void k_ring_adj_nl(GroupView g) {
  constexpr int M = 3 * S, PS = wave_row(S), NW = NT / 64, RT = NT / NR;
  static_assert(RT >= S && RT >= 384, "threads per ring");
  const int N = g.N, nlat = g.nlat;
  const int lat0 = NR * xcd_item(blockIdx.x, 8 / NR);  // XCD chunks of 8 latitudes
  if (lat0 >= nlat) return;
  const int b = blockIdx.y;
  extern __shared__ double2 lds[];
  const double2* tw = g.tw;  // twiddle half table, read through L1
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t fstride = (int64_t)(N + 1) * nlat;
  const int rr = threadIdx.x % NR, tt = threadIdx.x / NR;
  const bool rvalid = lat0 + rr < nlat;  // an odd last ring pair holds one ring
  const double2* F5 = g.Fa + (int64_t)b * 5 * fstride + lat0 + rr;

  // loads: thread t takes ring rr and order m = t' mod (N+1) of array
  // a = t' / (N+1), t' = t / NR (both fields of a forward pair, or the fifth
  // field for a = 2), all requested before the first LDS write
  constexpr int KI = (3 * (S + 1) + RT - 1) / RT;  // N + 1 <= S + 1
  const int n1 = N + 1;
  double2 ga[KI], gb[KI];
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int idx = tt + i * RT;
    ga[i] = gb[i] = make_double2(0.0, 0.0);
    if (idx < 3 * n1 && rvalid) {
      const int a = idx >= 2 * n1 ? 2 : (idx >= n1 ? 1 : 0), m = idx - a * n1;
      const double2* Fa = F5 + (int64_t)(2 * a) * fstride + (int64_t)m * nlat;
      ga[i] = Fa[0];
      if (a < 2) gb[i] = Fa[fstride];
    }
  }
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int idx = tt + i * RT;
    if (idx < 3 * n1) {
      const int a = idx >= 2 * n1 ? 2 : (idx >= n1 ? 1 : 0), m = idx - a * n1;
      double2* rows = lds + (9 * rr + 3 * a) * PS;
      const int k = M - m;
      if (a < 2) {
        if (m == 0) {
          rows[0] = make_double2(ga[i].x, gb[i].x);
        } else {
          rows[(m % 3) * PS + pad(m / 3)] = make_double2(ga[i].x - gb[i].y, ga[i].y + gb[i].x);
          rows[(k % 3) * PS + pad(k / 3)] = make_double2(ga[i].x + gb[i].y, gb[i].x - ga[i].y);
        }
      } else {
        // x_0 = Re Qbar_0, x_m = Qbar_m / 2, x_{M-m} = conj(Qbar_m) / 2
        if (m == 0) {
          rows[0] = make_double2(ga[i].x, 0.0);
        } else {
          rows[(m % 3) * PS + pad(m / 3)] = make_double2(0.5 * ga[i].x, 0.5 * ga[i].y);
          rows[(k % 3) * PS + pad(k / 3)] = make_double2(0.5 * ga[i].x, -0.5 * ga[i].y);
        }
      }
    }
  }
  // the zero band N < k < M - N of the three arrays of every ring
  const int zb = M - 2 * N - 1;
  for (int t = threadIdx.x; t < NR * 3 * zb; t += NT) {
    const int r = t / (3 * zb), u = t - r * 3 * zb;
    const int a = u >= 2 * zb ? 2 : (u >= zb ? 1 : 0);
    const int k = N + 1 + u - a * zb;
    lds[(9 * r + 3 * a + k % 3) * PS + pad(k / 3)] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int row = wave; row < 9 * NR; row += NW)
    wave_fft<S, 0, 1, 1, false>(lds + row * PS, tw, lane, 0.0, nullptr, 0, 0, 0);
  __syncthreads();
  // fused pass of ring r at n2: the grid values at S n1 + n2 of the three
  // arrays, gbar0 + i gbar1 = qb (g2, -g3) and gbar2 + i gbar3 = qb (g0, -g1)
  // with qb = c_lat qbar / s^2, and the forward radix 3 and twiddles of both
  {
    const int r = threadIdx.x / RT, n2 = threadIdx.x - r * RT;
    const int lat = lat0 + r;
    if (n2 < S && lat < nlat) {
      const int p = lat < g.nh ? lat : nlat - 1 - lat;  // northern node of the ring
      const double x = g.mu[p];
      const double inv_sin2 = 1.0 / ((1.0 - x) * (1.0 + x));
      const double clat = (6.283185307179586477 / M) * g.w[p];
      double2* rows = lds + 9 * r * PS;
      const double2 w1 = tw_full<M>(tw, n2), w2 = cmul(w1, w1);
      double2 y[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) y[a][k1] = rows[(3 * a + k1) * PS + pad(n2)];
        y[a][1] = cmul(y[a][1], make_double2(w1.x, -w1.y));
        y[a][2] = cmul(y[a][2], make_double2(w2.x, -w2.y));
        butterfly<3>(y[a], 1.0);
      }
      double2 z[2][3];
#pragma unroll
      for (int n1 = 0; n1 < 3; ++n1) {
        const double qb = clat * y[2][n1].x * inv_sin2;
        z[0][n1] = make_double2(qb * y[1][n1].x, -qb * y[1][n1].y);
        z[1][n1] = make_double2(qb * y[0][n1].x, -qb * y[0][n1].y);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        butterfly<3>(z[a], -1.0);
        z[a][1] = cmul(z[a][1], w1);
        z[a][2] = cmul(z[a][2], w2);
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) rows[(3 * a + k1) * PS + pad(n2)] = z[a][k1];
      }
    }
  }
  __syncthreads();
  for (int row = wave; row < 6 * NR; row += NW) {
    const int r = row / 6;
    wave_fft<S, 0, 1, -1, false>(lds + (9 * r + row - 6 * r) * PS, tw, lane, 0.0, nullptr, 0, 0, 0);
  }
  __syncthreads();
  // unpack two real transforms per array, Z_k at row 3 a + k mod 3, k / 3:
  // A_m = (Z_m + conj Z_{M-m}) / 2, B_m = (Z_m - conj Z_{M-m}) / (2 i); times 2 for m >= 1
  double2* Fb = g.Fbar + (int64_t)b * 4 * fstride + lat0 + rr;  // Fbar[b][f][m][lat]
  if (rvalid) {
    const double2* rows = lds + 9 * rr * PS;
    for (int m = tt; m <= N; m += RT) {
      const double sc = (m == 0) ? 0.5 : 1.0;
      const int mc = m == 0 ? 0 : M - m;
#pragma unroll
      for (int arr = 0; arr < 2; ++arr) {
        const double2 zm = rows[(3 * arr + m % 3) * PS + pad(m / 3)];
        const double2 zc = rows[(3 * arr + mc % 3) * PS + pad(mc / 3)];
        Fb[(int64_t)(2 * arr) * fstride + (int64_t)m * nlat] = make_double2(sc * (zm.x + zc.x), sc * (zm.y - zc.y));
        Fb[(int64_t)(2 * arr + 1) * fstride + (int64_t)m * nlat] = make_double2(sc * (zm.y + zc.y), -sc * (zm.x - zc.x));
      }
    }
  }
}

}  // namespace

size_t ring_lds_bytes(int M) { return sizeof(double2) * (size_t)(2 * padded_len(M) + M / 2); }

// One workgroup per ring; rings are taken in XCD-local chunks of eight
// neighbouring latitudes so that the strided reads of F share L2 lines.
// MAXM: the largest M of the size class this instance serves and NT its
// workgroup size (register arrays are sized from both).
// TWG: the stages read their twiddles from the global half table (L1-resident)
// instead of an LDS copy, which leaves 2 padded_len(M) entries of LDS per ring.
template <int MAXM, int NT, int CM, bool TWG = false>
__global__ __launch_bounds__(NT) void k_ring(GroupView g, FftPlan plan, int mode,
                                             double* grid_out) {
  constexpr int PTS = (MAXM + NT - 1) / NT;
  const int N = g.N, M = CM > 0 ? CM : g.M, nlat = g.nlat;
  const int lat = xcd_item(blockIdx.x, 8);
  if (lat >= nlat) return;
  const int b = blockIdx.y;
  const int p = lat < g.nh ? lat : nlat - 1 - lat;  // northern node of the ring
  const int PL = padded_len(M);
  extern __shared__ double2 lds[];
  double2* A0 = lds;
  double2* A1 = lds + PL;
  double2* twl = lds + 2 * PL;  // unused with TWG
  const double2* tw = TWG ? g.tw : twl;
  const double x = g.mu[p];
  const double sin2 = (1.0 - x) * (1.0 + x);
  const int64_t fstride = (int64_t)(N + 1) * nlat;
  const double2* F0 = g.F + (int64_t)b * 4 * fstride;

  if (mode == SYNTH_GRID) {
    // u_theta = f0 / sin, u_phi = -f1 / sin, zeta = f2
    const double rs = 1.0 / sqrt(sin2);
    load_ring<MAXM, NT, !TWG>(A0, A1, twl, g.tw, F0, F0 + fstride, F0 + 2 * fstride,
                              F0 + 2 * fstride, lat, N, M, nlat);
    __syncthreads();
    fft_any<2, MAXM, NT, CM>(A0, A1, plan, M, tw, 1.0);
    double* g0 = grid_out + ((int64_t)0 * nlat + lat) * M;
    double* g1 = grid_out + ((int64_t)1 * nlat + lat) * M;
    double* g2 = grid_out + ((int64_t)2 * nlat + lat) * M;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
      const double2 v0 = A0[pad(j)], v1 = A1[pad(j)];
      g0[j] = rs * v0.x;
      g1[j] = -rs * v0.y;
      g2[j] = v1.x;
    }
    return;
  }

  // inverse transforms of f0 + i f1 and f2 + i f3, then the grid product
  load_ring<MAXM, NT, !TWG>(A0, A1, twl, g.tw, F0, F0 + fstride, F0 + 2 * fstride,
                            F0 + 3 * fstride, lat, N, M, nlat);
  // an ended attempt of a device-controlled run (only nonlinear-mode launches
  // are gated): checked once the loads are in flight, nothing stored before
  if (gate_closed(g)) return;
  __syncthreads();
  const double inv_sin2 = 1.0 / sin2;
  if constexpr (CM > 0 && ct_fused<CM>()) {
    fft_ct_inverse_product<CM, 0, 1, NT>(A0, tw, inv_sin2);
  } else {
    fft_any<2, MAXM, NT, CM>(A0, A1, plan, M, tw, 1.0);
    // grid product, in place: each index j is read and rewritten by one thread
#pragma unroll
    for (int c = 0; c < PTS; ++c) {
      const int j = threadIdx.x + c * NT;
      if (j < M) {
        const double2 z01 = A0[pad(j)], z23 = A1[pad(j)];
        A0[pad(j)] = make_double2((z01.x * z23.x - z01.y * z23.y) * inv_sin2, 0.0);
      }
    }
    __syncthreads();
  }
  // quadrature factor (2 pi / M) w_p; the equator ring of an odd rule is its
  // own mirror and is folded twice by the analysis
  const double c = (6.283185307179586477 / M) * g.w[p] * (2 * p + 1 == nlat ? 0.5 : 1.0);
  // W[b][m][lat]: stride nlat between orders (the eight rings of an XCD chunk
  // fill whole cache lines of one order)
  double2* Wl = g.W + (int64_t)b * (N + 1) * nlat + lat;
  if constexpr (CM > 0 && ct_fused<CM>()) {
    fft_ct_forward_store<CM, 0, 1, NT>(A0, tw, c, Wl, nlat, N);
  } else {
    fft_any<1, MAXM, NT, CM>(A0, A1, plan, M, tw, -1.0);
    for (int m = threadIdx.x; m <= N; m += blockDim.x) {
      const double2 X = A0[pad(m)];
      Wl[(int64_t)m * nlat] = make_double2(c * X.x, c * X.y);
    }
  }
}

// Adjoint of the ring kernel (vector-Jacobian product on the real grid
// values): given the cotangent of the ring spectra Q (the fifth field of Fa,
// produced by the adjoint of the analysis), recompute the four forward grid
// fields of the ring, form
//   qbar_j = c_lat Re(Qbar_0 + sum_{m>=1} Qbar_m e^{i m phi_j})   (weighted r2c)^T
//   gbar0 = qbar g2 / s^2, gbar2 = qbar g0 / s^2, gbar1 = -qbar g3 / s^2, gbar3 = -qbar g1 / s^2
// and the cotangents of the field spectra (the c2r of the synthesis)^T:
//   Gbar_0 = sum_j gbar_j,  Gbar_m = 2 sum_j gbar_j e^{-i m phi_j}  (m >= 1),
// written to Fbar[b][f][m][lat]. c_lat = (2 pi / M) w_p.
template <int MAXM, int NT, int CM>
__global__ __launch_bounds__(NT) void k_ring_adj(GroupView g, FftPlan plan) {
  constexpr int PTS = (MAXM + NT - 1) / NT;
  const int N = g.N, M = CM > 0 ? CM : g.M, nlat = g.nlat;
  const int lat = xcd_item(blockIdx.x, 8);  // XCD-local chunks of 8 rings share L2 lines of Fa
  if (lat >= nlat) return;
  const int b = blockIdx.y;
  const int p = lat < g.nh ? lat : nlat - 1 - lat;
  const int PL = padded_len(M);
  extern __shared__ double2 lds[];
  double2* A0 = lds;
  double2* A1 = lds + PL;
  double2* tw = lds + 2 * PL;
  const double x = g.mu[p];
  const double inv_sin2 = 1.0 / ((1.0 - x) * (1.0 + x));
  const int64_t fstride = (int64_t)(N + 1) * nlat;
  const double2* F5 = g.Fa + (int64_t)b * 5 * fstride;

  // the ring's fifth field (the cotangent of its spectrum Q), requested now and
  // written to LDS after the forward transforms; 3N + 2 <= M <= MAXM bounds N + 1
  constexpr int KS = (MAXM / 3 + 1 + NT - 1) / NT;
  double2 qbar[KS];
#pragma unroll
  for (int i = 0; i < KS; ++i) {
    const int m = threadIdx.x + i * NT;
    qbar[i] = (m <= N) ? F5[4 * fstride + (int64_t)m * nlat + lat] : make_double2(0.0, 0.0);
  }
  // forward grid fields of this ring: f0 + i f1 and f2 + i f3 (pairs of one
  // kind, as in k_ring)
  load_ring<MAXM, NT>(A0, A1, tw, g.tw, F5, F5 + fstride, F5 + 2 * fstride, F5 + 3 * fstride, lat,
                      N, M, nlat);
  __syncthreads();
  fft_any<2, MAXM, NT, CM>(A0, A1, plan, M, tw, 1.0);
  double g0[PTS], g1[PTS], g2[PTS], g3[PTS];
#pragma unroll
  for (int c = 0; c < PTS; ++c) {
    const int j = threadIdx.x + c * NT;
    g0[c] = g1[c] = g2[c] = g3[c] = 0.0;
    if (j < M) {
      const double2 z01 = A0[pad(j)], z23 = A1[pad(j)];
      g0[c] = z01.x;
      g1[c] = z01.y;
      g2[c] = z23.x;
      g3[c] = z23.y;
    }
  }
  __syncthreads();
  // cotangent of the grid product: the real field of spectrum Qbar / 2 (m >= 1),
  // x_0 = Re Qbar_0, x_m = Qbar_m / 2, x_{M-m} = conj(Qbar_m) / 2, zero elsewhere
#pragma unroll
  for (int i = 0; i < KS; ++i) {
    const int m = threadIdx.x + i * NT;
    if (m == 0) {
      A0[0] = make_double2(qbar[i].x, 0.0);
    } else if (m <= N) {
      A0[pad(m)] = make_double2(0.5 * qbar[i].x, 0.5 * qbar[i].y);
      A0[pad(M - m)] = make_double2(0.5 * qbar[i].x, -0.5 * qbar[i].y);
    }
  }
  for (int j = N + 1 + threadIdx.x; j < M - N; j += NT) A0[pad(j)] = make_double2(0.0, 0.0);
  __syncthreads();
  fft_any<1, MAXM, NT, CM>(A0, A1, plan, M, tw, 1.0);
  const double clat = (6.283185307179586477 / M) * g.w[p];
  double qb[PTS];
#pragma unroll
  for (int c = 0; c < PTS; ++c) {
    const int j = threadIdx.x + c * NT;
    qb[c] = (j < M) ? clat * A0[pad(j)].x * inv_sin2 : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < PTS; ++c) {
    const int j = threadIdx.x + c * NT;
    if (j < M) {
      // gbar0 + i gbar1 (both of the vorticity-gradient size) and gbar2 + i gbar3
      A0[pad(j)] = make_double2(qb[c] * g2[c], -qb[c] * g3[c]);
      A1[pad(j)] = make_double2(qb[c] * g0[c], -qb[c] * g1[c]);
    }
  }
  __syncthreads();
  fft_any<2, MAXM, NT, CM>(A0, A1, plan, M, tw, -1.0);
  // unpack two real transforms per array: z = a + i b ->
  // A_m = (Z_m + conj Z_{M-m}) / 2, B_m = (Z_m - conj Z_{M-m}) / (2 i); times 2 for m >= 1
  double2* Fb = g.Fbar + (int64_t)b * 4 * fstride + lat;  // Fbar[b][f][m][lat]
  for (int m = threadIdx.x; m <= N; m += blockDim.x) {
    const double sc = (m == 0) ? 0.5 : 1.0;
#pragma unroll
    for (int arr = 0; arr < 2; ++arr) {
      const double2* X = arr ? A1 : A0;
      const double2 zm = X[pad(m)];
      const double2 zc = X[pad((M - m) % M)];
      const double2 ga = make_double2(sc * (zm.x + zc.x), sc * (zm.y - zc.y));
      const double2 gb = make_double2(sc * (zm.y + zc.y), -sc * (zm.x - zc.x));
      Fb[(int64_t)(arr ? 2 : 0) * fstride + (int64_t)m * nlat] = ga;
      Fb[(int64_t)(arr ? 3 : 1) * fstride + (int64_t)m * nlat] = gb;
    }
  }
}

// Longitude part of the projection (u, Z[l,m])_M of a grid velocity field:
// per ring, the real transforms Ut_m = sum_j u_theta e^{-i m phi_j} and
// Up_m = sum_j u_phi e^{-i m phi_j} (one complex FFT of u_theta + i u_phi),
// scaled by c = (2 pi / M) w_p / sin(theta_p) and written to
// Fbar[b][f][m][lat] as (c Ut, -c Up, 0, 0). The latitude sums and the degree
// coupling of d/dtheta are done by the unweighted analysis and the prologue
// transpose, since conj(Z[l,m]) = lambda^(-1/2) (-i m Pbar / sin, -dPbar/dtheta) e^{-i m phi}
// and sin(theta) dPbar/dtheta couples degrees l - 1 and l + 1.
template <int MAXM, int NT, int CM>
__global__ __launch_bounds__(NT) void k_ring_project(GroupView g, FftPlan plan,
                                                     const double* __restrict__ u_grid) {
  const int N = g.N, M = CM > 0 ? CM : g.M, nlat = g.nlat;
  const int lat = xcd_item(blockIdx.x, 8);
  if (lat >= g.nlat) return;
  const int b = blockIdx.y;
  const int p = lat < g.nh ? lat : nlat - 1 - lat;
  const int PL = padded_len(M);
  extern __shared__ double2 lds[];
  double2* A0 = lds;
  double2* tw = lds + 2 * PL;
  for (int j = threadIdx.x; j < M / 2; j += blockDim.x) tw[j] = g.tw[j];
  const double* ut = u_grid + ((int64_t)(2 * b) * nlat + lat) * M;
  const double* up = ut + (int64_t)nlat * M;
  for (int j = threadIdx.x; j < M; j += blockDim.x) A0[pad(j)] = make_double2(ut[j], up[j]);
  __syncthreads();
  fft_any<1, MAXM, NT, CM>(A0, A0, plan, M, tw, -1.0);
  const double x = g.mu[p];
  const double c = (6.283185307179586477 / M) * g.w[p] / sqrt((1.0 - x) * (1.0 + x));
  const int64_t fstride = (int64_t)(N + 1) * nlat;
  double2* Fb = g.Fbar + (int64_t)b * 4 * fstride + lat;  // Fbar[b][f][m][lat]
  for (int m = threadIdx.x; m <= N; m += blockDim.x) {
    const double2 zm = A0[pad(m)];
    const double2 zc = A0[pad((M - m) % M)];
    const double h = 0.5 * c;
    const int64_t mo = (int64_t)m * nlat;
    Fb[mo] = make_double2(h * (zm.x + zc.x), h * (zm.y - zc.y));
    Fb[fstride + mo] = make_double2(-h * (zm.y + zc.y), h * (zm.x - zc.x));
    Fb[2 * fstride + mo] = make_double2(0.0, 0.0);
    Fb[3 * fstride + mo] = make_double2(0.0, 0.0);
  }
}

// Calls launch(MAXM, NT, CM) (as integral constants) for the group's M: the
// compile-time instance when M = 3 * 2^k is one of the default grids, else
// the size class of the runtime plan.
template <typename F>
hipError_t ring_dispatch(int M, F&& launch) {
  using std::integral_constant;
  switch (M) {
    case 48: return launch(integral_constant<int, 48>{}, integral_constant<int, 64>{}, integral_constant<int, 48>{});
    case 96: return launch(integral_constant<int, 96>{}, integral_constant<int, 64>{}, integral_constant<int, 96>{});
    case 192: return launch(integral_constant<int, 192>{}, integral_constant<int, 128>{}, integral_constant<int, 192>{});
    case 320: return launch(integral_constant<int, 320>{}, integral_constant<int, 256>{}, integral_constant<int, 320>{});
    case 384: return launch(integral_constant<int, 384>{}, integral_constant<int, 256>{}, integral_constant<int, 384>{});
    case 768: return launch(integral_constant<int, 768>{}, integral_constant<int, 512>{}, integral_constant<int, 768>{});
    case 1536: return launch(integral_constant<int, 1536>{}, integral_constant<int, 1024>{}, integral_constant<int, 1536>{});
    default: break;
  }
  if (M <= 256) return launch(integral_constant<int, 256>{}, integral_constant<int, 128>{}, integral_constant<int, 0>{});
  if (M <= 512) return launch(integral_constant<int, 512>{}, integral_constant<int, 256>{}, integral_constant<int, 0>{});
  if (M <= 768) return launch(integral_constant<int, 768>{}, integral_constant<int, 256>{}, integral_constant<int, 0>{});
  if (M <= 1024) return launch(integral_constant<int, 1024>{}, integral_constant<int, 512>{}, integral_constant<int, 0>{});
  return launch(integral_constant<int, kMaxM>{}, integral_constant<int, 512>{}, integral_constant<int, 0>{});
}

// the split adjoint ring: nine rows of S + S/16 + 1 points (the twiddles are
// read from the global table; an LDS copy took the T255 ring from 8.2 to 8.8 us)
size_t ring_adj_nl_lds_bytes(int M) { return sizeof(double2) * (size_t)(9 * wave_row(M / 3)); }

hipError_t launch_ring_adjoint(const GroupView& g, const FftPlan& plan, hipStream_t s) {
  dim3 grid(xcd_grid(g.nlat, 8), g.nb);
  if (g.M == 384 || g.M == 768) {
    if (g.M == 768) {
      // two neighbouring rings per workgroup (at M = 384 the 96 ring pairs of
      // one member would leave most CUs idle)
      dim3 grid2(xcd_grid((g.nlat + 1) / 2, 4), g.nb);
      const size_t lds = 2 * ring_adj_nl_lds_bytes(g.M);
      hipLaunchKernelGGL((k_ring_adj_nl<256, 768, 2>), grid2, dim3(768), lds, s, g);
      return hipGetLastError();
    }
    const size_t lds = ring_adj_nl_lds_bytes(g.M);
    hipLaunchKernelGGL((k_ring_adj_nl<128, 384, 1>), grid, dim3(384), lds, s, g);
    return hipGetLastError();
  }
  const size_t lds = ring_lds_bytes(g.M);
  return ring_dispatch(g.M, [&](auto maxm, auto nt, auto cm) {
    constexpr int MAXM = decltype(maxm)::value, NT = decltype(nt)::value, CM = decltype(cm)::value;
    hipLaunchKernelGGL((k_ring_adj<MAXM, NT, CM>), grid, dim3(NT), lds, s, g, plan);
    return hipGetLastError();
  });
}

hipError_t launch_ring_project(const GroupView& g, const FftPlan& plan, const double* u_grid,
                               hipStream_t s) {
  dim3 grid(xcd_grid(g.nlat, 8), g.nb);
  const size_t lds = ring_lds_bytes(g.M);
  return ring_dispatch(g.M, [&](auto maxm, auto nt, auto cm) {
    constexpr int MAXM = decltype(maxm)::value, NT = decltype(nt)::value, CM = decltype(cm)::value;
    hipLaunchKernelGGL((k_ring_project<MAXM, NT, CM>), grid, dim3(NT), lds, s, g, plan, u_grid);
    return hipGetLastError();
  });
}

// the split ring: six rows of S + S/16 + 1 points per ring, and the twiddle
// half table with an LDS copy
size_t ring_nl_lds_bytes(int M, int nr, bool twl) {
  return sizeof(double2) * (size_t)(6 * nr * wave_row(M / 3) + (twl ? M / 2 : 0));
}

hipError_t launch_ring(const GroupView& g, const FftPlan& plan, int mode, double* grid_out,
                       hipStream_t s) {
  dim3 grid(xcd_grid(g.nlat, 8), g.nb);
  // the split kernel for M = 384 and 768 (T127, T255: ring 10.0 -> 9.4 us at
  // T255). At M = 1536 the radix-8/8/8/3 plan stays: three one-wave 512-point
  // transforms took 23.6 us, six 256-point ones with a radix-6 fused pass 26.8
  // us (twelve waves) and 25.8 us (six waves of two rows each, 52.7 KB of LDS:
  // still two rings per CU). Over 512 threads with the twiddles read from the
  // global table (52.3 KB of LDS, three rings per CU, the whole T511 launch
  // resident) it takes 19.4 us against 21.0 us over 1024 threads with an LDS
  // table (64.5 KB, two rings per CU).
  if (mode == SYNTH_NONLINEAR && g.M == 1536) {
    const size_t lds = sizeof(double2) * (size_t)(2 * padded_len(1536));
    hipLaunchKernelGGL((k_ring<1536, 512, 1536, true>), grid, dim3(512), lds, s, g, plan, mode,
                       grid_out);
    return hipGetLastError();
  }
  if (mode == SYNTH_NONLINEAR && (g.M == 384 || g.M == 768)) {
    // many members: one ring per workgroup with LDS twiddles (the ensemble's
    // 16 x N = 255 rings: 66 us against 76 us with the global table, its
    // 24 x N = 127 rings 58 against 75 us); few members: global twiddles, and
    // two rings per workgroup when there are more rings than CUs (one member
    // at T255: 7.6 us against 8.2 us with one ring per workgroup and 8.8 us
    // with LDS twiddles; at T127, 192 rings, one ring per workgroup: 5.7
    // against 7.0 us)
    if (g.nb >= 4) {
      const size_t lds = ring_nl_lds_bytes(g.M, 1, true);
      if (g.M == 384) hipLaunchKernelGGL((k_ring_nl<128, 384, true, 1>), grid, dim3(384), lds, s, g);
      else hipLaunchKernelGGL((k_ring_nl<256, 384, true, 1>), grid, dim3(384), lds, s, g);
    } else if ((int64_t)g.nlat * g.nb <= 256) {
      const size_t lds = ring_nl_lds_bytes(g.M, 1, false);
      if (g.M == 384) hipLaunchKernelGGL((k_ring_nl<128, 384, false, 1>), grid, dim3(384), lds, s, g);
      else hipLaunchKernelGGL((k_ring_nl<256, 384, false, 1>), grid, dim3(384), lds, s, g);
    } else {
      dim3 grid2(xcd_grid((g.nlat + 1) / 2, 4), g.nb);
      const size_t lds = ring_nl_lds_bytes(g.M, 2, false);
      if (g.M == 384) hipLaunchKernelGGL((k_ring_nl<128, 768, false, 2>), grid2, dim3(768), lds, s, g);
      else hipLaunchKernelGGL((k_ring_nl<256, 768, false, 2>), grid2, dim3(768), lds, s, g);
    }
    return hipGetLastError();
  }
  const size_t lds = ring_lds_bytes(g.M);
  return ring_dispatch(g.M, [&](auto maxm, auto nt, auto cm) {
    constexpr int MAXM = decltype(maxm)::value, NT = decltype(nt)::value, CM = decltype(cm)::value;
    hipLaunchKernelGGL((k_ring<MAXM, NT, CM>), grid, dim3(NT), lds, s, g, plan, mode, grid_out);
    return hipGetLastError();
  });
}

}  // namespace nse
