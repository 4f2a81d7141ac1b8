// Longitude transforms and the grid product (Section 4.2: FFT in the
// azimuthal direction at the M equispaced longitudes of eq. (quadrule)).
//
// One workgroup per northern/southern ring pair (p, nlat-1-p). The two rings
// share every complex FFT: for a field with Fourier coefficients G^N_m (north)
// and G^S_m (south), m = 0..N, the length-M sequence
//   x_m = G^N_m + i G^S_m,  x_{M-m} = conj(G^N_m) + i conj(G^S_m)
// has the inverse DFT g^N_j + i g^S_j (both rings' real grid values). The
// product q = (f0 f2 - f1 f3) / sin^2(theta) = u . Grad(zeta + 2 Omega cos theta)
// is formed in registers, then one forward FFT of q^N + i q^S gives both rings'
// spectra. The quadrature factor (2 pi / M) w_p of eq. (quadrule) is applied
// and the analysis input is written as even/odd combinations
//   We_m = c (Q^N_m + Q^S_m),  Wo_m = c (Q^N_m - Q^S_m),
// so that the Legendre analysis runs over northern latitudes only.
//
// The FFT is a mixed-radix (4, 5, 3, 2) Stockham transform in LDS: each stage
// reads R values at stride M/R, applies twiddles from a global table
// exp(-2 pi i k / M), performs a radix-R butterfly and writes in autosort
// order to the other LDS buffer.
#include "nse_internal.h"

namespace nse {

namespace {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// s * i * a for s = +-1
__device__ __forceinline__ double2 cmul_si(double2 a, double s) { return make_double2(-s * a.y, s * a.x); }

// cos/sin of 2 pi / 3, 2 pi / 5 and 4 pi / 5 in closed form:
// sqrt(3)/2, (sqrt(5)-1)/4, -(sqrt(5)+1)/4, sqrt(10+2 sqrt(5))/4, sqrt(10-2 sqrt(5))/4.
constexpr double kS3 = 0.86602540378443864676;
constexpr double kC1 = 0.30901699437494742410;
constexpr double kC2 = -0.80901699437494742410;
constexpr double kS1 = 0.95105651629515357212;
constexpr double kS2 = 0.58778525229247312917;

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
  }
}

// One Stockham stage of radix R from `in` to `out` (both LDS, length M).
// sign = -1 forward (exp(-2 pi i jk/M)), +1 inverse.
template <int R>
__device__ void stage(const double2* __restrict__ in, double2* __restrict__ out, int M, int Ns,
                      const double2* __restrict__ tw, double sign) {
  const int span = M / R;
  const int step = M / (Ns * R);
  for (int j = threadIdx.x; j < span; j += blockDim.x) {
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[j + r * span];
    const int k = j % Ns;
    if (k != 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double2 w = tw[(r * k * step) % M];
        w.y *= -sign;  // table holds exp(-2 pi i e / M); forward uses it as is
        v[r] = cmul(v[r], w);
      }
    }
    butterfly<R>(v, sign);
    const int idx = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[idx + r * Ns] = v[r];
  }
}

// Full transform; returns the buffer that holds the result.
__device__ double2* fft(double2* a, double2* b, const FftPlan& plan, int M,
                        const double2* __restrict__ tw, double sign) {
  int Ns = 1;
  for (int st = 0; st < plan.nstages; ++st) {
    const int R = plan.radix[st];
    switch (R) {
      case 2: stage<2>(a, b, M, Ns, tw, sign); break;
      case 3: stage<3>(a, b, M, Ns, tw, sign); break;
      case 4: stage<4>(a, b, M, Ns, tw, sign); break;
      default: stage<5>(a, b, M, Ns, tw, sign); break;
    }
    __syncthreads();
    double2* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// Loads the pair spectrum of field f into x (length M) for rings p (north) and ps.
__device__ void load_pair(double2* x, const double2* __restrict__ Fn, const double2* __restrict__ Fs,
                          int N, int M) {
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    double2 v = make_double2(0.0, 0.0);
    if (j == 0) {
      v = make_double2(Fn[0].x, Fs[0].x);
    } else if (j <= N) {
      const double2 gn = Fn[j], gs = Fs[j];
      v = make_double2(gn.x - gs.y, gn.y + gs.x);        // gn + i gs
    } else if (j >= M - N) {
      const double2 gn = Fn[M - j], gs = Fs[M - j];
      v = make_double2(gn.x + gs.y, -gn.y + gs.x);       // conj(gn) + i conj(gs)
    }
    x[j] = v;
  }
}

}  // namespace

template <int PTS>
__global__ __launch_bounds__(kRingThreads) void k_ring(GroupView g, FftPlan plan, int mode,
                                                       double* grid_out) {
  const int p = blockIdx.x;
  const int b = blockIdx.z;
  const int N = g.N, M = g.M, nlat = g.nlat;
  const int ps = nlat - 1 - p;
  extern __shared__ double2 lds[];
  double2* bufA = lds;
  double2* bufB = lds + M;
  const double x = g.mu[p];
  const double sin2 = (1.0 - x) * (1.0 + x);
  const double2* Fb = g.F + (int64_t)b * 4 * nlat * (N + 1);

  if (mode == SYNTH_GRID) {
    // u_theta = f0 / sin, u_phi = -f1 / sin, zeta = f2 for both rings.
    const double rs = 1.0 / sqrt(sin2);
    for (int f = 0; f < 3; ++f) {
      const double2* Ff = Fb + (int64_t)f * nlat * (N + 1);
      load_pair(bufA, Ff + (int64_t)p * (N + 1), Ff + (int64_t)ps * (N + 1), N, M);
      __syncthreads();
      const double2* res = fft(bufA, bufB, plan, M, g.tw, 1.0);
      const double sc = (f == 0) ? rs : (f == 1 ? -rs : 1.0);
      double* gn = grid_out + (((int64_t)b * 3 + f) * nlat + p) * M;
      double* gs = grid_out + (((int64_t)b * 3 + f) * nlat + ps) * M;
      for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double2 v = res[j];
        gn[j] = sc * v.x;
        if (ps != p) gs[j] = sc * v.y;
      }
      __syncthreads();
    }
    return;
  }

  double qn[PTS], qs[PTS], hn[PTS], hs[PTS];
  const double inv_sin2 = 1.0 / sin2;
  // field order f0, f2 (-> q = f0 f2), f1, f3 (-> q = (q - f1 f3) / sin^2)
  for (int oi = 0; oi < 4; ++oi) {
    const int f = (oi == 1) ? 2 : (oi == 2 ? 1 : oi);
    const double2* Ff = Fb + (int64_t)f * nlat * (N + 1);
    load_pair(bufA, Ff + (int64_t)p * (N + 1), Ff + (int64_t)ps * (N + 1), N, M);
    __syncthreads();
    const double2* res = fft(bufA, bufB, plan, M, g.tw, 1.0);
#pragma unroll
    for (int i = 0; i < PTS; ++i) {
      const int j = threadIdx.x + i * kRingThreads;
      double vn = 0.0, vs = 0.0;
      if (j < M) {
        const double2 v = res[j];
        vn = v.x;
        vs = v.y;
      }
      if (oi == 0 || oi == 2) {
        hn[i] = vn;
        hs[i] = vs;
      } else if (oi == 1) {
        qn[i] = hn[i] * vn;
        qs[i] = hs[i] * vs;
      } else {
        qn[i] = (qn[i] - hn[i] * vn) * inv_sin2;
        qs[i] = (qs[i] - hs[i] * vs) * inv_sin2;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < PTS; ++i) {
    const int j = threadIdx.x + i * kRingThreads;
    if (j < M) bufA[j] = make_double2(qn[i], qs[i]);
  }
  __syncthreads();
  const double2* X = fft(bufA, bufB, plan, M, g.tw, -1.0);
  const double c = (6.283185307179586477 / M) * g.w[p] * (ps == p ? 0.5 : 1.0);
  double2* Wb = g.W + (int64_t)b * (N + 1) * 2 * g.nh;
  for (int m = threadIdx.x; m <= N; m += blockDim.x) {
    const double2 xm = X[m];
    const double2 xc = X[(M - m) % M];
    // Q^N = (X_m + conj X_{M-m}) / 2,  Q^S = (X_m - conj X_{M-m}) / (2 i)
    const double2 qN = make_double2(0.5 * (xm.x + xc.x), 0.5 * (xm.y - xc.y));
    const double2 qS = make_double2(0.5 * (xm.y + xc.y), -0.5 * (xm.x - xc.x));
    Wb[((int64_t)m * 2 + 0) * g.nh + p] = make_double2(c * (qN.x + qS.x), c * (qN.y + qS.y));
    Wb[((int64_t)m * 2 + 1) * g.nh + p] = make_double2(c * (qN.x - qS.x), c * (qN.y - qS.y));
  }
}

hipError_t launch_ring(const GroupView& g, const FftPlan& plan, int mode, double* grid_out,
                       hipStream_t s) {
  dim3 block(kRingThreads);
  dim3 grid(g.nh, 1, g.nb);
  const size_t lds = 2 * sizeof(double2) * (size_t)g.M;
  const int pts = (g.M + kRingThreads - 1) / kRingThreads;
  if (pts <= 1)
    hipLaunchKernelGGL(k_ring<1>, grid, block, lds, s, g, plan, mode, grid_out);
  else if (pts <= 2)
    hipLaunchKernelGGL(k_ring<2>, grid, block, lds, s, g, plan, mode, grid_out);
  else if (pts <= 4)
    hipLaunchKernelGGL(k_ring<4>, grid, block, lds, s, g, plan, mode, grid_out);
  else if (pts <= 8)
    hipLaunchKernelGGL(k_ring<8>, grid, block, lds, s, g, plan, mode, grid_out);
  else
    hipLaunchKernelGGL(k_ring<16>, grid, block, lds, s, g, plan, mode, grid_out);
  return hipGetLastError();
}

}  // namespace nse
