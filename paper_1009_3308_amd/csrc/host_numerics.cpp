// Host-side numerics: the Gauss-Legendre rule of the Gauss-rectangle
// quadrature (Section 3, eq. (quadrule)) and the radix plan of the
// longitude FFTs (Section 4.2, FFT in the azimuthal direction).
#include <cmath>

#include "nse_internal.h"

namespace nse {

// Nodes mu_p of the n-point Gauss-Legendre rule in descending order (north
// pole first) and their weights. Newton's method on P_n in extended precision
// (x87 long double), P_n and P_n' from the three-term recurrence
// (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}, started from the asymptotic
// guess cos(pi (k - 1/4) / (n + 1/2)); w = 2 / ((1 - x^2) P_n'(x)^2) with
// 1 - x^2 formed as (1 - x)(1 + x).
void gauss_legendre(int n, std::vector<double>& mu, std::vector<double>& w) {
  mu.assign(n, 0.0);
  w.assign(n, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 1; k <= (n + 1) / 2; ++k) {
    long double x = std::cos(pi * (k - 0.25L) / (n + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = x;
      for (int j = 1; j < n; ++j) {
        long double p2 = ((2 * j + 1) * x * p1 - j * p0) / (j + 1);
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p0 = 1.0L;
      const long double omx2 = (1.0L - x) * (1.0L + x);
      dp = n * (p0 - x * p1) / omx2;
      const long double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-19L) {
        // one more evaluation of P_n' at the converged node
        p0 = 1.0L;
        p1 = x;
        for (int j = 1; j < n; ++j) {
          long double p2 = ((2 * j + 1) * x * p1 - j * p0) / (j + 1);
          p0 = p1;
          p1 = p2;
        }
        if (n == 1) p0 = 1.0L;
        dp = n * (p0 - x * p1) / ((1.0L - x) * (1.0L + x));
        break;
      }
    }
    if (2 * k - 1 == n) x = 0.0L;  // the equator node of an odd rule
    const long double wk = 2.0L / ((1.0L - x) * (1.0L + x) * dp * dp);
    mu[k - 1] = (double)x;
    mu[n - k] = (double)(-x);
    w[k - 1] = (double)wk;
    w[n - k] = (double)wk;
  }
}

// Splits M into radix-8 stages first, then 4, 2 and the odd radices 5, 3 last,
// so that the stride Ns = (product of earlier radices) is a power of two for
// every stage but those after an odd radix; false if M has another prime
// factor or too many stages.
bool fft_factor(int M, FftPlan& plan) {
  plan.nstages = 0;
  if (M < 2) return false;
  int r = M;
  const int rad[5] = {8, 4, 2, 5, 3};
  for (int i = 0; i < 5; ++i) {
    while (r % rad[i] == 0) {
      if (plan.nstages >= kMaxRadices) return false;
      plan.radix[plan.nstages++] = rad[i];
      r /= rad[i];
    }
  }
  if (r != 1) return false;
  int ns = 1;
  for (int st = 0; st < plan.nstages; ++st) {
    int lg = -1;
    for (int b = 0; b < 31; ++b)
      if ((1 << b) == ns) lg = b;
    plan.ns_log2[st] = lg;
    ns *= plan.radix[st];
  }
  return true;
}

}  // namespace nse
