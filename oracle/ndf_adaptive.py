"""Variable-order, variable-step NDF integrator: the time discretisation the paper
uses for its experiments (Section 4.2: the NDF_p formula (ode_disc) with p = 1..5
and the kappa_p listed there, the step chosen by comparing formulas of two orders;
Section 5, Example 2: orders one to five, adaptive steps at a relative tolerance).

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import this module. The product path never calls it and shares no
code, table or constant with it.

The system is y' = F(t, y) = f(t) - L y - n(y), with L >= 0 diagonal (the Stokes
term nu lambda_l, eq. (stok_eig)) and n the nonlinear term; every array is a 1-D
complex128 tensor. For the sphere, y = alpha and n = (B(u,u) + C u, Z)_M.

Method (backward-difference form of (ode_disc) at a quasi-constant step h). The
state holds D[j] = nabla^j y_n, j = 0..k+2, at spacing h. With
gamma_k = sum_{j<=k} 1/j and the predictor y0 = sum_{j=0}^{k} D[j] (so that
nabla^{k+1} y_{n+1} = y_{n+1} - y0 =: d), the identity
  sum_{m=1}^{k} (1/m) nabla^m y_{n+1} = gamma_k d + sum_{m=1}^{k} gamma_m D[m]
turns (ode_disc) into
  (1 - kappa_k) gamma_k d + psi - h F(t_{n+1}, y0 + d) = 0,  psi = sum_{m=1}^{k} gamma_m D[m].
The implicit part is iterated with the diagonal iteration matrix (L only):
  d_i = (h (f(t_{n+1}) - n(y_{i-1})) - h L y0 - psi) / ((1 - kappa_k) gamma_k + h L),
  y_i = y0 + d_i,  y_0 = y0.
Local error estimate: err = (kappa_k gamma_k + 1/(k+1)) ||d||, the leading error
constant of NDF_k times nabla^{k+1} y_{n+1}. On acceptance the differences are
updated: D[k+2] = d - D[k+1], D[k+1] = d, D[j] += D[j+1] for j = k..0.

Readings (the paper gives the formula, the orders, kappa, the tolerance and that
the error is estimated from formulas of two orders; the rest is chosen here and is
the same in the GPU library):
  * norm: ||v|| = max over coefficients |v_i| / max(|y_n,i|, |y_i,i|, atol/rtol), the
    modulus of each complex coefficient, y_i the current iterate; defaults
    rtol = 1e-3 (the paper's tolerance), atol = 1e-6;
  * Newton: at most `max_newton` sweeps (default 4); from the second sweep on,
    rho = ||d_i - d_{i-1}|| / ||d_{i-1} - d_{i-2}||; rho >= 0.9 fails, and the sweep
    converges when rho / (1 - rho) ||d_i - d_{i-1}|| <= 0.1 rtol or the correction is
    zero; a single sweep (max_newton = 1) is taken as converged;
  * a Newton failure multiplies h by 0.3;
  * an error failure (err > rtol): the first in a row multiplies h by
    max(0.1, 0.833 (rtol/err)^(1/(k+1))), or lowers the order when
    min(1, max(0.1, 0.769 (rtol/err_{k-1})^(1/k))) is larger, err_{k-1} =
    (kappa_{k-1} gamma_{k-1} + 1/k) ||D[k] + d||; later ones halve h, and from the
    third on the order drops to 1;
  * after an accepted step, once k + 2 steps in a row have used the same h and k,
    the ratios r_j = 1 / max(0.1, c_j (err_j / rtol)^(1/(j+1))) for j = k (c = 1.2),
    k-1 (c = 1.3, err_{k-1} from nabla^k y_{n+1}) and k+1 (c = 1.4, err_{k+1} from
    nabla^{k+2} y_{n+1}) are compared; the largest (ties: current order, then the
    lower) sets the new order and h <- r h, but only when r > 1;
  * h <= hmax, and a step that would end within 10 % of t_end is stretched or
    shortened to end there exactly;
  * a change of h rescales D[0..k] to the new spacing (the differences of the
    interpolating polynomial of y_n .. y_{n-k} taken at the new nodes) and zeroes
    D[k+1..];
  * first step: order 1, D[1] = h F(t0, y0), h = min(hmax, t_end - t0,
    0.8 sqrt(rtol) / ||F(t0, y0)||) unless h0 is given.
"""
from __future__ import annotations

import math
from fractions import Fraction

import torch

from .nse_oracle import NDF_KAPPA

ACCEPTED, ERROR_FAIL, NEWTON_FAIL = 0, 1, 2


def gamma(k: int) -> Fraction:
    return sum((Fraction(1, j) for j in range(1, k + 1)), Fraction(0))


def alpha_k(k: int) -> Fraction:
    """(1 - kappa_k) gamma_k: the coefficient of d in the corrector equation."""
    return (1 - NDF_KAPPA[k]) * gamma(k)


def error_constant(k: int) -> Fraction:
    """kappa_k gamma_k + 1/(k+1): leading error constant of NDF_k."""
    return NDF_KAPPA[k] * gamma(k) + Fraction(1, k + 1)


def step_change_matrix(k: int, rho: float):
    """Exact rational matrix R with D_new[j] = sum_i R[j][i] D[i], j, i = 0..k.

    Built from its definition: the past values y_{n-q} = (1 - nabla)^q y_n, the
    Lagrange polynomial through them at the nodes s = -q (units of the old h),
    evaluated at s = -q rho, and the backward differences of those values.
    """
    r = Fraction(rho)
    # values from differences: V[q][i] = (-1)^i C(q, i)
    V = [[Fraction((-1) ** i * math.comb(q, i)) if i <= q else Fraction(0) for i in range(k + 1)]
         for q in range(k + 1)]
    # Lagrange weights at s = -qq rho
    Lg = []
    for qq in range(k + 1):
        s = -qq * r
        row = []
        for q in range(k + 1):
            w = Fraction(1)
            for rr in range(k + 1):
                if rr != q:
                    w *= (s + rr) / (rr - q)
            row.append(w)
        Lg.append(row)
    # differences of the new values: Dn[j][qq] = (-1)^qq C(j, qq)
    Dn = [[Fraction((-1) ** qq * math.comb(j, qq)) if qq <= j else Fraction(0)
           for qq in range(k + 1)] for j in range(k + 1)]

    def mul(A, B):
        return [[sum((A[i][t] * B[t][j] for t in range(len(B))), Fraction(0))
                 for j in range(len(B[0]))] for i in range(len(A))]

    return mul(Dn, mul(Lg, V))


class AdaptiveNDF:
    """y' = f(t) - L y - n(y), variable order 1..max_order, variable step."""

    def __init__(self, lin: torch.Tensor, nonlinear, forcing, rtol=1e-3, atol=1e-6, h0=0.0,
                 hmax=0.0, max_order=5, max_newton=4, project=None):
        if not (1 <= max_order <= 5):
            raise ValueError("max_order must be 1..5")
        self.L = lin
        self.n = nonlinear
        self.f = forcing  # callable t -> tensor, or None
        self.rtol, self.atol = float(rtol), float(atol)
        self.h0, self.hmax = float(h0), (float(hmax) if hmax > 0 else math.inf)
        self.kmax, self.K = max_order, max_newton
        self.project = project if project is not None else (lambda y: y)
        self.log = []

    # -- pieces --------------------------------------------------------------
    def _forcing(self, t):
        return self.f(t) if self.f is not None else torch.zeros_like(self.D[0])

    def _F(self, t, y):
        return self.project(self._forcing(t) - self.L * y - self.n(y))

    def _norm(self, v, y_old, y_new):
        wt = torch.maximum(torch.maximum(y_old.abs(), y_new.abs()),
                           torch.full_like(y_old.real, self.atol / self.rtol))
        return float((v.abs() / wt).max())

    def _rescale(self, h_new):
        R = step_change_matrix(self.k, h_new / self.h)
        k = self.k
        new = [sum(float(R[j][i]) * self.D[i] for i in range(j, k + 1)) for j in range(k + 1)]
        self.D = new + [torch.zeros_like(self.D[0]) for _ in range(k + 1, self.kmax + 3)]
        self.h = h_new
        self.nconst = 0

    # -- interface -----------------------------------------------------------
    def begin(self, y0: torch.Tensor, t0: float):
        self.t = float(t0)
        self.D = [y0.clone()] + [torch.zeros_like(y0) for _ in range(self.kmax + 2)]
        self.k, self.h, self.nconst, self.started = 1, 0.0, 0, False
        self.F0 = self._F(self.t, y0)
        self.log = []

    def _start(self, t_end):
        wt = torch.maximum(self.D[0].abs(), torch.full_like(self.D[0].real, self.atol / self.rtol))
        fn = float((self.F0.abs() / wt).max())
        h = min(self.hmax, t_end - self.t)
        if self.h0 > 0:
            h = min(h, self.h0)
        elif fn > 0 and h * fn / (0.8 * math.sqrt(self.rtol)) > 1:
            h = 0.8 * math.sqrt(self.rtol) / fn
        self.h = h
        self.D[1] = h * self.F0
        self.started = True

    def advance(self, t_end: float):
        """Integrates until t = t_end exactly; returns y(t_end)."""
        if t_end < self.t:
            raise ValueError("t_end before the current time")
        if t_end == self.t:
            return self.D[0]
        if not self.started:
            self._start(t_end)
        nfail = 0
        while self.t < t_end:
            # clamp to hmax and to the end of the interval
            h_new = min(self.h, self.hmax)
            last = False
            if self.t + 1.1 * h_new >= t_end:
                h_new, last = t_end - self.t, True
            if h_new != self.h:
                self._rescale(h_new)
            if self.h <= 16 * 2.0 ** -52 * abs(self.t):
                raise RuntimeError("step size underflow")
            k, h, D = self.k, self.h, self.D
            t1 = self.t + h
            g = [float(gamma(j)) for j in range(k + 1)]
            y0 = sum(D[j] for j in range(k + 1))
            psi = sum(g[j] * D[j] for j in range(1, k + 1))
            f = self._forcing(t1)
            denom = float(alpha_k(k)) + h * self.L
            y, d_prev, dd_prev = y0, torch.zeros_like(y0), None
            converged, iters = False, 0
            for i in range(1, self.K + 1):
                iters = i
                d = self.project((h * (f - self.n(y)) - h * self.L * y0 - psi) / denom)
                y = y0 + d
                dd = self._norm(d - d_prev, D[0], y)
                if not math.isfinite(dd):
                    raise FloatingPointError("non-finite Newton correction")
                if self.K == 1:
                    converged = True
                    break
                if i >= 2:
                    if dd == 0.0:
                        converged = True
                        break
                    rho = dd / dd_prev if dd_prev > 0 else math.inf
                    if rho >= 0.9:
                        break
                    if rho / (1.0 - rho) * dd <= 0.1 * self.rtol:
                        converged = True
                        break
                d_prev, dd_prev = d, dd
            if not converged:
                self.log.append((self.t, h, k, iters, NEWTON_FAIL, math.nan))
                self._rescale(0.3 * h)
                continue
            err = float(error_constant(k)) * self._norm(d, D[0], y)
            if err > self.rtol:
                self.log.append((self.t, h, k, iters, ERROR_FAIL, err))
                nfail += 1
                if nfail == 1:
                    ratio = max(0.1, 0.833 * (self.rtol / err) ** (1.0 / (k + 1)))
                    if k > 1:
                        ekm1 = float(error_constant(k - 1)) * self._norm(D[k] + d, D[0], y)
                        rkm1 = (min(1.0, max(0.1, 0.769 * (self.rtol / ekm1) ** (1.0 / k)))
                                if ekm1 > 0 else 1.0)
                        if rkm1 > ratio:
                            ratio = rkm1
                            self.k = k - 1
                else:
                    ratio = 0.5
                    if nfail >= 3:
                        self.k = 1
                self._rescale(ratio * h)
                continue
            # accepted
            self.log.append((self.t, h, k, iters, ACCEPTED, err))
            nfail = 0
            ekm1 = float(error_constant(k - 1)) * self._norm(D[k] + d, D[0], y) if k > 1 else None
            ekp1 = (float(error_constant(k + 1)) * self._norm(d - D[k + 1], D[0], y)
                    if k < self.kmax else None)
            D[k + 2] = d - D[k + 1]
            D[k + 1] = d
            for j in range(k, -1, -1):
                D[j] = D[j] + D[j + 1]
            self.t = t_end if last else t1
            self.nconst += 1
            if self.nconst >= k + 2:
                def ratio_of(e, c, q):
                    return 1.0 / max(0.1, c * (e / self.rtol) ** (1.0 / (q + 1)))
                r = ratio_of(err, 1.2, k)
                knew = k
                if ekm1 is not None:
                    rm = ratio_of(ekm1, 1.3, k - 1)
                    if rm > r:
                        r, knew = rm, k - 1
                if ekp1 is not None:
                    rp = ratio_of(ekp1, 1.4, k + 1)
                    if rp > r:
                        r, knew = rp, k + 1
                if r > 1.0:
                    self.k = knew
                    self._rescale(min(r * h, self.hmax))
        return self.D[0]
