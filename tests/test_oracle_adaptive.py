"""Pins of the oracle's variable-order, variable-step NDF integrator.

Each check compares with something other than the integrator: exact rational
polynomial samples, the NDF_p formula (ode_disc) solved directly over values,
closed-form solutions of linear and nonlinear test equations.
"""
import math

import numpy as np
from fractions import Fraction

import pytest
import torch

from oracle import ndf_adaptive as A
from oracle import nse_oracle as O


def _poly(coeffs, t):
    return sum(c * t ** i for i, c in enumerate(coeffs))


def _differences(vals):
    """Backward differences nabla^j at the first entry of vals (newest first)."""
    out = []
    cur = list(vals)
    for _ in range(len(vals)):
        out.append(cur[0])
        cur = [cur[i] - cur[i + 1] for i in range(len(cur) - 1)]
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("rho", [0.3, 0.5, 1.0, 1.7, 4.0])
def test_step_change_matrix_exact_on_polynomials(k, rho):
    # a polynomial of degree k sampled at spacing h and rho h: the matrix maps the
    # first set of differences exactly onto the second (rational arithmetic)
    coeffs = [Fraction(3 * i + 1, 7 + i) * (-1) ** i for i in range(k + 1)]
    h = Fraction(1, 8)
    t_n = Fraction(5, 3)
    r = Fraction(rho)
    old = _differences([_poly(coeffs, t_n - q * h) for q in range(k + 1)])
    new = _differences([_poly(coeffs, t_n - q * r * h) for q in range(k + 1)])
    R = A.step_change_matrix(k, rho)
    got = [sum(R[j][i] * old[i] for i in range(k + 1)) for j in range(k + 1)]
    assert got == new
    # upper triangular, y_n unchanged
    assert all(R[j][i] == 0 for j in range(k + 1) for i in range(j))
    assert R[0][0] == 1


def test_error_constants_and_kappa():
    # BDF_k (kappa = 0) has error constant 1/(k+1); NDF_5 is BDF_5
    assert A.error_constant(5) == Fraction(1, 6)
    for k in range(1, 6):
        assert A.error_constant(k) == O.NDF_KAPPA[k] * A.gamma(k) + Fraction(1, k + 1)
    assert A.gamma(3) == Fraction(11, 6)


def _one_step_exact_history(k, h, deriv, exact):
    """One NDF_k step from an exact constant-step history of y(t) (L = n = 0)."""
    z = lambda v: torch.tensor([complex(v)], dtype=torch.complex128)
    integ = A.AdaptiveNDF(torch.zeros(1, dtype=torch.float64), lambda y: torch.zeros_like(y),
                          lambda t: z(deriv(t)), rtol=1e6, atol=1e6, max_order=5, max_newton=1)
    integ.begin(z(exact(0.0)), 0.0)
    vals = [exact(-q * h) for q in range(k + 1)]
    D = _differences(vals)
    integ.D = [z(v) for v in D] + [z(0.0) for _ in range(k + 1, 8)]
    integ.k, integ.h, integ.started, integ.nconst = k, h, True, 0
    return complex(integ.advance(h)[0])


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_one_step_solves_the_ndf_formula(k):
    # y' = (k+1) t^k, exact y = t^(k+1): the step must solve (ode_disc) over values,
    # sum_{m=1}^k (1/m) nabla^m y_{n+1} - kappa_k gamma_k nabla^{k+1} y_{n+1} = h f(t_{n+1})
    h = 0.125
    exact = lambda t: t ** (k + 1)
    deriv = lambda t: (k + 1) * t ** k
    got = _one_step_exact_history(k, h, deriv, exact)
    hh = Fraction(h)
    past = [Fraction(exact(-q * h)) for q in range(k + 1)]   # y_n .. y_{n-k}, exact
    rhs = hh * (k + 1) * hh ** k
    kap, gam = O.NDF_KAPPA[k], A.gamma(k)

    def residual(y1):
        vals = [y1] + past
        d = _differences(vals)
        return sum(Fraction(1, m) * d[m] for m in range(1, k + 1)) - kap * gam * d[k + 1] - rhs

    r0, r1 = residual(Fraction(0)), residual(Fraction(1))
    y1 = -r0 / (r1 - r0)  # the formula is affine in y_{n+1}
    assert abs(got.real - float(y1)) <= 1e-15 * max(1.0, abs(float(y1)))
    # and the local error equals E_k (k+1)! h^(k+1) / ((1 - kappa_k) gamma_k)
    lerr = float(A.error_constant(k) * math.factorial(k + 1) * hh ** (k + 1) / A.alpha_k(k))
    assert abs((got.real - exact(h)) - lerr) <= 1e-13 * abs(lerr) + 1e-17


def _linear_problem(n=12):
    a = torch.logspace(-2, 3, n, dtype=torch.float64)
    c = torch.linspace(0.5, 2.0, n, dtype=torch.float64).to(torch.complex128) * (1 + 0.5j)
    y0 = torch.linspace(1.0, -1.0, n, dtype=torch.float64).to(torch.complex128)

    def exact(t):
        yp = lambda s: c * (a * math.cos(s) + math.sin(s)) / (a * a + 1)
        return (y0 - yp(0.0)) * torch.exp(-a * t) + yp(t)

    forcing = lambda t: c * math.cos(t)
    return a, forcing, y0, exact


@pytest.mark.parametrize("rtol,bound", [(1e-3, 3e-3), (1e-6, 3e-6)])
def test_linear_stiff_system_meets_tolerance(rtol, bound):
    a, forcing, y0, exact = _linear_problem()
    integ = A.AdaptiveNDF(a, lambda y: torch.zeros_like(y), forcing, rtol=rtol, atol=rtol * 1e-3)
    integ.begin(y0, 0.0)
    y = integ.advance(4.0)
    assert integ.t == 4.0
    err = float(((y - exact(4.0)).abs() / exact(4.0).abs().clamp_min(1e-3)).max())
    assert err <= bound
    orders = {rec[2] for rec in integ.log if rec[4] == A.ACCEPTED}
    assert max(orders) >= 3          # the variable order is exercised
    # intermediate stops land exactly and do not change the answer beyond tolerance
    integ2 = A.AdaptiveNDF(a, lambda y: torch.zeros_like(y), forcing, rtol=rtol, atol=rtol * 1e-3)
    integ2.begin(y0, 0.0)
    for t in (0.5, 1.0, 2.5, 4.0):
        y2 = integ2.advance(t)
        assert integ2.t == t
    err2 = float(((y2 - exact(4.0)).abs() / exact(4.0).abs().clamp_min(1e-3)).max())
    assert err2 <= bound


def test_tolerance_proportionality():
    a, forcing, y0, exact = _linear_problem()
    errs = []
    for rtol in (1e-3, 1e-5, 1e-7):
        integ = A.AdaptiveNDF(a, lambda y: torch.zeros_like(y), forcing, rtol=rtol,
                              atol=rtol * 1e-3)
        integ.begin(y0, 0.0)
        y = integ.advance(3.0)
        errs.append(float(((y - exact(3.0)).abs() / exact(3.0).abs().clamp_min(1e-3)).max()))
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10


def test_nonlinear_riccati_with_newton():
    # y' = -y^2, y(0) = y0: y(t) = y0 / (1 + y0 t); n(y) = y^2 iterated by Newton sweeps
    y0 = torch.tensor([1.0 + 0.0j, 2.0 + 0.0j, 0.5 + 0.0j], dtype=torch.complex128)
    integ = A.AdaptiveNDF(torch.zeros(3, dtype=torch.float64), lambda y: y * y, None,
                          rtol=1e-4, atol=1e-8)
    integ.begin(y0, 0.0)
    y = integ.advance(5.0)
    ex = y0 / (1 + 5.0 * y0)
    assert float(((y - ex).abs() / ex.abs()).max()) <= 5e-4
    iters = [rec[3] for rec in integ.log if rec[4] == A.ACCEPTED]
    assert max(iters) >= 2


def test_rejections_recover():
    # a forcing that switches on sharply forces error failures and step reductions
    a = torch.tensor([1.0, 10.0], dtype=torch.float64)
    forcing = lambda t: torch.full((2,), complex(math.tanh(50.0 * (t - 1.0)) + 1.0),
                                   dtype=torch.complex128)
    integ = A.AdaptiveNDF(a, lambda y: torch.zeros_like(y), forcing, rtol=1e-3, atol=1e-6)
    integ.begin(torch.zeros(2, dtype=torch.complex128), 0.0)
    integ.advance(2.0)
    outcomes = [rec[4] for rec in integ.log]
    assert A.ERROR_FAIL in outcomes
    assert integ.t == 2.0


def test_example2_inputs():
    import nse_inputs as I
    N, nu = 30, 1e-4
    a = I.example2_state(N, nu)
    ls, ms = I.degrees_orders(N)
    L = np.arange(1, 21, dtype=np.float64)
    b = 2.0 / (L + (nu * L) ** 2.5)
    aL = b / np.linalg.norm(b)
    for l in range(1, N + 1):
        sel = ls == l
        if l <= 20:
            assert np.allclose(np.abs(a[sel]), aL[l - 1], rtol=1e-15, atol=0)
        else:
            assert not a[sel].any()
    assert not a[ls == 0].any()
    assert np.all(a[ms == 0].imag == 0)
    assert abs(np.sum(aL ** 2) - 1.0) < 1e-15
    # one phase per order, shared by every degree
    for m in range(1, 21):
        ph = np.angle(a[(ms == m) & (ls <= 20)])
        assert np.allclose(ph, ph[0], atol=1e-12)
    assert I.example2_force(10.0) == 1.0
    assert abs(I.example2_force(15.0) - math.cos(3 * math.pi) * math.exp(-1.0)) < 1e-15
