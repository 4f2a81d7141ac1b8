"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a library routine
(numpy, scipy), a closed form, an invariant of the method, brute force on tiny
inputs, or values printed in the paper (tests/golden/).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.special as sp
import torch

import nse_inputs as I
from oracle import nse_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
OMEGA = 2.0 * math.pi


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def _frac(s):
    return Fraction(s)


def _state(N, seed=I.SEED_INITIAL, scale=1.0):
    return O.to_tensor(I.spectrum(seed, N, scale))


def _wsum(N, x, y):
    """Real inner product of two real fields given by their m >= 0 coefficients."""
    w = torch.where(O.orders(N) > 0, 2.0, 1.0)
    return float((w * (x.conj() * y).real).sum())


# --------------------------------------------------------------------------- P1
def test_gauss_legendre_closed_forms():
    rows = _rows("gauss_legendre_small.txt")
    for n in (1, 2, 3):
        mu, w = O.gauss_legendre(n)
        exp = [(float(r[1]), float(r[2])) for r in rows if int(r[0]) == n]
        assert np.allclose(mu.numpy(), [e[0] for e in exp], atol=1e-15, rtol=0)
        assert np.allclose(w.numpy(), [e[1] for e in exp], atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", [24, 48, 96, 192, 384])
def test_gauss_legendre_vs_numpy_and_exactness(n):
    mu, w = O.gauss_legendre(n)
    xn, wn = np.polynomial.legendre.leggauss(n)
    assert np.all(np.diff(mu.numpy()) < 0)
    assert np.abs(mu.numpy()[::-1] - xn).max() < 1e-14
    # numpy's end weights carry ~1e-11 relative error; compare absolutely here and
    # relatively against a 40-digit Newton solve below.
    assert np.abs(w.numpy()[::-1] - wn).max() < 5e-14
    assert abs(float(w.sum()) - 2.0) < 1e-14
    for k in range(0, 2 * n, max(1, (2 * n) // 17)):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(float((w * mu ** k).sum()) - exact) < 1e-13


@pytest.mark.parametrize("n", [24, 96])
def test_gauss_legendre_vs_high_precision(n):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    mu, w = O.gauss_legendre(n)
    for i in range(0, n, max(1, n // 12)):
        x = mpmath.mpf(float(mu[i]))
        for _ in range(3):
            p0, p1 = mpmath.mpf(1), x
            for j in range(2, n + 1):
                p0, p1 = p1, ((2 * j - 1) * x * p1 - (j - 1) * p0) / j
            dp = n * (x * p1 - p0) / (x * x - 1)
            x = x - p1 / dp
        wx = 2 / ((1 - x * x) * dp * dp)
        assert abs(float(mu[i]) - float(x)) < 2e-16
        assert abs(float(w[i]) / float(wx) - 1.0) < 1e-12


# --------------------------------------------------------------------------- P2
@pytest.mark.parametrize("nlat,lmax", [(24, 20), (153, 100)])
def test_legendre_table_vs_scipy(nlat, lmax):
    g = O.Grid(nlat)
    th = np.arccos(g.mu.numpy())
    tab = O.LegendreTables(g, lmax, lmax)
    err = derr = 0.0
    for m in range(0, lmax + 1, 1 if lmax <= 20 else 7):
        for l in range(m, lmax + 1):
            v, d = sp.sph_legendre_p(l, m, th, diff_n=1)
            err = max(err, np.abs(tab.P[m][l - m].numpy() - v).max())
            derr = max(derr, np.abs(tab.dP[m][l - m].numpy() - d).max() / max(1.0, np.abs(d).max()))
    # both sides run degree recurrences up to l = 100: ~l ulps of accumulated rounding
    assert err < 5e-13
    assert derr < 5e-13


def test_discrete_orthonormality_full_table():
    # Q_M(Y[l,m] conj(Y[l',m])) = delta for all l, l' <= N+1 on the grid with M >= 3N+2.
    N = 31
    g = O.Grid(O.min_nlat(N))
    tab = O.LegendreTables(g, N + 1, N + 1)
    for m in range(N + 2):
        P = tab.P[m]
        gram = 2.0 * math.pi * (P * g.w) @ P.T
        assert torch.allclose(gram, torch.eye(P.shape[0], dtype=torch.float64), atol=1e-13)


# the full-size grids: every degree l <= N+1 of the selected orders, up to the
# sectoral end m = N+1 and orders above 400 at N = 511, where the values near the
# poles underflow (sin^m) and the recurrence runs over 500 degrees
@pytest.mark.parametrize("N,orders", [(255, (0, 1, 37, 128, 200, 255, 256)),
                                      (511, (0, 1, 37, 255, 400, 450, 500, 511, 512))])
def test_discrete_orthonormality_full_degree(N, orders):
    g = O.Grid(O.min_nlat(N))
    for m in orders:
        P = O.legendre_order(m, N + 1, g.mu, g.sin)
        gram = 2.0 * math.pi * (P * g.w) @ P.T
        err = float((gram - torch.eye(P.shape[0], dtype=torch.float64)).abs().max())
        assert err < 1e-13, (m, err)


@pytest.mark.parametrize("N", [255, 511])
def test_legendre_high_degree_vs_scipy(N):
    """Pbar[l,m] at the Gauss nodes against scipy's normalised associated Legendre
    function for degrees up to N+1 (the library runs its own recurrence; after
    ~500 degrees both carry ~l ulps of rounding on values up to sqrt((2l+1)/(4 pi)))."""
    g = O.Grid(O.min_nlat(N))
    th = np.arccos(g.mu.numpy())
    for m in (0, 1, 37, N // 2, 400 if N > 400 else N - 1, N, N + 1):
        P = O.legendre_order(m, N + 1, g.mu, g.sin).numpy()
        for l in sorted({m, min(m + 1, N + 1), (m + N + 1) // 2, N, N + 1}):
            if l < m:
                continue
            v = sp.sph_legendre_p(l, m, th)
            assert np.abs(P[l - m] - v).max() < 1e-11, (l, m)


# --------------------------------------------------------------------------- P3
@pytest.mark.parametrize("N", [7, 31])
def test_scalar_and_vector_round_trip(N):
    S = O.Sphere(N)
    a = _state(N)
    c = a * S.slam
    back = S.analyse_scalar(S.synth_scalar(c))
    assert float((back - O.clean(c, N)).abs().max()) < 1e-13 * float(c.abs().max())
    ut, up = S.velocity(a)
    assert float((S.project(ut, up) - O.clean(a, N)).abs().max()) < 1e-13 * float(a.abs().max())


def test_projection_of_solid_body_rotation():
    # u = omega0 sin(theta) phi_hat is Curl psi with psi = omega0 cos(theta) =
    # omega0 sqrt(4 pi/3) Y[1,0]; alpha[1,0] = sqrt(2) psi[1,0] (app_soln_rep).
    N = 6
    S = O.Sphere(N)
    om0 = 0.7
    ut = torch.zeros(S.grid.nlat, S.grid.M, dtype=torch.float64)
    up = om0 * S.grid.sin[:, None].expand(-1, S.grid.M).clone()
    a = S.project(ut, up)
    exp = torch.zeros_like(a)
    exp[1] = om0 * math.sqrt(8.0 * math.pi / 3.0)
    assert float((a - exp).abs().max()) < 1e-14


def test_vorticity_and_velocity_of_single_harmonic_match_scipy():
    # u = Z[l,m] + conj: zeta = sqrt(lambda) (Y + conj Y); u_phi = -lambda^(-1/2) dY/dtheta (+conj).
    N, l, m = 9, 5, 3
    S = O.Sphere(N)
    a = O.to_tensor(I.single_mode(N, {(l, m): 1.0 + 0.5j}))
    th = np.arccos(S.grid.mu.numpy())[:, None]
    ph = S.grid.phi.numpy()[None, :]
    y, dy = sp.sph_harm_y(l, m, th, ph, diff_n=1)
    lam = l * (l + 1)
    coef = 1.0 + 0.5j
    zeta = 2.0 * np.real(coef * math.sqrt(lam) * y)
    uphi = 2.0 * np.real(-coef * dy[..., 0] / math.sqrt(lam))
    utheta = 2.0 * np.real(coef * dy[..., 1] / np.sin(th) / math.sqrt(lam))
    ut, up = S.velocity(a)
    assert np.abs(S.vorticity(a).numpy() - zeta).max() < 1e-13
    assert np.abs(up.numpy() - uphi).max() < 1e-13
    assert np.abs(ut.numpy() - utheta).max() < 1e-13


# --------------------------------------------------------------------------- P4
def test_alias_free_exactness():
    N = 15
    a = _state(N)
    base = O.Sphere(N).nonlinear(a, OMEGA)
    for nlat in (O.min_nlat(N) + 3, 2 * O.min_nlat(N)):
        other = O.Sphere(N, nlat).nonlinear(a, OMEGA)
        assert float((other - base).abs().max()) < 1e-13 * float(base.abs().max())
    aliased = O.Sphere(N, N + 1).nonlinear(a, OMEGA)   # M = 2N + 2 < 3N + 2
    assert float((aliased - base).abs().max()) > 1e-8 * float(base.abs().max())


# --------------------------------------------------------------------------- P5 / P7
def test_single_degree_advection_vanishes():
    N = 12
    rng = np.random.default_rng(7)
    for l in (1, 4, 12):
        modes = {(l, m): complex(rng.standard_normal(), rng.standard_normal() if m else 0.0)
                 for m in range(0, l + 1)}
        a = O.to_tensor(I.single_mode(N, modes))
        S = O.Sphere(N)
        # the cancelling products are of size lambda |alpha|^2
        scale = l * (l + 1) * float(a.abs().max()) ** 2
        assert float(S.nonlinear(a, 0.0).abs().max()) < 1e-14 * scale
        lam = S.lam.clone()
        lam[0] = 1.0
        exp = O.clean(-2.0 * OMEGA * 1j * O.orders(N) * a / lam, N)
        assert float((S.nonlinear(a, OMEGA) - exp).abs().max()) < 1e-14 * scale


def test_coriolis_closed_form_and_invariants():
    N = 20
    S = O.Sphere(N)
    a = _state(N)
    lam = S.lam.clone()
    lam[0] = 1.0
    c = S.coriolis(a, OMEGA)
    exp = O.clean(-2.0 * OMEGA * 1j * O.orders(N) * a / lam, N)
    assert float((c - exp).abs().max()) < 1e-13
    scale = _wsum(N, a.abs(), c.abs() * S.lam)
    assert abs(_wsum(N, a, c)) < 1e-14 * scale
    assert abs(_wsum(N, a * S.lam, c)) < 1e-13 * scale


# --------------------------------------------------------------------------- P6
@pytest.mark.parametrize("l,omega0", [(4, 0.0), (4, 0.5), (7, -0.3)])
def test_rossby_haurwitz_closed_form(l, omega0):
    # Superrotation omega0 plus a degree-l wave: n[l,m] = i m (omega0 (1 - 2/lam) - 2 Omega/lam) alpha.
    N = 10
    rng = np.random.default_rng(l)
    modes = {(1, 0): omega0 * math.sqrt(8 * math.pi / 3)}
    for m in range(0, l + 1):
        modes[(l, m)] = complex(rng.standard_normal(), rng.standard_normal() if m else 0.0)
    a = O.to_tensor(I.single_mode(N, modes))
    S = O.Sphere(N)
    n = S.nonlinear(a, OMEGA)
    lam = float(l * (l + 1))
    exp = torch.zeros_like(a)
    for m in range(0, l + 1):
        k = I.index(N, l, m)
        exp[k] = 1j * m * (omega0 * (1 - 2 / lam) - 2 * OMEGA / lam) * a[k]
    assert float((n - exp).abs().max()) < 1e-13


# --------------------------------------------------------------------------- P8
@pytest.mark.parametrize("N", [15, 31])
def test_energy_and_enstrophy_conservation(N):
    S = O.Sphere(N)
    a = _state(N)
    n = S.nonlinear(a, OMEGA)
    scale = _wsum(N, a.abs() * S.lam, n.abs())
    assert abs(_wsum(N, a, n)) < 1e-13 * scale
    assert abs(_wsum(N, a * S.lam, n)) < 1e-13 * scale
    assert float(n.abs().max()) > 1e-3


# --------------------------------------------------------------------------- P9
def _brute_force_nonlinear(N, a_stored, omega):
    """Galerkin interaction sum over all (R,s), (J,k) basis pairs with scipy harmonics.

    (B(Z_R, Z_J), Z_L) = -sqrt(lam_R / (lam_J lam_L)) (Y_R Grad Y_J, xhat x Grad Y_L),
    evaluated on a 4x oversampled Gauss grid; Coriolis from its closed form.
    """
    nlat = 4 * O.min_nlat(N)
    mu, w = np.polynomial.legendre.leggauss(nlat)
    th = np.arccos(mu)[:, None]
    M = 2 * nlat
    ph = (2 * np.pi * np.arange(M) / M)[None, :]
    modes = [(l, m) for l in range(1, N + 1) for m in range(-l, l + 1)]
    Y, Yt, Yp = {}, {}, {}
    for (l, m) in modes:
        y, dy = sp.sph_harm_y(l, m, th, ph, diff_n=1)
        Y[l, m], Yt[l, m], Yp[l, m] = y, dy[..., 0], dy[..., 1] / np.sin(th)

    def coef(l, m):
        v = a_stored[I.index(N, l, abs(m))]
        return v if m >= 0 else (-1) ** m * np.conj(v)

    wq = (2 * np.pi / M) * w[:, None]
    # zeta-weighted gradient of psi, summed over the field first (bilinear in alpha)
    zeta = sum(coef(R, s) * math.sqrt(R * (R + 1)) * Y[R, s] for (R, s) in modes)
    gpt = sum(coef(J, k) / math.sqrt(J * (J + 1)) * Yt[J, k] for (J, k) in modes)
    gpp = sum(coef(J, k) / math.sqrt(J * (J + 1)) * Yp[J, k] for (J, k) in modes)
    out = np.zeros(I.coeff_count(N), dtype=np.complex128)
    for (L, m) in modes:
        if m < 0:
            continue
        lam = L * (L + 1)
        # xhat x Grad Y = (-Y_phi/sin, Y_theta); the inner product conjugates it
        ip = np.sum(wq * (zeta * (gpt * np.conj(-Yp[L, m]) + gpp * np.conj(Yt[L, m]))))
        out[I.index(N, L, m)] = -ip / math.sqrt(lam) - 2 * omega * 1j * m * coef(L, m) / lam
    return out


@pytest.mark.parametrize("N", [2, 4])
def test_tiny_n_brute_force(N):
    a = I.spectrum(11, N, 1.0)
    exp = _brute_force_nonlinear(N, a, OMEGA)
    got = O.Sphere(N).nonlinear(O.to_tensor(a), OMEGA).numpy()
    assert np.abs(got - exp).max() < 1e-13 * max(1.0, np.abs(exp).max())


# --------------------------------------------------------------------------- P10
def test_longitude_shift_equivariance_and_homogeneity():
    N = 15
    S = O.Sphere(N)
    a = _state(N)
    shift = O.clean(torch.exp(-1j * O.orders(N) * (2 * math.pi / S.grid.M) * 3).to(torch.complex128), N)
    shift[0] = 1.0
    n = S.nonlinear(a, OMEGA)
    n_shift = S.nonlinear(a * shift, OMEGA)
    assert float((n_shift - n * shift).abs().max()) < 1e-13 * float(n.abs().max())
    n0 = S.nonlinear(a, 0.0)
    assert float((S.nonlinear(2.5 * a, 0.0) - 6.25 * n0).abs().max()) < 1e-13 * 6.25 * float(n0.abs().max())


# --------------------------------------------------------------------------- time stepping
def test_ndf_coefficients_match_paper_and_textbook():
    kappa = {int(r[0]): _frac(r[1]) for r in _rows("ndf_kappa.txt")}
    assert kappa == O.NDF_KAPPA
    for r in _rows("bdf_coefficients.txt"):
        q = int(r[0])
        assert O.ndf_coefficients(q, False) == [_frac(x) for x in r[1:]]
    named = {r[0]: [_frac(x) for x in r[1:]] for r in _rows("ndf2_coefficients.txt")}
    assert O.ndf_coefficients(1, True) == named["NDF1"]
    assert O.ndf_coefficients(2, True) == named["NDF2"]


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_ndf_order_conditions(q):
    # sum_j c_j y(t_{n+1} - j h) = h y'(t_{n+1}) exactly for polynomials of degree <= q.
    for with_kappa in (False, True):
        c = O.ndf_coefficients(q, with_kappa)
        assert sum(c) == 0
        assert sum(cj * (-j) for j, cj in enumerate(c)) == 1
        for r in range(2, q + 1):
            assert sum(cj * Fraction(-j) ** r for j, cj in enumerate(c)) == 0


def test_predictor_extrapolates_polynomials():
    for d in range(0, 6):
        pi = O.predictor_coefficients(d)
        for r in range(0, d + 1):
            # y(t) = t^r sampled at t = -i, extrapolated to t = 1
            assert sum(p * Fraction(-i) ** r for i, p in enumerate(pi)) == 1


def test_viscous_decay_order_of_convergence():
    # Omega = 0, one degree, no forcing: alpha(t) = alpha(0) exp(-nu lambda t).
    N, l, nu, T = 8, 6, 0.05, 0.4
    S = O.Sphere(N)
    a0 = O.to_tensor(I.single_mode(N, {(l, 2): 0.3 - 0.4j, (l, 0): 0.2}))
    for p, expect in ((1, 2.0), (2, 4.0)):
        errs = []
        for steps in (40, 80):
            st = O.Stepper(S, nu, 0.0, T / steps, order=p)
            hist = st.run(a0, torch.zeros_like(a0), steps)
            exact = a0 * math.exp(-nu * l * (l + 1) * T)
            errs.append(float((hist[0] - exact).abs().max()))
        assert abs(errs[0] / errs[1] - expect) < 0.35 * expect


def test_rossby_haurwitz_viscous_wave_in_time():
    # alpha(t) = alpha(0) exp(-nu lam t - i m [(1 - 2/lam) w0 (1 - e^{-2 nu t})/(2 nu) - 2 Omega t/lam]),
    # alpha[1,0](t) = alpha[1,0](0) e^{-2 nu t}; second-order convergence for NDF2.
    N, l, m, nu, w0, T = 6, 4, 4, 1e-3, 0.5, 0.5
    S = O.Sphere(N)
    a0 = O.to_tensor(I.single_mode(N, {(1, 0): w0 * math.sqrt(8 * math.pi / 3), (l, m): 0.5}))
    lam = l * (l + 1)
    phase = (1 - 2 / lam) * w0 * (1 - math.exp(-2 * nu * T)) / (2 * nu) - 2 * OMEGA * T / lam
    exact = a0.clone()
    exact[I.index(N, l, m)] = 0.5 * complex(math.exp(-nu * lam * T)) * np.exp(-1j * m * phase)
    exact[I.index(N, 1, 0)] = a0[I.index(N, 1, 0)] * math.exp(-2 * nu * T)
    errs = []
    for steps in (50, 100, 200):
        st = O.Stepper(S, nu, OMEGA, T / steps, order=2)
        hist = st.run(a0, torch.zeros_like(a0), steps)
        errs.append(float((hist[0] - exact).abs().max()))
    assert errs[-1] < 1e-4
    assert 3.3 < errs[1] / errs[2] < 4.7


def test_forcing_steady_state():
    # Linear, Omega = 0, single degree: the fixed point is alpha = f / (nu lambda).
    N, l = 5, 3
    S = O.Sphere(N)
    f = O.to_tensor(I.single_mode(N, {(l, 1): 0.02 + 0.01j}))
    st = O.Stepper(S, 0.5, 0.0, 0.05, order=2)
    hist = st.run(torch.zeros_like(f), f, 400)
    exp = f / (0.5 * l * (l + 1))
    assert float((hist[0] - exp).abs().max()) < 1e-12


# --------------------------------------------------------------------------- P12 / adjoint
def test_misfit_grid_equals_parseval():
    N = 12
    S = O.Sphere(N)
    a, t = _state(N), _state(N, I.SEED_TARGET)
    g = float(O.misfit_grid(S, a, t))
    s = float(O.misfit_spectral(N, a, t))
    assert abs(g - s) < 1e-13 * s


def test_oracle_gradient_vs_central_differences():
    N, steps = 7, 5
    S = O.Sphere(N)
    a0 = _state(N)
    f = _state(N, I.SEED_FORCING, 1e-2)
    tgt = _state(N, I.SEED_TARGET)
    st = O.Stepper(S, 1e-3, OMEGA, 1e-2, order=2)

    def loss_of(real_view):
        a = O.clean(torch.view_as_complex(real_view), N)
        hist = st.run(a, f, steps)
        return O.misfit_spectral(N, hist[0], tgt)

    x = torch.view_as_real(a0).clone().requires_grad_(True)
    L = loss_of(x)
    (g,) = torch.autograd.grad(L, x)
    rng = np.random.default_rng(3)
    for _ in range(4):
        d = torch.view_as_real(O.clean(O.to_tensor(I.spectrum(int(rng.integers(1 << 30)), N)), N))
        eps = 1e-6
        with torch.no_grad():
            fd = (loss_of(x + eps * d) - loss_of(x - eps * d)) / (2 * eps)
        ad = float((g * d).sum())
        assert abs(fd - ad) < 1e-7 * max(1.0, abs(ad))


def test_oracle_vjp_dot_product_exact():
    """n and one step are quadratic in the state, so the central difference
    (F(a + d) - F(a - d)) / 2 equals J d up to rounding, for any size of d:
    <J d, c> must equal <d, J^T c> from autograd to rounding."""
    N = 9
    S = O.Sphere(N)
    a = O.to_tensor(I.initial_state(N))
    d = O.to_tensor(I.directions(N, 1)[0])
    c = O.to_tensor(I.cotangent(N))
    x = a.clone().requires_grad_(True)
    (g,) = torch.autograd.grad((c.conj() * S.nonlinear(x, OMEGA)).real.sum(), x)
    with torch.no_grad():
        jd = (S.nonlinear(a + d, OMEGA) - S.nonlinear(a - d, OMEGA)) / 2
    lhs, rhs = float((jd.conj() * c).real.sum()), float((d.conj() * g).real.sum())
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)

    st = O.Stepper(S, 1e-3, OMEGA, 1e-2, order=3)
    f = O.to_tensor(I.forcing(N))
    hist = [O.to_tensor(I.member_state(j, N)) for j in range(4)]
    dh = [O.to_tensor(I.directions(N, 5)[j + 1]) for j in range(4)]
    ch = [O.to_tensor(I.cotangent(N, j)) for j in range(4)]
    xs = [h.clone().requires_grad_(True) for h in hist]
    new = st.step(xs, f, 4)
    gs = torch.autograd.grad(sum((cj.conj() * y).real.sum() for cj, y in zip(ch, new)), xs,
                             allow_unused=True)
    with torch.no_grad():
        up = st.step([h + e for h, e in zip(hist, dh)], f, 4)
        dn = st.step([h - e for h, e in zip(hist, dh)], f, 4)
    lhs = sum(float(((u - v) / 2).conj().mul(cj).real.sum()) for u, v, cj in zip(up, dn, ch))
    rhs = sum(float((e.conj() * gj).real.sum()) for e, gj in zip(dh, gs) if gj is not None)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


# --------------------------------------------------------------------------- Example 1
def _example1_run(N, nu, dt, T, omega=OMEGA):
    """The oracle's NDF2 trajectory of the manufactured flow of Example 1, with the
    force f(t) = alpha'(t) + nu lambda alpha(t) + n(alpha(t)) of the exact coefficients."""
    S = O.Sphere(N)
    st = O.Stepper(S, nu, omega, dt, order=2)
    a0 = O.to_tensor(I.example1_state(N, N, 0.0, nu))
    hist = [a0] + [torch.zeros_like(a0) for _ in range(2)]
    steps = int(round(T / dt))
    for k in range(steps):
        t1 = (k + 1) * dt
        ae = O.to_tensor(I.example1_state(N, N, t1, nu))
        f = O.to_tensor(I.example1_state(N, N, t1, nu, rate=True)) + nu * S.lam * ae \
            + S.nonlinear(ae, omega)
        hist = st.step(hist, O.clean(f, N), k)
    exact = O.to_tensor(I.example1_state(N, N, steps * dt, nu))
    return float((hist[0] - exact).abs().norm() / exact.abs().norm())


def test_example1_manufactured_solution_second_order():
    """Example 1 (manufactured exact solution, nu = 0.1 chosen since the paper does not
    state it): the NDF2 error at T = 0.2 falls by 4 when the step halves, and the
    generator's time derivative matches central differences of the coefficients."""
    N, nu = 6, 0.1
    t, d = 0.37, 1e-5
    num = (I.example1_state(N, N, t + d, nu) - I.example1_state(N, N, t - d, nu)) / (2 * d)
    assert np.abs(num - I.example1_state(N, N, t, nu, rate=True)).max() < 1e-8
    e1 = _example1_run(N, nu, 4e-3, 0.2)
    e2 = _example1_run(N, nu, 2e-3, 0.2)
    assert e2 < 1e-3
    assert 3.3 < e1 / e2 < 4.7
