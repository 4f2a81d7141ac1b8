"""FP64 CPU oracle of the pseudospectral quadrature method for the Navier-Stokes
equations on the rotating unit sphere.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import this module. The product path (the HIP library and its
Python binding) never calls it, and shares no code, table or constant with it.

Everything here is plain and slow on purpose: torch CPU float64/complex128, a
Python loop over the azimuthal order m, a dense explicit DFT matrix in longitude
(no FFT) and direct quadrature sums. The nonlinear term is evaluated in the vector
weak form of the paper, not in the scalar advective form the GPU path uses.

Conventions (paper Section 2, eqs. (Curl), (stok_eig), (sph_har); Section 3,
(quadrule)):
  * theta is colatitude, mu = cos(theta), phi longitude, dS = sin(theta) dtheta dphi.
  * Y[l,m] = Pbar[l,m](mu) exp(i m phi) with the Condon-Shortley phase and
    int_{-1}^{1} Pbar^2 dmu = 1/(2 pi) (orthonormal on the sphere).
  * Curl v = -xhat x Grad v, Z[l,m] = lambda_l^(-1/2) Curl Y[l,m], lambda_l = l(l+1).
    In (theta, phi) components Z[l,m] = lambda^(-1/2) (Y_phi / sin(theta), -Y_theta).
  * The velocity is u = sum alpha[l,m] Z[l,m] over 1 <= l <= N, |m| <= l, with
    alpha[l,-m] = (-1)^m conj(alpha[l,m]); only m >= 0 is stored (storage order of
    nse_inputs), so every m > 0 term counts twice (2 Re) in a grid sum.
  * The grid is M/2 Gauss-Legendre latitudes (mu descending, north first) times M
    equispaced longitudes phi_j = 2 pi j / M, j = 0..M-1 (the same point set as the
    paper's q = 1..M); Q_M(g) = (2 pi / M) sum_j sum_p w_p g(theta_p, phi_j).

Readings of the paper taken here (each is also listed with its reason in the
design notes of the repository):
  * Sign of the nonlinear term: from (short_nonlin1), (Curl) and (stok_eig),
    B(u,u) + C u = (zeta + 2 Omega cos(theta)) xhat x u up to a surface gradient,
    which is orthogonal to every Z[l,m]. The printed interaction formula
    (eval_nonlin1) carries the opposite overall sign; the Rossby-Haurwitz closed
    form in the tests fixes the sign used here.
  * The Coriolis term is evaluated together with the advection (absolute vorticity),
    which is exactly equal to the diagonal closed form (Coriolis_ZLm).
  * Time stepping: the NDF_p formula (ode_disc) at a fixed step h, the nonlinear term
    at the extrapolated predictor, the Stokes term implicit and diagonal, with
    `newton_iters` fixed-point sweeps; order ramp-up q = min(p, k+1) with kappa_q only
    once q+1 past states exist.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import torch

F64 = torch.float64
C128 = torch.complex128

# ---------------------------------------------------------------------------
# Index helpers (storage order of one member: m-major, l fastest, m >= 0).
# ---------------------------------------------------------------------------


def coeff_count(N: int) -> int:
    return (N + 1) * (N + 2) // 2


def m_offset(N: int, m: int) -> int:
    return m * (2 * N + 3 - m) // 2


def split_by_m(alpha: torch.Tensor, N: int):
    """List over m of the coefficient vectors alpha[m..N, m]."""
    return [alpha[m_offset(N, m): m_offset(N, m) + N + 1 - m] for m in range(N + 1)]


def join_by_m(parts) -> torch.Tensor:
    return torch.cat(list(parts))


def degrees(N: int) -> torch.Tensor:
    return torch.cat([torch.arange(m, N + 1, dtype=F64) for m in range(N + 1)])


def orders(N: int) -> torch.Tensor:
    return torch.cat([torch.full((N + 1 - m,), float(m), dtype=F64) for m in range(N + 1)])


def stokes_eigenvalues(N: int) -> torch.Tensor:
    """lambda_l = l(l+1) per storage slot (stok_eig)."""
    l = degrees(N)
    return l * (l + 1.0)


def clean(alpha: torch.Tensor, N: int) -> torch.Tensor:
    """Zero the (0,0) slot and the imaginary part of every m = 0 coefficient."""
    out = alpha.clone()
    m0 = slice(0, N + 1)
    out[m0] = out[m0].real.to(C128)
    out[0] = 0.0
    return out


# ---------------------------------------------------------------------------
# Quadrature (Section 3, (quadrule)).
# ---------------------------------------------------------------------------


def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes (descending, in (-1, 1)) and weights.

    Newton's method on the Legendre polynomial P_n, evaluated by its three-term
    recurrence, from the asymptotic guesses cos(pi (k - 1/4)/(n + 1/2)).
    Weights w = 2 / ((1 - x^2) P_n'(x)^2), with 1 - x^2 formed as (1 - x)(1 + x).
    """
    k = torch.arange(1, n + 1, dtype=F64)
    x = torch.cos(math.pi * (k - 0.25) / (n + 0.5))
    for it in range(100):
        p_prev = torch.ones_like(x)
        p = x.clone()
        for j in range(2, n + 1):
            p_prev, p = p, ((2 * j - 1) * x * p - (j - 1) * p_prev) / j
        dp = n * (p_prev - x * p) / ((1.0 - x) * (1.0 + x))
        dx = p / dp
        x = x - dx
        if float(dx.abs().max()) < 1e-16:
            break
    p_prev = torch.ones_like(x)
    p = x.clone()
    for j in range(2, n + 1):
        p_prev, p = p, ((2 * j - 1) * x * p - (j - 1) * p_prev) / j
    dp = n * (p_prev - x * p) / ((1.0 - x) * (1.0 + x))
    w = 2.0 / ((1.0 - x) * (1.0 + x) * dp * dp)
    return x, w


class Grid:
    """Gauss-rectangle grid of (quadrule): nlat = M/2 latitudes, nlon = M longitudes."""

    def __init__(self, nlat: int):
        if nlat < 1:
            raise ValueError("nlat must be positive")
        self.nlat = nlat
        self.M = 2 * nlat
        self.mu, self.w = gauss_legendre(nlat)
        # (1 - mu)(1 + mu) keeps full relative accuracy next to the poles
        self.sin = torch.sqrt((1.0 - self.mu) * (1.0 + self.mu))
        self.phi = 2.0 * math.pi * torch.arange(self.M, dtype=F64) / self.M

    def quad(self, g: torch.Tensor) -> torch.Tensor:
        """Q_M(g) for a grid field g[p, j] (real or complex)."""
        return (2.0 * math.pi / self.M) * (self.w.to(g.dtype) @ g.sum(dim=1))


def min_nlat(N: int) -> int:
    """Smallest nlat with M = 2 nlat >= 3N + 2 (M_choice, M even)."""
    return (3 * N + 2 + 1) // 2


# ---------------------------------------------------------------------------
# Normalised associated Legendre functions (sph_har).
# ---------------------------------------------------------------------------


def legendre_order(m: int, lmax: int, mu: torch.Tensor, sin: torch.Tensor) -> torch.Tensor:
    """Pbar[l, m](mu) for l = m..lmax as a tensor [lmax - m + 1, len(mu)].

    Textbook normalised recurrences:
      Pbar[0,0] = 1/sqrt(4 pi),
      Pbar[m,m] = -sqrt((2m+1)/(2m)) sin Pbar[m-1,m-1]          (Condon-Shortley),
      Pbar[m+1,m] = sqrt(2m+3) mu Pbar[m,m],
      Pbar[l,m] = a(l,m) (mu Pbar[l-1,m] - Pbar[l-2,m] / a(l-1,m)),
      a(l,m) = sqrt((4 l^2 - 1) / (l^2 - m^2)).
    Values below the double range near the poles flush to zero.
    """
    if lmax < m:
        return torch.zeros((0, mu.numel()), dtype=F64)
    pmm = torch.full_like(mu, 1.0 / math.sqrt(4.0 * math.pi))
    for k in range(1, m + 1):
        pmm = -math.sqrt((2 * k + 1) / (2 * k)) * sin * pmm
    rows = [pmm]
    if lmax > m:
        rows.append(math.sqrt(2 * m + 3) * mu * pmm)
    for l in range(m + 2, lmax + 1):
        a_l = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
        a_lm1 = math.sqrt((4.0 * (l - 1) ** 2 - 1.0) / ((l - 1) ** 2 - m * m))
        rows.append(a_l * (mu * rows[-1] - rows[-2] / a_lm1))
    return torch.stack(rows)


class LegendreTables:
    """Pbar[l,m](mu_p) and dPbar/dtheta for m = 0..mmax, l = m..lmax on a grid.

    The theta-derivative uses the ladder identity in the order m,
      dPbar[l,m]/dtheta = (sqrt((l-m)(l+m+1)) Pbar[l,m+1] - sqrt((l+m)(l-m+1)) Pbar[l,m-1]) / 2,
    with Pbar[l,-1] = -Pbar[l,1] (Condon-Shortley), so it draws on the neighbouring
    orders and not on the degree recurrence.
    """

    def __init__(self, grid: Grid, lmax: int, mmax: int):
        self.lmax, self.mmax = lmax, mmax
        mu, s = grid.mu, grid.sin
        full = [legendre_order(m, lmax, mu, s) for m in range(min(mmax + 1, lmax) + 1)]
        while len(full) < mmax + 2:
            full.append(torch.zeros((0, mu.numel()), dtype=F64))
        self.P = full[: mmax + 1]
        self.dP = []
        for m in range(mmax + 1):
            rows = []
            for l in range(m, lmax + 1):
                up = full[m + 1][l - (m + 1)] if l >= m + 1 else torch.zeros_like(mu)
                if m == 0:
                    down = -full[1][l - 1] if l >= 1 else torch.zeros_like(mu)
                else:
                    down = full[m - 1][l - (m - 1)]
                rows.append(0.5 * (math.sqrt((l - m) * (l + m + 1)) * up
                                   - math.sqrt((l + m) * (l - m + 1)) * down))
            self.dP.append(torch.stack(rows) if rows else torch.zeros((0, mu.numel()), dtype=F64))


# ---------------------------------------------------------------------------
# Direct synthesis and quadrature analysis (no FFT).
# ---------------------------------------------------------------------------


def _dft_synthesis_matrix(grid: Grid, mmax: int) -> torch.Tensor:
    """E[m, j] = c_m exp(i m phi_j), c_0 = 1, c_m = 2 for m > 0 (real-field sum)."""
    m = torch.arange(mmax + 1, dtype=F64)
    E = torch.exp(1j * torch.outer(m, grid.phi).to(C128))
    c = torch.full((mmax + 1,), 2.0, dtype=F64)
    c[0] = 1.0
    return E * c[:, None].to(C128)


def _dft_analysis_matrix(grid: Grid, mmax: int) -> torch.Tensor:
    """A[j, m] = (2 pi / M) exp(-i m phi_j)."""
    m = torch.arange(mmax + 1, dtype=F64)
    return (2.0 * math.pi / grid.M) * torch.exp(-1j * torch.outer(grid.phi, m).to(C128))


class Sphere:
    """Truncation N on a Gauss-rectangle grid with nlat latitudes (M = 2 nlat)."""

    def __init__(self, N: int, nlat: int | None = None):
        self.N = N
        self.grid = Grid(nlat if nlat is not None else min_nlat(N))
        self.tab = LegendreTables(self.grid, N, N)
        self.Es = _dft_synthesis_matrix(self.grid, N)
        self.Ea = _dft_analysis_matrix(self.grid, N)
        self.lam = stokes_eigenvalues(N)
        lam = self.lam.clone()
        lam[0] = 1.0
        self.rlam = 1.0 / torch.sqrt(lam)       # lambda^(-1/2), slot (0,0) unused
        self.slam = torch.sqrt(self.lam)        # lambda^(+1/2)

    # -- scalar fields -------------------------------------------------------
    def synth_scalar(self, c: torch.Tensor) -> torch.Tensor:
        """g = sum c[l,m] Y[l,m] (real field) on the grid, [nlat, M]."""
        N = self.N
        parts = split_by_m(c, N)
        G = torch.stack([parts[m] @ self.tab.P[m].to(C128) for m in range(N + 1)], dim=1)
        return (G @ self.Es).real

    def analyse_scalar(self, g: torch.Tensor) -> torch.Tensor:
        """(g, Y[l,m])_M for 0 <= m <= l <= N (discrete inner product (disc_ip))."""
        N = self.N
        G = g.to(C128) @ self.Ea                      # [nlat, N+1]
        wG = G * self.grid.w[:, None].to(C128)
        return join_by_m(self.tab.P[m].to(C128) @ wG[:, m] for m in range(N + 1))

    # -- divergence-free vector fields ---------------------------------------
    def velocity(self, alpha: torch.Tensor):
        """(u_theta, u_phi) of u = sum alpha Z on the grid."""
        N = self.N
        a = split_by_m(alpha * self.rlam, N)
        s = self.grid.sin.to(C128)[:, None]
        Gt, Gp = [], []
        for m in range(N + 1):
            # Z components: lambda^(-1/2) (i m Pbar / sin, -dPbar/dtheta) e^{i m phi}
            Gt.append(a[m] @ self.tab.P[m].to(C128) * (1j * m))
            Gp.append(-(a[m] @ self.tab.dP[m].to(C128)))
        Gt = torch.stack(Gt, dim=1) / s
        Gp = torch.stack(Gp, dim=1)
        return (Gt @ self.Es).real, (Gp @ self.Es).real

    def vorticity(self, alpha: torch.Tensor) -> torch.Tensor:
        """zeta = xhat . Curln u = sum lambda^(1/2) alpha Y (Vort Z = lambda^(1/2) xhat Y)."""
        return self.synth_scalar(alpha * self.slam)

    def stream_function(self, alpha: torch.Tensor) -> torch.Tensor:
        """psi with u = Curl psi: psi = sum lambda^(-1/2) alpha Y (the paper's Psi_N is -psi)."""
        return self.synth_scalar(alpha * self.rlam)

    def project(self, v_theta: torch.Tensor, v_phi: torch.Tensor) -> torch.Tensor:
        """(v, Z[l,m])_M = Q_M(v . conj(Z[l,m])) for 1 <= l <= N (disc_vec_orth_proj)."""
        N = self.N
        Vt = v_theta.to(C128) @ self.Ea
        Vp = v_phi.to(C128) @ self.Ea
        w = self.grid.w.to(C128)
        s = self.grid.sin.to(C128)
        out = []
        for m in range(N + 1):
            # conj(Z) = lambda^(-1/2) (-i m Pbar / sin, -dPbar/dtheta) e^{-i m phi}
            ct = (w * (-1j * m) / s * Vt[:, m])
            cp = -(w * Vp[:, m])
            out.append(self.tab.P[m].to(C128) @ ct + self.tab.dP[m].to(C128) @ cp)
        res = join_by_m(out) * self.rlam
        return res

    # -- the hot-path quantity -----------------------------------------------
    def nonlinear(self, alpha: torch.Tensor, omega: float) -> torch.Tensor:
        """n[l,m] = (B(u,u) + C u, Z[l,m])_M (app1_weak_form, B and C terms).

        B(u,u) + C u = (zeta + 2 Omega cos(theta)) xhat x u plus a surface gradient
        (short_nonlin1, (C)); xhat x u = (-u_phi, u_theta).
        """
        ut, up = self.velocity(alpha)
        za = self.vorticity(alpha) + 2.0 * omega * self.grid.mu[:, None]
        return clean(self.project(-za * up, za * ut), self.N)

    def coriolis(self, alpha: torch.Tensor, omega: float) -> torch.Tensor:
        """(C u, Z[l,m])_M with (C v)(x) = 2 Omega cos(theta) xhat x v ((C))."""
        ut, up = self.velocity(alpha)
        f = 2.0 * omega * self.grid.mu[:, None]
        return clean(self.project(-f * up, f * ut), self.N)


# ---------------------------------------------------------------------------
# Time stepping (ode_disc).
# ---------------------------------------------------------------------------

NDF_KAPPA = {1: Fraction(-185, 1000), 2: Fraction(-1, 9), 3: Fraction(-823, 10000),
             4: Fraction(-415, 10000), 5: Fraction(0)}


def _binom(n: int, k: int) -> int:
    return math.comb(n, k)


def backward_difference(order: int):
    """Coefficients d_j of nabla^order y_{n+1} = sum_j d_j y_{n+1-j}."""
    return [Fraction((-1) ** j * _binom(order, j)) for j in range(order + 1)]


def ndf_coefficients(q: int, with_kappa: bool):
    """c_j of sum_{m=1}^q (1/m) nabla^m y_{n+1} - kappa_q gamma_q nabla^{q+1} y_{n+1}.

    With these, (ode_disc) reads sum_j c_j y_{n+1-j} = h F(t_{n+1}, y_{n+1}).
    gamma_q = sum_{j=1}^q 1/j. Without kappa the formula is BDF_q.
    """
    length = q + 2 if with_kappa else q + 1
    c = [Fraction(0)] * length
    for m in range(1, q + 1):
        for j, d in enumerate(backward_difference(m)):
            c[j] += Fraction(1, m) * d
    if with_kappa:
        gamma = sum(Fraction(1, j) for j in range(1, q + 1))
        for j, d in enumerate(backward_difference(q + 1)):
            c[j] -= NDF_KAPPA[q] * gamma * d
    return c


def predictor_coefficients(d: int):
    """pi_i of sum_{j=0}^d nabla^j y_n = sum_i pi_i y_{n-i} (extrapolation)."""
    pi = [Fraction(0)] * (d + 1)
    for j in range(d + 1):
        for i, v in enumerate(backward_difference(j)):
            pi[i] += v
    return pi


def step_scheme(k: int, p: int):
    """(c, pi) used at global step index k (k = 0 is the first step) for order p."""
    q = min(p, k + 1)
    with_kappa = k >= q and NDF_KAPPA[q] != 0
    c = ndf_coefficients(q, with_kappa)
    pi = predictor_coefficients(min(q, k))
    return c, pi


class Stepper:
    """Fixed-step NDF_p integrator of d alpha/dt = f - nu lambda alpha - n(alpha)."""

    def __init__(self, sphere: Sphere, nu: float, omega: float, dt: float, order: int = 2,
                 newton_iters: int = 1):
        if not (1 <= order <= 5):
            raise ValueError("order must be 1..5")
        self.S, self.nu, self.omega, self.dt = sphere, nu, omega, dt
        self.p, self.K = order, newton_iters

    def step(self, hist, forcing: torch.Tensor, k: int):
        """One step. hist[0] is the newest state; returns the new history list."""
        c, pi = step_scheme(k, self.p)
        h = self.dt
        pred = sum(float(pi[i]) * hist[i] for i in range(len(pi)))
        rhs_hist = sum(float(c[j]) * hist[j - 1] for j in range(1, len(c)))
        denom = float(c[0]) + h * self.nu * self.S.lam
        a = pred
        for _ in range(self.K):
            n = self.S.nonlinear(a, self.omega)
            a = clean((h * (forcing - n) - rhs_hist) / denom, self.S.N)
        depth = self.p + 1
        new = [a] + list(hist[: depth - 1])
        while len(new) < depth:
            new.append(torch.zeros_like(a))
        return new

    def run(self, alpha0: torch.Tensor, forcing: torch.Tensor, nsteps: int, step0: int = 0,
            hist=None):
        if hist is None:
            hist = [alpha0] + [torch.zeros_like(alpha0) for _ in range(self.p)]
        for k in range(step0, step0 + nsteps):
            hist = self.step(hist, forcing, k)
        return hist


# ---------------------------------------------------------------------------
# Diagnostics of the experiments (Section 5.2 and 5.3).
# ---------------------------------------------------------------------------


def energy_spectrum(alpha: torch.Tensor, N: int) -> torch.Tensor:
    """E(L) = sum_{|m| <= L} |alpha[L,m]|^2 for L = 0..N (energy); the stored m > 0
    coefficient stands for m and -m."""
    w = torch.where(orders(N) > 0, 2.0, 1.0).to(F64)
    E = torch.zeros(N + 1, dtype=F64)
    E.index_add_(0, degrees(N).long(), w * alpha.abs() ** 2)
    return E


def stream_function_psi(sphere: "Sphere", alpha: torch.Tensor) -> torch.Tensor:
    """Psi_N = -sum lambda^(-1/2) alpha[L,m] Y[L,m] on the grid (eq:vort_app)."""
    return -sphere.stream_function(alpha)


def embed(alpha: torch.Tensor, n_src: int, n_dst: int, lmax: int) -> torch.Tensor:
    """The coefficients of degree <= lmax of a truncation-n_src state, stored in
    truncation n_dst (zero elsewhere): the orthogonal projection P_lmax."""
    out = torch.zeros(coeff_count(n_dst), dtype=C128)
    for m in range(min(n_src, n_dst, lmax) + 1):
        for l in range(m, min(n_src, n_dst, lmax) + 1):
            out[m_offset(n_dst, m) + l - m] = alpha[m_offset(n_src, m) + l - m]
    return out


def inertial_manifold(sphere: "Sphere", alpha: torch.Tensor, n_src: int, N1: int,
                      forcing, nu: float, omega: float) -> torch.Tensor:
    """Phi = (nu A + C)^(-1) (P_N' - P_N1) [f - B(u1, u1)], u1 = P_N1 u (eq:p-p),
    N' = sphere.N. B is the advection term alone (the Coriolis part is the C of the
    inverse); (nu A + C) is diagonal on Z[L,m]: nu lambda_L - 2 i Omega m / lambda_L
    ((stok_eig), (Coriolis_ZLm))."""
    N = sphere.N
    u1 = embed(alpha, n_src, N, N1)
    b = sphere.nonlinear(u1, 0.0)
    r = -b if forcing is None else forcing - b
    lam = sphere.lam.clone()
    lam[0] = 1.0
    diag = nu * lam - 2j * omega * orders(N) / lam
    band = degrees(N) > N1
    return clean(torch.where(band, r / diag, torch.zeros_like(r)), N)


# ---------------------------------------------------------------------------
# Misfit of the final state.
# ---------------------------------------------------------------------------


def misfit_grid(sphere: Sphere, alpha: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """0.5 Q_M(|u - u_target|^2) over the quadrature grid."""
    ut, up = sphere.velocity(alpha - target)
    return 0.5 * sphere.grid.quad(ut * ut + up * up)


def misfit_spectral(N: int, alpha: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """0.5 sum over all (l, |m| <= l) of |alpha - target|^2 (m > 0 counted twice)."""
    d = (alpha - target)
    w = torch.where(orders(N) > 0, 2.0, 1.0).to(F64)
    return 0.5 * (w * (d.real ** 2 + d.imag ** 2)).sum()


def to_tensor(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a), dtype=C128)
