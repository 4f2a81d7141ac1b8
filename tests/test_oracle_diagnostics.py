"""Pins of the oracle's diagnostics of the experiments: the energy spectrum E(L)
(eq. (energy)), the stream function Psi_N (eq. (eq:vort_app)) and the approximate
inertial manifold (eq. (eq:p-p)).

Each is checked against something other than its own formula: quadrature of the
grid velocity (Parseval), the Laplacian relation of the vorticity, the Coriolis
and Stokes operators applied by quadrature, and the degree bound of the product.
"""
import math

import numpy as np
import pytest
import torch

import nse_inputs as I
from oracle import nse_oracle as O


def _state(N, seed=I.SEED_INITIAL):
    return O.to_tensor(I.spectrum(seed, N))


@pytest.mark.parametrize("N", [7, 20])
def test_energy_spectrum_parseval(N):
    S = O.Sphere(N)
    a = _state(N)
    E = O.energy_spectrum(a, N)
    ut, up = S.velocity(a)
    total = float(S.grid.quad(ut * ut + up * up))
    assert abs(float(E.sum()) - total) <= 1e-13 * total
    assert float(E[0]) == 0.0
    # a single degree carries all of the energy in its own bin
    L = 5
    single = torch.where(O.degrees(N) == L, a, torch.zeros_like(a))
    E1 = O.energy_spectrum(single, N)
    ut, up = S.velocity(single)
    assert abs(float(E1[L]) - float(S.grid.quad(ut * ut + up * up))) <= 1e-13 * float(E1[L])
    assert float(E1.sum() - E1[L]) == 0.0


def test_stream_function_laplacian_and_velocity():
    N = 16
    S = O.Sphere(N)
    a = _state(N)
    psi = O.stream_function_psi(S, a)
    # Vort u = xhat Delta Psi_N: Delta Y = -lambda Y, so the Y-coefficients of Psi_N are
    # -lambda^(-1/2) alpha and those of the vorticity lambda^(1/2) alpha
    c = S.analyse_scalar(psi)
    lam = S.lam.clone()
    lam[0] = 1.0
    assert float((c - O.clean(-a / torch.sqrt(lam), N)).abs().max()) < 1e-14
    zeta_c = S.analyse_scalar(S.vorticity(a))
    assert float((-lam * c - zeta_c)[1:].abs().max()) < 1e-13
    # u = -xhat x Grad Psi_N ... in components u_phi = -dPsi/dtheta with the sign of
    # Psi_N: check u_theta = -(1/sin) dPsi_N/dphi against the velocity synthesis by a
    # spectral derivative in longitude
    ut, up = S.velocity(a)
    M = S.grid.M
    k = torch.fft.fftfreq(M, d=1.0 / M)
    dpsi = torch.fft.ifft(1j * k * torch.fft.fft(psi, dim=1), dim=1).real
    assert float((ut + dpsi / S.grid.sin[:, None]).abs().max()) < 1e-12


def test_inertial_manifold_inverts_stokes_and_coriolis():
    N1, Np, nu, omega = 6, 12, 3e-3, 1.3
    S = O.Sphere(Np)
    a = _state(N1)
    f = _state(Np, I.SEED_FORCING) * 0.01
    phi = O.inertial_manifold(S, a, N1, N1, f, nu, omega)
    band = O.degrees(Np) > N1
    assert float(phi[~band].abs().max()) == 0.0
    # (nu A + C) phi, with C applied by quadrature, returns the band part of f - B(u1, u1)
    lhs = nu * S.lam * phi + S.coriolis(phi, omega)
    u1 = O.embed(a, N1, Np, N1)
    b = S.nonlinear(u1, omega) - S.coriolis(u1, omega)       # B alone, by linearity of C
    r = torch.where(band, f - b, torch.zeros_like(f))
    assert float((lhs - O.clean(r, Np)).abs().max()) <= 1e-12 * float(r.abs().max())


def test_inertial_manifold_degree_bound_and_truncation():
    # B(u1, u1) of a field of degree <= N1 has no component above 2 N1: with no forcing
    # the manifold vanishes above 2 N1; and only P_N1 of the input matters
    N1, Np, nu, omega = 5, 14, 1e-3, 1.0
    S = O.Sphere(Np)
    a = _state(9)
    phi = O.inertial_manifold(S, a, 9, N1, None, nu, omega)
    deg = O.degrees(Np)
    assert float(phi[deg > 2 * N1].abs().max()) < 1e-13 * float(phi.abs().max())
    assert float(phi[(deg > N1) & (deg <= 2 * N1)].abs().max()) > 0
    a_cut = O.embed(a, 9, 9, N1)
    phi2 = O.inertial_manifold(S, a_cut, 9, N1, None, nu, omega)
    assert float((phi - phi2).abs().max()) == 0.0
