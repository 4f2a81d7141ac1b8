"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This module holds the workload recipes only (random draws, spectral shapes and
the coefficient storage order). It holds none of the method's arithmetic: no
quadrature, no Legendre functions, no transforms, no time stepping.

Storage order of one member's coefficients (complex128, m >= 0 only):
    index(l, m) = m*(2N+3-m)/2 + (l-m),   0 <= m <= l <= N,
i.e. m-major, l fastest. The slot (l=0, m=0) is always 0 (the divergence-free
space starts at degree 1). A real velocity field needs
alpha[l,-m] = (-1)^m conj(alpha[l,m]), so negative orders are not stored and the
imaginary part of every m = 0 coefficient is 0.

Spectral recipe (the workloads of the paper's experiments are synthetic
band-limited spectra, Section 5): a stream-function coefficient
    psi[l,m] = scale * x * (l(l+1))^(-1.5) * exp(-l/8)
with x ~ N(0,1) for m = 0 and x = (z1 + i z2)/sqrt(2), z ~ N(0,1) for m > 0,
drawn from numpy.random.default_rng(seed) in storage order. The state
coefficient of the divergence-free basis is alpha = sqrt(l(l+1)) * psi, because
Z[l,m] = (l(l+1))^(-1/2) Curl Y[l,m] and u = Curl psi.

Seeds used by the tests and the benchmark:
    1 initial state, 2 forcing (scale 1e-2), 3 target state, 4 finite-difference
    directions, 5 ensemble viscosities, 6 adjoint cotangents (flat spectrum),
    7 phases of Example 2's random initial flow, 8 flat spectra (every degree
    weighted alike), 100+i ensemble member i.
"""
from __future__ import annotations

import numpy as np

SEED_INITIAL = 1
SEED_FORCING = 2
SEED_TARGET = 3
SEED_DIRECTIONS = 4
SEED_ENSEMBLE_NU = 5
SEED_COTANGENT = 6
SEED_MEMBER0 = 100


def coeff_count(N: int) -> int:
    """Complex slots per member: (N+1)(N+2)/2."""
    return (N + 1) * (N + 2) // 2


def index(N: int, l: int, m: int) -> int:
    """Storage slot of (l, m), 0 <= m <= l <= N."""
    if not (0 <= m <= l <= N):
        raise ValueError(f"(l={l}, m={m}) outside 0 <= m <= l <= {N}")
    return m * (2 * N + 3 - m) // 2 + (l - m)


def degrees_orders(N: int):
    """Arrays (l, m) of length coeff_count(N) in storage order."""
    ls, ms = [], []
    for m in range(N + 1):
        for l in range(m, N + 1):
            ls.append(l)
            ms.append(m)
    return np.array(ls, dtype=np.int64), np.array(ms, dtype=np.int64)


def spectrum(seed: int, N: int, scale: float = 1.0, efold: float = 8.0) -> np.ndarray:
    """State coefficients alpha (complex128, storage order) of the seeded spectrum."""
    rng = np.random.default_rng(seed)
    out = np.zeros(coeff_count(N), dtype=np.complex128)
    k = 0
    for m in range(N + 1):
        for l in range(m, N + 1):
            if l == 0:
                k += 1
                continue
            if m == 0:
                x = complex(rng.standard_normal(), 0.0)
            else:
                z1, z2 = rng.standard_normal(2)
                x = complex(z1, z2) / np.sqrt(2.0)
            lam = float(l * (l + 1))
            psi = scale * x * lam ** -1.5 * np.exp(-l / efold)
            out[k] = np.sqrt(lam) * psi
            k += 1
    return out


def initial_state(N: int) -> np.ndarray:
    return spectrum(SEED_INITIAL, N, 1.0)


def forcing(N: int) -> np.ndarray:
    return spectrum(SEED_FORCING, N, 1e-2)


def target_state(N: int) -> np.ndarray:
    return spectrum(SEED_TARGET, N, 1.0)


def directions(N: int, count: int) -> np.ndarray:
    """count seeded directions of the same spectral shape, shape [count, slots]."""
    return np.stack([spectrum(SEED_DIRECTIONS * 1000 + i, N, 1.0) for i in range(count)])


def cotangent(N: int, index: int = 0) -> np.ndarray:
    """A seeded cotangent with unit-variance entries at every degree (no decay),
    zero at l = 0 and real at m = 0, for adjoint tests."""
    rng = np.random.default_rng(SEED_COTANGENT * 1000 + index)
    ls, ms = degrees_orders(N)
    z = rng.standard_normal((len(ls), 2))
    out = (z[:, 0] + 1j * z[:, 1]).astype(np.complex128)
    out[ms == 0] = z[ms == 0, 0]
    out[ls == 0] = 0.0
    return out


SEED_FLAT = 8


def flat_spectrum(N: int, index: int = 0, scale: float = 1.0) -> np.ndarray:
    """A state with the same law at every degree (no decay): alpha[l,m] = scale * x,
    x ~ N(0,1) for m = 0 and (z1 + i z2)/sqrt(2) for m > 0, zero at l = 0, drawn
    in storage order from default_rng(SEED_FLAT * 1000 + index). Every degree and
    order carries weight, so a full-size comparison sees every coefficient."""
    rng = np.random.default_rng(SEED_FLAT * 1000 + index)
    ls, ms = degrees_orders(N)
    z = rng.standard_normal((len(ls), 2))
    out = ((z[:, 0] + 1j * z[:, 1]) / np.sqrt(2.0)).astype(np.complex128)
    out[ms == 0] = z[ms == 0, 0]
    out[ls == 0] = 0.0
    return scale * out


def grid_noise(seed: int, nlat: int, M: int, fields: int = 2) -> np.ndarray:
    """Seeded N(0,1) grid values [fields][nlat][M] (a field with every scale,
    not divergence-free), for projection tests."""
    return np.random.default_rng(seed).standard_normal((fields, nlat, M))


def ensemble_viscosities(count: int, lo: float = 1e-5, hi: float = 1e-3) -> np.ndarray:
    """nu_i log-uniform in [lo, hi]."""
    rng = np.random.default_rng(SEED_ENSEMBLE_NU)
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=count)


def member_state(i: int, N: int) -> np.ndarray:
    return spectrum(SEED_MEMBER0 + i, N, 1.0)


def ensemble_truncations():
    """The mixed-truncation ensemble: 24 x N=63, 24 x N=127, 16 x N=255."""
    return [63] * 24 + [127] * 24 + [255] * 16


def single_mode(N: int, modes) -> np.ndarray:
    """A state with the given {(l, m): value} entries and zeros elsewhere."""
    out = np.zeros(coeff_count(N), dtype=np.complex128)
    for (l, m), v in modes.items():
        out[index(N, l, m)] = v
    return out


def example1_g(t: float, nu: float):
    """g(t) = nu e^-t (sin 5t + cos 10t) of the manufactured flow of the paper's
    Example 1, and its derivative."""
    e = nu * np.exp(-t)
    s = np.sin(5 * t) + np.cos(10 * t)
    ds = 5 * np.cos(5 * t) - 10 * np.sin(10 * t)
    return e * s, e * (ds - s)


def example1_state(N0: int, N: int, t: float, nu: float, rate: bool = False) -> np.ndarray:
    """Coefficients of the manufactured velocity of Example 1,
    u = t g(t) sum_{L<=N0} [Z_{L,0} + 2 sum_{m>=1} Re Z_{L,m}] + g(t) W1 + (t - 1) g(t) W2,
    W1 = Z_{1,0} + 2 Re Z_{1,1},  W2 = Z_{2,0} + 2 Re(Z_{2,1} + Z_{2,2}),
    in the storage of truncation N >= N0 (2 Re Z_{L,m} is the stored coefficient 1
    at (L, m)); with rate=True the time derivative of those coefficients."""
    g, dg = example1_g(t, nu)
    a1 = g + t * dg if rate else t * g                 # coefficient of the sum
    aw1 = dg if rate else g
    aw2 = (g + (t - 1) * dg) if rate else (t - 1) * g
    out = np.zeros(coeff_count(N), dtype=np.complex128)
    ls, ms = degrees_orders(N)
    out[(ls >= 1) & (ls <= N0)] = a1
    for (l, m) in ((1, 0), (1, 1)):
        out[index(N, l, m)] += aw1
    for (l, m) in ((2, 0), (2, 1), (2, 2)):
        out[index(N, l, m)] += aw2
    return out


SEED_EXAMPLE2 = 7


def example2_state(N: int, nu: float = 1e-4, seed: int = SEED_EXAMPLE2, Lmax: int = 20) -> np.ndarray:
    """Random initial velocity of the paper's Example 2 in the storage of truncation
    N >= Lmax: alpha[L,m] = a_L exp(i phi_m) for 1 <= L <= Lmax, 0 <= m <= L, zero
    above Lmax, with phi_0 = 0, phi_m ~ U(0, 2 pi) for m >= 1 (one phase per order,
    drawn from numpy.random.default_rng(seed) for m = 1..Lmax), a_L = b_L / |b|,
    b_L = 2 / (L + (nu L)^2.5)."""
    if N < Lmax:
        raise ValueError("N must be >= Lmax")
    rng = np.random.default_rng(seed)
    phi = np.concatenate([[0.0], rng.uniform(0.0, 2.0 * np.pi, size=Lmax)])
    L = np.arange(1, Lmax + 1, dtype=np.float64)
    b = 2.0 / (L + (nu * L) ** 2.5)
    a = b / np.linalg.norm(b)
    out = np.zeros(coeff_count(N), dtype=np.complex128)
    for l in range(1, Lmax + 1):
        for m in range(0, l + 1):
            out[index(N, l, m)] = a[l - 1] * np.exp(1j * phi[m])
    return out


def example2_force(t: float) -> float:
    """f_{3,0}(t) of Example 2, the only non-zero forcing coefficient: 1 for
    t <= 10, cos(pi t / 5) exp(-(t - 10) / 5) after."""
    return 1.0 if t <= 10.0 else float(np.cos(np.pi * t / 5.0) * np.exp(-(t - 10.0) / 5.0))


def example2_schedule() -> dict:
    """The same f_{3,0}(t) as parameters of the switched-on decaying oscillation
    s(t) = before (t <= t_on), amp cos(omega t + phase) exp(-decay (t - t_on))."""
    return {"t_on": 10.0, "before": 1.0, "amp": 1.0, "omega": np.pi / 5.0, "phase": 0.0,
            "decay": 0.2}


def as_real_view(alpha: np.ndarray) -> np.ndarray:
    """Interleaved (re, im) float64 view of a complex128 array."""
    return np.ascontiguousarray(alpha).view(np.float64)
