"""Diagnostics of the experiments on the GPU against the oracle: the energy spectrum
E(L) (eq. (energy)), the stream function Psi_N (eq. (eq:vort_app)) and the
approximate inertial manifold (eq. (eq:p-p)), through the C ABI. Bar 1e-12
relative (FP64 path); for the manifold every coefficient against the largest
coefficient of the band (N1, N'], on inputs whose product fills that band."""
import math
import os

import numpy as np
import pytest
import torch

import nse_inputs as I
import paper_1009_3308_amd as pkg
from oracle import nse_oracle as O

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1009_3308_amd import build
        build.build()
    torch.cuda.set_device(0)


def test_energy_spectrum_members():
    Ns = (31, 63, 7)
    _say(f"case energy spectrum N={Ns}")
    s = pkg.Sphere([(N, 0, 1e-3) for N in Ns], omega=2 * math.pi, dt=1e-3)
    a = s.new_state()
    states = [I.member_state(i, N) for i, N in enumerate(Ns)]
    for i, st in enumerate(states):
        a[s.member_slice(i)] = pkg.to_device(st)
    E = s.energy_spectrum(a).cpu()
    off = 0
    for N, st in zip(Ns, states):
        ref = O.energy_spectrum(O.to_tensor(st), N)
        got = E[off:off + N + 1]
        assert float((got - ref).abs().max()) <= 1e-14 * float(ref.max())
        off += N + 1
    s.close()


@pytest.mark.parametrize("N,prec", [(31, "fp64"), (255, "fp64"), (63, "fp32"), (63, "bf16x3")])
def test_stream_function(N, prec):
    _say(f"case stream function N={N} {prec}")
    s = pkg.Sphere([(N, 0, 1e-3)], omega=2 * math.pi, dt=1e-3, precision=prec)
    a = I.initial_state(N)
    ad = pkg.to_device(a)
    g = s.synthesize_psi(ad)[0]
    plain = s.synthesize(ad)[0]
    S = O.Sphere(N, s.nlat[0])
    ref = O.stream_function_psi(S, O.to_tensor(a))
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert float((g[2].cpu() - ref).abs().max()) <= tol * float(ref.abs().max())
    # the velocity fields are those of nse_synthesize
    assert torch.equal(g[:2], plain[:2])
    s.close()


@pytest.mark.parametrize("N1,Np,n_src,nu,omega", [
    (10, 20, 10, 1e-3, 2 * math.pi),
    (10, 20, 15, 1e-3, 2 * math.pi),     # source stored at a larger truncation
    (75, 150, 100, 1e-4, 1.0),           # Example 2 sizes: N = 100, N1 = 75, N' = 2 N1
])
def test_inertial_manifold(N1, Np, n_src, nu, omega):
    _say(f"case inertial manifold N1={N1} N'={Np} n_src={n_src}")
    if n_src == 100:
        # a flat spectrum gives u1 = P_N1 u weight at every degree <= N1, so that
        # B(u1, u1) fills the whole band (N1, 2 N1] with values of one size
        a = I.flat_spectrum(n_src, 3)
        f = np.zeros(I.coeff_count(Np), dtype=np.complex128)
        f[I.index(Np, 3, 0)] = 1.0
    else:
        a = I.spectrum(I.SEED_INITIAL, n_src)
        f = 0.01 * I.spectrum(I.SEED_FORCING, Np)
    s = pkg.Sphere([(Np, 0, nu)], omega=omega, dt=1e-3)
    phi = s.inertial_manifold(pkg.to_device(a), n_src, N1, pkg.to_device(f)).cpu()
    phi0 = s.inertial_manifold(pkg.to_device(a), n_src, N1, None).cpu()
    s.close()
    S = O.Sphere(Np)
    ref = O.inertial_manifold(S, O.to_tensor(a), n_src, N1, O.to_tensor(f), nu, omega)
    ref0 = O.inertial_manifold(S, O.to_tensor(a), n_src, N1, None, nu, omega)
    deg = torch.as_tensor(I.degrees_orders(Np)[0])
    band = (deg > N1) & (deg <= Np)
    for got, r in ((phi, ref), (phi0, ref0)):
        # every band degree that B(u1, u1) can reach (N1 < L <= 2 N1 - 2; the two top
        # degrees of the product of two degree-N1 fields vanish) carries content, so
        # this is no comparison of rounding with rounding
        rms = [float(r[deg == L].abs().pow(2).mean().sqrt()) for L in range(N1 + 1, 2 * N1 - 1)]
        assert min(rms) > 1e-6 * max(rms)
        e = float((got - r).abs().max()) / float(r[band].abs().max())
        _say(f"  max coefficient err / max {e:.3e}; band degree RMS spread {min(rms) / max(rms):.2e}")
        assert e <= 1e-12
    assert float(phi[deg <= N1].abs().max()) == 0.0


def test_inertial_manifold_members_and_errors():
    N1, Np = 8, 16
    _say(f"case inertial manifold two members N1={N1}")
    nus = (1e-3, 4e-3)
    s = pkg.Sphere([(Np, 0, nus[0]), (Np, 0, nus[1])], omega=1.0, dt=1e-3)
    a = np.concatenate([I.member_state(0, N1), I.member_state(1, N1)])
    phi = s.inertial_manifold(pkg.to_device(a), N1, N1).cpu()
    S = O.Sphere(Np)
    P = I.coeff_count(N1)
    for i in range(2):
        ref = O.inertial_manifold(S, O.to_tensor(a[i * P:(i + 1) * P]), N1, N1, None, nus[i], 1.0)
        got = phi[s.member_slice(i)]
        assert float((got - ref).abs().max()) <= 1e-12 * float(ref.abs().max())
    ad = pkg.to_device(a)
    for n_src, n1 in ((N1, N1 + 1), (N1, 0), (N1, Np + 1)):
        with pytest.raises(pkg.NseError) as e:
            s.inertial_manifold(ad, n_src, n1)
        assert e.value.status == pkg.NSE_ERR_ARG
    s.close()
    s = pkg.Sphere([(Np, 0, 0.0)], omega=1.0, dt=1e-3)
    with pytest.raises(pkg.NseError) as e:
        s.inertial_manifold(pkg.to_device(I.member_state(0, N1)), N1, N1)
    assert e.value.status == pkg.NSE_ERR_ARG
    s.close()
