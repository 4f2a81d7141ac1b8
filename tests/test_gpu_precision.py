"""Reduced-precision Legendre contractions (FP32 and split bf16x3 on MFMA) against
the FP64 oracle and the FP64 GPU path.

Bars: one nonlinear-term evaluation within 1e-6 relative l2 of the FP64 oracle;
grid fields (u_theta, u_phi, zeta) after 200 T511 steps within 1e-6 of the FP64
run. Everything but the contractions (recurrences, weights, FFTs, products, the
viscous update) is FP64 in all modes.
"""
import math
import os

import numpy as np
import pytest
import torch

import nse_inputs as I
import paper_1009_3308_amd as pkg
from oracle import nse_oracle as O

pytestmark = pytest.mark.gpu
OMEGA = 2.0 * math.pi


def _say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1009_3308_amd import build
        build.build()
    torch.cuda.set_device(0)


# N = 400 runs on its default grid of 625 latitudes (313 northern, the middle one on
# the equator): the FP32 recurrence kernels with two latitudes per lane in the
# synthesis and five in the analysis
@pytest.mark.parametrize("prec,N", [(p, n) for p in ("fp32", "bf16x3") for n in (15, 31, 255, 511)]
                         + [("fp32", 400)])
def test_nonlinear_reduced_precision_vs_oracle(prec, N):
    _say(f"case: nonlinear {prec} N={N}")
    s = pkg.Sphere([(N, 0, 1e-5)], omega=OMEGA, dt=1e-3, precision=prec)
    a = I.initial_state(N)
    got = s.nonlinear(pkg.to_device(a)).cpu().numpy()
    ref = O.Sphere(N, s.nlat[0]).nonlinear(O.to_tensor(a), OMEGA).numpy()
    e = rel(got, ref)
    _say(f"  rel err {e:.3e}")
    assert e < 1e-6
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_synthesis_reduced_precision_vs_oracle(prec):
    N = 255
    _say(f"case: synthesis {prec} N={N}")
    s = pkg.Sphere([(N, 0, 0.0)], omega=OMEGA, dt=1e-3, precision=prec)
    a = I.initial_state(N)
    ut, up, ze = s.synthesize(pkg.to_device(a))[0].cpu().numpy()
    S = O.Sphere(N, s.nlat[0])
    rt, rp = S.velocity(O.to_tensor(a))
    for got, ref in ((ut, rt), (up, rp), (ze, S.vorticity(O.to_tensor(a)))):
        assert rel(got, ref.numpy()) < 1e-6
    s.close()


def _fields(sph64, alpha):
    return sph64.synthesize(alpha)[0].cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_t511_trajectory_fields_vs_fp64(prec):
    N, steps = 511, 200
    _say(f"case: T511 {prec} {steps} steps")
    a0, f = pkg.to_device(I.initial_state(N)), pkg.to_device(I.forcing(N))
    out = {}
    for p in ("fp64", prec):
        s = pkg.Sphere([(N, 0, 1e-5)], omega=OMEGA, dt=1e-3, precision=p)
        h = s.new_history()
        h[0] = a0
        s.step(h, f, 0, 1)
        one = h[0].clone()
        s.step(h, f, 1, steps - 1)
        out[p] = (one, h[0].clone())
        s.close()
    s64 = pkg.Sphere([(N, 0, 1e-5)], omega=OMEGA, dt=1e-3)
    for idx, label in ((0, "1 step"), (1, f"{steps} steps")):
        g64 = _fields(s64, out["fp64"][idx])
        glp = _fields(s64, out[prec][idx])
        errs = [rel(glp[i], g64[i]) for i in range(3)]
        _say(f"  {label}: rel err u_theta {errs[0]:.3e} u_phi {errs[1]:.3e} zeta {errs[2]:.3e}")
        assert max(errs) < 1e-6
    s64.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_reduced_precision_graph_equals_eager_bitwise(prec):
    N, steps = 127, 37
    _say(f"case: {prec} graph vs eager N={N}")
    stream = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(stream):
        a0, f = pkg.to_device(I.initial_state(N)), pkg.to_device(I.forcing(N))
        for graph in (False, True):
            s = pkg.Sphere([(N, 0, 1e-4)], omega=OMEGA, dt=1e-3, precision=prec, graph=graph,
                           stream=stream)
            h = s.new_history()
            h[0] = a0
            s.step(h, f, 0, steps)
            s.step(h, f, steps, steps)
            s.sync()
            outs.append(h.clone())
            s.close()
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_reduced_precision_members(prec):
    """Several members (two truncation groups) in one reduced-precision context:
    each member's nonlinear term within 1e-6 of the FP64 oracle and bitwise equal
    to the same member alone."""
    specs = [(63, 0, 1e-4), (31, 0, 1e-3), (63, 0, 5e-4)]
    _say(f"case: {prec} members {specs}")
    s = pkg.Sphere(specs, omega=OMEGA, dt=1e-3, precision=prec)
    a = s.new_state()
    host = []
    for i, (N, _, _) in enumerate(specs):
        host.append(I.member_state(i, N))
        a[s.member_slice(i)] = pkg.to_device(host[i])
    got = s.nonlinear(a).cpu().numpy()
    for i, spec in enumerate(specs):
        N = spec[0]
        sl = s.member_slice(i)
        ref = O.Sphere(N, s.nlat[i]).nonlinear(O.to_tensor(host[i]), OMEGA).numpy()
        assert rel(got[sl], ref) < 1e-6
        one = pkg.Sphere([spec], omega=OMEGA, dt=1e-3, precision=prec)
        assert np.array_equal(one.nonlinear(pkg.to_device(host[i])).cpu().numpy(), got[sl])
        one.close()
    s.close()
