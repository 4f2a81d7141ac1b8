"""Adaptive NDF integration on the GPU against the oracle's integrator.

The GPU controller takes the same decisions as the oracle's (orders 1..5 of eq.
(ode_disc), step and order control at a relative tolerance), whether it runs on
the host (forcing callbacks) or on the device (no callback): the attempt logs
must agree in order, outcome and corrector sweeps exactly, in t and h to 1e-9
relative, and the states to 1e-10 of their largest coefficient (the nonlinear
terms agree to ~1e-14 per evaluation; the step-size feedback amplifies that by a
few orders over a run). Example 1's manufactured flow is recovered to the
tolerance.
"""
import ctypes
import math
import os

import numpy as np
import pytest
import torch

import nse_inputs as I
import paper_1009_3308_amd as pkg
from oracle import ndf_adaptive as A
from oracle import nse_oracle as O

pytestmark = pytest.mark.gpu
OMEGA = 2.0 * math.pi


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


def _compare_logs(glog, olog, label, stops=()):
    """Attempt logs: order, sweeps and outcome exactly, t to 1e-9 (absolute below
    1), h to 1e-9 relative, except for a step shortened or stretched to end at a
    stop, whose h = stop - t carries the absolute deviation of t."""
    assert len(glog) == len(olog), (label, len(glog), len(olog))
    for i, (g, o) in enumerate(zip(glog, olog)):
        gt, gh, gk, gs, gout, gerr = g
        ot, oh, ok, osw, oout, oerr = o
        assert (gk, gs, gout) == (ok, osw, oout), (label, i, g, o)
        tol_t = 1e-9 * max(1.0, abs(ot))
        assert abs(gt - ot) <= tol_t, (label, i, g, o)
        at_stop = any(abs(ot + oh - t) <= 1e-12 * max(1.0, t) for t in stops)
        assert abs(gh - oh) <= (tol_t if at_stop else 1e-9 * oh), (label, i, g, o)
        if oout != A.NEWTON_FAIL:
            assert abs(gerr - oerr) <= 1e-7 * oerr + 1e-300, (label, i, g, o)


def _oracle_integrator(N, nus, forcing, omega=OMEGA, nlat=None, **kw):
    """One system of len(nus) members of truncation N (states concatenated)."""
    S = O.Sphere(N, nlat)
    P = O.coeff_count(N)
    L = torch.cat([(nu * S.lam).to(torch.float64) for nu in nus])

    def nonlinear(y):
        return torch.cat([S.nonlinear(y[i * P:(i + 1) * P], omega) for i in range(len(nus))])

    def project(y):
        return torch.cat([O.clean(y[i * P:(i + 1) * P], N) for i in range(len(nus))])

    return A.AdaptiveNDF(L, nonlinear, forcing, project=project, **kw)


@pytest.mark.parametrize("N,nu,T,rtol,max_newton", [
    (31, 1e-3, 5.0, 1e-3, 4),     # orders 1..4, error failures, 3-sweep attempts
    (31, 1e-3, 2.0, 1e-5, 4),     # order 5
    (63, 1e-4, 2.0, 1e-3, 4),
    (31, 1e-3, 1.0, 1e-3, 1),     # one sweep per attempt
])
def test_adaptive_matches_oracle(N, nu, T, rtol, max_newton):
    _say(f"case adaptive N={N} nu={nu} T={T} rtol={rtol} K={max_newton}")
    a0 = I.initial_state(N)
    f = I.forcing(N)
    s = pkg.Sphere([(N, 0, nu)], omega=OMEGA, dt=1e-3, order=2)
    s.adaptive_begin(pkg.to_device(a0), 0.0, rtol=rtol, atol=1e-6, max_newton=max_newton,
                     forcing=pkg.to_device(f))
    out, stats = s.adaptive_advance(T)
    glog = s.adaptive_log()
    g = out.cpu()
    s.close()
    ft = O.to_tensor(f)
    integ = _oracle_integrator(N, [nu], lambda t: ft, rtol=rtol, atol=1e-6,
                               max_newton=max_newton)
    integ.begin(O.to_tensor(a0), 0.0)
    o = integ.advance(T)
    _compare_logs(glog, integ.log, f"N={N}", (T,))
    scale = float(o.abs().max())
    diff = float((g - o).abs().max())
    _say(f"  attempts {len(glog)} accepted {stats['accepted']} evals {stats['evaluations']} "
         f"state diff {diff / scale:.3e}")
    assert stats["t"] == T
    assert stats["accepted"] == sum(1 for r in glog if r[4] == A.ACCEPTED)
    assert diff <= 1e-10 * scale
    # no callback: the controller ran on the device, the host waited once for
    # F(t0) and once per batch of attempts
    assert stats["waits"] <= 2 + len(glog) // 4, stats


@pytest.mark.parametrize("N", [140, 60])
def test_adaptive_wide_grid_matches_oracle(N):
    """The device-controlled sweeps on a grid of 200 northern latitudes (four
    latitudes per analysis lane, four latitude tiles per synthesis order): at
    N = 60 the synthesis also runs the slot's controller step (every tile
    forming its order's predictor from the old differences, the analysis
    epilogue storing the new ones), at N = 140 (a launch too large to stay
    resident with the controller's registers) the step kernel does."""
    nlat, nu, T = 400, 1e-3, 0.3
    _say(f"case adaptive N={N} nlat={nlat} T={T}")
    a0 = I.initial_state(N)
    f = I.forcing(N)
    s = pkg.Sphere([(N, nlat, nu)], omega=OMEGA, dt=1e-3, order=2)
    s.adaptive_begin(pkg.to_device(a0), 0.0, rtol=1e-4, atol=1e-6, forcing=pkg.to_device(f))
    out, stats = s.adaptive_advance(T)
    glog = s.adaptive_log()
    g = out.cpu()
    s.close()
    ft = O.to_tensor(f)
    integ = _oracle_integrator(N, [nu], lambda t: ft, nlat=nlat, rtol=1e-4, atol=1e-6)
    integ.begin(O.to_tensor(a0), 0.0)
    o = integ.advance(T)
    _compare_logs(glog, integ.log, f"N={N} nlat={nlat}", (T,))
    scale = float(o.abs().max())
    diff = float((g - o).abs().max())
    _say(f"  attempts {len(glog)} state diff {diff / scale:.3e}")
    assert stats["t"] == T
    assert diff <= 1e-10 * scale


def test_adaptive_stops_and_time_dependent_forcing():
    # several stops, a forcing refreshed by a callback at every time level
    N, nu = 31, 1e-3
    _say(f"case adaptive stops N={N}")
    a0 = I.initial_state(N)
    f0 = I.forcing(N)
    fd = pkg.to_device(f0)
    s = pkg.Sphere([(N, 0, nu)], omega=OMEGA, dt=1e-3, order=2)
    seen = []

    def forcing(t):
        seen.append(t)
        return fd * math.cos(3.0 * t)

    s.adaptive_begin(pkg.to_device(a0), 0.25, forcing=forcing)
    stops = (0.5, 0.75, 1.5, 1.5, 2.0)
    gouts = []
    for t in stops:
        out, stats = s.adaptive_advance(t)
        assert stats["t"] == t
        gouts.append(out.cpu())
    glog = s.adaptive_log()
    s.close()
    assert seen[0] == 0.25 and len(seen) == len(glog) + 1
    ft = O.to_tensor(f0)
    integ = _oracle_integrator(N, [nu], lambda t: ft * math.cos(3.0 * t))
    integ.begin(O.to_tensor(a0), 0.25)
    for t, g in zip(stops, gouts):
        o = integ.advance(t)
        assert float((g - o).abs().max()) <= 1e-10 * float(o.abs().max())
    _compare_logs(glog, integ.log, "stops", stops)


def _schedule_scale(sc, t):
    """s(t) of a forcing schedule, as the header defines it."""
    if t <= sc.t_on:
        return sc.before
    return sc.amp * math.cos(sc.omega * t + sc.phase) * math.exp(-sc.decay * (t - sc.t_on))


def test_adaptive_device_schedule_and_stops():
    # a forcing scale switched on inside the run and evaluated by the device,
    # several stops (each advance a new batch sequence on the same graph)
    N, nu = 31, 1e-3
    _say(f"case adaptive device schedule N={N}")
    a0 = I.initial_state(N)
    f0 = I.forcing(N)
    sc = pkg.ForcingSchedule(t_on=0.6, before=1.0, amp=1.3, omega=7.0, phase=0.4, decay=2.0)
    s = pkg.Sphere([(N, 0, nu)], omega=OMEGA, dt=1e-3, order=2)
    s.adaptive_begin(pkg.to_device(a0), 0.25, forcing=(pkg.to_device(f0), sc))
    stops = (0.5, 0.75, 1.5, 1.5, 2.0)
    gouts = []
    for t in stops:
        out, stats = s.adaptive_advance(t)
        assert stats["t"] == t
        gouts.append(out.cpu())
    glog = s.adaptive_log()
    s.close()
    ft = O.to_tensor(f0)
    integ = _oracle_integrator(N, [nu], lambda t: ft * _schedule_scale(sc, t))
    integ.begin(O.to_tensor(a0), 0.25)
    for t, g in zip(stops, gouts):
        o = integ.advance(t)
        assert float((g - o).abs().max()) <= 1e-10 * float(o.abs().max())
    _compare_logs(glog, integ.log, "schedule stops", stops)
    _say(f"  attempts {len(glog)} waits {stats['waits']}")
    assert stats["waits"] <= 1 + len(stops) + len(glog) // 4


def test_adaptive_members_form_one_system():
    N, nus = 31, (1e-3, 3e-3)
    _say(f"case adaptive two members N={N}")
    a0 = np.concatenate([I.member_state(0, N), I.member_state(1, N)])
    f = np.concatenate([I.forcing(N), 0.5 * I.forcing(N)])
    s = pkg.Sphere([(N, 0, nus[0]), (N, 0, nus[1])], omega=OMEGA, dt=1e-3, order=2)
    s.adaptive_begin(pkg.to_device(a0), 0.0, forcing=pkg.to_device(f))
    out, _ = s.adaptive_advance(1.5)
    glog = s.adaptive_log()
    g = out.cpu()
    s.close()
    ft = O.to_tensor(f)
    integ = _oracle_integrator(N, nus, lambda t: ft)
    integ.begin(O.to_tensor(a0), 0.0)
    o = integ.advance(1.5)
    _compare_logs(glog, integ.log, "members", (1.5,))
    assert float((g - o).abs().max()) <= 1e-10 * float(o.abs().max())


@pytest.mark.parametrize("rtol", [1e-3, 1e-5])
def test_adaptive_example1_recovers_exact_flow(rtol):
    # Example 1: f = alpha' + nu lambda alpha + n(alpha) of the exact coefficients;
    # the adaptive integration must track the exact flow to the tolerance and
    # agree with the oracle's integrator
    N, NU, T = 10, 0.1, 1.0
    _say(f"case adaptive example 1 N={N} rtol={rtol}")
    s = pkg.Sphere([(N, 0, NU)], omega=OMEGA, dt=1e-3, order=2)
    ls = torch.as_tensor(I.degrees_orders(N)[0], dtype=torch.float64, device="cuda")
    lam = ls * (ls + 1)

    def force(t):
        ae = pkg.to_device(I.example1_state(N, N, t, NU))
        return pkg.to_device(I.example1_state(N, N, t, NU, rate=True)) + NU * lam * ae \
            + s.nonlinear(ae)

    s.adaptive_begin(pkg.to_device(I.example1_state(N, N, 0.0, NU)), 0.0, rtol=rtol,
                     atol=rtol * 1e-3, forcing=force)
    out, stats = s.adaptive_advance(T)
    glog = s.adaptive_log()
    g = out.cpu()
    s.close()
    ex = O.to_tensor(I.example1_state(N, N, T, NU))
    err = float((g - ex).abs().max()) / float(ex.abs().max())
    _say(f"  attempts {len(glog)} error vs exact {err:.3e}")
    assert err <= 5 * rtol
    S = O.Sphere(N)
    L = (NU * S.lam).to(torch.float64)

    def oforce(t):
        ae = O.to_tensor(I.example1_state(N, N, t, NU))
        return O.to_tensor(I.example1_state(N, N, t, NU, rate=True)) + L * ae \
            + S.nonlinear(ae, OMEGA)

    integ = A.AdaptiveNDF(L, lambda y: S.nonlinear(y, OMEGA), oforce, rtol=rtol,
                          atol=rtol * 1e-3, project=lambda y: O.clean(y, N))
    integ.begin(O.to_tensor(I.example1_state(N, N, 0.0, NU)), 0.0)
    o = integ.advance(T)
    _compare_logs(glog, integ.log, "example1", (T,))
    assert float((g - o).abs().max()) <= 1e-10 * float(o.abs().max())


def test_adaptive_argument_errors():
    N = 15
    s = pkg.Sphere([(N, 0, 1e-3)], omega=OMEGA, dt=1e-3, order=2)
    a0 = pkg.to_device(I.initial_state(N))
    with pytest.raises(pkg.NseError) as e:
        s.adaptive_advance(1.0)
    assert e.value.status == pkg.NSE_ERR_STATE
    for kw in ({"rtol": 0.0}, {"atol": -1.0}, {"max_order": 6}, {"max_order": 0},
               {"max_newton": 9}, {"h0": -1.0}, {"hmax": -0.5}):
        with pytest.raises(pkg.NseError) as e:
            s.adaptive_begin(a0, 0.0, **kw)
        assert e.value.status == pkg.NSE_ERR_ARG
    bad = pkg.ForcingSchedule(t_on=0.0, before=1.0, amp=math.nan, omega=1.0, phase=0.0, decay=0.0)
    with pytest.raises(pkg.NseError) as e:
        s.adaptive_begin(a0, 0.0, forcing=(s.new_state(), bad))
    assert e.value.status == pkg.NSE_ERR_ARG
    s.adaptive_begin(a0, 1.0)
    with pytest.raises(pkg.NseError) as e:
        s.adaptive_advance(0.5)
    assert e.value.status == pkg.NSE_ERR_ARG
    out, stats = s.adaptive_advance(1.0)      # no-op: returns the initial state
    assert torch.equal(out, a0) and stats["accepted"] == 0
    s.close()


def test_adaptive_hmax_and_h0():
    N, nu = 31, 1e-3
    _say(f"case adaptive hmax/h0 N={N}")
    a0 = I.initial_state(N)
    f = I.forcing(N)
    s = pkg.Sphere([(N, 0, nu)], omega=OMEGA, dt=1e-3, order=2)
    s.adaptive_begin(pkg.to_device(a0), 0.0, h0=1e-3, hmax=0.02, forcing=pkg.to_device(f))
    out, _ = s.adaptive_advance(1.0)
    glog = s.adaptive_log()
    s.close()
    assert glog[0][1] == 1e-3
    assert max(r[1] for r in glog) <= 0.02
    ft = O.to_tensor(f)
    integ = _oracle_integrator(N, [nu], lambda t: ft, h0=1e-3, hmax=0.02)
    integ.begin(O.to_tensor(a0), 0.0)
    o = integ.advance(1.0)
    _compare_logs(glog, integ.log, "hmax", (1.0,))
    assert float((out.cpu() - o).abs().max()) <= 1e-10 * float(o.abs().max())


@pytest.mark.parametrize("control", ["host", "device"])
def test_adaptive_example2_matches_oracle(control):
    # the paper's Example 2 setting (N = 100, nu = 1e-4, Omega = 1, random initial
    # flow of degrees 1..20, forcing f_{3,0}) over a short interval; its forcing
    # scale as a host callback (host control) or as a device schedule
    N, nu, omega, T = 100, 1e-4, 1.0, 0.08
    _say(f"case adaptive example 2 N={N} T={T} control={control}")
    a0 = I.example2_state(N, nu)
    s = pkg.Sphere([(N, 0, nu)], omega=omega, dt=1e-3, order=2)
    F = s.new_state()
    F[I.index(N, 3, 0)] = 1.0
    scale = (I.example2_force if control == "host"
             else pkg.ForcingSchedule(**I.example2_schedule()))
    s.adaptive_begin(pkg.to_device(a0), 0.0, forcing=(F, scale))
    out, stats = s.adaptive_advance(T)
    glog = s.adaptive_log()
    g = out.cpu()
    s.close()
    Fo = torch.zeros(O.coeff_count(N), dtype=torch.complex128)
    Fo[I.index(N, 3, 0)] = 1.0
    integ = _oracle_integrator(N, [nu], lambda t: Fo * I.example2_force(t), omega=omega)
    integ.begin(O.to_tensor(a0), 0.0)
    o = integ.advance(T)
    _say(f"  attempts {len(glog)} sweeps {sum(r[3] for r in glog)}")
    _compare_logs(glog, integ.log, "example2", (T,))
    assert float((g - o).abs().max()) <= 1e-10 * float(o.abs().max())


def test_adaptive_forcing_callback_error_propagates():
    N = 15
    s = pkg.Sphere([(N, 0, 1e-3)], omega=OMEGA, dt=1e-3, order=2)
    F = pkg.to_device(I.forcing(N))

    def scale(t):
        if t > 0.3:
            raise ZeroDivisionError("forcing undefined")
        return 1.0

    s.adaptive_begin(pkg.to_device(I.initial_state(N)), 0.0, forcing=(F, scale))
    with pytest.raises(ZeroDivisionError):
        s.adaptive_advance(1.0)
    s.close()

