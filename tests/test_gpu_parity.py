"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Floating-point bar: relative l2 error <= 1e-12 per nonlinear-term evaluation
and per short trajectory (FP64 on both sides; differences come from summation
order, FMA contraction and the FFT versus the direct DFT).
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
TOL = 1e-12


def _say(*a):
    print(*a, flush=True)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1009_3308_amd import build
        build.build()
    torch.cuda.set_device(0)


_SPHERES = {}


def oracle_sphere(N, nlat):
    key = (N, nlat)
    if key not in _SPHERES:
        _SPHERES[key] = O.Sphere(N, nlat)
    return _SPHERES[key]


def test_gauss_legendre_nodes_match_oracle():
    for N in (9, 31, 255):
        _say(f"case: grid N={N}")
        s = pkg.Sphere([(N, 0, 0.0)], omega=OMEGA, dt=1e-3)
        mu, w = s.grid(0)
        mo, wo = O.gauss_legendre(s.nlat[0])
        assert np.abs(mu - mo.numpy()).max() < 1e-15
        # a weight near a pole depends on 1 - |x|, which a node rounded to FP64
        # carries only to ~1e-16 absolute: at the polar nodes (1 - |x| ~ 1e-5 at
        # N = 255) two correct FP64 rules may differ by ~1e-11 relative, so the
        # bar is absolute (which still bounds the polar weights to 1e-10 relative)
        assert np.abs(w - wo.numpy()).max() < 1e-15
        assert abs(w.sum() - 2.0) < 1e-14
        s.close()


@pytest.mark.parametrize("N", [9, 31, 255, 511])
def test_legendre_table_matches_oracle(N):
    _say(f"case: legendre table N={N}")
    s = pkg.Sphere([(N, 0, 0.0)], omega=OMEGA, dt=1e-3)
    g = O.Grid(s.nlat[0])
    nh = (s.nlat[0] + 1) // 2
    mu, sn = g.mu[:nh], g.sin[:nh]
    ms = range(N + 1) if N <= 31 else [0, 1, 2, 7, N // 3, N // 2, N - 1, N]
    for m in ms:
        got = s.legendre_values(0, m).cpu().numpy()
        ref = O.legendre_order(m, N + 1, mu, sn).numpy()
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(got - ref).max() <= 1e-13 * scale * max(1, N / 31), (m,)
    s.close()


# the FP64 synthesis takes 1, 2 or 3 latitudes per lane by grid size (nh <= 192,
# 256 <= nh with nh % 192 != 0, nh = 384): (400, 640) and (511, 0) cover 2 and 3
@pytest.mark.parametrize("N,nlat", [(9, 0), (31, 0), (31, 60), (255, 0), (400, 640), (511, 0)])
def test_synthesis_matches_oracle(N, nlat):
    _say(f"case: synthesis N={N} nlat={nlat}")
    s = pkg.Sphere([(N, nlat, 0.0)], omega=OMEGA, dt=1e-3)
    a = I.initial_state(N)
    ut, up, ze = s.synthesize(pkg.to_device(a))[0].cpu().numpy()
    S = oracle_sphere(N, s.nlat[0])
    rt, rp = S.velocity(O.to_tensor(a))
    rz = S.vorticity(O.to_tensor(a))
    assert rel(ut, rt.numpy()) < TOL
    assert rel(up, rp.numpy()) < TOL
    assert rel(ze, rz.numpy()) < TOL
    s.close()


# the FP64 analysis takes ceil(nh / 64) latitudes per lane: every count 1..6 occurs
# ((127, 0): 2, (255, 0): 3, (300, 480): 4, (400, 640): 5, (511, 0): 6)
@pytest.mark.parametrize("N,nlat", [(1, 0), (2, 0), (9, 0), (15, 0), (31, 0), (31, 60),
                                    (63, 0), (127, 0), (255, 0), (300, 480), (400, 640),
                                    (511, 0)])
def test_nonlinear_matches_oracle(N, nlat):
    _say(f"case: nonlinear N={N} nlat={nlat}")
    s = pkg.Sphere([(N, nlat, 1e-3)], omega=OMEGA, dt=1e-3)
    a = I.initial_state(N)
    got = s.nonlinear(pkg.to_device(a)).cpu().numpy()
    ref = oracle_sphere(N, s.nlat[0]).nonlinear(O.to_tensor(a), OMEGA).numpy()
    e = rel(got, ref)
    _say(f"  rel err {e:.3e}")
    assert e < TOL
    assert got[0] == 0 and np.all(got[: N + 1].imag == 0)
    s.close()


def test_nonlinear_closed_forms_at_full_size():
    N = 255
    _say(f"case: closed forms N={N}")
    s = pkg.Sphere([(N, 0, 0.0)], omega=OMEGA, dt=1e-3)
    rng = np.random.default_rng(5)
    # single degree: advection vanishes, Coriolis = -2 Omega i m alpha / lambda
    l = 40
    a = I.single_mode(N, {(l, m): complex(rng.standard_normal(), rng.standard_normal() if m else 0)
                          for m in range(l + 1)})
    got = s.nonlinear(pkg.to_device(a)).cpu().numpy()
    _, ms = I.degrees_orders(N)
    exp = -2 * OMEGA * 1j * ms * a / (l * (l + 1))
    assert np.abs(got - exp).max() < 1e-13 * l * (l + 1) * np.abs(a).max() ** 2
    # Rossby-Haurwitz wave with superrotation w0
    w0, lr = 0.5, 4
    a = I.single_mode(N, {(1, 0): w0 * math.sqrt(8 * math.pi / 3), (lr, 4): 0.5, (lr, 2): 0.1j})
    got = s.nonlinear(pkg.to_device(a)).cpu().numpy()
    lam = lr * (lr + 1)
    exp = np.zeros_like(a)
    for m in (2, 4):
        k = I.index(N, lr, m)
        exp[k] = 1j * m * (w0 * (1 - 2 / lam) - 2 * OMEGA / lam) * a[k]
    assert np.abs(got - exp).max() < 1e-13
    s.close()


@pytest.mark.parametrize("N", [255, 511])
def test_energy_and_enstrophy_conservation_on_gpu(N):
    _say(f"case: invariants N={N}")
    s = pkg.Sphere([(N, 0, 0.0)], omega=OMEGA, dt=1e-3)
    a = I.initial_state(N)
    n = s.nonlinear(pkg.to_device(a)).cpu().numpy()
    ls, ms = I.degrees_orders(N)
    w = np.where(ms > 0, 2.0, 1.0)
    lam = ls * (ls + 1.0)
    scale = np.sum(w * np.abs(a) * np.abs(n) * lam)
    assert abs(np.sum(w * (np.conj(a) * n).real)) < 1e-13 * scale
    assert abs(np.sum(w * lam * (np.conj(a) * n).real)) < 1e-13 * scale
    s.close()


@pytest.mark.parametrize("N,order,iters,steps", [(31, 2, 1, 100), (15, 1, 1, 30), (15, 3, 1, 30),
                                                  (15, 5, 1, 30), (15, 2, 3, 20)])
def test_step_matches_oracle(N, order, iters, steps):
    _say(f"case: step N={N} p={order} K={iters} steps={steps}")
    nu, dt = 1e-3, 1e-3
    s = pkg.Sphere([(N, 0, nu)], omega=OMEGA, dt=dt, order=order, newton_iters=iters)
    a0, f = I.initial_state(N), I.forcing(N)
    hist = s.new_history()
    hist[0] = pkg.to_device(a0)
    s.step(hist, pkg.to_device(f), 0, steps)
    got = hist.cpu().numpy()
    st = O.Stepper(oracle_sphere(N, s.nlat[0]), nu, OMEGA, dt, order=order, newton_iters=iters)
    ref = st.run(O.to_tensor(a0), O.to_tensor(f), steps)
    for j in range(order + 1):
        e = rel(got[j], ref[j].numpy())
        _say(f"  slot {j} rel err {e:.3e}")
        assert e < TOL
    s.close()


def test_step_in_two_calls_equals_one_call():
    N = 31
    _say(f"case: split step calls N={N}")
    s = pkg.Sphere([(N, 0, 1e-3)], omega=OMEGA, dt=1e-3, order=3)
    a0, f = pkg.to_device(I.initial_state(N)), pkg.to_device(I.forcing(N))
    h1 = s.new_history()
    h1[0] = a0
    s.step(h1, f, 0, 17)
    h2 = s.new_history()
    h2[0] = a0
    s.step(h2, f, 0, 2)
    s.step(h2, f, 2, 15)
    assert torch.equal(h1, h2)
    s.close()


def test_step_t255_matches_oracle():
    N, steps = 255, 3
    _say(f"case: step N={N} steps={steps}")
    nu, dt = 1e-5, 1e-3
    s = pkg.Sphere([(N, 0, nu)], omega=OMEGA, dt=dt, order=2)
    a0, f = I.initial_state(N), I.forcing(N)
    hist = s.new_history()
    hist[0] = pkg.to_device(a0)
    s.step(hist, pkg.to_device(f), 0, steps)
    ref = O.Stepper(oracle_sphere(N, s.nlat[0]), nu, OMEGA, dt).run(O.to_tensor(a0),
                                                                      O.to_tensor(f), steps)
    assert rel(hist[0].cpu().numpy(), ref[0].numpy()) < TOL
    s.close()


def test_graph_replay_equals_eager_bitwise():
    N, steps = 63, 47
    _say(f"case: graph vs eager N={N}")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a0, f = pkg.to_device(I.initial_state(N)), pkg.to_device(I.forcing(N))
        outs = []
        for graph in (False, True):
            s = pkg.Sphere([(N, 0, 1e-4)], omega=OMEGA, dt=1e-3, graph=graph, stream=stream)
            h = s.new_history()
            h[0] = a0
            s.step(h, f, 0, steps)
            s.step(h, f, steps, steps)      # replays the cached graph
            s.sync()
            outs.append(h.clone())
            s.close()
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


def test_multi_member_context_equals_single_members():
    specs = [(31, 0, 1e-3), (63, 0, 1e-4), (31, 0, 5e-4), (15, 30, 2e-3)]
    _say("case: multi-member context (per-member kernels)")
    multi = pkg.Sphere(specs, omega=OMEGA, dt=1e-3)
    for i in range(len(specs)):
        multi.set_member_blocks(i, 0, 0)  # the batched products are tested in test_gpu_ensemble
    states = [I.member_state(i, N) for i, (N, _, _) in enumerate(specs)]
    forc = [I.spectrum(200 + i, N, 1e-2) for i, (N, _, _) in enumerate(specs)]
    a = pkg.to_device(np.concatenate(states))
    f = pkg.to_device(np.concatenate(forc))
    n_multi = multi.nonlinear(a).cpu().numpy()
    hist = multi.new_history()
    hist[0] = a
    multi.step(hist, f, 0, 12)
    hm = hist.cpu().numpy()
    for i, spec in enumerate(specs):
        single = pkg.Sphere([spec], omega=OMEGA, dt=1e-3)
        sl = multi.member_slice(i)
        n1 = single.nonlinear(pkg.to_device(states[i])).cpu().numpy()
        assert np.array_equal(n1, n_multi[sl])
        h1 = single.new_history()
        h1[0] = pkg.to_device(states[i])
        single.step(h1, pkg.to_device(forc[i]), 0, 12)
        assert np.array_equal(h1.cpu().numpy(), hm[:, sl])
        single.close()
    multi.close()


def test_rossby_haurwitz_wave_t255_against_closed_form():
    # alpha(t) = alpha(0) exp(-nu lam t - i m [(1-2/lam) w0 (1-e^{-2 nu t})/(2 nu) - 2 Omega t/lam])
    N, nu, dt, steps, w0 = 255, 1e-5, 1e-3, 1000, 0.5
    _say(f"case: viscous Rossby-Haurwitz N={N} steps={steps}")
    s = pkg.Sphere([(N, 0, nu)], omega=OMEGA, dt=dt, order=2, graph=True,
                   stream=torch.cuda.current_stream())
    a0 = I.single_mode(N, {(1, 0): w0 * math.sqrt(8 * math.pi / 3), (4, 4): 0.5})
    hist = s.new_history()
    hist[0] = pkg.to_device(a0)
    s.step(hist, None, 0, steps)
    got = hist[0].cpu().numpy()
    T = steps * dt
    lam = 20.0
    phase = (1 - 2 / lam) * w0 * (1 - math.exp(-2 * nu * T)) / (2 * nu) - 2 * OMEGA * T / lam
    exp = np.zeros_like(a0)
    exp[I.index(N, 4, 4)] = 0.5 * math.exp(-nu * lam * T) * np.exp(-4j * phase)
    exp[I.index(N, 1, 0)] = a0[I.index(N, 1, 0)] * math.exp(-2 * nu * T)
    err = np.abs(got - exp).max()
    _say(f"  max err {err:.3e}")
    assert err < 2e-6          # second-order time error at h = 1e-3 over t = 1
    others = np.ones(len(a0), bool)
    others[[I.index(N, 4, 4), I.index(N, 1, 0)]] = False
    assert np.abs(got[others]).max() < 1e-12


def test_check_finite_flag():
    N = 31
    _say("case: non-finite detection")
    s = pkg.Sphere([(N, 0, 1e-3)], omega=OMEGA, dt=1e-3, check_finite=True)
    a = I.initial_state(N)
    a[5] = np.nan
    hist = s.new_history()
    hist[0] = pkg.to_device(a)
    s.step(hist, None, 0, 1)
    with pytest.raises(pkg.NseError) as ei:
        s.sync()
    assert ei.value.status == pkg.NSE_ERR_NONFINITE
    s.sync()  # the flag is cleared after being reported
    s.close()


def test_argument_errors_through_binding():
    s = pkg.Sphere([(31, 0, 1e-3)], omega=OMEGA, dt=1e-3)
    a = s.new_state()
    p = pkg._ptr(a, torch.complex128)
    with pytest.raises(pkg.NseError) as ei:
        pkg._check(pkg.lib().nse_nonlinear(s._h, p, p), s._h)      # aliasing in/out
    assert ei.value.status == pkg.NSE_ERR_ARG
    with pytest.raises(pkg.NseError) as ei:
        s.step(s.new_history(), None, -1, 1)
    assert ei.value.status == pkg.NSE_ERR_ARG
    with pytest.raises(ValueError):
        s.nonlinear(torch.zeros(5, dtype=torch.complex128, device="cuda"))
    s.close()


@pytest.mark.parametrize("iters", [1, 2])
def test_profiled_steps_equal_plain_steps_bitwise(iters):
    """Timing mode repeats every launch between its events; the history after
    profiled steps must be bitwise that of plain steps."""
    N = 63
    _say(f"case: profiled steps N={N} newton_iters={iters}")
    a, f = pkg.to_device(I.initial_state(N)), pkg.to_device(I.forcing(N))
    out = []
    for repeat in (0, 5):
        s = pkg.Sphere([(N, 0, 1e-4)], omega=OMEGA, dt=1e-3, newton_iters=iters)
        h = s.new_history()
        h[0] = a
        if repeat:
            s.profile(True, repeat=repeat)
        s.step(h, f, 0, 12)
        if repeat:
            prof = s.profile_read()
            assert prof["synthesis"][0] == 12 * iters and prof["analysis"][0] == 12 * iters
            assert all(ms > 0 for _, ms in prof.values())
            s.profile(False)
        s.sync()
        out.append(h.clone())
        s.close()
    assert torch.equal(out[0], out[1])
