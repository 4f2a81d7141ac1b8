"""Member-batched contractions of truncation groups (FP64 MFMA products in which
one table pass serves a block of members) and the mixed-truncation ensemble.

Bars: every member's nonlinear term and short trajectory within 1e-12 of the
FP64 oracle; batched and per-member kernels within 1e-13 of each other; graph
replay bitwise equal to eager launches.
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
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


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
    if (N, nlat) not in _SPHERES:
        _SPHERES[(N, nlat)] = O.Sphere(N, nlat)
    return _SPHERES[(N, nlat)]


def _states(s, specs, seed0=0):
    a = s.new_state()
    host = []
    for i, (N, _, _) in enumerate(specs):
        x = I.member_state(seed0 + i, N)
        host.append(x)
        a[s.member_slice(i)] = pkg.to_device(x)
    return a, host


@pytest.mark.parametrize("sb,ab", [(2, 2), (4, 4), (8, 8), (8, 2), (2, 8), (0, 8), (8, 0)])
def test_member_blocks_nonlinear_vs_oracle(sb, ab):
    specs = [(31, 0, 1e-3)] * 5 + [(15, 0, 1e-3)] * 3   # partial blocks in both groups
    _say(f"case: member blocks synth={sb} anal={ab}, {len(specs)} members")
    s = pkg.Sphere(specs, omega=OMEGA, dt=1e-3)
    s.set_member_blocks(0, sb, ab)
    s.set_member_blocks(5, sb, ab)
    assert s.member_blocks(0) == (sb, ab)
    a, host = _states(s, specs)
    got = s.nonlinear(a).cpu().numpy()
    ref_s = pkg.Sphere(specs, omega=OMEGA, dt=1e-3)
    ref_s.set_member_blocks(0, 0, 0)
    ref_s.set_member_blocks(5, 0, 0)
    per_member = ref_s.nonlinear(a).cpu().numpy()
    worst, worst_pm = 0.0, 0.0
    for i, (N, _, _) in enumerate(specs):
        sl = s.member_slice(i)
        ref = oracle_sphere(N, s.nlat[i]).nonlinear(O.to_tensor(host[i]), OMEGA).numpy()
        worst = max(worst, rel(got[sl], ref))
        worst_pm = max(worst_pm, rel(got[sl], per_member[sl]))
    _say(f"  worst rel err vs oracle {worst:.3e}, vs per-member kernels {worst_pm:.3e}")
    assert worst < TOL and worst_pm < 1e-13
    s.close()
    ref_s.close()


def test_ensemble_steps_vs_oracle():
    specs = [(31, 0, 1e-3), (31, 0, 3e-4), (31, 0, 2e-3), (15, 0, 1e-3), (15, 0, 5e-3)]
    steps = 20
    _say(f"case: ensemble steps, {len(specs)} members, {steps} steps")
    s = pkg.Sphere(specs, omega=OMEGA, dt=1e-3, graph=True)
    assert s.member_blocks(0)[0] >= 2
    a, host = _states(s, specs, 10)
    f = s.new_state()
    forc = []
    for i, (N, _, _) in enumerate(specs):
        forc.append(I.spectrum(300 + i, N, 1e-2))
        f[s.member_slice(i)] = pkg.to_device(forc[i])
    h = s.new_history()
    h[0] = a
    s.step(h, f, 0, steps)
    got = h.cpu().numpy()
    for i, (N, _, nu) in enumerate(specs):
        st = O.Stepper(oracle_sphere(N, s.nlat[i]), nu, OMEGA, 1e-3, 2)
        ref = st.run(O.to_tensor(host[i]), O.to_tensor(forc[i]), steps)
        e = rel(got[0, s.member_slice(i)], ref[0].numpy())
        _say(f"  member {i} N={N} nu={nu}: rel err {e:.3e}")
        assert e < TOL
    s.close()


def test_ensemble_graph_equals_eager_bitwise():
    specs = [(63, 0, 1e-4)] * 4 + [(31, 0, 1e-3)] * 3
    _say("case: ensemble graph vs eager")
    stream = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(stream):
        for graph in (False, True):
            s = pkg.Sphere(specs, omega=OMEGA, dt=1e-3, graph=graph, stream=stream)
            a, _ = _states(s, specs)
            h = s.new_history()
            h[0] = a
            s.step(h, None, 0, 33)
            s.sync()
            outs.append(h.clone())
            s.close()
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


def test_autotune_picks_valid_blocks_and_same_results():
    specs = [(63, 0, 1e-4)] * 6
    _say("case: autotune")
    s = pkg.Sphere(specs, omega=OMEGA, dt=1e-3, autotune=True)
    sb, ab = s.member_blocks(0)
    _say(f"  chosen blocks synth={sb} anal={ab}")
    assert sb in (0, 2, 4, 8) and ab in (0, 2, 4, 8)
    a, _ = _states(s, specs)
    got = s.nonlinear(a).cpu().numpy()
    d = pkg.Sphere(specs, omega=OMEGA, dt=1e-3)
    d.set_member_blocks(0, 0, 0)
    ref = d.nonlinear(a).cpu().numpy()
    assert rel(got, ref) < 1e-13
    s.close()
    d.close()


def test_invalid_member_blocks_rejected():
    s = pkg.Sphere([(31, 0, 1e-3)] * 2, omega=OMEGA, dt=1e-3)
    for sb, ab in ((3, 2), (2, 16), (16, 2), (-1, 0), (32, 0)):
        with pytest.raises(pkg.NseError) as ei:
            s.set_member_blocks(0, sb, ab)
        assert ei.value.status == pkg.NSE_ERR_ARG
    with pytest.raises(pkg.NseError):
        s.set_member_blocks(5, 2, 2)
    s.close()


def test_mixed_truncation_ensemble_full_size_members_vs_oracle():
    """The 64-member mixed-truncation ensemble (24 x N=63, 24 x N=127, 16 x N=255):
    one nonlinear evaluation of every member in one call; the first and last member
    of each truncation checked against the oracle."""
    Ns = I.ensemble_truncations()
    nus = I.ensemble_viscosities(len(Ns))
    specs = [(N, 0, float(nu)) for N, nu in zip(Ns, nus)]
    _say(f"case: mixed-truncation ensemble, {len(specs)} members")
    s = pkg.Sphere(specs, omega=OMEGA, dt=1e-3)
    a, host = _states(s, specs)
    got = s.nonlinear(a).cpu().numpy()
    assert np.isfinite(got).all()
    for i in (0, 23, 24, 47, 48, 63):
        N = specs[i][0]
        ref = oracle_sphere(N, s.nlat[i]).nonlinear(O.to_tensor(host[i]), OMEGA).numpy()
        e = rel(got[s.member_slice(i)], ref)
        _say(f"  member {i} N={N}: rel err {e:.3e}")
        assert e < TOL
    s.close()
