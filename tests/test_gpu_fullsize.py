"""Full-size parity of the HIP path (through the C ABI) with the FP64 oracle on
inputs that carry weight at every degree and order.

The seeded workload spectrum decays like e^(-l/8), so a global relative norm on it
cannot see coefficients above l ~ 150. Here the inputs are flat spectra
(`nse_inputs.flat_spectrum`: the same law at every degree) and N(0,1) grid noise,
and every output is checked twice:

  * relative l2 error <= 1e-12 (the FP64 bar per evaluation), which on these
    inputs weighs every degree and order alike;
  * every coefficient: |got - ref| <= 5e-11 S, S the largest per-degree RMS of the
    reference. For these inputs every degree's RMS is within a factor ~1e4 of S,
    so an error in any one coefficient (a wrong index, order, seed row, tile or
    XCD mapping) is far above this bar. The bar is set by the rounding of the
    formulation, not by the oracle: the GPU evaluates the advection in the scalar
    form u . Grad(zeta_a), whose rounding error grows like |u| |Grad zeta_a|,
    a factor of order N above the vector form the oracle uses. An FP64 CPU
    evaluation of the scalar form (exact-phase transforms) lies 1.9e-12 S (N =
    255) and 1.0e-11 S (N = 511) from an 80-bit evaluation, the oracle 2.9e-13 S
    and 8.5e-13 S;
  * grid outputs: every point |got - ref| <= 1e-11 RMS of the reference field
    (FP64 rounding of the Gauss nodes moves values of degree ~N by ~N^2 ulps at
    the polar rows; the oracle itself is 1.8e-12 RMS from an 80-bit evaluation
    there at N = 255).
The error relative to each degree's own RMS is reported and held to 1e-6 (at
N = 511 the degree-1 RMS is 1e-4 S).

Trajectories (the seeded workload spectrum, as the workloads define it) are
compared with oracle trajectories stored by `tests/golden/make_trajectories.py`
(oracle only; the stored input hash is checked first).
"""
import hashlib
import json
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
TOL = 1e-12          # relative l2 (and trajectories)
COEF_TOL = 5e-11     # every coefficient, against the largest per-degree RMS
POINT_TOL = 1e-11    # every grid point, against the field's RMS
DEGREE_TOL = 1e-6    # every coefficient, against its own degree's RMS
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


_SPHERES = {}


def oracle_sphere(N, nlat=None):
    key = (N, nlat)
    if key not in _SPHERES:
        _SPHERES.clear()          # one full-size oracle at a time (T511 holds ~2 GB)
        _SPHERES[key] = O.Sphere(N, nlat)
    return _SPHERES[key]


def spectral_errors(got, ref, N):
    """(max |got - ref| / S, max over degrees of max |got - ref| / RMS_l, worst l)."""
    ls, _ = I.degrees_orders(N)
    err = np.abs(np.asarray(got) - np.asarray(ref))
    cnt = np.bincount(ls, minlength=N + 1)
    rms = np.sqrt(np.bincount(ls, weights=np.abs(ref) ** 2, minlength=N + 1) / cnt)
    S = rms[1:].max()
    emax = np.zeros(N + 1)
    np.maximum.at(emax, ls, err)
    per = np.where(rms > 0, emax / np.where(rms > 0, rms, 1.0), 0.0)
    per[0] = 0.0
    return float(err.max() / S), float(per.max()), int(per.argmax()), float(rms[1:].min() / S)


def check_spectral(got, ref, N, label):
    e, ed, lw, spread = spectral_errors(got, ref, N)
    r = float(np.linalg.norm(np.asarray(got) - ref) / np.linalg.norm(ref))
    _say(f"  {label}: rel l2 {r:.3e}; max coefficient err / S {e:.3e}; worst per-degree "
         f"{ed:.3e} at l={lw} (min/max degree RMS {spread:.2e})")
    assert r <= TOL, (label, r)
    assert e <= COEF_TOL, (label, e)
    assert ed <= DEGREE_TOL, (label, ed, lw)


@pytest.mark.parametrize("N", [255, 511])
def test_flat_nonlinear_every_coefficient(N):
    _say(f"case: flat-spectrum nonlinear N={N}")
    s = pkg.Sphere([(N, 0, 1e-5)], omega=OMEGA, dt=1e-3)
    a = I.flat_spectrum(N, 0)
    got = s.nonlinear(pkg.to_device(a)).cpu().numpy()
    s.close()
    ref = oracle_sphere(N).nonlinear(O.to_tensor(a), OMEGA).numpy()
    check_spectral(got, ref, N, "n")
    _, ms = I.degrees_orders(N)
    assert np.abs(ref[ms > 400] if N > 400 else ref[ms > N - 40]).max() > 0


@pytest.mark.parametrize("N", [255, 511])
def test_flat_synthesis_every_point(N):
    _say(f"case: flat-spectrum synthesis N={N}")
    s = pkg.Sphere([(N, 0, 0.0)], omega=OMEGA, dt=1e-3)
    a = I.flat_spectrum(N, 1)
    ut, up, ze = s.synthesize(pkg.to_device(a))[0].cpu().numpy()
    s.close()
    S = oracle_sphere(N)
    rt, rp = (x.numpy() for x in S.velocity(O.to_tensor(a)))
    rz = S.vorticity(O.to_tensor(a)).numpy()
    for name, g, r in (("u_theta", ut, rt), ("u_phi", up, rp), ("zeta", ze, rz)):
        rms = float(np.sqrt(np.mean(r ** 2)))
        e = float(np.abs(g - r).max()) / rms
        rl = float(np.linalg.norm(g - r) / np.linalg.norm(r))
        _say(f"  {name}: rel l2 {rl:.3e}; max point err / RMS {e:.3e}")
        assert rl <= TOL, (name, rl)
        assert e <= POINT_TOL, (name, e)


@pytest.mark.parametrize("N", [255, 511])
def test_grid_noise_projection_every_coefficient(N):
    _say(f"case: grid-noise projection N={N}")
    s = pkg.Sphere([(N, 0, 1e-5)], omega=OMEGA, dt=1e-3)
    nl = s.nlat[0]
    u = I.grid_noise(21, nl, 2 * nl)
    got = s.analyze_velocity([torch.as_tensor(u, device="cuda")]).cpu().numpy()
    s.close()
    S = oracle_sphere(N)
    ref = O.clean(S.project(torch.as_tensor(u[0]), torch.as_tensor(u[1])), N).numpy()
    check_spectral(got, ref, N, "(u, Z)_M")


@pytest.mark.parametrize("N", [255, 511])
def test_flat_nonlinear_adjoint_every_coefficient(N):
    _say(f"case: flat-spectrum nonlinear adjoint N={N}")
    s = pkg.Sphere([(N, 0, 1e-5)], omega=OMEGA, dt=1e-3)
    a, nb = I.flat_spectrum(N, 2), I.cotangent(N, 9)
    got = s.nonlinear_adjoint(pkg.to_device(a), pkg.to_device(nb)).cpu().numpy()
    s.close()
    S = oracle_sphere(N)
    at = O.to_tensor(a).requires_grad_(True)
    L = (O.to_tensor(nb).conj() * S.nonlinear(at, OMEGA)).real.sum()
    (g,) = torch.autograd.grad(L, at)
    check_spectral(got, g.numpy(), N, "J^T n_bar")


def _stored(name):
    with open(os.path.join(GOLDEN, f"traj_{name}.json")) as fh:
        meta = json.load(fh)
    N = meta["N"]
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(I.initial_state(N)).tobytes())
    h.update(np.ascontiguousarray(I.forcing(N)).tobytes())
    assert h.hexdigest() == meta["input_sha256"], "seeded inputs changed since the oracle run"
    with np.load(os.path.join(GOLDEN, f"traj_{name}.npz"), allow_pickle=False) as z:
        arrays = {k: z[k] for k in z.files}
    for k, v in arrays.items():
        assert hashlib.sha256(np.ascontiguousarray(v).tobytes()).hexdigest() == meta["arrays"][k]
    return meta, arrays


def trajectory_errors(got, ref):
    """(relative l2 error, max coefficient error / max |ref|)."""
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return rel, float(np.abs(got - ref).max() / np.abs(ref).max())


def _run(meta, steps, precision="fp64", graph=True):
    N = meta["N"]
    s = pkg.Sphere([(N, 0, meta["nu"])], omega=meta["omega"], dt=meta["dt"], order=meta["order"],
                   precision=precision, graph=graph, stream=torch.cuda.current_stream())
    assert s.nlat[0] == meta["nlat"]
    hist = s.new_history()
    hist[0] = pkg.to_device(I.initial_state(N))
    f = pkg.to_device(I.forcing(N))
    out, done = {}, 0
    for k in steps:
        s.step(hist, f, done, k - done)
        done = k
        out[k] = hist[0].cpu().numpy()
    s.close()
    return out


def test_t255_1000_steps_vs_stored_oracle():
    meta, ref = _stored("t255")
    _say(f"case: {meta['workload']}, 1000 steps vs the stored oracle trajectory")
    got = _run(meta, [1000])[1000]
    r, e = trajectory_errors(got, ref["step1000"])
    _say(f"  1000 steps: rel l2 {r:.3e}, max coefficient err / max {e:.3e}")
    assert r <= TOL and e <= TOL


def test_t511_fp64_steps_vs_stored_oracle():
    meta, ref = _stored("t511")
    _say(f"case: {meta['workload']}, FP64, 1 and 200 steps vs the stored oracle trajectory")
    got = _run(meta, [1, 200])
    for k in (1, 200):
        r, e = trajectory_errors(got[k], ref[f"step{k}"])
        _say(f"  {k} steps: rel l2 {r:.3e}, max coefficient err / max {e:.3e}")
        assert r <= TOL and e <= TOL


def _field_errors(sph, got, ref):
    g = sph.synthesize(pkg.to_device(got))[0].cpu().numpy()
    r = sph.synthesize(pkg.to_device(ref))[0].cpu().numpy()
    return [float(np.linalg.norm(g[i] - r[i]) / np.linalg.norm(r[i])) for i in range(3)]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_t511_reduced_precision_fields_vs_stored_oracle(prec):
    """Relative error of each grid field (u_theta, u_phi, zeta) against the FP64
    oracle's trajectory after 1 and after 200 steps; bar 1e-6. Both states are
    put on the grid by the FP64 synthesis (a linear map checked above)."""
    meta, ref = _stored("t511")
    _say(f"case: {meta['workload']}, {prec}, fields after 1 and 200 steps vs the oracle")
    got = _run(meta, [1, 200], precision=prec)
    s64 = pkg.Sphere([(meta["N"], 0, 0.0)], omega=OMEGA, dt=1e-3)
    for k in (1, 200):
        errs = _field_errors(s64, got[k], ref[f"step{k}"])
        _say(f"  {k} steps: u_theta {errs[0]:.3e} u_phi {errs[1]:.3e} zeta {errs[2]:.3e}")
        assert max(errs) < 1e-6
    s64.close()
