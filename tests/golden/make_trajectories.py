"""Writes the stored oracle trajectories used by the full-length parity tests.

Calls only the FP64 CPU oracle (`oracle/nse_oracle.py`) and the seeded input
recipes (`nse_inputs`); nothing here touches the HIP library.

Workloads (fixed-step NDF2 of eq. (ode_disc), one nonlinear evaluation per step,
Omega = 2 pi, dt = 1e-3, nu = 1e-5, seeded initial spectrum (seed 1) and
constant forcing (seed 2, scale 1e-2)):
  * t255: N = 255 on 384 x 768, the state after 1000 steps;
  * t511: N = 511 on 768 x 1536, the states after 1 and after 200 steps.

Output per workload: `traj_<name>.npz` (complex128 arrays named `step<k>`, the
newest history slot after k steps) and `traj_<name>.json` (parameters, the
SHA-256 of the initial state and forcing bytes, and of each stored array).

Usage: python tests/golden/make_trajectories.py [t255] [t511]
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import nse_inputs as I  # noqa: E402
from oracle import nse_oracle as O  # noqa: E402

OMEGA = 2.0 * math.pi
WORKLOADS = {
    "t255": dict(N=255, nu=1e-5, dt=1e-3, order=2, save=(1000,)),
    "t511": dict(N=511, nu=1e-5, dt=1e-3, order=2, save=(1, 200)),
}


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def input_hash(N: int) -> str:
    """SHA-256 over the bytes of the initial state and the forcing."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(I.initial_state(N)).tobytes())
    h.update(np.ascontiguousarray(I.forcing(N)).tobytes())
    return h.hexdigest()


def run(name: str) -> None:
    w = WORKLOADS[name]
    N = w["N"]
    a0, f = I.initial_state(N), I.forcing(N)
    S = O.Sphere(N)
    st = O.Stepper(S, w["nu"], OMEGA, w["dt"], order=w["order"])
    hist = [O.to_tensor(a0)] + [torch.zeros(len(a0), dtype=O.C128) for _ in range(w["order"])]
    out = {}
    t0 = time.time()
    for k in range(max(w["save"])):
        hist = st.step(hist, O.to_tensor(f), k)
        if k + 1 in w["save"]:
            out[f"step{k + 1}"] = hist[0].numpy().copy()
        if (k + 1) % 50 == 0:
            print(f"{name}: step {k + 1} ({time.time() - t0:.0f} s)", flush=True)
    np.savez(os.path.join(HERE, f"traj_{name}.npz"), **out)
    meta = {
        "workload": f"NDF2 fixed step, N={N}, nlat={S.grid.nlat}, M={S.grid.M}, "
                    f"nu={w['nu']}, Omega=2pi, dt={w['dt']}, newton_iters=1",
        "N": N, "nlat": S.grid.nlat, "nu": w["nu"], "dt": w["dt"], "order": w["order"],
        "omega": OMEGA,
        "initial_state": "nse_inputs.initial_state(N) (seed 1)",
        "forcing": "nse_inputs.forcing(N) (seed 2, scale 1e-2)",
        "input_sha256": input_hash(N),
        "arrays": {k: sha256(v) for k, v in out.items()},
        "writer": "tests/golden/make_trajectories.py (FP64 CPU oracle only)",
    }
    with open(os.path.join(HERE, f"traj_{name}.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
        fh.write("\n")
    print(f"{name}: done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(WORKLOADS):
        run(name)
