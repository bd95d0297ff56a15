"""Central finite differences of the FP64 oracle for the differentiated
droplet run (writes adjoint_droplet_fd.json beside this file).

Objective: J = y_c(N) - y_c(0), the displacement of the order-parameter
centroid y_c = sum c y / sum c (the droplet migration of Sec. IV C) after
N steps of the 256 x 512 droplet workload.  Controls: sigmaT and the bottom
wall temperature vector Tw_bot (256 values); the initial temperature field
is the steady conduction field of the walls, so it moves with Tw_bot.
Derivatives: (J(x + h e) - J(x - h e)) / (2 h) with h = 1e-6 along sigmaT,
along two seeded directions of Tw_bot and along three unit vectors.  The wall
derivatives are small (|J| / |dJ/dTw[i]| ~ 1e3), so the round-off of J limits
the h = 1e-6 differences to a few 1e-4 relative; they are repeated with
h = 1e-3, over which J is linear in the wall values to far below that.

Only the oracle and the input generator are called.  Takes about 18
minutes on eight cores:  python tests/golden/make_adjoint_fd.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle  # noqa: E402
from paper_1412_6238_amd import workloads as wl  # noqa: E402

H = 1e-6
H_WALL = 1e-3
NSTEPS = 4000
COMPONENTS = (0, 100, 200)


def directions(nx):
    """Two seeded directions in the wall-temperature space."""
    rng = np.random.default_rng(14126238)
    d1 = rng.normal(0.0, 1.0, nx)
    x = np.arange(nx) + 0.5
    d2 = np.cos(2.0 * np.pi * 3.0 * x / nx)
    return [d1, d2]


def objective(sigmaT, tb, nsteps=NSTEPS):
    w = wl.make("adjoint_droplet", sigmaT=sigmaT)
    p = w["params"]
    tt = w["Twall_top"]
    T0 = wl.conduction_field(tb, tt[0], p["ny"])
    o = oracle.Oracle(p, tb, tt)
    o.init(w["phi0"], T0)
    y0 = o.diag()["centroid_y"]
    o.step(nsteps)
    return o.diag()["centroid_y"] - y0


def main():
    w = wl.make("adjoint_droplet")
    s0 = w["params"]["sigmaT"]
    tb = w["Twall_bot"]
    nx = tb.size
    t0 = time.time()
    out = {"workload": "adjoint_droplet", "nsteps": NSTEPS, "h": H,
           "objective": "centroid_y(N) - centroid_y(0)", "threads": oracle.threads()}
    out["J"] = objective(s0, tb)
    print(f"J = {out['J']!r}  ({time.time() - t0:.0f} s)", flush=True)
    out["dJ_dsigmaT"] = (objective(s0 + H, tb) - objective(s0 - H, tb)) / (2 * H)
    print(f"dJ/dsigmaT = {out['dJ_dsigmaT']!r}  ({time.time() - t0:.0f} s)", flush=True)
    out["h_wall"] = H_WALL

    def wall_fd(d, h):
        return (objective(s0, tb + h * d) - objective(s0, tb - h * d)) / (2 * h)

    dirs = []
    for d in directions(nx):
        v, v3 = wall_fd(d, H), wall_fd(d, H_WALL)
        dirs.append({"direction": d.tolist(), "dJ": v, "dJ_h_wall": v3})
        print(f"dJ/dTw . d = {v!r} / {v3!r}  ({time.time() - t0:.0f} s)", flush=True)
    out["Twall_directions"] = dirs
    comps, comps3 = {}, {}
    for i in COMPONENTS:
        e = np.zeros(nx)
        e[i] = 1.0
        comps[str(i)], comps3[str(i)] = wall_fd(e, H), wall_fd(e, H_WALL)
        print(f"dJ/dTw[{i}] = {comps[str(i)]!r} / {comps3[str(i)]!r}  ({time.time() - t0:.0f} s)",
              flush=True)
    out["Twall_components"] = comps
    out["Twall_components_h_wall"] = comps3
    with open(os.path.join(HERE, "adjoint_droplet_fd.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
