"""Central finite differences of the FP64 oracle for the differentiated
droplet run (writes adjoint_droplet_fd.json beside this file).

Objective: J = y_c(N) - y_c(0), the displacement of the order-parameter
centroid y_c = sum c y / sum c (the droplet migration of Sec. IV C) after
N steps of the 256 x 512 droplet workload.  Controls: sigmaT and the bottom
wall temperature vector Tw_bot (256 values); the initial temperature field
is the steady conduction field of the walls, so it moves with Tw_bot.
Derivatives: (J(x + h e) - J(x - h e)) / (2 h) with h = 1e-6 along sigmaT,
along eight seeded Gaussian directions of Tw_bot and along sixteen seeded
unit vectors (wall components).  The wall derivatives are small
(|J| / |dJ/dTw[i]| ~ 1e3 or more), so the round-off of J limits the h = 1e-6
differences to a few 1e-4 relative; each is repeated with h = 1e-3, over
which J is linear in the wall values to far below that.

Only the oracle and the input generator are called.  The 99 oracle runs are
spread over worker processes (two OpenMP threads each); about 70 minutes
on eight cores:  python tests/golden/make_adjoint_fd.py
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

H = 1e-6
H_WALL = 1e-3
NSTEPS = 4000
N_COMPONENTS = 16
N_DIRECTIONS = 8
THREADS_PER_WORKER = 2


def components(nx):
    """Sixteen seeded wall components (distinct column indices, sorted)."""
    rng = np.random.default_rng(62381412)
    return sorted(int(i) for i in rng.choice(nx, N_COMPONENTS, replace=False))


def directions(nx):
    """Eight seeded Gaussian directions in the wall-temperature space."""
    rng = np.random.default_rng(14126238)
    return [rng.normal(0.0, 1.0, nx) for _ in range(N_DIRECTIONS)]


def objective(sigmaT, tb, nsteps=NSTEPS):
    from oracle import oracle
    from paper_1412_6238_amd import workloads as wl
    w = wl.make("adjoint_droplet", sigmaT=sigmaT)
    p = w["params"]
    tt = w["Twall_top"]
    T0 = wl.conduction_field(tb, tt[0], p["ny"])
    o = oracle.Oracle(p, tb, tt)
    o.init(w["phi0"], T0)
    y0 = o.diag()["centroid_y"]
    o.step(nsteps)
    return o.diag()["centroid_y"] - y0


def _job(args):
    sigmaT, tb = args
    return objective(sigmaT, np.asarray(tb))


def main():
    os.environ["OMP_NUM_THREADS"] = str(THREADS_PER_WORKER)
    from oracle import oracle
    from paper_1412_6238_amd import workloads as wl
    w = wl.make("adjoint_droplet")
    s0 = w["params"]["sigmaT"]
    tb = w["Twall_bot"]
    nx = tb.size
    comps = components(nx)
    dirs = directions(nx)
    # every objective evaluation, in a fixed order
    jobs = [("J", None, 0.0, s0, tb)]
    jobs += [("sT", None, sgn, s0 + sgn * H, tb) for sgn in (1, -1)]
    for k, d in enumerate(dirs):
        for h in (H, H_WALL):
            jobs += [("dir", (k, h), sgn, s0, tb + sgn * h * d) for sgn in (1, -1)]
    for i in comps:
        e = np.zeros(nx)
        e[i] = 1.0
        for h in (H, H_WALL):
            jobs += [("comp", (i, h), sgn, s0, tb + sgn * h * e) for sgn in (1, -1)]
    workers = max(1, (os.cpu_count() or 8) // THREADS_PER_WORKER)
    t0 = time.time()
    vals = []
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for k, v in enumerate(ex.map(_job, [(j[3], j[4]) for j in jobs])):
            vals.append(v)
            print(f"{k + 1}/{len(jobs)} {jobs[k][0]} {jobs[k][1]} {jobs[k][2]:+g}: {v!r} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    res = {}
    for (kind, key, sgn, _, _), v in zip(jobs, vals):
        res[(kind, key, sgn)] = v
    out = {"workload": "adjoint_droplet", "nsteps": NSTEPS, "h": H, "h_wall": H_WALL,
           "objective": "centroid_y(N) - centroid_y(0)",
           "threads": THREADS_PER_WORKER, "processes": workers,
           "oracle_threads_check": oracle.threads()}
    out["J"] = res[("J", None, 0.0)]
    out["dJ_dsigmaT"] = (res[("sT", None, 1)] - res[("sT", None, -1)]) / (2 * H)
    out["Twall_directions"] = [
        {"direction": d.tolist(),
         "dJ": (res[("dir", (k, H), 1)] - res[("dir", (k, H), -1)]) / (2 * H),
         "dJ_h_wall": (res[("dir", (k, H_WALL), 1)] - res[("dir", (k, H_WALL), -1)]) /
                      (2 * H_WALL)}
        for k, d in enumerate(dirs)]
    out["Twall_components"] = {
        str(i): (res[("comp", (i, H), 1)] - res[("comp", (i, H), -1)]) / (2 * H) for i in comps}
    out["Twall_components_h_wall"] = {
        str(i): (res[("comp", (i, H_WALL), 1)] - res[("comp", (i, H_WALL), -1)]) / (2 * H_WALL)
        for i in comps}
    with open(os.path.join(HERE, "adjoint_droplet_fd.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
