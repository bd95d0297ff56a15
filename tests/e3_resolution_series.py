"""E3 resolution series (run by hand on a GPU; not collected by pytest).

The droplet of Sec. IV C refined at fixed Re, Ma, Ca and Cahn-Hilliard
Peclet number with the interface width fixed (workloads.paper_case("e3",
R, height)), in the potential and the curvature form of the capillary force.
For each reference time t_r it prints u_r / U_YGB averaged over that t_r (the
diagnostic of the printed formula, over the c >= 1/2 region), the velocity
of the c >= 1/2 centroid over the same t_r and the c >= 1/2 mass against its
start, and at the end one line "JSON [...]" with every figure.

    python tests/e3_resolution_series.py --radii 20 40 80 --t-r 6
    python tests/e3_resolution_series.py --radii 160 --forms 0 --t-r 2

R = 160 takes 1280 x 2400 sites and 1.28 M steps per t_r (about 3.5 minutes
per t_r in the FP32 form).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_1412_6238_amd import lbe_csf, workloads as wl  # noqa: E402


def run(R, form, n_tr, height, precision):
    w = wl.paper_case("e3", R=R, height=height, csf_form=form)
    m, p = w["meta"], w["params"]
    t_r = m["t_r"]
    every = max(1, t_r // 1600)   # 400 diagnostic records per quarter t_r
    sim = lbe_csf.Simulation(p, w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                             precision=precision, diag_every=every)

    def centroid():
        phi = sim.fields(("phi",))["phi"].cpu().numpy()
        c = 0.5 * (phi + 1.0)
        Y, _ = wl.coords(c.shape[1], c.shape[0])
        inside = c >= 0.5
        return float((c * Y)[inside].sum() / c[inside].sum()), float(c[inside].sum())

    y0, mass0 = centroid()
    t0 = time.time()
    u_r, vel, ys = [], [], [y0]
    for k in range(n_tr):
        hist = []
        for quarter in range(4):
            sim.step(t_r // 4)
            hist += sim.diag_history(4096)
            print(f"  R={R:g} form={form} t_r {k}+{quarter + 1}/4 ({time.time() - t0:.0f} s)",
                  flush=True)
        u_r.append(float(np.mean([d["u_r"] for d in hist]) / m["U_YGB"]))
        yc, mass = centroid()
        ys.append(yc)
        vel.append((ys[-1] - ys[-2]) / t_r / m["U_YGB"])
        print(f"R={R:g} form={form} t_r {k + 1}: u_r/U_YGB {u_r[-1]:.4f}  centroid/U_YGB "
              f"{vel[-1]:.4f}  mass(c>=1/2) {mass / mass0:.4f}", flush=True)
    return dict(R=R, form=form, height=height, precision=precision, nx=p["nx"], ny=p["ny"],
                t_r=t_r, u_r=u_r, centroid=vel)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--radii", type=float, nargs="+", default=[20.0, 40.0, 80.0])
    ap.add_argument("--forms", type=int, nargs="+", default=[0, 1], choices=(0, 1),
                    help="0 potential form, 1 curvature form")
    ap.add_argument("--t-r", type=int, default=6, help="reference times to run")
    ap.add_argument("--height", type=float, default=4.0,
                    help="droplet centre above the bottom wall, in radii")
    ap.add_argument("--precision", default="fp32_dev", choices=("fp32_dev", "fp64"))
    args = ap.parse_args()
    out = [run(R, form, args.t_r, args.height, args.precision)
           for R in args.radii for form in args.forms]
    print("JSON " + json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
