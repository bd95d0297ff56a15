"""Benchmark of the fused CSF lattice Boltzmann step on one MI355X.

A step is one pass of the whole path (three coupled D2Q9 lattices: stream,
moments, stencils, CSF force, three collisions, and the FP64 diagnostics
every --diag-every steps) over the 4096 x 4096 multi-droplet workload
(200 seeded droplets, R in [16, 48], dT/dy = 0.002), with every input already
resident in HBM.  Metric: million lattice updates per second (all three
lattices at one site = one update).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 2000] [--warmup 10] [--precision fp32_dev]
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# algorithmic bytes per site update: the 27 distributions read once and
# written once, 4 bytes each in the FP32 form (216) and 8 in FP64 (432)
BYTES_PER_SITE = {"fp32_dev": 216, "fp64": 432}
# bytes the state layout actually moves per site update: the FP32 form keeps
# the rest population g_0 in FP64, 2 x (26 x 4 + 8) = 224
STORED_BYTES_PER_SITE = {"fp32_dev": 224, "fp64": 432}
REPEATS = 5
# the step kernel and its launch shape and store policy (host_layout.h)
KERNEL_SOURCES = ("paper_1412_6238_amd/csrc/step_kernel.h", "paper_1412_6238_amd/csrc/lattice.h",
                  "paper_1412_6238_amd/csrc/host_layout.h")


def _code_only(text):
    """C++ source without its comments and with runs of white space made one
    space: what the compiler sees of it, up to formatting."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash():
    """Hash of the code of the step kernel's sources (comments and
    formatting excluded, so that editing them keeps the counter figures)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(_code_only(open(os.path.join(ROOT, f)).read()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, precision, sites, csf_form=0):
    """Measured HBM bytes per launch from the committed counter summary, if it
    was taken on the current kernel source (else None)."""
    form = "_curvature" if csf_form == 1 else ""
    path = os.path.join(ROOT, "profiles", f"traffic_step_{workload}_{precision}{form}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def _oracle_band_mlups(w, rows, seconds, threads=None):
    """MLUPS of the FP64 oracle stepping the lowest `rows` rows (full width,
    with the bottom wall) of workload w for about `seconds`."""
    from oracle import oracle
    p = w["params"]
    nx = p["nx"]
    rows = min(rows, p["ny"])
    o = oracle.Oracle(p, w["Twall_bot"], w["Twall_top"], window=(0, 0, nx, rows))
    o.init(np.ascontiguousarray(w["phi0"][:rows]), np.ascontiguousarray(w["T0"][:rows]))
    with oracle.thread_limit(threads):
        used = oracle.threads()
        t0 = time.perf_counter()
        o.step(1)
        t1 = time.perf_counter()
        n = max(1, int((seconds - (t1 - t0)) / max(t1 - t0, 1e-3)))
        o.step(n)
        t2 = time.perf_counter()
    steps = n + 1
    return nx * rows * steps / (t2 - t0) / 1e6, used, steps, t2 - t0, rows


def cpu_baseline(w, seconds=15.0):
    """The FP64 oracle on the host cores, on bands of the same workload (the
    lowest rows, full width, with the bottom wall): all threads for about
    `seconds` on 512 rows, then one thread for about seconds / 2 on 64 rows;
    MLUPS over each band's sites."""
    nx, ny = w["params"]["nx"], w["params"]["ny"]
    m_all, used, st_all, t_all, r_all = _oracle_band_mlups(w, 512, seconds)
    m_one, _, st_one, t_one, r_one = _oracle_band_mlups(w, 64, seconds / 2, threads=1)
    return {"value": round(m_all, 3), "unit": "MLUPS", "cores": used, "kind": "oracle",
            "single_thread": round(m_one, 3),
            "sample": f"FP64 oracle on the {nx}x{ny} workload's lowest rows (bottom wall "
                      f"included): rows 0-{r_all - 1} for {st_all} steps on {used} threads "
                      f"({t_all:.1f} s), rows 0-{r_one - 1} for {st_one} steps on 1 thread "
                      f"({t_one:.1f} s)"}


# the oracle's step counts per workload: the full run where it is feasible,
# else the first steps (the per-step cost does not change over a run)
ORACLE_TABLE = (("poiseuille", 20000), ("planar_marangoni", 50000), ("droplet", 1000),
                ("adjoint_droplet", 4000), ("multi_droplet", 20))


def oracle_table(single_fraction=0.1):
    """The FP64 oracle on each workload, on all host threads at the step
    counts above and on one thread for single_fraction of them (at least one
    step); prints one JSON line per run and a markdown table."""
    from oracle import oracle
    from paper_1412_6238_amd import workloads as wl
    rows = []
    for name, steps in ORACLE_TABLE:
        w = wl.make(name)
        p = w["params"]
        n = p["nx"] * p["ny"]
        for threads, nsteps in ((None, steps), (1, max(1, int(steps * single_fraction)))):
            o = oracle.Oracle(p, w["Twall_bot"], w["Twall_top"])
            o.init(w["phi0"], w["T0"])
            with oracle.thread_limit(threads):
                used = oracle.threads()
                t0 = time.perf_counter()
                o.step(nsteps)
                dt = time.perf_counter() - t0
            del o
            r = {"workload": f"{name} {p['nx']}x{p['ny']}", "steps": nsteps, "threads": used,
                 "seconds": round(dt, 2), "mlups": round(n * nsteps / dt / 1e6, 3)}
            rows.append(r)
            print(json.dumps(r), flush=True)
    print("| workload | steps | threads | s | MLUPS |\n|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['workload']} | {r['steps']} | {r['threads']} | {r['seconds']} | {r['mlups']} |")


def adjoint_bench(args, torch, lbe_csf, wl):
    """Cost of the gradient of a differentiated droplet run (default the
    256 x 512 run of 4000 steps; --adjoint-workload adjoint_droplet_wide is
    4096 x 1024, 400 steps): wall time of lbe_csf_backward (segment replay +
    adjoint sweep) over the wall time of the same N forward steps without
    recording, and over the recorded forward run; all timed with events on
    the handle's stream, the second of two repetitions reported."""
    w = wl.make(args.adjoint_workload)
    p = w["params"]
    nx, ny = p["nx"], p["ny"]
    N = args.adjoint_steps or w["nsteps"]
    prec = args.precision
    dev = torch.device("cuda:0")
    y = torch.arange(ny, dtype=torch.float64, device=dev)[:, None] + 0.5
    out = None
    for rep in range(2):
        plain = lbe_csf.Simulation(p, w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                                   precision=prec)
        ep = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ep[0].record(plain.stream)
        plain.step(N)
        ep[1].record(plain.stream)
        torch.cuda.synchronize()
        t_p = ep[0].elapsed_time(ep[1])
        del plain
        sim = lbe_csf.Simulation(p, w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                                 precision=prec, record_steps=N)
        st = sim.stream
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        e[0].record(st)
        sim.step(N, record=True)
        e[1].record(st)
        cN = 0.5 * (1.0 + sim.fields(("phi",))["phi"])
        seed = ((y - (cN * y).sum() / cN.sum()) / cN.sum()).expand(ny, nx).contiguous()
        torch.cuda.synchronize()
        e[2].record(st)
        g = sim.backward(seed, want_T0=True)   # synchronises at its end
        e[3].record(st)
        torch.cuda.synchronize()
        t_f = e[0].elapsed_time(e[1])
        t_b = e[2].elapsed_time(e[3])
        dtb = g["Twall"][0].cpu().numpy() + wl.conduction_field_T(g["T0"].cpu().numpy(), ny)
        out = {"metric": "adjoint cost (backward / forward)", "value": round(t_b / t_p, 3),
               "unit": "ratio", "higher_is_better": False, "n_gpus": 1,
               "backward_over_recorded_forward": round(t_b / t_f, 3),
               "forward_plain_ms": round(t_p, 3),
               "config": {"workload": f"{args.adjoint_workload} {nx}x{ny}", "steps": N,
                          "precision": prec, "checkpoint_spacing": int(np.ceil(np.sqrt(N)))},
               "forward_ms": round(t_f, 3), "backward_ms": round(t_b, 3),
               "forward_mlups": round(nx * ny * N / (t_f / 1e3) / 1e6, 1),
               "dJ_dsigmaT": g["sigmaT"], "dJ_dTw_bot_norm": float(np.linalg.norm(dtb)),
               "rep": rep}
        del sim
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp32_dev", choices=("fp32_dev", "fp64"))
    ap.add_argument("--workload", default="multi_droplet",
                    help="a named synthetic workload (poiseuille, planar_marangoni, droplet, "
                         "adjoint_droplet, multi_droplet, multi_droplet_slab) or one of the "
                         "paper's cases (paper_e1, paper_e2, paper_e3)")
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--rho2", type=float, default=0.0,
                    help="density of the c = 1 fluid (two densities; 0: one density)")
    ap.add_argument("--csf-form", type=int, default=0, choices=(0, 1),
                    help="capillary part of the CSF force: 0 potential form (default), "
                         "1 curvature form as printed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error-check", action="store_true",
                    help="skip the FP64 run that states the FP32 form's error")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--adjoint", action="store_true",
                    help="time the differentiated droplet run instead: a recorded forward "
                         "run and lbe_csf_backward (replay + reverse sweep); prints one JSON line")
    ap.add_argument("--adjoint-workload", default="adjoint_droplet",
                    help="workload of --adjoint (adjoint_droplet 256x512, or "
                         "adjoint_droplet_wide 4096x1024)")
    ap.add_argument("--adjoint-steps", type=int, default=0,
                    help="steps of --adjoint (default: the workload's)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of known size (for scaling HBM "
                         "byte counters) and exit")
    ap.add_argument("--oracle-table", action="store_true",
                    help="time only the FP64 oracle on every workload (all host threads, "
                         "then one thread) and exit")
    args = ap.parse_args()
    if args.oracle_table:
        oracle_table()
        return
    if args.calibrate_copy:
        import torch
        nbytes = 1 << 31
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_copy": nbytes,
                          "bytes_written_per_copy": nbytes, "copies": 10}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1412_6238_amd import lbe_csf, workloads as wl

    if args.adjoint:
        adjoint_bench(args, torch, lbe_csf, wl)
        return
    extra = {"rho2": args.rho2} if args.rho2 > 0 else {}
    if args.workload.startswith("paper_"):
        # the paper's own cases of Sec. IV at their printed sizes
        w = wl.paper_case(args.workload[len("paper_"):], csf_form=args.csf_form, **extra)
    else:
        w = wl.make(args.workload, csf_form=args.csf_form, **extra)
    p = w["params"]
    nx, ny = p["nx"], p["ny"]
    sites = nx * ny
    sim = lbe_csf.Simulation(p, w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                             precision=args.precision, diag_every=args.diag_every)
    stream = sim.stream
    torch.cuda.synchronize()
    sim.step(args.warmup)
    torch.cuda.synchronize()

    # REPEATS timed windows of exactly --steps steps each, every window
    # bracketed by a synchronisation, timed with HIP events on the handle's
    # stream (where the step kernel runs); the median window is reported
    windows = []
    t0 = time.perf_counter()
    for _ in range(REPEATS):
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        sim.step(args.steps)      # ends with one synchronising check of the diagnostics
        stop.record(stream)
        torch.cuda.synchronize()
        windows.append(start.elapsed_time(stop))
    wall = time.perf_counter() - t0
    ms = float(np.median(windows))
    ms_per_step = ms / args.steps
    mlups = sites * args.steps / (ms / 1e3) / 1e6
    hist = sim.diag_history()
    d_last = sim.diagnostics()
    mass_drift = None
    if hist:
        mass_drift = d_last["mass"] / hist[0]["mass"] - 1.0
    diag_in_windows = len([h for h in hist if h["step"] >= args.warmup])

    # dominant kernel: the fused step, one launch per step; its average
    # launch time is the window time over the steps (the window also holds
    # one small reduction launch per diagnostic step)
    bps = BYTES_PER_SITE[args.precision]
    stored = STORED_BYTES_PER_SITE[args.precision]
    if args.rho2 > 0:
        # two densities: the pressure pass reads the 27 values (half the
        # step's bytes) and writes the FP64 pressure of Eq. 9 (8 B), which
        # the step then reads (8 B)
        bps += bps // 2 + 8 + 8
        stored += stored // 2 + 8 + 8
    achieved = bps * sites / (ms_per_step / 1e3) / 1e9
    traffic = (traffic_from_profile(args.workload, args.precision, sites, args.csf_form)
               if args.rho2 <= 0 else None)
    out = {
        "metric": "MLUPS (3 coupled D2Q9 lattices)",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32_dev" else "f64",
        "data": "synthetic (seeded droplets, linear temperature)",
        "config": {"workload": f"{args.workload} {nx}x{ny}", "precision": args.precision,
                   "sites": sites, "diag_every": args.diag_every,
                   "capillary_form": "curvature" if args.csf_form == 1 else "potential",
                   "densities": [p["rho"], args.rho2] if args.rho2 > 0 else [p["rho"]],
                   "bytes_per_site_update": bps, "stored_bytes_per_site_update": stored},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic},
        "timing": {"windows": REPEATS, "steps_per_window": args.steps,
                   "ms_per_step_each": [round(t / args.steps, 5) for t in windows],
                   "statistic": "median window", "diag_steps_in_windows": diag_in_windows},
        "stored_bytes_frac": round(stored * sites / (ms_per_step / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
        "wall_s": round(wall, 3),
        "mass_drift": mass_drift,
        "n_nonfinite": d_last["n_nonfinite"],
        "kernel_hash": kernel_hash(),
    }
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / (bps * sites), 4)
    if args.precision == "fp32_dev" and not args.no_error_check:
        # the FP32 form's error at this step count: the FP64 path run from the
        # same inputs for the same number of steps (outside the timed region)
        a = sim.fields()
        del sim
        torch.cuda.empty_cache()
        ref = lbe_csf.Simulation(p, w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                                 precision="fp64", diag_every=0)
        ref.step(args.warmup + REPEATS * args.steps)
        b = ref.fields()
        del ref
        rel = lambda x, y: float(torch.linalg.norm(x - y) / torch.linalg.norm(y))
        out["fp32_vs_fp64"] = {
            "steps": args.warmup + REPEATS * args.steps,
            "phi": rel(a["phi"], b["phi"]),
            "u": rel(torch.stack([a["ux"], a["uy"]]), torch.stack([b["ux"], b["uy"]])),
            "T": rel(a["T"], b["T"]),
            "measure": "relative L2 of the FP32 form's fields against the FP64 path"}
        del a, b
    else:
        del sim
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
