"""The paper's own three test cases at their printed parameters (Sec. IV), on
the GPU through the C ABI.

  E1  layered thermal Poiseuille flow, 40 x 100, eta_r = 10, lambda_r in
      {1, 10, 100}, h/H in {1, 1/9, 9} (Sec. IV A, Eqs. 28-29)
  E2  two superimposed planar fluids, 200 x 100, lambda_r in {1, 0.1}
      (Sec. IV B, the Pendse-Esmaeeli fields)
  E3  thermocapillary droplet, R = 20 in 160 x 300, |grad T| = 0.1
      (Sec. IV C, u_r / U_YGB)

Each case first runs a short FP64 parity check against the CPU oracle, then
the full run.  The bars are physical: E1 against the steady diffuse-interface
solution (viscosity and conductivity linear in c across the tanh profile) and
against the sharp-interface Eqs. 28-29; E2 against the corrected
Pendse-Esmaeeli solution; E3 against the migration velocity printed in
Sec. IV C, which the method reaches only where the interface relaxes fast
(large mobility).  Every figure is printed for the record.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_1412_6238_amd import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
import analytic as an  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbe():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_6238_amd import lbe_csf
    return lbe_csf


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _sim(lbe, w, precision="fp64", **kw):
    return lbe.Simulation(w["params"], w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                          precision=precision, **kw)


def _fields(sim):
    return {k: v.cpu().numpy() for k, v in sim.fields().items()}


def _parity(lbe, oracle_mod, w, nsteps, floor=False):
    """FP64 GPU against the oracle on the case's own parameters, run in the
    p0 = 0 gauge (exact for the method; it keeps the populations near the
    size of what they encode) and with p compared in the p0 = 1/3 gauge.
    With ``floor`` the velocity is held to ten times the oracle's own
    round-off sensitivity where that exceeds 1e-12: on a flat interface the
    Marangoni flow is the residue of capillary terms that cancel, and the
    oracle itself moves by ~1e-12 when its initial phi is perturbed at 2e-16."""
    w = dict(w, params=dict(w["params"], p0=0.0))
    sim = _sim(lbe, w)
    orc = oracle_mod.Oracle(w["params"], w["Twall_bot"], w["Twall_top"]).init(w["phi0"], w["T0"])
    sim.step(nsteps)
    orc.step(nsteps)
    g, o = _fields(sim), orc.fields()
    ug, uo = np.stack([g["ux"], g["uy"]]), np.stack([o["ux"], o["uy"]])
    errs = {k: _rel(g[k], o[k]) for k in ("phi", "T")}
    errs["p"] = _rel(g["p"] + 1 / 3, o["p"] + 1 / 3)
    errs["u"] = _rel(ug, uo)
    bar_u = 1e-12
    if floor:
        rng = np.random.default_rng(0)
        phi_b = w["phi0"] * (1 + 2e-16 * rng.choice([-1.0, 1.0], w["phi0"].shape))
        ob = oracle_mod.Oracle(w["params"], w["Twall_bot"], w["Twall_top"]).init(phi_b, w["T0"])
        ob.step(nsteps)
        fb = ob.fields()
        fl = _rel(np.stack([fb["ux"], fb["uy"]]), uo)
        bar_u = max(1e-12, 10 * fl)
        _say(f"  oracle round-off floor of u {fl:.1e}")
    _say("  parity vs oracle " + " ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= (bar_u if k == "u" else 1e-12), (k, v)


# ---- E1 -------------------------------------------------------------------------
E1 = [(1, 1.0), (10, 1.0), (100, 1.0), (10, 1.0 / 9.0), (10, 9.0)]


@pytest.mark.parametrize("lam_r,h_r", E1)
def test_e1_layered_poiseuille(lbe, oracle_mod, lam_r, h_r):
    """Sec. IV A.  After about two viscous times the x-averaged profiles match
    the steady diffuse-interface solution (u within 2e-3; T within 1e-3 where
    the run spans several thermal times, 1.5e-2 at lambda_r = 100, whose
    thermal time 2.5e6 exceeds the run); their distance from the
    sharp-interface Eqs. 28-29 is the diffuse-interface error of the
    eta_r = 10 viscosity jump (7-10%) and of the conductivity jump."""
    w = wl.paper_case("e1", lam_r=lam_r, h_r=h_r)
    m, p = w["meta"], w["params"]
    _say(f"case E1 lam_r={lam_r} h_r={h_r:.4f}: parity 3000 steps, then {w['nsteps']} steps")
    _parity(lbe, oracle_mod, w, 3000)
    sim = _sim(lbe, w)
    sim.step(w["nsteps"])
    f = _fields(sim)
    ny = p["ny"]
    u_d, T_d = an.layered_1d_steady(ny, m["h"], p["width"], m["eta1"], m["eta2"], m["lam1"],
                                    m["lam2"], m["ax"], m["Tc"], m["Th"])
    yr = np.arange(ny) + 0.5 - m["h"]
    u_s = an.poiseuille_ux(yr, m["h"], m["H"], m["eta1"], m["eta2"], 1.0, m["ax"])
    T_s = an.poiseuille_T(yr, m["h"], m["H"], m["lam1"], m["lam2"], m["Tc"], m["Th"])
    ux, T = f["ux"].mean(axis=1), f["T"].mean(axis=1)
    e = dict(u_diffuse=_rel(ux, u_d), T_diffuse=_rel(T, T_d), u_sharp=_rel(ux, u_s),
             T_sharp=_rel(T, T_s))
    _say("  " + " ".join(f"{k} {v:.2e}" for k, v in e.items()) +
         f"  (u_max {np.abs(u_s).max():.2e}, a_x {m['ax']:.3e})")
    assert np.abs(f["ux"] - ux[:, None]).max() <= 1e-12 * np.abs(ux).max()
    assert np.abs(f["uy"]).max() <= 1e-6 * np.abs(ux).max()
    assert e["u_diffuse"] <= 2e-3
    assert e["T_diffuse"] <= (1.5e-2 if lam_r == 100 else 1e-3)
    assert e["u_sharp"] <= 0.12
    assert e["T_sharp"] <= (1e-10 if lam_r == 1 else 0.15)


# ---- E2 -------------------------------------------------------------------------
@pytest.mark.parametrize("lam_r,form,bar_u,bar_T", [(1.0, 1, 0.06, 1e-3), (0.1, 1, 0.10, 2e-2),
                                                    (1.0, 0, 0.30, 1e-3)])
def test_e2_planar_marangoni(lbe, oracle_mod, lam_r, form, bar_u, bar_T):
    """Sec. IV B after three thermal times of the less conducting layer.  With
    the curvature form of Eq. 4 the velocity is within 6% (lambda_r = 1) and
    10% (lambda_r = 0.1) of the sharp-interface solution, the deviation
    growing as lambda_r falls, as the paper reports.  The potential form at
    the printed mobility is 25% low: its capillary term resists the
    stretching of the interface profile by the Marangoni flow (a stress of
    order sigma0 times the profile's departure from equilibrium, which the
    Cahn-Hilliard relaxation at rate ~M/W^2 keeps small only for large M)."""
    w = wl.paper_case("e2", lam_r=lam_r, csf_form=form)
    m, p = w["meta"], w["params"]
    _say(f"case E2 lam_r={lam_r} form={form}: parity 1000 steps, then {w['nsteps']} steps")
    if form == 1:
        _parity(lbe, oracle_mod, w, 1000, floor=True)
    sim = _sim(lbe, w)
    sim.step(w["nsteps"])
    f = _fields(sim)
    nx, ny = p["nx"], p["ny"]
    Y, X = wl.coords(nx, ny)
    ux, uy, T, _ = an.planar_marangoni(X, Y - ny / 2, nx, m["h"], m["H"], m["eta1"], m["eta2"],
                                       m["lam1"], m["lam2"], m["Tc"], m["Th"], m["Tr"],
                                       m["sigma_T"])
    e = dict(ux=_rel(f["ux"], ux), uy=_rel(f["uy"], uy), T=_rel(f["T"], T))
    _say("  vs Pendse-Esmaeeli " + " ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert e["ux"] <= bar_u and e["uy"] <= bar_u and e["T"] <= bar_T
    # the interface flows from the hot (x = 0) to the cold side
    assert f["ux"][ny // 2, nx // 4] > 0
    if form == 0:
        assert e["ux"] >= 0.15     # the documented deviation of this form


def test_e2_potential_form_converges_with_mobility(lbe):
    """The potential form's deviation on E2 is set by sigma0 / M: at ten times
    the printed mobility (tau_g = 5.5, Gamma = 0.1) it falls below 5%."""
    w = wl.paper_case("e2", lam_r=1.0, csf_form=0, mobility=0.5, tau_g=5.5)
    m, p = w["meta"], w["params"]
    _say("case E2 potential form M = 0.5")
    sim = _sim(lbe, w)
    sim.step(w["nsteps"])
    f = _fields(sim)
    Y, X = wl.coords(p["nx"], p["ny"])
    ux, uy, T, _ = an.planar_marangoni(X, Y - p["ny"] / 2, p["nx"], 50.0, 50.0, 0.2, 0.2, 0.2,
                                       0.2, m["Tc"], m["Th"], m["Tr"], m["sigma_T"])
    e = (_rel(f["ux"], ux), _rel(f["uy"], uy))
    _say(f"  u_x {e[0]:.2e} u_y {e[1]:.2e}")
    assert max(e) <= 0.05


# ---- E3 -------------------------------------------------------------------------
def _migration(lbe, w, nsteps=200000, every=50, precision="fp64"):
    """u_r / U_YGB averaged over each t_r (20000 steps at R = 20; the printed
    formula, sites with c >= 1/2), and the displacement of the thresholded
    droplet centroid per t_r in units of U_YGB."""
    m = w["meta"]
    sim = _sim(lbe, w, precision=precision, diag_every=every)

    def cen():
        f = _fields(sim)
        c = 0.5 * (f["phi"] + 1)
        Y, _ = wl.coords(*c.shape[::-1])
        msk = c >= 0.5
        return float((c * Y)[msk].sum() / c[msk].sum())

    y0 = cen()
    hist = []
    for _ in range(nsteps // m["t_r"]):
        sim.step(m["t_r"])
        hist += sim.diag_history(4096)
    y1 = cen()
    st = np.array([d["step"] for d in hist])
    ur = np.array([d["u_r"] for d in hist]) / m["U_YGB"]
    win = [float(ur[(st >= k * m["t_r"]) & (st < (k + 1) * m["t_r"])].mean())
           for k in range(nsteps // m["t_r"])]
    vc = (y1 - y0) / nsteps / m["U_YGB"]
    return win, vc


@pytest.mark.parametrize("form", [0, 1])
def test_e3_isothermal_droplet_rests(lbe, oracle_mod, form):
    """Without a surface-tension gradient the saturated droplet does not move
    (|u_r| below 0.1 U_YGB next to the wall; the printed geometry)."""
    w = wl.paper_case("e3", csf_form=form, sigmaT=0.0)
    _say(f"case E3 isothermal form={form}: parity 300 steps, then 200000 steps")
    _parity(lbe, oracle_mod, w, 300)
    win, vc = _migration(lbe, w)
    _say("  u_r/U_YGB per t_r " + " ".join(f"{v:.3f}" for v in win) + f"  centroid {vc:.3f}")
    assert max(abs(v) for v in win) <= 0.1 and abs(vc) <= 0.1


def test_e3_droplet_migration(lbe):
    """Sec. IV C at the printed parameters (potential form, mobility 5e-2, the
    matrix at the droplet's saturation).  The droplet migrates towards the
    hot wall, u_r and the displacement of its c >= 1/2 centroid agree, but
    at 0.12 U_YGB, far below the printed u_r / U_YGB ~ 0.8 (Fig. 9): the
    ratio sigma0 W^2 / (M eta R) = 8 keeps the interface profile far from
    equilibrium under the Marangoni flow.  Raising the mobility at fixed
    Gamma = 0.1 (tau_g = 1/2 + 10 M) raises u_r monotonically, to the
    printed value at M = 2; there, however, the Cahn-Hilliard flux lets the
    fluid pass through the interface and the droplet itself moves at a
    fraction of u_r.  No mobility gives both at once."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    printed = g["u_r_over_U_YGB_droplet"]["value"]
    res, cen = {}, {}
    for M in (0.05, 0.5, 2.0):
        w = wl.paper_case("e3", mobility=M, tau_g=0.5 + M / 0.1)
        _say(f"case E3 potential form M={M} 200000 steps")
        win, vc = _migration(lbe, w)
        res[M], cen[M] = float(np.mean(win[2:])), vc
        _say("  u_r/U_YGB per t_r " + " ".join(f"{v:.3f}" for v in win) +
             f"  mean(t_r 2-10) {res[M]:.3f}  thresholded centroid {vc:.3f}")
    assert 0.05 <= res[0.05] <= 0.3 and abs(cen[0.05] - res[0.05]) <= 0.05
    assert res[0.05] < res[0.5] < res[2.0]
    assert abs(res[2.0] - printed) <= 0.2
    assert cen[2.0] <= 0.5 * res[2.0]


def test_e3_curvature_form_at_printed_mobility(lbe):
    """With the curvature form at the printed mobility the same profile
    response acts as a net normal force (sigma0 times the thinning of the
    profile at the hot pole and its thickening at the cold pole) that exceeds
    the Marangoni propulsion: the droplet moves towards the cold wall.  Kept
    as a recorded property of the method at these parameters."""
    w = wl.paper_case("e3", csf_form=1)
    _say("case E3 curvature form M=0.05 60000 steps")
    win, vc = _migration(lbe, w, nsteps=60000)
    _say("  u_r/U_YGB per t_r " + " ".join(f"{v:.3f}" for v in win) + f"  centroid {vc:.3f}")
    assert max(win) < 0 and vc < 0


def test_e3_resolution_trend(lbe):
    """The droplet of Sec. IV C refined at fixed Re, Ma, Ca and Cahn-Hilliard
    Peclet number with the interface width fixed (R = 20 and 40, so the
    Cahn number W / R halves), 4R above the bottom wall, both capillary
    forms, in the FP32 form.  u_r / U_YGB rises with R in both forms and the
    gap between the forms closes: the printed geometry is far from the
    sharp-interface limit, which both forms approach from below (at R = 80:
    0.49 potential, 0.18 curvature; R = 20: 0.14 and -1.27)."""
    res = {}
    for R in (20.0, 40.0):
        for form in (0, 1):
            w = wl.paper_case("e3", R=R, height=4.0, csf_form=form)
            t_r = w["meta"]["t_r"]
            _say(f"case E3 R={R:.0f} form={form}, 3 t_r = {3 * t_r} steps, fp32_dev")
            win, vc = _migration(lbe, w, nsteps=3 * t_r, every=max(1, t_r // 400),
                                 precision="fp32_dev")
            res[(R, form)] = float(np.mean(win[1:]))
            _say("  u_r/U_YGB per t_r " + " ".join(f"{v:.3f}" for v in win) +
                 f"  mean(t_r 2-3) {res[(R, form)]:.3f}  thresholded centroid {vc:.3f}")
    assert res[(40.0, 0)] > res[(20.0, 0)] + 0.1
    assert res[(40.0, 1)] > res[(20.0, 1)] + 0.4
    gap20 = abs(res[(20.0, 0)] - res[(20.0, 1)])
    gap40 = abs(res[(40.0, 0)] - res[(40.0, 1)])
    assert gap40 < 0.75 * gap20


@pytest.mark.parametrize("name,kw", [("e1", dict(lam_r=10, h_r=1.0)), ("e2", dict(lam_r=1.0)),
                                     ("e2", dict(lam_r=1.0, csf_form=1)), ("e3", {})])
def test_paper_cases_fp32_matches_fp64(lbe, name, kw):
    """The FP32 deviation form against the FP64 path over the full runs of
    the paper's cases (500,000 / 37,500 / 200,000 steps): relative L2 on phi,
    u and T within 1e-4."""
    w = wl.paper_case(name, **kw)
    _say(f"case paper {name} {kw} fp32_dev vs fp64, {w['nsteps']} steps")
    res = {}
    for prec in ("fp64", "fp32_dev"):
        sim = _sim(lbe, w, precision=prec)
        sim.step(w["nsteps"])
        res[prec] = _fields(sim)
        del sim
    a, b = res["fp32_dev"], res["fp64"]
    e = dict(phi=_rel(a["phi"], b["phi"]),
             u=_rel(np.stack([a["ux"], a["uy"]]), np.stack([b["ux"], b["uy"]])),
             T=_rel(a["T"], b["T"]))
    _say("  " + " ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert max(e.values()) <= 1e-4
