"""The inputs of the paper's own cases (Sec. IV) carry the printed numbers:
meshes, transport coefficients and their ratios, surface tension, wall
temperatures, droplet size and place; and the seeded generators are
reproducible."""
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_1412_6238_amd import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
import analytic as an  # noqa: E402

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
eta = lambda tau: (tau - 0.5) / 3.0     # rho = 1
lam = lambda tau: (tau - 0.5) / 3.0     # rho = cv = 1


@pytest.mark.parametrize("lam_r,h_r", [(1, 1.0), (10, 1.0), (100, 1.0), (10, 1 / 9), (10, 9.0)])
def test_e1_inputs(lam_r, h_r):
    w = wl.paper_case("e1", lam_r=lam_r, h_r=h_r)
    p, m = w["params"], w["meta"]
    assert [p["nx"], p["ny"]] == GOLD["mesh_poiseuille"]["value"]
    # fluid 1 (c = 0) below with eta1 = lambda1 = 0.1; eta_r = 10; lambda_r as asked
    assert eta(p["tau_f"][0]) == pytest.approx(0.1) and lam(p["tau_T"][0]) == pytest.approx(0.1)
    assert eta(p["tau_f"][0]) / eta(p["tau_f"][1]) == pytest.approx(10.0)
    assert lam(p["tau_T"][0]) / lam(p["tau_T"][1]) == pytest.approx(lam_r)
    assert m["h"] / m["H"] == pytest.approx(h_r) and m["h"] + m["H"] == p["ny"]
    assert p["width"] == pytest.approx(2 * math.sqrt(2)) and p["beta"] == 0.25
    # Re = u1 h / eta1 = 1 with u1 = rho a h^2 / (2 eta1), unless capped at |u| = 0.01
    u1 = p["force"][0] * m["h"] ** 2 / (2 * 0.1)
    yr = np.linspace(-m["h"], m["H"], 2001)
    umax = np.abs(an.poiseuille_ux(yr, m["h"], m["H"], 0.1, 0.01, 1.0, p["force"][0])).max()
    assert u1 * m["h"] / 0.1 == pytest.approx(1.0) or umax == pytest.approx(0.01, rel=1e-3)
    # the initial temperature is the sharp conduction profile between 0 and 1
    Y, _ = wl.coords(p["nx"], p["ny"])
    Ta = an.poiseuille_T(Y[:, 0] - m["h"], m["h"], m["H"], m["lam1"], m["lam2"], 0.0, 1.0)
    np.testing.assert_allclose(w["T0"][:, 0], Ta, rtol=0, atol=1e-14)
    assert np.all(w["Twall_bot"] == 0.0) and np.all(w["Twall_top"] == 1.0)


@pytest.mark.parametrize("lam_r", [1.0, 0.1])
def test_e2_inputs(lam_r):
    w = wl.paper_case("e2", lam_r=lam_r)
    p, m = w["params"], w["meta"]
    assert [p["nx"], p["ny"]] == GOLD["mesh_planar"]["value"]
    assert p["sigmaT"] == 5e-4 and m["sigma_T"] == -5e-4           # sigma_T = -5e-4
    assert p["sigma0"] == 2.5e-2 and p["Tref"] == 10.0 and p["mobility"] == 5e-2
    assert eta(p["tau_f"][0]) == pytest.approx(0.2) and eta(p["tau_f"][1]) == pytest.approx(0.2)
    # lambda2 = 0.2 below (c = 0), lambda1 = lambda_r lambda2 above (fluid 1 upper)
    assert lam(p["tau_T"][0]) == pytest.approx(0.2)
    assert lam(p["tau_T"][1]) == pytest.approx(0.2 * lam_r)
    x = np.arange(p["nx"]) + 0.5
    np.testing.assert_allclose(w["Twall_bot"], 20.0 + 4.0 * np.cos(2 * np.pi * x / p["nx"]))
    assert np.all(w["Twall_top"] == 10.0)
    # interface halfway: phi = 0 between rows 49 and 50
    assert w["phi0"][49, 0] < 0 < w["phi0"][50, 0]


def test_e3_inputs():
    w = wl.paper_case("e3")
    p, m = w["params"], w["meta"]
    R = m["R"]
    assert (p["nx"], p["ny"]) == (8 * R, 15 * R)
    assert eta(p["tau_f"][0]) == pytest.approx(0.1) and lam(p["tau_T"][0]) == pytest.approx(0.1)
    assert p["tau_f"][0] == p["tau_f"][1] and p["tau_T"][0] == p["tau_T"][1]
    assert p["sigma0"] == 0.1 and p["Tref"] == 0.0
    assert np.all(w["Twall_bot"] == 0.0) and np.all(w["Twall_top"] == 30.0)
    # |grad T| = 0.1 and the printed U_YGB from these parameters
    u = an.ygb_velocity(-p["sigmaT"], 30.0 / p["ny"], R, 0.1, 1.0, 1.0)
    assert u == pytest.approx(GOLD["U_YGB_droplet"]["value"], rel=1e-12)
    assert m["U_YGB"] == pytest.approx(u, rel=1e-12) and m["t_r"] == R / 1e-3
    # droplet centred at x = 80, 2R above the bottom wall, radius R (c = 1/2
    # contour, with the matrix raised to the droplet's saturation)
    c = 0.5 * (w["phi0"] + 1)
    sat = c.min()
    assert 0.005 < sat < 0.02
    inside = c >= 0.5 + sat
    Y, X = wl.coords(p["nx"], p["ny"])
    area = inside.sum()
    assert area == pytest.approx(math.pi * R * R, rel=0.02)
    assert X[inside].mean() == pytest.approx(80.0, abs=0.05)
    assert Y[inside].mean() == pytest.approx(2 * R, abs=0.05)


def test_generators_are_seeded():
    a, b = wl.random_case(37, 21, 5), wl.random_case(37, 21, 5)
    np.testing.assert_array_equal(a["phi0"], b["phi0"])
    assert a["params"] == b["params"]
    np.testing.assert_array_equal(wl.random_state(20, 10, 3), wl.random_state(20, 10, 3))
    np.testing.assert_array_equal(wl.make("adjoint_droplet")["Twall_bot"],
                                  wl.make("adjoint_droplet")["Twall_bot"])


def test_conduction_field_torch_and_its_transpose():
    """The torch form of the conduction field equals the numpy form, and
    autograd through it equals conduction_field_T (the transpose the wall
    gradient of the differentiated run needs)."""
    import torch
    rng = np.random.default_rng(11)
    nx, ny = 48, 30
    tb = rng.normal(0.0, 0.1, nx)
    a = wl.conduction_field(tb, 2.5, ny)
    t = torch.tensor(tb, requires_grad=True)
    b = wl.conduction_field_torch(t, 2.5, ny)
    assert np.abs(a - b.detach().numpy()).max() <= 1e-14
    G = rng.normal(size=(ny, nx))
    (b * torch.tensor(G)).sum().backward()
    assert np.abs(t.grad.numpy() - wl.conduction_field_T(G, ny)).max() <= 1e-13
    # the field solves the discrete boundary values: rows approach the walls
    assert np.abs(b.detach().numpy()[-1] - 2.5).max() < 0.1
