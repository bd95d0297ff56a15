"""Pins of the oracle's single-site collision by its moments (closed forms).

The moment identities follow from the equilibria and forcing terms of the
three lattice Boltzmann equations (Sec. II Eqs. 6-9, 12-15; Sec. III Eqs. 22,
25-26) and the D2Q9 moment sums of Gamma_i(u): sum Gamma = 1,
sum xi Gamma = u, sum xi xi Gamma = cs^2 I + u u.  A dropped term, a wrong
sign or a wrong relaxation factor in any of the three collisions changes one
of them.
"""
import math

import numpy as np
import pytest

XI = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]],
              dtype=np.float64)
CS2 = 1.0 / 3.0


def _random_params(rng):
    from paper_1412_6238_amd import workloads as wl
    return wl.base_params(
        16, 16, tau_f=tuple(rng.uniform(0.55, 2.0, 2)), tau_T=tuple(rng.uniform(0.55, 2.0, 2)),
        tau_g=float(rng.uniform(0.6, 2.0)), mobility=float(rng.uniform(0.01, 0.2)),
        width=float(rng.uniform(1.0, 5.0)), beta=float(rng.uniform(0.1, 1.0)),
        sigma0=float(rng.uniform(0.0, 0.1)), sigmaT=float(rng.uniform(-1e-2, 1e-2)),
        Tref=float(rng.uniform(-1, 1)), force=tuple(rng.uniform(-1e-3, 1e-3, 2)),
        rho=float(rng.uniform(0.5, 2.0)), cv=float(rng.uniform(0.5, 2.0)))


def _random_site(rng):
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    pre = np.empty(27)
    pre[:9] = w * 0.33 * (1 + 0.2 * rng.standard_normal(9))
    pre[9:18] = w * rng.uniform(-0.1, 1.1) + 0.02 * rng.standard_normal(9)
    pre[18:] = w * rng.uniform(0.5, 2.0) * (1 + 0.2 * rng.standard_normal(9))
    st = 0.05 * rng.standard_normal(7)
    return pre, st


@pytest.mark.parametrize("seed", range(40))
def test_collision_moments(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    p = _random_params(rng)
    pre, st = _random_site(rng)
    post, a = oracle_mod.collide_site(p, pre, st)
    f, g, h = pre[:9], pre[9:18], pre[18:]
    fs, gs, hs = post[:9], post[9:18], post[18:]
    rho, cv = p["rho"], p["cv"]
    u = np.array([a["ux"], a["uy"]])
    F = np.array([a["Fx"], a["Fy"]])
    Fbar = F - st[5:7]                       # grad p is the last stencil pair
    c, T, pr = g.sum(), h.sum() / (rho * cv), f.sum()
    assert a["c"] == pytest.approx(c, abs=1e-15)
    assert a["T"] == pytest.approx(T, rel=1e-14)
    wf, wT, wg = a["wf"], a["wT"], a["wg"]
    tol = dict(rel=1e-11, abs=1e-15)
    # zeroth moments: p, c and rho cv T are collision invariants
    assert fs.sum() == pytest.approx(pr, **tol)
    assert gs.sum() == pytest.approx(c, **tol)
    assert hs.sum() == pytest.approx(rho * cv * T, **tol)
    # first moments: relaxation towards the equilibrium flux plus the
    # first moment of the forcing term
    j = XI.T @ f
    np.testing.assert_allclose(
        XI.T @ fs, (1 - wf) * j + wf * rho * CS2 * u + (1 - wf / 2) * CS2 * F, rtol=1e-10, atol=1e-16)
    np.testing.assert_allclose(
        XI.T @ gs, (1 - wg) * (XI.T @ g) + wg * c * u + (1 - wg / 2) * c * Fbar / rho,
        rtol=1e-10, atol=1e-16)
    np.testing.assert_allclose(
        XI.T @ hs, (1 - wT) * (XI.T @ h) + wT * rho * cv * T * u + (1 - wT / 2) * cv * T * Fbar,
        rtol=1e-10, atol=1e-15)
    # second moment of f: the equilibrium carries p cs^2 I + rho cs^2 u u
    # (exact for D2Q9 with the second-order equilibrium)
    M2 = np.einsum("ia,ib,i->ab", XI, XI, f)
    M2s = np.einsum("ia,ib,i->ab", XI, XI, fs)
    Seq = pr * CS2 * np.eye(2) + rho * CS2 * np.outer(u, u)
    # second moment of the forcing term: sum xi_a xi_b (xi - u).F Gamma_i
    # = cs^2 (u_a F_b + u_b F_a) - (u.F) u_a u_b on D2Q9
    SF = CS2 * (np.outer(u, F) + np.outer(F, u)) - np.dot(u, F) * np.outer(u, u)
    np.testing.assert_allclose(M2s, (1 - wf) * M2 + wf * Seq + (1 - wf / 2) * SF,
                               rtol=1e-10, atol=1e-15)
    # second moment of g: Gamma mu I + c u u
    Gam = p["mobility"] / (p["tau_g"] - 0.5)
    G2 = np.einsum("ia,ib,i->ab", XI, XI, g)
    G2s = np.einsum("ia,ib,i->ab", XI, XI, gs)
    Geq = Gam * a["mu"] * np.eye(2) + c * np.outer(u, u)
    SG = c / (rho * CS2) * (CS2 * (np.outer(u, Fbar) + np.outer(Fbar, u))
                            - np.dot(u, Fbar) * np.outer(u, u))
    np.testing.assert_allclose(G2s, (1 - wg) * G2 + wg * Geq + (1 - wg / 2) * SG,
                               rtol=1e-10, atol=1e-15)


def test_relaxation_rates_and_interpolation(oracle_mod):
    """omega = 1/tau, with tau linear in the clamped order parameter."""
    rng = np.random.default_rng(7)
    p = _random_params(rng)
    for cval in (-0.3, 0.0, 0.25, 0.5, 1.0, 1.4):
        pre, st = _random_site(rng)
        pre[9:18] *= cval / pre[9:18].sum()
        _, a = oracle_mod.collide_site(p, pre, st)
        ch = min(max(cval, 0.0), 1.0)
        assert a["wf"] == pytest.approx(1 / (p["tau_f"][0] + ch * (p["tau_f"][1] - p["tau_f"][0])))
        assert a["wT"] == pytest.approx(1 / (p["tau_T"][0] + ch * (p["tau_T"][1] - p["tau_T"][0])))
        assert a["wg"] == pytest.approx(1 / p["tau_g"])


def test_equilibrium_is_fixed_point_without_force(oracle_mod):
    """A state at rest with uniform fields and no force does not change."""
    from paper_1412_6238_amd import workloads as wl
    p = wl.base_params(8, 8, sigma0=0.0, sigmaT=0.0)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    pre = np.concatenate([w * 0.4, np.eye(9)[0] * 1.0, w * 2.5])   # c = 1: mu0(1) = 0
    post, a = oracle_mod.collide_site(p, pre, np.zeros(7))
    np.testing.assert_allclose(post, pre, rtol=0, atol=1e-16)
    assert a["mu"] == 0.0


def test_paper_printed_constants(oracle_mod):
    """alpha = 6 sqrt(2) for c1 = 0, c2 = 1 and the planar profile of Sec. II;
    the normalisation eps alpha int c'^2 dz = 1 and kcap sigma_fe = 1."""
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    from paper_1412_6238_amd import workloads as wl
    p = wl.base_params(8, 8, width=2 * math.sqrt(2), beta=0.25)
    d = oracle_mod.derived(p)
    assert d["alpha"] == pytest.approx(gold["alpha"]["value"], rel=1e-15)
    assert d["eps"] == pytest.approx(1.0, rel=1e-15)
    for W, beta in ((2 * math.sqrt(2), 0.25), (4.0, 0.25), (3.0, 0.6)):
        d = oracle_mod.derived(wl.base_params(8, 8, width=W, beta=beta))
        # eps alpha int (c')^2 dz with c = 1/2 + 1/2 tanh(z/W), by quadrature
        z = np.linspace(-40 * W, 40 * W, 400001)
        cp = 0.5 / W / np.cosh(z / W) ** 2
        integral = np.trapezoid(cp ** 2, z)
        assert d["eps"] * d["alpha"] * integral == pytest.approx(1.0, rel=1e-9)
        # the planar profile solves mu = 0 for this eps: eps^2 c'' = mu0(c)
        c = 0.5 + 0.5 * np.tanh(z / W)
        cpp = -np.tanh(z / W) / W * 2 * cp
        mu0 = 2 * beta * c * (c - 1) * (2 * c - 1)
        assert np.max(np.abs(d["eps"] ** 2 * cpp - mu0)) < 1e-12
        # free-energy tension sigma_fe = eps^2 int c'^2, and kcap sigma_fe = 1
        assert d["kcap"] * d["eps"] ** 2 * integral == pytest.approx(1.0, rel=1e-9)


@pytest.mark.parametrize("theta", [0.3, 1.1, 2.5, 4.0, 5.6])
def test_curvature_force_closed_form(oracle_mod, theta):
    """Curvature form of the capillary force, Eq. 4: -sigma kappa n delta with
    n = grad c/|grad c|, kappa = div n, delta = eps alpha |grad c|^2.  For a
    radial profile c = f(r) the gradient is f' r_hat and the Hessian is
    f'' r_hat r_hat + (f'/r)(I - r_hat r_hat), so div n = -1/r (n points
    inwards for a droplet) and the force is -sigma eps alpha f'^2 / r r_hat,
    pointing inwards with magnitude sigma delta / r.  Fed with these exact
    derivatives at a generic angle, the site closure must return exactly that
    (a swapped tangent and normal, a wrong sign of the mixed derivative or of
    the force fails)."""
    from paper_1412_6238_amd import workloads as wl
    W, R, r = 2.5, 30.0, 31.2
    p = wl.base_params(8, 8, width=W, beta=0.3, sigma0=0.07, sigmaT=0.0, Tref=0.0,
                       csf_form=1)
    d = oracle_mod.derived(p)
    sech2 = 1.0 / math.cosh((R - r) / W) ** 2
    f1 = -0.5 * sech2 / W                                      # f'(r)
    # f''(r) of the tanh profile plus an offset: the profile is then off its
    # equilibrium, where the potential form (exact on the equilibrium
    # profile) and the curvature form differ; the curvature form does not
    # depend on f'' at all
    f2 = -sech2 * math.tanh((R - r) / W) / W ** 2 + 0.01
    e = np.array([math.cos(theta), math.sin(theta)])
    H = f2 * np.outer(e, e) + (f1 / r) * (np.eye(2) - np.outer(e, e))
    g = f1 * e
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    cval = 0.5 + 0.5 * math.tanh((R - r) / W)
    pre = np.concatenate([w * 0.33, w * cval, w * 1.0])
    st = np.array([g[0], g[1], np.trace(H), 0.0, 0.0, 0.0, 0.0, H[0, 0], H[0, 1], H[1, 1]])
    _, a = oracle_mod.collide_site(p, pre, st)
    expect = -p["sigma0"] * d["eps"] * d["alpha"] * f1 * f1 / r * e
    assert a["Fx"] == pytest.approx(expect[0], rel=1e-12, abs=1e-18)
    assert a["Fy"] == pytest.approx(expect[1], rel=1e-12, abs=1e-18)
    # the potential form at the same site differs off equilibrium
    _, a0 = oracle_mod.collide_site(dict(p, csf_form=0), pre, st)
    assert abs(a0["Fx"] - a["Fx"]) > 1e-6 * abs(a["Fx"])


def test_curvature_force_vanishes_on_flat_profile(oracle_mod):
    """A planar profile c(y) has no curvature: with grad c along y and the
    Hessian's only entry d2c/dy2, the capillary force of the curvature form is
    zero whatever the profile, leaving the Marangoni part alone."""
    from paper_1412_6238_amd import workloads as wl
    p = wl.base_params(8, 8, sigma0=0.05, sigmaT=2e-3, Tref=1.0, csf_form=1)
    d = oracle_mod.derived(p)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    pre = np.concatenate([w * 0.33, w * 0.4, w * 1.3])
    gy, hyy, gTx, gTy = 0.11, -0.02, 0.03, -0.01
    st = np.array([0.0, gy, hyy, gTx, gTy, 0.0, 0.0, 0.0, 0.0, hyy])
    _, a = oracle_mod.collide_site(p, pre, st)
    # Marangoni part: eps alpha (|g|^2 grad sigma - (g . grad sigma) g) with
    # grad sigma = -sigmaT grad T; along x only for g along y
    ea = d["eps"] * d["alpha"]
    assert a["Fx"] == pytest.approx(ea * gy * gy * (-p["sigmaT"] * gTx), rel=1e-13)
    assert a["Fy"] == 0.0


@pytest.mark.parametrize("seed", range(12))
def test_collision_moments_two_densities(oracle_mod, seed):
    """Two densities, rho(c) = rho1 + c (rho2 - rho1) (the closure the paper
    leaves open): T = sum hbar / (rho(c) cv) (Eq. 26); the pressure of Eq. 9
    is p = sum f + (1/2) u.grad(rho cs^2); the density term of Eq. 6,
    (xi - u).grad(rho cs^2)(Gamma_i(u) - Gamma_i(0)), has zero first moment,
    and with the pressure's own correction the collision adds exactly
    cs^2 u.grad rho to sum f; the first moments use the local rho;
    the g forcing uses F - grad p (Eq. 12) and the hbar forcing F-bar =
    grad(rho cs^2) - grad p + F (Sec. III)."""
    rng = np.random.default_rng(100 + seed)
    p = dict(_random_params(rng), rho2=float(rng.uniform(0.3, 4.0)))
    pre, st = _random_site(rng)
    post, a = oracle_mod.collide_site(p, pre, st)
    f, g, h = pre[:9], pre[9:18], pre[18:]
    fs, gs, hs = post[:9], post[9:18], post[18:]
    c = g.sum()
    rho = p["rho"] + c * (p["rho2"] - p["rho"])
    cv = p["cv"]
    grad_rho = (p["rho2"] - p["rho"]) * st[0:2]
    gradp = st[5:7]
    T = h.sum() / (rho * cv)
    assert a["T"] == pytest.approx(T, rel=1e-14)
    u = np.array([a["ux"], a["uy"]])
    F = np.array([a["Fx"], a["Fy"]])
    j = XI.T @ f
    # u from the f moments with the local density (Eq. 9, reading A1)
    np.testing.assert_allclose(u, 3 * j / rho + F / (2 * rho), rtol=1e-12, atol=1e-16)
    assert a["p"] == pytest.approx(f.sum() + 0.5 * CS2 * u @ grad_rho, rel=1e-13, abs=1e-16)
    wf, wT, wg = a["wf"], a["wT"], a["wg"]
    assert fs.sum() - f.sum() == pytest.approx(CS2 * u @ grad_rho, rel=1e-9, abs=1e-15)
    np.testing.assert_allclose(XI.T @ fs, (1 - wf) * j + wf * rho * CS2 * u + (1 - wf / 2) * CS2 * F,
                               rtol=1e-10, atol=1e-16)
    np.testing.assert_allclose(
        XI.T @ gs, (1 - wg) * (XI.T @ g) + wg * c * u + (1 - wg / 2) * c * (F - gradp) / rho,
        rtol=1e-10, atol=1e-16)
    Fbar = CS2 * grad_rho - gradp + F
    np.testing.assert_allclose(
        XI.T @ hs, (1 - wT) * (XI.T @ h) + wT * rho * cv * T * u + (1 - wT / 2) * cv * T * Fbar,
        rtol=1e-10, atol=1e-15)
    assert gs.sum() == pytest.approx(c, rel=1e-12)
    assert hs.sum() == pytest.approx(h.sum(), rel=1e-12)
