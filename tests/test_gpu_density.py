"""GPU parity of the two-density step (rho2 != rho, FP64 form).

rho(c) = rho + c (rho2 - rho) brings in the density terms of Eq. 6, the
pressure of Eq. 9 (p = sum f + (1/2) u.grad(rho cs^2), computed by a pressure
pass before every step) and F-bar of Sec. III.  The HIP path is held to the
FP64 oracle at 1e-12 on random states, grids with walls and periodic y,
ragged strips, both capillary forms and the 4096 x 4096 grid on sampled
windows; strip shapes agree bitwise; the layered channel reaches its
diffuse-interface steady state.  The FP32 deviation form is held to the FP64
path at 1e-4 relative L2 on phi, u and T over long runs.  The adjoint
refuses two densities.
"""
import os
import sys

import numpy as np
import pytest

from paper_1412_6238_amd import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
import analytic as an  # noqa: E402

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "ux", "uy", "p", "T")


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
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _cmp(gpu, orc, tol=1e-12, what=""):
    g, o = dict(gpu), dict(orc)
    if "ux" in o:
        g["u"] = np.stack([g.pop("ux"), g.pop("uy")])
        o["u"] = np.stack([o.pop("ux"), o.pop("uy")])
    errs = {}
    for k in o:
        gk, ok = np.asarray(g[k]), np.asarray(o[k])
        scale = max(np.abs(ok).max(), 1e-300)
        assert np.all(np.isfinite(gk)), (what, k)
        errs[k] = _rel(gk, ok)
        assert errs[k] <= tol, (what, k, errs[k])
        assert np.abs(gk - ok).max() <= 10 * tol * scale, (what, k, np.abs(gk - ok).max() / scale)
    _say(f"  {what}: rel L2 " + " ".join(f"{k} {v:.1e}" for k, v in errs.items()))


def _fields_np(sim):
    return {k: v.cpu().numpy() for k, v in sim.fields().items()}


def _two(case, rho2, **kw):
    case = dict(case)
    case["params"] = dict(case["params"], rho2=rho2, **kw)
    return case


def _pair(lbe, oracle_mod, case):
    p = case["params"]
    sim = lbe.Simulation(p, case["phi0"], case["T0"], case["Twall_bot"], case["Twall_top"])
    orc = oracle_mod.Oracle(p, case["Twall_bot"], case["Twall_top"]).init(case["phi0"], case["T0"])
    return sim, orc


GRIDS = [(8, 8, 1, 2.0), (37, 21, 1, 0.4), (70, 9, 0, 3.0), (130, 7, 1, 5.0), (600, 5, 0, 1.5),
         (64, 64, 1, 0.25)]


@pytest.mark.parametrize("nx,ny,walls,ratio", GRIDS)
def test_two_densities_fp64_vs_oracle(lbe, oracle_mod, nx, ny, walls, ratio):
    base = wl.random_case(nx, ny, seed=5 * nx + ny, walls_y=walls)
    case = _two(base, ratio * base["params"]["rho"], p0=0.0)
    _say(f"case two densities random {nx}x{ny} walls={walls} ratio={ratio}")
    sim, orc = _pair(lbe, oracle_mod, case)
    _cmp({"F": sim.get_state().cpu().numpy()}, {"F": orc.state()}, what="F0")
    for n in (1, 3, 12):
        sim.step(n)
        orc.step(n)
        _cmp({"F": sim.get_state().cpu().numpy()}, {"F": orc.state()}, what=f"F after +{n}")
        _cmp(_fields_np(sim), orc.fields(), what=f"fields after +{n}")


@pytest.mark.parametrize("form", [0, 1])
def test_two_densities_random_state(lbe, oracle_mod, form):
    """Arbitrary non-equilibrium states (large u and density gradients), both
    capillary forms, and the diagnostics."""
    base = wl.random_case(90, 33, seed=9 + form, walls_y=1)
    case = _two(base, 3.0 * base["params"]["rho"], csf_form=form)
    F = wl.random_state(90, 33, seed=23 + form)
    _say(f"case two densities random state 90x33 form={form}")
    sim, orc = _pair(lbe, oracle_mod, case)
    sim.set_state(F)
    orc.set_state(F)
    sim.step(4)
    orc.step(4)
    _cmp({"F": sim.get_state().cpu().numpy()}, {"F": orc.state()}, what="F")
    _cmp(_fields_np(sim), orc.fields(), what="fields")
    d, e = sim.diagnostics(), orc.diag()
    for k in ("mass", "energy", "sum_cy", "mass_thr", "sum_cuy_thr"):
        assert d[k] == pytest.approx(e[k], rel=1e-12, abs=1e-15), k


def test_two_densities_launch_shapes_agree(lbe, monkeypatch):
    """Strip widths of 1, 2, 4, 8 waves and chunk heights give the same state,
    bit for bit (an asked-for row pipeline other than one row ahead is
    ignored with two densities)."""
    base = wl.random_case(300, 40, seed=44, walls_y=1)
    case = _two(base, 2.5 * base["params"]["rho"])
    out = []
    monkeypatch.setenv("LBE_CSF_TILE", "0")   # the row-marching kernel
    for pipe, nw, rows in (("1", "4", "40"), ("0", "1", "7"), ("2", "2", "9"), ("1", "8", "13")):
        monkeypatch.setenv("LBE_CSF_PIPE", pipe)
        monkeypatch.setenv("LBE_CSF_NW", nw)
        monkeypatch.setenv("LBE_CSF_ROWS", rows)
        _say(f"case two densities launch pipe={pipe} nw={nw} rows={rows}")
        sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                             case["Twall_top"])
        sim.step(5)
        out.append(sim.get_state().cpu().numpy())
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])


def test_two_densities_channel_steady_state(lbe):
    """The layered channel of the oracle's pin (rho 1 below, 3 above, driven
    along x), run to its steady state on the GPU: within 5e-3 (u) and 4e-3
    (T) of the diffuse-interface balances, the second-order discretisation
    error at W = 4."""
    nx, ny = 4, 64
    p = wl.base_params(nx, ny, tau_f=(0.8, 0.8), tau_T=(0.8, 1.1), tau_g=2.5, mobility=0.1,
                       width=4.0, sigma0=1e-3, sigmaT=0.0, force=(1e-6, 0.0), rho=1.0, rho2=3.0)
    phi0 = wl.tanh_layer(nx, ny, ny / 2, 4.0)
    Y, _ = wl.coords(nx, ny)
    _say("case two densities channel 4x64 60000 steps")
    sim = lbe.Simulation(p, phi0, Y / ny, np.zeros(nx), np.ones(nx))
    sim.step(60000)
    f = _fields_np(sim)
    u_d, T_d = an.layered_1d_steady(ny, ny / 2, 4.0, 0, 0, 0, 0, 1e-6, 0.0, 1.0, rho1=1.0,
                                    rho2=3.0, tau=(p["tau_f"], p["tau_T"]))
    eu, eT = _rel(f["ux"].mean(axis=1), u_d), _rel(f["T"].mean(axis=1), T_d)
    _say(f"  u {eu:.2e} T {eT:.2e}")
    assert eu <= 5e-3 and eT <= 4e-3


@pytest.mark.parametrize("name,nsteps", [("e1", 2000), ("e3", 200)])
def test_two_densities_paper_geometries(lbe, oracle_mod, name, nsteps):
    """The paper's layered channel and droplet geometries with a density
    ratio of 2 (the paper's cases use one density), p0 = 0 gauge."""
    w = wl.paper_case(name, rho2=2.0, p0=0.0)
    _say(f"case two densities paper {name} {nsteps} steps")
    sim, orc = _pair(lbe, oracle_mod, w)
    sim.step(nsteps)
    orc.step(nsteps)
    g, o = _fields_np(sim), orc.fields()
    g["p"], o["p"] = g["p"] + 1 / 3, o["p"] + 1 / 3
    _cmp(g, o, what=name)


def test_two_densities_full_size_sampled(lbe, oracle_mod):
    """4096 x 4096 multi-droplet workload with droplets twice as dense as the
    matrix, FP64: k GPU steps, the oracle on windows centred on interfaces
    (the dependence cone is three sites per step: the pressure's stencil of
    u), fields compared on the valid centres."""
    w = wl.make("multi_droplet", rho2=2.0)
    p = w["params"]
    nx, ny = p["nx"], p["ny"]
    k = 2
    _say(f"case two densities full-size multi_droplet fp64 {k} steps")
    sim = lbe.Simulation(p, w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"])
    sim.step(k)
    g = {kk: v.cpu().numpy() for kk, v in sim.fields().items()}
    del sim
    umax = np.hypot(g["ux"], g["uy"]).max()
    trange = w["T0"].max() - w["T0"].min()
    rng = np.random.default_rng(11)
    m = 3 + 3 * k
    size = 2 * m + 8
    iy, ix = np.nonzero(np.abs(w["phi0"]) < 0.5)
    wins = []
    for t in rng.choice(len(iy), 8, replace=False):
        y0 = int(min(max(iy[t] - m - 4, 0), ny - size))
        wins.append((int((ix[t] - m - 4) % nx), y0, size, size))
    checked = 0
    for (x0, y0, wx, wy) in wins:
        cols = np.arange(x0, x0 + wx) % nx
        sub = lambda a: np.ascontiguousarray(a[y0:y0 + wy][:, cols])
        o = oracle_mod.Oracle(p, w["Twall_bot"], w["Twall_top"], window=(x0, y0, wx, wy))
        o.init(sub(w["phi0"]), sub(w["T0"]))
        o.step(k)
        of = o.fields()
        jj, ii = np.meshgrid(np.arange(wy), np.arange(wx), indexing="ij")
        dist_x = np.minimum(ii, wx - 1 - ii)
        dist_bot = jj if y0 > 0 else np.full_like(jj, 10 ** 6)
        dist_top = (wy - 1 - jj) if y0 + wy < ny else np.full_like(jj, 10 ** 6)
        valid = np.minimum(np.minimum(dist_x, dist_bot), dist_top) >= 3 + 3 * k
        assert valid.sum() >= 64
        gw = {f: sub(g[f])[valid] for f in FIELDS}
        ow = {f: of[f][valid] for f in FIELDS}
        for f in FIELDS:
            assert np.all(np.isfinite(ow[f])), f
        du = np.hypot(gw["ux"] - ow["ux"], gw["uy"] - ow["uy"]).max()
        assert du <= 1e-12 * umax, ("u", x0, y0, du / umax)
        assert np.abs(gw["phi"] - ow["phi"]).max() <= 1e-12, ("phi", x0, y0)
        assert np.abs(gw["T"] - ow["T"]).max() <= 1e-12 * trange, ("T", x0, y0)
        assert np.abs(gw["p"] - ow["p"]).max() <= 1e-12 * np.abs(ow["p"]).max(), ("p", x0, y0)
        checked += int(valid.sum())
    _say(f"  compared {checked} sites in {len(wins)} windows")


def test_two_densities_refuse_recording(lbe):
    """The adjoint covers one density only: a recorded run is refused."""
    base = wl.random_case(16, 16, seed=3)
    case = _two(base, 2.0 * base["params"]["rho"])
    for prec in ("fp64", "fp32_dev"):
        sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                             case["Twall_top"], precision=prec, record_steps=8)
        with pytest.raises(lbe.LbeCsfError) as e:
            sim.step(4, record=True)
        assert e.value.status == lbe.LBE_CSF_EINVAL
        sim.step(4)


def _fp32_vs_fp64(lbe, w, nsteps, what, tol=1e-4, state=False):
    """Run both forms from the same inputs; relative L2 of the FP32 form's
    phi, u and T against the FP64 path (and of the 27 distributions as
    get_state returns them, with state=True)."""
    res, F = {}, {}
    for prec in ("fp64", "fp32_dev"):
        sim = lbe.Simulation(w["params"], w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                             precision=prec)
        sim.step(nsteps)
        assert sim.diagnostics()["n_nonfinite"] == 0
        res[prec] = _fields_np(sim)
        if state:
            F[prec] = sim.get_state().cpu().numpy()
        del sim
    a, b = res["fp32_dev"], res["fp64"]
    e = {"phi": _rel(a["phi"], b["phi"]),
         "u": _rel(np.stack([a["ux"], a["uy"]]), np.stack([b["ux"], b["uy"]])),
         "T": _rel(a["T"], b["T"])}
    if state:
        e["F"] = _rel(F["fp32_dev"], F["fp64"])
    _say(f"  {what}: fp32_dev vs fp64 " + " ".join(f"{k} {v:.2e}" for k, v in e.items()))
    for k, v in e.items():
        assert v <= tol, (what, k, v)
    return a, b


@pytest.mark.parametrize("nx,ny,walls,ratio", GRIDS)
def test_two_densities_fp32_random(lbe, nx, ny, walls, ratio):
    """The FP32 form on the random cases of the parity test (density ratios
    0.25 to 5, walls and periodic y), 50 steps; fields and the distributions
    read back through get_state."""
    base = wl.random_case(nx, ny, seed=5 * nx + ny, walls_y=walls)
    case = _two(base, ratio * base["params"]["rho"], p0=0.0)
    _say(f"case two densities fp32 random {nx}x{ny} walls={walls} ratio={ratio}")
    _fp32_vs_fp64(lbe, case, 50, f"{nx}x{ny}", state=True)


@pytest.mark.parametrize("name,nsteps,kw", [("e1", 100000, {}), ("e3", 40000, {}),
                                            ("e3", 40000, {"csf_form": 1}),
                                            ("e1", 100000, {"rho2": 5.0})])
def test_two_densities_fp32_paper_geometries(lbe, name, nsteps, kw):
    """The paper's layered channel and droplet with a density ratio of 2 (5
    for one channel run), both force forms: the FP32 form against FP64 over
    long runs."""
    kw = dict({"rho2": 2.0}, **kw)
    w = wl.paper_case(name, **kw)
    _say(f"case two densities fp32 paper {name} {kw} {nsteps} steps")
    _fp32_vs_fp64(lbe, w, nsteps, name)


def test_two_densities_fp32_channel(lbe):
    """The layered channel (rho 1 below, 3 above) to its steady state in the
    FP32 form: within 1e-4 of the FP64 path and within the same bars of the
    diffuse-interface balances as the FP64 run."""
    nx, ny = 4, 64
    p = wl.base_params(nx, ny, tau_f=(0.8, 0.8), tau_T=(0.8, 1.1), tau_g=2.5, mobility=0.1,
                       width=4.0, sigma0=1e-3, sigmaT=0.0, force=(1e-6, 0.0), rho=1.0, rho2=3.0,
                       T_shift=0.0, T_grad=1.0 / ny)
    Y, _ = wl.coords(nx, ny)
    w = dict(params=p, phi0=wl.tanh_layer(nx, ny, ny / 2, 4.0), T0=Y / ny,
             Twall_bot=np.zeros(nx), Twall_top=np.ones(nx))
    _say("case two densities fp32 channel 4x64 60000 steps")
    a, _ = _fp32_vs_fp64(lbe, w, 60000, "channel")
    u_d, T_d = an.layered_1d_steady(ny, ny / 2, 4.0, 0, 0, 0, 0, 1e-6, 0.0, 1.0, rho1=1.0,
                                    rho2=3.0, tau=(p["tau_f"], p["tau_T"]))
    eu, eT = _rel(a["ux"].mean(axis=1), u_d), _rel(a["T"].mean(axis=1), T_d)
    _say(f"  u {eu:.2e} T {eT:.2e}")
    assert eu <= 5e-3 and eT <= 4e-3


def test_two_densities_fp32_multi_droplet(lbe):
    """4096 x 4096 multi-droplet workload with droplets twice as dense as the
    matrix, 2000 steps in each form."""
    w = wl.make("multi_droplet", rho2=2.0)
    _say("case two densities fp32 multi_droplet 4096x4096 2000 steps")
    _fp32_vs_fp64(lbe, w, 2000, "multi_droplet")


@pytest.mark.parametrize("nx", [150, 196])
@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_two_densities_tile_kernel_matches_row_kernel(lbe, monkeypatch, precision, nx):
    """Two densities in tiles (the pressure pass, then the step, each with its
    frame of wrapped or ghost cells) against the row-marching kernel on a
    grid ragged in both directions, diagnostics included: FP64 bitwise, FP32
    to rounding (the compiler fuses the FP32 multiply-adds differently).
    196 columns: four tiles, the last of 4 columns, whose other lanes collide
    their wrapped sites (pressure pass included) and write what the owning
    lanes write."""
    base = wl.random_case(nx, 45, seed=46, walls_y=1)
    case = _two(base, 2.5 * base["params"]["rho"])
    out = []
    for tile in ("0", "1"):
        monkeypatch.setenv("LBE_CSF_TILE", tile)
        _say(f"case two densities tile kernel={tile} {nx}x45 {precision}")
        sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                             case["Twall_top"], precision=precision, diag_every=3)
        sim.step(7)
        out.append((sim.get_state().cpu().numpy(), sim.diag_history()))
    if precision == "fp64":
        np.testing.assert_array_equal(out[1][0], out[0][0])
    else:
        a, b = out[1][0], out[0][0]
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-6
    assert len(out[0][1]) == len(out[1][1]) >= 2
    for d, e in zip(out[1][1], out[0][1]):
        assert d["mass"] == pytest.approx(e["mass"], rel=1e-12 if precision == "fp64" else 1e-6)


def test_two_densities_fp32_launch_shapes_agree(lbe, monkeypatch):
    """FP32 form: strip widths and chunk heights give the same state, bit for
    bit."""
    base = wl.random_case(300, 40, seed=45, walls_y=1)
    case = _two(base, 2.5 * base["params"]["rho"])
    out = []
    monkeypatch.setenv("LBE_CSF_TILE", "0")   # the row-marching kernel
    for nw, rows in (("4", "40"), ("1", "7"), ("2", "9"), ("8", "13")):
        monkeypatch.setenv("LBE_CSF_NW", nw)
        monkeypatch.setenv("LBE_CSF_ROWS", rows)
        _say(f"case two densities fp32 launch nw={nw} rows={rows}")
        sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                             case["Twall_top"], precision="fp32_dev")
        sim.step(5)
        out.append(sim.get_state().cpu().numpy())
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])
