"""GPU parity: the HIP step (through the C ABI) against the FP64 CPU oracle.

FP64: every field and every distribution within 1e-12 relative L2 (and
1e-11 of the field's maximum elementwise).  FP32 deviations: against the FP64
path at the error the precision allows.  Cases cover several strips and
chunks with ragged tails, walls and periodic y, random non-equilibrium states,
the workloads at oracle-feasible sizes, and the full 4096 x 4096 workload on
sampled windows.
"""
import os
import sys

import numpy as np
import pytest

from paper_1412_6238_amd import workloads as wl

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
    """Relative L2 error <= tol per field, and elementwise <= 10 tol of the
    field's largest magnitude.  The velocity is compared as one vector field
    (a component that is only round-off, like u_y of a parallel flow, has no
    meaningful relative error of its own)."""
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


def _pair(lbe, oracle_mod, case, precision="fp64", state=None):
    p = case["params"]
    sim = lbe.Simulation(p, case["phi0"], case["T0"], case["Twall_bot"], case["Twall_top"],
                         precision=precision)
    orc = oracle_mod.Oracle(p, case["Twall_bot"], case["Twall_top"]).init(case["phi0"], case["T0"])
    if state is not None:
        sim.set_state(state)
        orc.set_state(state)
    return sim, orc


GRIDS = [(8, 8, 1), (16, 12, 0), (37, 21, 1), (70, 9, 1), (130, 7, 0), (600, 5, 1), (2100, 4, 1),
         (64, 64, 0)]


@pytest.mark.parametrize("nx,ny,walls", GRIDS)
def test_fp64_initial_state_and_steps(lbe, oracle_mod, nx, ny, walls):
    case = wl.random_case(nx, ny, seed=nx * 131 + ny, walls_y=walls)
    _say(f"case random {nx}x{ny} walls={walls} fp64 from init")
    sim, orc = _pair(lbe, oracle_mod, case)
    _cmp({"F": sim.get_state().cpu().numpy()}, {"F": orc.state()}, what="F0")
    _cmp(_fields_np(sim), orc.fields(), what="fields0")
    for n in (1, 2, 4):
        sim.step(n)
        orc.step(n)
        _cmp({"F": sim.get_state().cpu().numpy()}, {"F": orc.state()}, what=f"F after +{n}")
        _cmp(_fields_np(sim), orc.fields(), what=f"fields after +{n}")


@pytest.mark.parametrize("nx,ny,walls", [(3, 3, 1), (3, 5, 0), (4, 3, 1), (65, 3, 1), (3, 70, 1)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_smallest_grids(lbe, oracle_mod, nx, ny, walls, precision):
    """Degenerate shapes: three columns (the halo columns wrap onto the
    strip's own sites), three rows between two walls (every row touches a
    wall), one column past a full wave.  FP64 against the oracle at 1e-12,
    FP32 deviations at 1e-5."""
    case = wl.random_case(nx, ny, seed=900 + 7 * nx + ny, walls_y=walls, n_drops=1)
    _say(f"case smallest grid {nx}x{ny} walls={walls} {precision}")
    p = case["params"]
    sim = lbe.Simulation(p, case["phi0"], case["T0"], case["Twall_bot"], case["Twall_top"],
                         precision=precision)
    orc = oracle_mod.Oracle(p, case["Twall_bot"], case["Twall_top"]).init(case["phi0"], case["T0"])
    sim.step(7)
    orc.step(7)
    tol = 1e-12 if precision == "fp64" else 1e-5
    _cmp(_fields_np(sim), orc.fields(), tol=tol, what="fields")
    if precision == "fp64":
        _cmp({"F": sim.get_state().cpu().numpy()}, {"F": orc.state()}, what="F")


@pytest.mark.parametrize("nx,ny,walls", GRIDS[:6])
def test_fp64_random_state(lbe, oracle_mod, nx, ny, walls):
    """Arbitrary non-equilibrium states, loaded through set_state."""
    case = wl.random_case(nx, ny, seed=7 + nx, walls_y=walls)
    F = wl.random_state(nx, ny, seed=nx + 3 * ny)
    _say(f"case random state {nx}x{ny} walls={walls} fp64")
    sim, orc = _pair(lbe, oracle_mod, case, state=F)
    sim.step(3)
    orc.step(3)
    _cmp({"F": sim.get_state().cpu().numpy()}, {"F": orc.state()}, what="F")
    _cmp(_fields_np(sim), orc.fields(), what="fields")


def test_fp64_diagnostics(lbe, oracle_mod):
    case = wl.random_case(90, 40, seed=4, walls_y=1)
    _say("case diagnostics 90x40")
    sim, orc = _pair(lbe, oracle_mod, case)
    sim.step(5)
    orc.step(5)
    d, e = sim.diagnostics(), orc.diag()
    for k in ("mass", "energy", "sum_cy", "sum_cx", "mass_thr", "sum_cuy_thr", "centroid_y", "u_r"):
        assert d[k] == pytest.approx(e[k], rel=1e-12, abs=1e-15), k
    assert d["n_nonfinite"] == 0 and d["step"] == 5


@pytest.mark.parametrize("name,nsteps,p0", [("poiseuille", 20000, 1 / 3),
                                            ("planar_marangoni", 50000, 0.0),
                                            ("droplet", 1000, 0.0), ("adjoint_droplet", 4000, 0.0)])
def test_fp64_workloads(lbe, oracle_mod, name, nsteps, p0):
    """The workloads at their stated step counts (the 512 x 1024 droplet at
    its first 1,000 of 100,000).  Droplet and planar cases
    run in the p0 = 0 gauge (an exact symmetry of the method): at p0 = 1/3 the
    populations are ~1e4 times the velocity they encode and the FP64
    round-off of u alone approaches 1e-12.  The planar case is weaker still:
    its Marangoni flow (|u| ~ 1e-6) is the small residue of capillary terms of
    size ~1e-1 that cancel in mu, so its velocity is compared against the
    round-off floor of the comparison itself: the oracle against the same
    oracle source compiled with fused multiply-adds, after the same steps
    (GPU within ten times that)."""
    w = wl.make(name, p0=p0)
    _say(f"case workload {name} fp64 {nsteps} steps p0={p0:.3f}")
    sim, orc = _pair(lbe, oracle_mod, w)
    sim.step(nsteps)
    orc.step(nsteps)
    g, o = _fields_np(sim), orc.fields()
    # pressure compared in the p0 = 1/3 gauge (the same physical state)
    g["p"] = g["p"] + (1 / 3 - p0)
    o["p"] = o["p"] + (1 / 3 - p0)
    if name == "planar_marangoni":
        # the floor: the same oracle source built with fused multiply-adds
        # (the GPU's kind of rounding), against the oracle
        ob = oracle_mod.Oracle(w["params"], w["Twall_bot"], w["Twall_top"], variant="fma")
        ob.init(w["phi0"], w["T0"])
        ob.step(nsteps)
        fb = ob.fields()
        floor = _rel(np.stack([fb["ux"], fb["uy"]]), np.stack([o["ux"], o["uy"]]))
        err = _rel(np.stack([g["ux"], g["uy"]]), np.stack([o["ux"], o["uy"]]))
        _say(f"  u: GPU vs oracle {err:.2e}, oracle round-off floor {floor:.2e}")
        assert err <= max(1e-12, 10 * floor)
        for k in ("ux", "uy"):
            g.pop(k), o.pop(k)
    _cmp(g, o, what=name)


@pytest.mark.parametrize("pipe", ["0", "1", "2"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_row_pipelines_agree(lbe, oracle_mod, monkeypatch, pipe, precision):
    """The ways of feeding rows (loaded twice, one row ahead, two rows ahead)
    give the same state, bit for bit, and FP64 matches the oracle."""
    case = wl.random_case(136, 40, seed=21, walls_y=1)
    monkeypatch.setenv("LBE_CSF_TILE", "0")   # the row-marching kernel
    monkeypatch.setenv("LBE_CSF_PIPE", pipe)
    monkeypatch.setenv("LBE_CSF_ROWS", "7")
    _say(f"case pipeline {pipe} {precision} 136x40")
    sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                         case["Twall_top"], precision=precision)
    sim.step(5)
    F = sim.get_state().cpu().numpy()
    monkeypatch.setenv("LBE_CSF_PIPE", "1")
    ref = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                         case["Twall_top"], precision=precision)
    ref.step(5)
    np.testing.assert_array_equal(F, ref.get_state().cpu().numpy())
    if precision == "fp64":
        orc = oracle_mod.Oracle(case["params"], case["Twall_bot"], case["Twall_top"])
        orc.init(case["phi0"], case["T0"]).step(5)
        _cmp({"F": F}, {"F": orc.state()}, what="F")


@pytest.mark.parametrize("extra", [{}, {"csf_form": 1}])
def test_fp32_store_policy_does_not_matter(lbe, monkeypatch, extra):
    """The FP32 form's whole-line stores with and without the cache bypass
    (chosen by state size; forced both ways here) give the same state, bit
    for bit.  (The two-density step has no bypass variant.)"""
    case = wl.random_case(136, 40, seed=31, walls_y=1)
    monkeypatch.setenv("LBE_CSF_TILE", "0")   # the row-marching kernel
    p = dict(case["params"], **extra)
    out = []
    for policy in ("0", "1"):
        monkeypatch.setenv("LBE_CSF_STREAM", policy)
        _say(f"case fp32 store policy {policy} {extra}")
        sim = lbe.Simulation(p, case["phi0"], case["T0"], case["Twall_bot"], case["Twall_top"],
                             precision="fp32_dev")
        sim.step(6)
        out.append(sim.get_state().cpu().numpy())
    np.testing.assert_array_equal(out[0], out[1])


@pytest.mark.parametrize("name,nx,ny,walls,extra", [
    ("poiseuille", 8, 64, 1, {}), ("random", 37, 13, 0, {"csf_form": 1}),
    ("random", 16, 30, 1, {}), ("random", 17, 19, 1, {}), ("random", 3, 5, 0, {})])
@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_small_grid_path_matches_per_step(lbe, monkeypatch, name, nx, ny, walls, extra,
                                          precision):
    """Small grids (up to 512 sites) run their plain steps many per launch
    of one block (small_step_kernel, the moments of the whole grid in LDS, and
    both states too where they fit: every one of these grids in FP32, 17 x 19
    and 3 x 5 in FP64); the states are bitwise those of one launch per step,
    with diagnostics every 7 steps interleaved and an odd number of steps.
    LBE_CSF_SMALL: 0 one launch per step, 1 the moments-only kernel, 2 the
    default (states resident where they fit)."""
    if name == "poiseuille":
        w = wl.make("poiseuille")
    else:
        w = wl.random_case(nx, ny, seed=nx + ny, walls_y=walls, **extra)
    out = []
    for small in ("0", "1", "2"):
        monkeypatch.setenv("LBE_CSF_SMALL", small)
        _say(f"case small-grid path={small} {name} {nx}x{ny} {precision} {extra}")
        sim = lbe.Simulation(dict(w["params"], **extra), w["phi0"], w["T0"], w["Twall_bot"],
                             w["Twall_top"], precision=precision, diag_every=7)
        sim.step(53)
        sim.step(4)
        out.append((sim.get_state().cpu().numpy(), sim.diag_history(), sim.step_count))
    for o in out[1:]:
        np.testing.assert_array_equal(o[0], out[0][0])
        assert o[1] == out[0][1] and o[2] == out[0][2] == 57


@pytest.mark.parametrize("nx,ny,walls,extra", [(600, 389, 1, {}), (520, 400, 0, {"csf_form": 1})])
def test_one_block_per_cu_ragged(lbe, oracle_mod, monkeypatch, nx, ny, walls, extra):
    """The default launch on grids where one block per CU marches chunks of
    a few rows, with a part-filled last strip and a short last chunk
    (600 x 389: FP64 strips of 256 columns, 88 in the last, 5-row chunks,
    4 in the last; FP32 strips of 512 columns, 4-row chunks, 1 in the last).
    FP64 against the oracle at 1e-12, both forms bitwise equal to another
    launch shape, and the FP32 form within 1e-5 of FP64."""
    case = wl.random_case(nx, ny, seed=nx + 11 * ny, walls_y=walls, n_drops=6, **extra)
    for k in ("LBE_CSF_NW", "LBE_CSF_ROWS", "LBE_CSF_PIPE"):
        monkeypatch.delenv(k, raising=False)
    monkeypatch.setenv("LBE_CSF_TILE", "0")   # the row-marching kernel
    _say(f"case one block per CU {nx}x{ny} walls={walls} {extra} fp64")
    sim, orc = _pair(lbe, oracle_mod, case)
    for n in (1, 3):
        sim.step(n)
        orc.step(n)
        _cmp({"F": sim.get_state().cpu().numpy()}, {"F": orc.state()}, what=f"F after +{n}")
    f64 = _fields_np(sim)
    _say(f"case one block per CU {nx}x{ny} fp32_dev")
    s32 = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                         case["Twall_top"], precision="fp32_dev")
    s32.step(4)
    _cmp(_fields_np(s32), f64, tol=1e-5, what="fp32 fields")
    F32 = s32.get_state().cpu().numpy()
    F64 = sim.get_state().cpu().numpy()
    monkeypatch.setenv("LBE_CSF_NW", "2")
    monkeypatch.setenv("LBE_CSF_ROWS", "7")
    for precision, F in (("fp64", F64), ("fp32_dev", F32)):
        _say(f"case one block per CU {nx}x{ny} {precision} against 2-wave 7-row chunks")
        alt = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                             case["Twall_top"], precision=precision)
        alt.step(4)
        np.testing.assert_array_equal(alt.get_state().cpu().numpy(), F)


@pytest.mark.parametrize("nx,ny,walls,extra", [(40, 100, 1, {}), (37, 21, 0, {"csf_form": 1}),
                                               (130, 7, 1, {}), (65, 70, 0, {}), (3, 600, 1, {}),
                                               (200, 3, 1, {"csf_form": 1}), (1030, 1000, 1, {})])
@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_tile_kernel_matches_row_kernel(lbe, monkeypatch, nx, ny, walls, extra, precision):
    """Steps in tiles of one site per lane (tile_step_kernel, with its frame
    of wrapped or ghost cells), diagnostic steps included, against the
    row-marching kernel; grids narrower and shorter than a tile, ragged in
    both directions, walls and periodic, and a ragged grid of a million sites
    (4,000 tiles: the diagnostic partials at the size where the tiles end).  FP64: the states bitwise the same.
    FP32: the same arithmetic, but the compiler fuses the FP32 multiply-adds
    of the collision differently in the two kernels, so the states agree to
    FP32 rounding (relative L2 under 1e-6).  The diagnostics are FP64 sums of
    per-block partials over different blocks: equal to rounding."""
    case = wl.random_case(nx, ny, seed=3 * nx + ny, walls_y=walls, n_drops=2, **extra)
    out = []
    for tile in ("0", "1"):
        monkeypatch.setenv("LBE_CSF_TILE", tile)
        _say(f"case tile kernel={tile} {nx}x{ny} walls={walls} {extra} {precision}")
        sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                             case["Twall_top"], precision=precision, diag_every=4)
        sim.step(9)
        out.append((sim.get_state().cpu().numpy(), sim.diag_history()))
    if precision == "fp64":
        np.testing.assert_array_equal(out[1][0], out[0][0])
    else:
        assert _rel(out[1][0], out[0][0]) < 1e-6
    assert len(out[1][1]) == len(out[0][1]) >= 2
    for a, b in zip(out[1][1], out[0][1]):
        assert a["step"] == b["step"]
        for k in ("mass", "energy", "n_nonfinite"):
            assert a[k] == pytest.approx(b[k], rel=1e-12 if precision == "fp64" else 1e-6), k


@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_tile_kernel_short_last_tile_outputs(lbe, monkeypatch, precision):
    """A grid two tiles wide whose last tile holds 6 columns: the tile
    kernel's lanes beyond the last column collide their wrapped sites and
    store what the owning lanes store.  Every output against the row-marching
    kernel: the fields, the diagnostics, and the gradients of a recorded run
    (its tape written by the tile kernel).  FP64 bitwise, FP32 to rounding."""
    import torch
    case = wl.random_case(70, 30, seed=77, walls_y=1, n_drops=2)
    rng = np.random.default_rng(77)
    seed_field = torch.as_tensor(rng.standard_normal((30, 70)))
    out = []
    for tile in ("0", "1"):
        monkeypatch.setenv("LBE_CSF_TILE", tile)
        _say(f"case short last tile kernel={tile} 70x30 {precision}")
        sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                             case["Twall_top"], precision=precision, diag_every=2,
                             record_steps=9)
        sim.step(9, record=True)
        g = sim.backward(seed_field, want_F0=True, want_T0=True)
        f = sim.fields()
        torch.cuda.synchronize()
        out.append(dict(state=sim.get_state().cpu().numpy(),
                        **{k: v.cpu().numpy() for k, v in f.items()},
                        sigmaT=np.array([g["sigmaT"]]), Twall=g["Twall"].cpu().numpy(),
                        F0=g["F0"].cpu().numpy(), T0=g["T0"].cpu().numpy(),
                        mass=np.array([d["mass"] for d in sim.diag_history()])))
    assert out[0]["mass"].size >= 4
    for key in out[0]:
        a, b = out[1][key], out[0][key]
        if precision == "fp64" and key != "mass":
            np.testing.assert_array_equal(a, b, err_msg=key)
        else:
            # FP32: states and fields to rounding, gradients through a tape
            # that differs at that rounding
            tol = 1e-5 if key in ("sigmaT", "Twall", "F0", "T0") else 1e-6
            assert _rel(a, b) < tol, key


def test_fp64_chunking_does_not_matter(lbe, oracle_mod, monkeypatch):
    """Different strip widths and chunk heights give bitwise-identical states."""
    case = wl.random_case(200, 60, seed=12, walls_y=1)
    monkeypatch.setenv("LBE_CSF_TILE", "0")   # the row-marching kernel
    out = []
    for nw, rows in (("1", "3"), ("2", "7"), ("4", "60"), ("1", "1"), ("8", "13")):
        monkeypatch.setenv("LBE_CSF_NW", nw)
        monkeypatch.setenv("LBE_CSF_ROWS", rows)
        _say(f"case chunking nw={nw} rows={rows}")
        sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                             case["Twall_top"])
        sim.step(6)
        out.append(sim.get_state().cpu().numpy())
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])


def test_determinism(lbe):
    w = wl.make("adjoint_droplet")
    res = []
    for _ in range(2):
        _say("case determinism adjoint_droplet fp32_dev 50 steps")
        sim = lbe.Simulation(w["params"], w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                             precision="fp32_dev", diag_every=10)
        sim.step(50)
        res.append((sim.get_state().cpu().numpy(), sim.diag_history()))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]
    assert [r["step"] for r in res[0][1]] == [0, 10, 20, 30, 40]


def test_diag_history_wraps(lbe):
    """The device keeps the last 4096 diagnostic records: after 4200 steps with
    a record every step, lbe_csf_diag_history returns steps 104-4199 in order
    (the ring wrapped), or the oldest `max` of them, and then starts over."""
    case = wl.random_case(8, 8, seed=3, walls_y=1)
    _say("case diag ring 8x8, 4200 steps, every step")
    sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                         case["Twall_top"], diag_every=1)
    sim.step(4200)
    last = sim.diagnostics()
    h = sim.diag_history(4096)
    assert [r["step"] for r in h] == list(range(104, 4200))
    assert all(r["n_nonfinite"] == 0 for r in h)
    assert abs(h[-1]["mass"] / last["mass"] - 1.0) < 1e-12
    sim.step(10)
    h2 = sim.diag_history(4)
    assert [r["step"] for r in h2] == [4200, 4201, 4202, 4203]
    assert sim.diag_history(4096) == []


def test_nonfinite_is_reported(lbe):
    case = wl.random_case(32, 16, seed=1)
    phi0 = case["phi0"].copy()
    phi0[5, 7] = np.nan
    _say("case non-finite injection")
    sim = lbe.Simulation(case["params"], phi0, case["T0"], case["Twall_bot"], case["Twall_top"],
                         diag_every=1)
    with pytest.raises(lbe.LbeCsfError) as e:
        sim.step(3)
    assert e.value.status == lbe.LBE_CSF_ENONFINITE
    assert sim.diagnostics()["n_nonfinite"] > 0


def test_backward_requires_record(lbe):
    case = wl.random_case(16, 16, seed=2)
    sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                         case["Twall_top"], record_steps=8)
    sim.step(4)
    with pytest.raises(lbe.LbeCsfError) as e:
        sim.backward(np.zeros((16, 16)))
    assert e.value.status == lbe.LBE_CSF_ENOTRECORDED


# ---- FP32 deviation form --------------------------------------------------------
@pytest.mark.parametrize("name,nsteps,tol", [("planar_marangoni", 50000, 1e-4),
                                             ("poiseuille", 20000, 1e-4),
                                             ("droplet", 100000, 1e-4),
                                             ("multi_droplet", 2000, 1e-4)])
def test_fp32_dev_vs_fp64(lbe, name, nsteps, tol):
    """FP32 deviation storage against the FP64 path after the stated steps
    (the FP64 path matches the oracle to 1e-12): relative L2 on phi, u and T
    within tol; mass drift reported."""
    import torch
    w = wl.make(name)
    _say(f"case fp32_dev vs fp64 {name} {nsteps}")
    res = {}
    for prec in ("fp64", "fp32_dev"):
        sim = lbe.Simulation(w["params"], w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                             precision=prec)
        m0 = sim.diagnostics()["mass"]
        sim.step(nsteps)
        res[prec] = (sim.fields(), sim.diagnostics()["mass"] / m0 - 1)
        del sim
    a, b = res["fp32_dev"][0], res["fp64"][0]
    rel = lambda x, y: (torch.linalg.norm(x - y) / torch.linalg.norm(y)).item()
    ua, ub = torch.stack([a["ux"], a["uy"]]), torch.stack([b["ux"], b["uy"]])
    errs = {"phi": rel(a["phi"], b["phi"]), "u": rel(ua, ub), "T": rel(a["T"], b["T"]),
            "T-Tmin": rel(a["T"] - b["T"].min(), b["T"] - b["T"].min())}
    _say(f"  errors " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()) +
         f"  mass drift fp64 {res['fp64'][1]:.2e} fp32 {res['fp32_dev'][1]:.2e}")
    for k in ("phi", "u", "T"):
        assert errs[k] <= tol, (k, errs[k])


def test_plain_fp32_would_fail_where_deviations_pass(lbe):
    """Ablation (storage only): rounding the FP64 state to plain FP32 values
    (not deviations) once destroys the Marangoni velocity of the planar case,
    while the deviation form keeps it; this is why deviations are stored."""
    import torch
    w = wl.make("planar_marangoni")
    sim = lbe.Simulation(w["params"], w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"])
    sim.step(5000)
    F = sim.get_state()
    ref = _fields_np(sim)
    sim.set_state(F.float().double())
    plain = _fields_np(sim)
    dev = lbe.Simulation(w["params"], w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"],
                         precision="fp32_dev")
    dev.set_state(F)
    devf = _fields_np(dev)
    e_plain, e_dev = _rel(plain["ux"], ref["ux"]), _rel(devf["ux"], ref["ux"])
    _say(f"  u_x error after one FP32 rounding: plain {e_plain:.2e}, deviations {e_dev:.2e}")
    assert e_dev < 1e-5 < e_plain


# ---- full size, sampled -------------------------------------------------------------
def _windows(nx, ny, k, rng, n):
    """n windows of (2m+8) x (2m+8) sites, m = 2 + 2k, some touching the walls
    and some wrapping in x; the centre 8 x 8 is valid after k steps."""
    m = 2 + 2 * k
    size = 2 * m + 8
    wins = [(nx - m - 4, 0, size, m + 8), (3, ny - (m + 8), size, m + 8)]   # walls, x wrap
    while len(wins) < n:
        x0 = int(rng.integers(0, nx))
        y0 = int(rng.integers(0, ny - size))
        wins.append((x0, y0, size, size))
    return wins, m


@pytest.mark.parametrize("precision,tol", [("fp32_dev", 1e-5), ("fp64", 1e-12)])
def test_full_size_sampled(lbe, oracle_mod, precision, tol):
    """The 4096 x 4096 multi-droplet workload in the benchmark's launch
    configuration: k steps on the GPU, the oracle on windows around sampled
    sites (its dependence cone is 2 sites per step), fields compared on the
    windows' valid centres."""
    w = wl.make("multi_droplet")
    p = w["params"]
    nx, ny = p["nx"], p["ny"]
    k = 20
    _say(f"case full-size multi_droplet {precision} {k} steps")
    sim = lbe.Simulation(p, w["phi0"], w["T0"], w["Twall_bot"], w["Twall_top"], precision=precision)
    sim.step(k)
    g = {kk: v.cpu().numpy() for kk, v in sim.fields().items()}
    del sim
    umax = np.hypot(g["ux"], g["uy"]).max()
    trange = w["T0"].max() - w["T0"].min()
    rng = np.random.default_rng(99)
    wins, m = _windows(nx, ny, k, rng, 12)
    # also windows centred on droplet interfaces (where the force acts)
    phi = w["phi0"]
    iy, ix = np.nonzero(np.abs(phi) < 0.5)
    for t in rng.choice(len(iy), 6, replace=False):
        y0 = int(min(max(iy[t] - m - 4, 0), ny - (2 * m + 8)))
        wins.append((int((ix[t] - m - 4) % nx), y0, 2 * m + 8, 2 * m + 8))
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
        valid = np.minimum(np.minimum(dist_x, dist_bot), dist_top) >= 2 + 2 * k
        assert valid.sum() >= 64
        gw = {f: sub(g[f])[valid] for f in FIELDS}
        ow = {f: of[f][valid] for f in FIELDS}
        for f in FIELDS:
            assert np.all(np.isfinite(ow[f]))
        # u against the largest speed of the whole field, T against its range
        du = np.hypot(gw["ux"] - ow["ux"], gw["uy"] - ow["uy"]).max()
        assert du <= tol * umax, ("u", x0, y0, du / umax)
        assert np.abs(gw["phi"] - ow["phi"]).max() <= tol, ("phi", x0, y0)
        assert np.abs(gw["T"] - ow["T"]).max() <= tol * trange, ("T", x0, y0)
        assert np.abs(gw["p"] - ow["p"]).max() <= tol * np.abs(ow["p"]).max(), ("p", x0, y0)
        checked += int(valid.sum())
    _say(f"  compared {checked} sites in {len(wins)} windows")
