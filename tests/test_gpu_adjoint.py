"""GPU adjoint: lbe_csf_backward (and the autograd Function above it) against
central finite differences of the FP64 CPU oracle.

Small cases: J = sum_x s(x) c_N(x) with a seeded weight s, N steps spanning
several checkpoint segments (the last one partial), grids with several
adjoint strips and row chunks (ragged), walls and periodic y.  Every control
is checked: sigmaT, the bottom and top wall temperatures (along a seeded
direction), the initial temperature field and the whole initial state (along
seeded directions).  FP64 within 1e-6 relative of the oracle's differences
(their own error is below 1e-7 at these step sizes), FP32 deviations within
1e-3.

Full size: the 256 x 512 droplet run of 4000 steps through CSFDroplet,
gradient of the centroid displacement w.r.t. sigmaT and the bottom wall
temperatures (16 seeded components, 8 seeded directions) against the stored
oracle differences (tests/golden/adjoint_droplet_fd.json): FP32 within 1e-3
relative, FP64 within 1e-6 (sigmaT) and 1e-4 (walls).
"""
import json
import os
import sys
import time

import numpy as np
import pytest

from paper_1412_6238_amd import workloads as wl

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lbe():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_6238_amd import lbe_csf
    return lbe_csf


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_J(oracle_mod, case, N, s, sigmaT=None, tb=None, tt=None, T0=None, F0=None):
    p = dict(case["params"])
    if sigmaT is not None:
        p["sigmaT"] = sigmaT
    o = oracle_mod.Oracle(p, case["Twall_bot"] if tb is None else tb,
                          case["Twall_top"] if tt is None else tt)
    o.init(case["phi0"], case["T0"] if T0 is None else T0)
    if F0 is not None:
        o.set_state(F0)
    o.step(N)
    c = 0.5 * (1.0 + o.fields()["phi"])
    return float((s * c).sum())


def _fd(f, h):
    return (f(h) - f(-h)) / (2.0 * h)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# relaxation times that vary with c use the full-state replay; constant ones
# the moment tape
CONST_TAU = dict(tau_f=(0.9, 0.9), tau_T=(0.8, 0.8))
CASES = [
    # nx, ny, walls, seed, N, precision, parameter overrides
    (37, 21, 1, 5, 12, "fp64", {}),
    (130, 13, 1, 11, 10, "fp64", {}),
    (70, 9, 0, 7, 12, "fp64", {}),
    (37, 21, 1, 5, 12, "fp32_dev", {}),
    (130, 13, 1, 11, 10, "fp32_dev", {}),
    (37, 21, 1, 5, 12, "fp64", CONST_TAU),
    (130, 13, 1, 11, 10, "fp64", CONST_TAU),
    (70, 9, 0, 7, 12, "fp64", CONST_TAU),
    (130, 13, 1, 11, 10, "fp32_dev", CONST_TAU),
    # the capillary force in the curvature form (Eq. 4)
    (37, 21, 1, 5, 12, "fp64", dict(csf_form=1)),
    (70, 9, 0, 7, 12, "fp64", dict(csf_form=1)),
    (130, 13, 1, 11, 10, "fp32_dev", dict(csf_form=1)),
    (130, 13, 1, 11, 10, "fp64", dict(CONST_TAU, csf_form=1)),
]


@pytest.mark.parametrize("nx,ny,walls,seed,N,prec,over", CASES)
def test_adjoint_vs_oracle_fd(lbe, oracle_mod, nx, ny, walls, seed, N, prec, over):
    import torch
    _say(f"adjoint vs oracle FD: {nx}x{ny} walls={walls} seed={seed} N={N} {prec} {over}")
    case = wl.random_case(nx, ny, seed, walls_y=walls, **over)
    rng = np.random.default_rng(1000 + seed)
    s = rng.standard_normal((ny, nx))
    # weights near the walls make the wall-temperature derivative sizeable
    sw = np.zeros((ny, nx))
    sw[:3] = rng.standard_normal((3, nx))
    sw[-3:] = rng.standard_normal((3, nx))
    tol = 1e-6 if prec == "fp64" else 1e-3
    p = case["params"]

    def grads(seed_field):
        sim = lbe.Simulation(p, case["phi0"], case["T0"], case["Twall_bot"] if walls else None,
                             case["Twall_top"] if walls else None, precision=prec,
                             record_steps=N)
        sim.step(N, record=True)
        g = sim.backward(torch.as_tensor(seed_field), want_F0=True, want_T0=True)
        torch.cuda.synchronize()
        return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in g.items()}

    g = grads(s)
    st0 = p["sigmaT"]
    fd = _fd(lambda h: _oracle_J(oracle_mod, case, N, s, sigmaT=st0 + h), 1e-5)
    _say(f"  dJ/dsigmaT gpu {g['sigmaT']!r} fd {fd!r} rel {_rel(g['sigmaT'], fd):.2e}")
    assert _rel(g["sigmaT"], fd) <= tol

    dT = rng.standard_normal((ny, nx))
    fd = _fd(lambda h: _oracle_J(oracle_mod, case, N, s, T0=case["T0"] + h * dT), 1e-5)
    ad = float((g["T0"] * dT).sum())
    _say(f"  dJ/dT0 . d gpu {ad!r} fd {fd!r} rel {_rel(ad, fd):.2e}")
    assert _rel(ad, fd) <= tol

    o = oracle_mod.Oracle(p, case["Twall_bot"], case["Twall_top"])
    o.init(case["phi0"], case["T0"])
    F0 = o.state()
    dF = 0.01 * rng.standard_normal(F0.shape)
    fd = _fd(lambda h: _oracle_J(oracle_mod, case, N, s, F0=F0 + h * dF), 1e-5)
    ad = float((g["F0"] * dF).sum())
    _say(f"  dJ/dF0 . d gpu {ad!r} fd {fd!r} rel {_rel(ad, fd):.2e}")
    assert _rel(ad, fd) <= tol

    if walls:
        gw = grads(sw)
        for side, key in ((0, "tb"), (1, "tt")):
            d = rng.standard_normal(nx)
            base = case["Twall_bot"] if side == 0 else case["Twall_top"]
            # J is linear in the wall values to ~1e-7 over this step, which keeps
            # the round-off of the differences of these small derivatives low
            fd = _fd(lambda h: _oracle_J(oracle_mod, case, N, sw, **{key: base + h * d}), 1e-2)
            ad = float((gw["Twall"][side] * d).sum())
            _say(f"  dJ/dTw[{side}] . d gpu {ad!r} fd {fd!r} rel {_rel(ad, fd):.2e}")
            assert _rel(ad, fd) <= tol
    else:
        assert np.all(g["Twall"] == 0.0)


def test_adjoint_deterministic_and_state_kept(lbe):
    """Two backward passes give bitwise equal gradients; the forward state is
    unchanged by them; a backward needs a recorded run ending at the state."""
    import torch
    _say("adjoint determinism 130x13 fp64")
    case = wl.random_case(130, 13, 3, walls_y=1)
    sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                         case["Twall_top"], precision="fp64", record_steps=20)
    sim.step(17, record=True)
    f_before = sim.get_state().cpu().numpy()
    seed = torch.as_tensor(np.random.default_rng(4).standard_normal((13, 130)))
    g1 = sim.backward(seed, want_F0=True)
    g2 = sim.backward(seed, want_F0=True)
    assert g1["sigmaT"] == g2["sigmaT"]
    assert torch.equal(g1["Twall"], g2["Twall"]) and torch.equal(g1["F0"], g2["F0"])
    assert np.array_equal(sim.get_state().cpu().numpy(), f_before)
    sim.step(1)
    with pytest.raises(lbe.LbeCsfError) as e:
        sim.backward(seed)
    assert e.value.status == lbe.LBE_CSF_ENOTRECORDED
    with pytest.raises(lbe.LbeCsfError):
        sim.step(21, record=True)            # beyond the workspace's record capacity


def test_adjoint_segments_agree(lbe):
    """The checkpoint spacing only changes what is recomputed: a run recorded
    in one call and the same run with a larger record capacity give the same
    gradient bitwise (K = ceil(sqrt N) of the run, not of the capacity)."""
    import torch
    case = wl.random_case(37, 21, 8, walls_y=1)
    seed = torch.as_tensor(np.random.default_rng(5).standard_normal((21, 37)))
    out = []
    for cap in (9, 50):
        sim = lbe.Simulation(case["params"], case["phi0"], case["T0"], case["Twall_bot"],
                             case["Twall_top"], precision="fp64", record_steps=cap)
        sim.step(9, record=True)
        out.append(sim.backward(seed, want_F0=True))
    assert out[0]["sigmaT"] == out[1]["sigmaT"]
    assert torch.equal(out[0]["F0"], out[1]["F0"])


def test_autograd_function(lbe):
    """torch.autograd through LbeRun: J computed in torch from phi_N; the
    gradients equal those of a direct lbe_csf_backward with dJ/dc = 2 dJ/dphi."""
    import torch
    case = wl.random_case(37, 21, 5, walls_y=1)
    p = case["params"]
    dev = torch.device("cuda:0")
    sT = torch.tensor(p["sigmaT"], dtype=torch.float64, requires_grad=True)
    tb = torch.tensor(case["Twall_bot"], device=dev, requires_grad=True)
    tt = torch.tensor(case["Twall_top"], device=dev, requires_grad=True)
    T0 = torch.tensor(case["T0"], device=dev, requires_grad=True)
    phi = lbe.run_phi(p, case["phi0"], T0, tb, tt, 8, sT, precision="fp64")
    y = torch.arange(21, dtype=torch.float64, device=dev)[:, None] + 0.5
    c = 0.5 * (1.0 + phi)
    J = (c * y).sum() / c.sum()
    J.backward()
    # direct call with the same seed
    sim = lbe.Simulation(p, case["phi0"], case["T0"], case["Twall_bot"], case["Twall_top"],
                         precision="fp64", record_steps=8)
    sim.step(8, record=True)
    cN = 0.5 * (1.0 + sim.fields(("phi",))["phi"])
    seed = (y - (cN * y).sum() / cN.sum()) / cN.sum()
    g = sim.backward(seed.expand(21, 37).contiguous())
    assert abs(sT.grad.item() - g["sigmaT"]) <= 1e-12 * abs(g["sigmaT"])
    assert torch.allclose(tb.grad, g["Twall"][0], rtol=1e-12, atol=0)
    assert torch.allclose(tt.grad, g["Twall"][1], rtol=1e-12, atol=0)
    assert torch.allclose(T0.grad, g["T0"], rtol=1e-12, atol=0)


def test_csf_droplet_function(lbe, oracle_mod):
    """CSFDroplet: J = y_c(N) - y_c(0) with T0 the conduction field of the
    walls built with torch operations, so that autograd adds the path through
    T0 to the direct wall derivative.  J, dJ/dsigmaT and the total wall
    derivative along a seeded direction against the FP64 oracle (central
    differences), within 1e-6."""
    import torch
    nx, ny, N = 37, 21, 12
    case = wl.random_case(nx, ny, 5, walls_y=1)
    p = case["params"]
    T_top = 1.5
    dev = torch.device("cuda:0")
    sT = torch.tensor(p["sigmaT"], dtype=torch.float64, requires_grad=True)
    tb = torch.tensor(case["Twall_bot"], device=dev, requires_grad=True)
    tt = torch.full((nx,), T_top, dtype=torch.float64, device=dev)
    T0 = wl.conduction_field_torch(tb, T_top, ny)
    J = lbe.CSFDroplet.apply(sT, tb, tt, T0, p, case["phi0"], N, "fp64")
    J.backward()

    def orc_J(sigmaT, tbv):
        o = oracle_mod.Oracle(dict(p, sigmaT=sigmaT), tbv, np.full(nx, T_top))
        o.init(case["phi0"], wl.conduction_field(tbv, T_top, ny))
        y0 = o.diag()["centroid_y"]
        o.step(N)
        return o.diag()["centroid_y"] - y0

    J_o = orc_J(p["sigmaT"], case["Twall_bot"])
    _say(f"  CSFDroplet J gpu {J.item()!r} oracle {J_o!r}")
    assert abs(J.item() - J_o) <= 1e-12 * ny
    fd = _fd(lambda h: orc_J(p["sigmaT"] + h, case["Twall_bot"]), 1e-5)
    _say(f"  dJ/dsigmaT gpu {sT.grad.item()!r} fd {fd!r}")
    assert _rel(sT.grad.item(), fd) <= 1e-6
    d = np.random.default_rng(17).standard_normal(nx)
    fd = _fd(lambda h: orc_J(p["sigmaT"], case["Twall_bot"] + h * d), 1e-2)
    ad = float((tb.grad.cpu().numpy() * d).sum())
    _say(f"  dJ/dTw_bot . d (total) gpu {ad!r} fd {fd!r}")
    assert _rel(ad, fd) <= 1e-6


GOLDEN = os.path.join(HERE, "golden", "adjoint_droplet_fd.json")


def _droplet_gradient(lbe, w, N, precision):
    """CSFDroplet on the differentiated droplet run: returns (J, dJ/dsigmaT,
    total dJ/dTw_bot, forward seconds, backward seconds).  T0 is the
    conduction field of the walls, built with torch operations, so the wall
    gradient includes the path through the initial temperature field."""
    import torch
    p = w["params"]
    ny = p["ny"]
    dev = torch.device("cuda:0")
    sT = torch.tensor(p["sigmaT"], dtype=torch.float64, requires_grad=True)
    tb = torch.tensor(w["Twall_bot"], device=dev, requires_grad=True)
    tt = torch.tensor(w["Twall_top"], device=dev)
    T0 = wl.conduction_field_torch(tb, float(w["Twall_top"][0]), ny)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = lbe.CSFDroplet.apply(sT, tb, tt, T0, p, w["phi0"], N, precision)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    return J.item(), sT.grad.item(), tb.grad.cpu().numpy(), t_fwd, t_bwd


def _vec_rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden differences not generated")
@pytest.mark.parametrize("precision,tol,tol_wall",
                         [("fp32_dev", 1e-3, 1e-3), ("fp64", 1e-6, 1e-4)])
def test_adjoint_droplet_full(lbe, precision, tol, tol_wall):
    """256 x 512 droplet, 4000 steps with sqrt(N) checkpoints, through
    CSFDroplet: gradient of the centroid displacement against the FP64
    oracle's central differences -- sigmaT (h = 1e-6), eight seeded
    directions and sixteen seeded components of the bottom-wall temperatures
    (h = 1e-3, where the differences are not limited by the round-off of J).
    The wall derivatives are compared as vectors (relative 2-norm) and one by
    one.  FP32 within 1e-3.  FP64 within 1e-6 on sigmaT and 1e-4 on the wall
    derivatives, the accuracy of the differences themselves (h = 1e-6 and
    h = 1e-3 differ by up to ~1e-4 on the smallest components)."""
    ref = json.load(open(GOLDEN))
    w = wl.make("adjoint_droplet")
    N = ref["nsteps"]
    _say(f"adjoint droplet 256x512 N={N} {precision}")
    J, dsT, dtb, t_fwd, t_bwd = _droplet_gradient(lbe, w, N, precision)
    _say(f"  J gpu {J!r} oracle {ref['J']!r}; forward {t_fwd:.3f} s backward {t_bwd:.3f} s "
         f"ratio {t_bwd / t_fwd:.2f}")
    assert abs(J - ref["J"]) <= (1e-4 if precision == "fp32_dev" else 1e-9) * abs(ref["J"])
    rel = _rel(dsT, ref["dJ_dsigmaT"])
    _say(f"  dJ/dsigmaT gpu {dsT!r} fd {ref['dJ_dsigmaT']!r} rel {rel:.2e}")
    assert rel <= tol
    ad_d, fd_d = [], []
    for d in ref["Twall_directions"]:
        fd = d.get("dJ_h_wall", d["dJ"])
        ad = float(np.dot(dtb, np.asarray(d["direction"])))
        ad_d.append(ad)
        fd_d.append(fd)
        _say(f"  dJ/dTw . d gpu {ad!r} fd {fd!r} (h=1e-6: {d['dJ']!r}) rel {_rel(ad, fd):.2e}")
        assert _rel(ad, fd) <= tol_wall
    comps = ref.get("Twall_components_h_wall", ref["Twall_components"])
    ad_c = [float(dtb[int(i)]) for i in comps]
    fd_c = [float(v) for v in comps.values()]
    for (i, v), a in zip(comps.items(), ad_c):
        _say(f"  dJ/dTw[{i}] gpu {a!r} fd {v!r} (h=1e-6: {ref['Twall_components'][i]!r}) "
             f"rel {_rel(a, v):.2e}")
        assert _rel(a, v) <= tol_wall
    rd, rc = _vec_rel(ad_d, fd_d), _vec_rel(ad_c, fd_c)
    _say(f"  {len(ad_d)} directions: relative 2-norm {rd:.2e}; {len(ad_c)} components: {rc:.2e}")
    assert rd <= tol_wall and rc <= tol_wall
