"""Seeded synthetic inputs: parameter sets and initial fields of the workloads.

This module only generates inputs (parameters, initial order parameter and
temperature fields, wall temperatures, random states for parity checks).  It
holds none of the lattice Boltzmann arithmetic: both the HIP library and the
CPU oracle receive exactly these arrays and derive everything else on their
own.

The workloads are the paper's three validation problems (Sec. IV) at the
sizes of the build's benchmark set, plus a large multi-droplet throughput
case and a differentiated droplet case:

  poiseuille        8 x 64      thermal two-layer Poiseuille flow (Sec. IV A)
  planar_marangoni  256 x 128   two superimposed planar fluids (Sec. IV B)
  droplet           512 x 1024  one migrating droplet (Sec. IV C)
  adjoint_droplet   256 x 512   droplet case differentiated w.r.t. sigmaT, T_wall
  multi_droplet     4096 x 4096 200 seeded droplets, throughput
  multi_droplet_slab  4096 x 516  one of eight y-slabs of it, with 2 + 2 halo rows

Grid convention: sites (i, j) at x = i + 1/2, y = j + 1/2; x periodic; when
``walls_y`` is 1 the walls sit halfway, at y = 0 and y = ny.  Arrays are
(ny, nx) float64, x fastest.  phi = 2c - 1 with c = 1 inside droplets and in
the upper layer.

T_shift and T_grad set the linear temperature T_shift + T_grad y that the
FP32 deviation form stores hbar relative to; each workload uses the linear
profile its walls impose (only the FP32 form reads them).

Relaxation times are stated directly; the comments give the transport
coefficients they stand for (eta = (tau_f - 1/2)/3, lambda = (tau_T - 1/2)/3
at rho = cv = 1).
"""
from __future__ import annotations

import math

import numpy as np

W_DEFAULT = 2.0 * math.sqrt(2.0)   # tanh width for eps = 1 at beta = 1/4

PARAM_KEYS = ("nx", "ny", "walls_y", "rho", "cv", "tau_f", "tau_T", "tau_g",
              "mobility", "width", "beta", "sigma0", "sigmaT", "Tref", "force",
              "p0", "T_shift", "T_grad", "csf_form")

WORKLOADS = ("poiseuille", "planar_marangoni", "droplet", "adjoint_droplet",
             "multi_droplet", "adjoint_droplet_wide")


def base_params(nx: int, ny: int, **kw) -> dict:
    p = dict(nx=nx, ny=ny, walls_y=1, rho=1.0, cv=1.0, tau_f=(1.0, 1.0),
             tau_T=(1.0, 1.0), tau_g=1.0, mobility=0.05, width=W_DEFAULT,
             beta=0.25, sigma0=1e-2, sigmaT=0.0, Tref=0.0, force=(0.0, 0.0),
             p0=1.0 / 3.0, T_shift=0.0, T_grad=0.0, csf_form=0)
    p.update(kw)
    return p


def coords(nx: int, ny: int):
    """Site centre coordinates (Y, X), each (ny, nx)."""
    y = np.arange(ny, dtype=np.float64) + 0.5
    x = np.arange(nx, dtype=np.float64) + 0.5
    return np.meshgrid(y, x, indexing="ij")


def tanh_layer(nx, ny, y_if, width, upper_is_one=True):
    Y, _ = coords(nx, ny)
    s = 1.0 if upper_is_one else -1.0
    return np.tanh(s * (Y - y_if) / width)


def droplet_phi(nx, ny, drops, width, periodic_x=True):
    """phi for droplets [(xc, yc, R), ...]: c = max_k 1/2 + 1/2 tanh((R_k - r_k)/W).

    Each droplet is evaluated on its bounding box (R + 64 lattice units, where
    the tanh tail is below 1e-19); phi = -1 elsewhere."""
    phi = -np.ones((ny, nx))
    for xc, yc, R in drops:
        m = int(math.ceil(R + 64))
        j0, j1 = max(0, int(yc) - m), min(ny, int(yc) + m + 1)
        ii = np.arange(int(xc) - m, int(xc) + m + 1)
        if periodic_x:
            cols = np.mod(ii, nx)
            if len(ii) >= nx:
                ii = np.arange(nx)
                cols = ii
        else:
            ii = ii[(ii >= 0) & (ii < nx)]
            cols = ii
        y = np.arange(j0, j1) + 0.5
        x = ii + 0.5
        dx = x[None, :] - xc
        if periodic_x:
            dx = (dx + nx / 2.0) % nx - nx / 2.0
        r = np.sqrt(dx ** 2 + (y[:, None] - yc) ** 2)
        val = np.tanh((R - r) / width)
        sub = phi[j0:j1][:, cols]
        phi[j0:j1, cols] = np.maximum(sub, val)
    return phi


def place_droplets(nx, ny, n_drops, seed, rmin, rmax, gap=8.0,
                   max_tries=200000):
    """Seeded non-overlapping droplets: R ~ U[rmin, rmax], x ~ U[0, nx),
    y ~ U[R + gap, ny - R - gap]; a candidate is rejected if it comes closer
    than R_a + R_b + gap to a placed one (x distance periodic)."""
    rng = np.random.default_rng(seed)
    drops = []
    tries = 0
    while len(drops) < n_drops:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place droplets")
        R = rng.uniform(rmin, rmax)
        x = rng.uniform(0.0, nx)
        y = rng.uniform(R + gap, ny - R - gap)
        ok = True
        for (xb, yb, Rb) in drops:
            dx = abs(x - xb)
            dx = min(dx, nx - dx)
            if math.hypot(dx, y - yb) < R + Rb + gap:
                ok = False
                break
        if ok:
            drops.append((x, y, R))
    return drops


# ---- steady conduction field between the walls (adjoint_droplet) -------------
def _conduction_kernel(nx, ny):
    """B[j, m]: response at row j of wall mode m (rfft order) of the bottom
    wall, for Laplace's equation with the top wall held at 0.  Mode 0 is
    linear, mode m is sinh(k (ny - y)) / sinh(k ny), written in overflow-free
    exponential form."""
    y = np.arange(ny, dtype=np.float64) + 0.5
    m = np.arange(nx // 2 + 1, dtype=np.float64)
    k = 2.0 * np.pi * m / nx
    B = np.empty((ny, m.size))
    B[:, 0] = 1.0 - y / ny
    kk = k[None, 1:]
    yy = y[:, None]
    B[:, 1:] = (np.exp(-kk * yy) * (1.0 - np.exp(-2.0 * kk * (ny - yy)))
                / (1.0 - np.exp(-2.0 * kk * ny)))
    return B


def conduction_field(Tw_bot, T_top, ny):
    """T0 solving Laplace's equation, periodic in x, T = Tw_bot on y = 0 and
    T = T_top on y = ny (linear in (Tw_bot, T_top))."""
    Tw_bot = np.asarray(Tw_bot, dtype=np.float64)
    nx = Tw_bot.size
    B = _conduction_kernel(nx, ny)
    Fw = np.fft.rfft(Tw_bot)
    T = np.fft.irfft(Fw[None, :] * B, n=nx, axis=1)
    y = np.arange(ny, dtype=np.float64) + 0.5
    return T + (T_top * y / ny)[:, None]


def conduction_field_T(G, ny):
    """Transpose of ``conduction_field`` w.r.t. Tw_bot: given G = dJ/dT0
    (ny, nx) returns dJ/dTw_bot (nx,).  Each row map is a symmetric circulant,
    so the transpose applies the same kernel."""
    G = np.asarray(G, dtype=np.float64)
    nx = G.shape[1]
    B = _conduction_kernel(nx, ny)
    return np.fft.irfft(np.fft.rfft(G, axis=1) * B, n=nx, axis=1).sum(axis=0)


def conduction_field_torch(Tw_bot, T_top, ny):
    """``conduction_field`` written with torch operations on the wall tensor's
    device and dtype, so that autograd carries gradients of T0 back to Tw_bot
    (the transpose of this linear map)."""
    import torch
    nx = Tw_bot.shape[0]
    B = torch.as_tensor(_conduction_kernel(nx, ny), dtype=Tw_bot.dtype, device=Tw_bot.device)
    T = torch.fft.irfft(torch.fft.rfft(Tw_bot)[None, :] * B, n=nx, dim=1)
    y = torch.arange(ny, dtype=Tw_bot.dtype, device=Tw_bot.device) + 0.5
    return T + (T_top * y / ny)[:, None]


# ---- the workloads -----------------------------------------------------------
def _droplet_physics(**kw):
    # eta = 0.0715542, lambda = 7.15542e-3: Re = 1 and Ma = 10 for R = 32,
    # sigmaT = 5e-4, |grad T| = 0.01 (U = sigmaT |grad T| R / eta)
    return dict(tau_f=(0.7146625, 0.7146625), tau_T=(0.5214663, 0.5214663),
                tau_g=1.0, mobility=0.05, width=W_DEFAULT, beta=0.25,
                sigma0=1e-2, sigmaT=5e-4, Tref=0.0, **kw)


def make(name: str, **overrides) -> dict:
    """Return dict(params, phi0, T0, Twall_bot, Twall_top, nsteps, precision,
    meta) for a named workload.  ``overrides`` replace parameter entries."""
    if name == "poiseuille":
        nx, ny = 8, 64
        # eta 0.1 / 0.3 (1:3), lambda 0.1 / 0.2 (1:2); c = 0 lower layer
        p = base_params(nx, ny, tau_f=(0.8, 1.4), tau_T=(0.8, 1.1), tau_g=2.5,
                        mobility=0.1, width=4.0, sigma0=1e-3, sigmaT=1e-4,
                        Tref=10.0, force=(1e-6, 0.0), T_shift=20.0, T_grad=-10.0 / 64.0)
        phi0 = tanh_layer(nx, ny, ny / 2, 4.0)
        Y, _ = coords(nx, ny)
        T0 = 20.0 - 10.0 * Y / ny
        tb, tt = np.full(nx, 20.0), np.full(nx, 10.0)
        nsteps, prec = 20000, "fp64"
    elif name == "planar_marangoni":
        nx, ny = 256, 128
        # eta = lambda = 0.2 in both fluids; Re = Ma = 1e-3 (U_max = 3.125e-6)
        p = base_params(nx, ny, tau_f=(1.1, 1.1), tau_T=(1.1, 1.1), tau_g=1.0,
                        mobility=5e-2, width=W_DEFAULT, sigma0=2.5e-2,
                        sigmaT=4.661e-6, Tref=10.0, T_shift=10.0)
        phi0 = tanh_layer(nx, ny, ny / 2, W_DEFAULT)
        T0 = np.full((ny, nx), 10.0)
        x = np.arange(nx) + 0.5
        tb = 10.0 + 4.0 * np.cos(2.0 * np.pi * x / nx)
        tt = np.full(nx, 10.0)
        nsteps, prec = 50000, "fp32_dev"
    elif name == "droplet":
        nx, ny = 512, 1024
        p = base_params(nx, ny, T_shift=0.0, T_grad=0.01, **_droplet_physics())
        phi0 = droplet_phi(nx, ny, [(256.0, 128.0, 32.0)], W_DEFAULT)
        Y, _ = coords(nx, ny)
        T0 = 0.01 * Y
        tb, tt = np.zeros(nx), np.full(nx, 0.01 * ny)
        nsteps, prec = 100000, "fp32_dev"
    elif name == "adjoint_droplet":
        nx, ny = 256, 512
        p = base_params(nx, ny, T_shift=0.0, T_grad=0.01, **_droplet_physics())
        phi0 = droplet_phi(nx, ny, [(128.0, 96.0, 24.0)], W_DEFAULT)
        rng = np.random.default_rng(6238)
        tb = 0.0 + rng.normal(0.0, 0.1, nx)
        tt = np.full(nx, 0.01 * ny)
        T0 = conduction_field(tb, tt[0], ny)
        nsteps, prec = 4000, "fp32_dev"
    elif name == "adjoint_droplet_wide":
        # the differentiated run at a size where HBM bandwidth is the bound:
        # 4096 x 1024, sixteen droplets of radius 24 a row above the bottom
        # wall (as in adjoint_droplet), bottom wall N(0, 0.1^2), T0 the
        # conduction field of the walls; 400 steps (20 checkpoints)
        nx, ny = 4096, 1024
        p = base_params(nx, ny, T_shift=0.0, T_grad=0.01, **_droplet_physics())
        drops = [(128.0 + 256.0 * k, 96.0, 24.0) for k in range(16)]
        phi0 = droplet_phi(nx, ny, drops, W_DEFAULT)
        rng = np.random.default_rng(62380)
        tb = 0.0 + rng.normal(0.0, 0.1, nx)
        tt = np.full(nx, 0.01 * ny)
        T0 = conduction_field(tb, tt[0], ny)
        nsteps, prec = 400, "fp32_dev"
    elif name == "multi_droplet":
        nx, ny = 4096, 4096
        p = base_params(nx, ny, T_shift=0.0, T_grad=0.002, **_droplet_physics())
        drops = place_droplets(nx, ny, 200, 1412, 16.0, 48.0)
        phi0 = droplet_phi(nx, ny, drops, W_DEFAULT)
        Y, _ = coords(nx, ny)
        T0 = 0.002 * Y
        tb, tt = np.zeros(nx), np.full(nx, 0.002 * ny)
        nsteps, prec = 2000, "fp32_dev"
    elif name == "multi_droplet_slab":
        # one GPU's share of the 4096 x 4096 run split into eight y-slabs:
        # 512 rows plus two halo rows on each side, taken from the middle of
        # the full field; walls at the band's edges hold the full field's
        # temperatures there (the stand-in for the exchanged halo rows)
        full = make("multi_droplet")
        y0, y1 = 2048 - 258, 2048 + 258
        p = dict(full["params"], ny=y1 - y0, T_shift=0.002 * y0)
        phi0 = full["phi0"][y0:y1]
        T0 = full["T0"][y0:y1]
        tb, tt = np.full(4096, 0.002 * y0), np.full(4096, 0.002 * y1)
        nsteps, prec = 2000, "fp32_dev"
    else:
        raise KeyError(name)
    p.update(overrides)
    return dict(params=p, phi0=np.ascontiguousarray(phi0),
                T0=np.ascontiguousarray(T0), Twall_bot=np.ascontiguousarray(tb),
                Twall_top=np.ascontiguousarray(tt), nsteps=nsteps,
                precision=prec, name=name)


# ---- the paper's own test cases at their printed parameters (Sec. IV) --------
def paper_case(name: str, lam_r: float = 1.0, h_r: float = 1.0, R: float = 20.0,
               height: float = 2.0, **overrides) -> dict:
    """Sec. IV as printed: "e1" layered Poiseuille flow (40 x 100, eta_r = 10,
    lam_r in {1, 10, 100}, h_r = h/H in {1, 1/9, 9}), "e2" two superimposed
    planar fluids (200 x 100, lam_r = lam1/lam2 in {1, 0.1}, fluid 1 upper),
    "e3" the migrating droplet (160 x 300, R = 20).  eps = 1 (W = 2 sqrt 2),
    beta = 1/4, rho = cv = 1 throughout.  Values the text leaves open:
    mobility 5e-2 with tau_g = 1 in every case (the one printed M); e1 with
    T = 0 / 1 on the walls, sigma0 = 1e-3, and a body force from Re = 1 unless
    that drives the low-viscosity layer above |u| = 0.01 (h_r = 1/9), where it
    is scaled down to that bound; e1 starts from the steady two-layer
    conduction profile (its thermal time reaches 2.5e6 steps at lam_r = 100);
    e3 with sigmaT = 5e-5, the value that the printed U_YGB = 1.333e-4
    implies, and the matrix at the droplet's saturation: the order parameter
    is the tanh droplet raised by mu_R / (2 beta) everywhere, mu_R =
    sigma_fe / R the chemical potential of a droplet of radius R with the
    free-energy tension sigma_fe = eps^2 / (3 W) of the double well.  Below
    a critical radius, which R = 20 in 160 x 300 is, a droplet in a pure
    matrix dissolves into it; the saturated matrix keeps it in equilibrium.

    e3 also takes R (default 20) and height (the droplet centre above the
    bottom wall in radii, default 2): a resolution series of the same
    droplet at fixed Re = U R / nu, Ma = U R / kappa, Ca = U eta / sigma0 and
    Cahn-Hilliard Peclet number U R / M, with the interface width W fixed
    (so the Cahn number W / R falls as 1 / R).  With s = R / 20 the box is
    8R x 15R, |grad T| = 0.1, sigmaT = 5e-5 / s^2, sigma0 = 0.1 / s, nu,
    kappa and M unchanged; U = 1e-3 / s, t_r = R / U = 2e4 s^2."""
    W = W_DEFAULT
    if name == "e1":
        nx, ny = 40, 100
        h = ny * h_r / (1.0 + h_r)
        H = ny - h
        eta1, lam1 = 0.1, 0.1
        eta2, lam2 = eta1 / 10.0, lam1 / lam_r
        u1 = eta1 / h                                   # Re = u1 h / eta1 = 1
        ax = 2.0 * eta1 * u1 / (h * h)
        # largest |u| of the two-layer profile (upper-layer maximum or the
        # interface value)
        yy = np.linspace(-h, H, 4001)
        lo = ax * h * h / (2 * eta1) * (-(yy / h) ** 2 + ((H * H / (h * h) * eta1 - eta2)
                                        / (H / h * eta1 + eta2)) * yy / h
                                        + (1 + H / h) * H * eta1 / (eta1 * H + eta2 * h))
        up = ax * H * H / (2 * eta2) * (-(yy / H) ** 2 + ((eta1 - h * h / (H * H) * eta2)
                                        / (eta1 + h / H * eta2)) * yy / H
                                        + (1 + h / H) * h * eta2 / (eta1 * H + eta2 * h))
        umax = float(np.abs(np.where(yy < 0, lo, up)).max())
        if umax > 0.01:
            ax *= 0.01 / umax
        p = base_params(nx, ny, tau_f=(3 * eta1 + 0.5, 3 * eta2 + 0.5),
                        tau_T=(3 * lam1 + 0.5, 3 * lam2 + 0.5), tau_g=1.0, mobility=5e-2,
                        width=W, sigma0=1e-3, sigmaT=0.0, Tref=0.0, force=(ax, 0.0),
                        T_shift=0.0, T_grad=1.0 / ny)
        phi0 = tanh_layer(nx, ny, h, W)
        Y, _ = coords(nx, ny)
        yr = Y - h
        d = lam1 * H + lam2 * h
        b = (lam2 * h * 1.0) / d                        # T = 0 at y = -h, 1 at y = H
        T0 = np.where(yr < 0, lam2 / d * yr + b, lam1 / d * yr + b)
        tb, tt = np.zeros(nx), np.ones(nx)
        nsteps = int(2.0 * max(h * h / eta1, H * H / eta2))
        meta = dict(h=h, H=H, eta1=eta1, eta2=eta2, lam1=lam1, lam2=lam2, ax=ax, Tc=0.0, Th=1.0)
    elif name == "e2":
        nx, ny = 200, 100
        lam2, lam1 = 0.2, 0.2 * lam_r                   # fluid 1 upper (c = 1)
        p = base_params(nx, ny, tau_f=(1.1, 1.1), tau_T=(3 * lam2 + 0.5, 3 * lam1 + 0.5),
                        tau_g=1.0, mobility=5e-2, width=W, sigma0=2.5e-2, sigmaT=5e-4,
                        Tref=10.0, T_shift=20.0, T_grad=-0.1)
        phi0 = tanh_layer(nx, ny, ny / 2, W)
        Y, _ = coords(nx, ny)
        T0 = 20.0 - 10.0 * Y / ny
        x = np.arange(nx) + 0.5
        tb = 20.0 + 4.0 * np.cos(2.0 * np.pi * x / nx)
        tt = np.full(nx, 10.0)
        nsteps = int(3.0 * 50 * 50 / min(lam1, lam2))
        meta = dict(h=50.0, H=50.0, eta1=0.2, eta2=0.2, lam1=lam1, lam2=lam2, Tc=10.0,
                    Th=20.0, Tr=4.0, sigma_T=-5e-4)
    elif name == "e3":
        sc = R / 20.0
        nx, ny = int(round(8 * R)), int(round(15 * R))   # 160 x 300 at R = 20
        p = base_params(nx, ny, tau_f=(0.8, 0.8), tau_T=(0.8, 0.8), tau_g=1.0, mobility=5e-2,
                        width=W, sigma0=0.1 / sc, sigmaT=5e-5 / sc ** 2, Tref=0.0,
                        T_shift=0.0, T_grad=0.1)
        eps = W * math.sqrt(0.25 / 2.0)
        sat = (eps * eps / (3.0 * W)) / R / (2.0 * 0.25)
        phi0 = droplet_phi(nx, ny, [(nx / 2.0, height * R, R)], W) + 2.0 * sat
        Y, _ = coords(nx, ny)
        T0 = 0.1 * Y
        tb, tt = np.zeros(nx), np.full(nx, 0.1 * ny)
        t_r = int(round(20000 * sc * sc))               # t_r = R / U
        nsteps = 10 * t_r
        meta = dict(R=R, U=1e-3 / sc, U_YGB=1.0 / 7500.0 / sc, t_r=t_r)
    else:
        raise KeyError(name)
    p.update(overrides)
    return dict(params=p, phi0=np.ascontiguousarray(phi0), T0=np.ascontiguousarray(T0),
                Twall_bot=np.ascontiguousarray(tb), Twall_top=np.ascontiguousarray(tt),
                nsteps=nsteps, precision="fp64", name=f"paper_{name}", meta=meta)


def random_case(nx, ny, seed, walls_y=1, n_drops=2, amp_T=0.5, **kw):
    """Small seeded case for parity checks: a few droplets (radius 2-5 sites
    smaller than the grid), a random temperature field around 1 and random
    wall temperatures, with parameters drawn in stable ranges.  The reference
    pressure is 0 (an exact symmetry of the method), so the populations are
    of the size of their deviations and FP64 comparisons of u and p are not
    swamped by the round-off of a large constant part."""
    rng = np.random.default_rng(seed)
    tau_g = float(rng.uniform(0.8, 1.3))
    width = float(rng.uniform(1.5, 3.0))
    # mobility kept below 0.1 (tau_g - 1/2) / eps^2 with eps^2 = W^2 beta / 2:
    # larger values make the shortest lattice waves of c grow
    mobility = float(rng.uniform(0.3, 1.0)) * 0.1 * (tau_g - 0.5) / (width ** 2 / 8.0)
    p = base_params(
        nx, ny, walls_y=walls_y,
        tau_f=tuple(rng.uniform(0.6, 1.4, 2)), tau_T=tuple(rng.uniform(0.55, 1.2, 2)),
        tau_g=tau_g, mobility=mobility, width=width, beta=0.25,
        sigma0=float(rng.uniform(5e-3, 2e-2)), sigmaT=float(rng.uniform(-2e-3, 2e-3)),
        Tref=float(rng.uniform(0.5, 1.5)),
        force=tuple(rng.uniform(-1e-4, 1e-4, 2)), p0=0.0, T_shift=1.0,
        T_grad=(float(np.random.default_rng(seed + 100003).uniform(-0.02, 0.02))
                if walls_y else 0.0))
    p.update(kw)
    drops = []
    for _ in range(n_drops):
        R = float(rng.uniform(2.0, max(2.5, min(nx, ny) / 4)))
        drops.append((float(rng.uniform(0, nx)), float(rng.uniform(0, ny)), R))
    phi0 = droplet_phi(nx, ny, drops, p["width"])
    phi0 = np.clip(phi0 + 0.05 * rng.standard_normal((ny, nx)), -1.2, 1.2)
    T0 = 1.0 + amp_T * rng.standard_normal((ny, nx))
    tb = 1.0 + 0.3 * rng.standard_normal(nx)
    tt = 1.0 + 0.3 * rng.standard_normal(nx)
    return dict(params=p, phi0=np.ascontiguousarray(phi0), T0=np.ascontiguousarray(T0),
                Twall_bot=tb, Twall_top=tt, name=f"random_{nx}x{ny}_s{seed}")


def random_state(nx, ny, seed, p0=1.0 / 3.0, T=1.0):
    """A seeded non-equilibrium state (27, ny, nx): rest-weight values with
    10% relative noise for f and hbar, and order-parameter populations that
    sum to a c field in [-0.1, 1.1]."""
    rng = np.random.default_rng(seed)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    F = np.empty((27, ny, nx))
    F[0:9] = w[:, None, None] * p0 * (1.0 + 0.1 * rng.standard_normal((9, ny, nx)))
    cfield = rng.uniform(-0.1, 1.1, (ny, nx))
    gn = 0.02 * rng.standard_normal((9, ny, nx))
    F[9:18] = w[:, None, None] * cfield[None] + gn
    F[18:27] = w[:, None, None] * T * (1.0 + 0.1 * rng.standard_normal((9, ny, nx)))
    return F
