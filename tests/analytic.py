"""Closed-form solutions the paper gives for its validation problems (Sec. IV).

Used only as pins of the CPU oracle.  Coordinates follow the paper: y is
measured from the interface (lower layer -h <= y < 0, upper layer
0 < y <= H), x from the centre of the periodic cell.
"""
from __future__ import annotations

import math

import numpy as np


def poiseuille_ux(y, h, H, eta1, eta2, rho, ax):
    """Two-layer Poiseuille velocity, Sec. IV A, Eq. (28); fluid 1 below."""
    y = np.asarray(y, dtype=np.float64)
    lo = rho * ax * h * h / (2 * eta1) * (
        -(y / h) ** 2 + ((H * H / (h * h) * eta1 - eta2) / (H / h * eta1 + eta2)) * y / h
        + (1 + H / h) * H * eta1 / (eta1 * H + eta2 * h))
    up = rho * ax * H * H / (2 * eta2) * (
        -(y / H) ** 2 + ((eta1 - h * h / (H * H) * eta2) / (eta1 + h / H * eta2)) * y / H
        + (1 + h / H) * h * eta2 / (eta1 * H + eta2 * h))
    return np.where(y < 0, lo, up)


def poiseuille_T(y, h, H, lam1, lam2, Tc, Th):
    """Two-layer conduction profile, Sec. IV A, Eq. (29): T = Tc at y = -h,
    T = Th at y = H."""
    y = np.asarray(y, dtype=np.float64)
    d = lam1 * H + lam2 * h
    b = (lam1 * H * Tc + lam2 * h * Th) / d
    return np.where(y < 0, lam2 * (Th - Tc) / d * y + b, lam1 * (Th - Tc) / d * y + b)


def planar_marangoni(x, y, L, h, H, eta1, eta2, lam1, lam2, Tc, Th, Tr, sigma_T):
    """Pendse-Esmaeeli solution for two superimposed planar fluids (Sec. IV B,
    Eqs. 32-43), fluid 1 in the upper layer 0 < y <= H, fluid 2 below.

    Three misprints are corrected: cost(kx) is cos(kx); the first lower-layer
    coefficient is C^h_1 (printed as a second C^h_2); and the lower-layer C^h_3
    carries the opposite sign, (sinh 2b - 2b) / (2 [sinh^2 b - b^2]), which is
    the sign that makes u_x and u_y vanish on the lower wall (the printed
    upper-layer coefficients already vanish on the upper wall).
    ``sigma_T`` is the paper's d(sigma)/dT (negative for most fluids).
    Returns (u_x, u_y, T)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    k = 2 * math.pi / L
    a, b = H * k, h * k
    lr, er = lam1 / lam2, eta1 / eta2
    sh, ch = math.sinh, math.cosh
    f = 1.0 / (lr * ch(a) * sh(b) + sh(a) * ch(b))
    Da, Db = sh(a) ** 2 - a * a, sh(b) ** 2 - b * b
    CH1, CH2, CH3 = sh(a) ** 2 / Da, -H * a / Da, (2 * a - sh(2 * a)) / (2 * Da)
    Ch1, Ch2, Ch3 = sh(b) ** 2 / Db, -h * b / Db, (sh(2 * b) - 2 * b) / (2 * Db)
    g = sh(a) * f
    hh = Da * Db / (er * Db * (sh(2 * a) - 2 * a) + Da * (sh(2 * b) - 2 * b))
    Umax = -Tr * sigma_T / eta2 * g * hh

    def vel(C1, C2, C3):
        ux = Umax * ((C1 + k * (C2 + C3 * y)) * np.cosh(k * y)
                     + (C3 + k * C1 * y) * np.sinh(k * y)) * np.sin(k * x)
        uy = -k * Umax * (C1 * y * np.cosh(k * y)
                          + (C2 + C3 * y) * np.sinh(k * y)) * np.cos(k * x)
        return ux, uy

    uxu, uyu = vel(CH1, CH2, CH3)
    uxl, uyl = vel(Ch1, Ch2, Ch3)
    Tu = ((Tc - Th) * y + lr * Tc * h + Th * H) / (H + lr * h) \
        + Tr * f * np.sinh(a - k * y) * np.cos(k * x)
    Tl = (lr * (Tc - Th) * y + lr * Tc * h + Th * H) / (H + lr * h) \
        + Tr * f * (sh(a) * np.cosh(k * y) - lr * np.sinh(k * y) * ch(a)) * np.cos(k * x)
    up = y >= 0
    return np.where(up, uxu, uxl), np.where(up, uyu, uyl), np.where(up, Tu, Tl), Umax


def ygb_velocity(sigma_T, gradT, R, eta2, lam_r, eta_r):
    """Young-Goldstein-Block migration velocity, Sec. IV C, Eqs. (44)-(45)."""
    U = -sigma_T * gradT * R / eta2
    return 2 * U / ((2 + lam_r) * (2 + 3 * eta_r))


def layered_1d_steady(ny, h, width, eta1, eta2, lam1, lam2, ax, Tc, Th, n=400001,
                      rho1=1.0, rho2=None, tau=None):
    """Steady two-layer channel flow and conduction with the diffuse interface
    of the method: c(y) = 1/2 + 1/2 tanh((y - h)/W) between walls at y = 0 and
    y = ny (fluid 1, c = 0, below), viscosity and conductivity linear in c
    (the reading of the unstated interpolation).  The x-momentum balance
    d/dy(eta u') = -rho a_x with u = 0 on both walls and the heat balance
    (lam T')' = 0 with T = Tc, Th on the walls are integrated by quadrature:
        eta u' = -a_x (R(y) - R*),  R(y) = int_0^y rho,
        R* = int(R/eta) / int(1/eta)   (u vanishes on both walls),
        T = Tc + (Th - Tc) int_0^y dy/lam / int_0^ny dy/lam.
    With one density (rho2 None) rho = rho1 throughout.  With two densities
    rho(c) = rho1 + c (rho2 - rho1), and ``tau`` = (tau_f, tau_T), each a
    pair for c = 0 and c = 1, gives eta = rho (tau_f(c) - 1/2)/3 and
    lam = rho cv (tau_T(c) - 1/2)/3 (cv = 1) with tau linear in c; eta1..lam2
    are then ignored.  Returns (u, T) at the site centres y = j + 1/2.  The
    sharp-interface limit (W -> 0) with one density is Eqs. (28)-(29)."""
    y = np.linspace(0.0, float(ny), n)
    c = 0.5 + 0.5 * np.tanh((y - h) / width)
    rho = rho1 + c * ((rho1 if rho2 is None else rho2) - rho1)
    if tau is None:
        eta = eta1 + c * (eta2 - eta1)
        lam = lam1 + c * (lam2 - lam1)
    else:
        (tf0, tf1), (tT0, tT1) = tau
        eta = rho * (tf0 + c * (tf1 - tf0) - 0.5) / 3.0
        lam = rho * (tT0 + c * (tT1 - tT0) - 0.5) / 3.0

    def cumint(f):
        return np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(y))])

    R = rho1 * y if rho2 is None else cumint(rho)
    i0, i1, il = cumint(1.0 / eta), cumint(R / eta), cumint(1.0 / lam)
    u = -ax * (i1 - (i1[-1] / i0[-1]) * i0)
    T = Tc + (Th - Tc) * il / il[-1]
    yc = np.arange(ny) + 0.5
    return np.interp(yc, y, u), np.interp(yc, y, T)
