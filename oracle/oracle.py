"""ctypes front end of the FP64 CPU oracle (``liblbe_oracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product package.  The
oracle shares no code with the HIP library; this wrapper marshals arguments
and nothing else (all arithmetic lives in ``lbe_oracle.c``).

Parameters are the same plain dict the workload generator returns (keys
``nx ny walls_y rho cv tau_f tau_T tau_g mobility width beta sigma0 sigmaT
Tref force p0``); the oracle derives eps, alpha, kcap and Gamma itself.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbe_oracle.so")
SRC_PATH = os.path.join(_HERE, "lbe_oracle.c")

N_DIAG = 7
DIAG_KEYS = ("mass", "energy", "sum_cy", "sum_cx", "mass_thr", "sum_cuy_thr",
             "n_nonfinite")
INTERMEDIATE_KEYS = ("c", "T", "p", "jx", "jy", "gcx", "gcy", "lapc", "gTx",
                     "gTy", "gpx", "gpy", "mu", "Fx", "Fy", "ux", "uy", "hxx",
                     "hxy", "hyy")


class _Params(ctypes.Structure):
    _fields_ = [
        ("NX", ctypes.c_int32), ("NY", ctypes.c_int32),
        ("x0", ctypes.c_int32), ("y0", ctypes.c_int32),
        ("wx", ctypes.c_int32), ("wy", ctypes.c_int32),
        ("walls_y", ctypes.c_int32), ("csf_form", ctypes.c_int32),
        ("rho", ctypes.c_double), ("cv", ctypes.c_double),
        ("tau_f", ctypes.c_double * 2), ("tau_T", ctypes.c_double * 2),
        ("tau_g", ctypes.c_double), ("mobility", ctypes.c_double),
        ("width", ctypes.c_double), ("beta", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("sigmaT", ctypes.c_double),
        ("Tref", ctypes.c_double), ("force", ctypes.c_double * 2),
        ("p0", ctypes.c_double), ("rho2", ctypes.c_double),
    ]


# Builds of the one source.  "" is the oracle (-ffp-contract=off: every
# product and sum rounded as written).  "fma" lets the compiler fuse
# multiply-adds and "rev" sums over the lattice directions in reverse order:
# the same arithmetic with different rounding.  The tests use them only to
# measure how far two correct FP64 evaluations drift apart on an
# ill-conditioned case (the round-off floor of a comparison).
VARIANTS = {"": ["-ffp-contract=off"], "fma": ["-ffp-contract=fast", "-mfma"],
            "rev": ["-ffp-contract=off", "-DORC_REVERSED_SUMS"],
            # the oracle itself under AddressSanitizer and UndefinedBehaviorSanitizer
            # (tests/test_sanitizers.py loads it with the ASan runtime preloaded)
            "asan": ["-ffp-contract=off", "-g", "-fno-omit-frame-pointer",
                     "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]}


def lib_path(variant: str = "") -> str:
    return LIB_PATH if not variant else os.path.join(_HERE, f"liblbe_oracle_{variant}.so")


def build(verbose: bool = False, extra=(), variant: str = "") -> str:
    """Compile the oracle with gcc (-O2, OpenMP; -ffp-contract=off for the
    oracle itself)."""
    import subprocess
    out = lib_path(variant)
    # written beside the library and renamed into place, so that processes
    # that have the previous build loaded keep a consistent file
    tmp = f"{out}.tmp{os.getpid()}"
    cmd = ["gcc", "-O2", *VARIANTS[variant], "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", *extra, "-o", tmp, SRC_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


_libs = {}


def lib(variant: str = ""):
    if variant not in _libs:
        path = lib_path(variant)
        if not os.path.exists(path) or (os.path.getmtime(path) < os.path.getmtime(SRC_PATH)):
            build(variant=variant)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(_Params), dp, dp]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_init.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_set_state.argtypes = [ctypes.c_void_p, dp]
        L.orc_get_state.argtypes = [ctypes.c_void_p, dp]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp]
        L.orc_intermediates.argtypes = [ctypes.c_void_p, dp]
        L.orc_diag.argtypes = [ctypes.c_void_p, dp]
        L.orc_collide_site.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp]
        L.orc_derived.argtypes = [ctypes.POINTER(_Params), dp]
        L.orc_sizeof_params.restype = ctypes.c_int
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        assert L.orc_sizeof_params() == ctypes.sizeof(_Params)
        _libs[variant] = L
    return _libs[variant]


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _make_params(p: dict, window=None) -> _Params:
    nx, ny = int(p["nx"]), int(p["ny"])
    x0, y0, wx, wy = window if window is not None else (0, 0, nx, ny)
    P = _Params()
    P.NX, P.NY, P.x0, P.y0, P.wx, P.wy = nx, ny, x0, y0, wx, wy
    P.walls_y = int(p.get("walls_y", 1))
    P.csf_form = int(p.get("csf_form", 0))
    P.rho, P.cv = float(p["rho"]), float(p["cv"])
    P.tau_f[0], P.tau_f[1] = map(float, p["tau_f"])
    P.tau_T[0], P.tau_T[1] = map(float, p["tau_T"])
    P.tau_g, P.mobility = float(p["tau_g"]), float(p["mobility"])
    P.width, P.beta = float(p["width"]), float(p["beta"])
    P.sigma0, P.sigmaT, P.Tref = (float(p["sigma0"]), float(p["sigmaT"]),
                                  float(p["Tref"]))
    P.force[0], P.force[1] = map(float, p["force"])
    P.p0 = float(p["p0"])
    P.rho2 = float(p.get("rho2", p["rho"]))
    return P


def threads() -> int:
    """OpenMP threads the oracle's passes run on."""
    return int(lib().orc_threads())


class thread_limit:
    """Context manager: run the oracle's passes on n threads (None: leave
    the count as it is); the previous count is restored on exit."""

    def __init__(self, n=None):
        self.n = n

    def __enter__(self):
        self.prev = threads()
        if self.n is not None:
            lib().orc_set_threads(int(self.n))
        return self

    def __exit__(self, *exc):
        lib().orc_set_threads(self.prev)
        return False


def derived(p: dict, variant: str = "") -> dict:
    out = np.zeros(4)
    lib(variant).orc_derived(ctypes.byref(_make_params(p)), _ptr(out))
    return dict(eps=out[0], alpha=out[1], kcap=out[2], Gamma=out[3])


def collide_site(p: dict, pre27, stencil, variant: str = ""):
    """Single-site collision: returns (post[27], aux dict).  ``stencil`` holds
    (gcx, gcy, lapc, gTx, gTy, gpx, gpy) and optionally the Hessian of c
    (hxx, hxy, hyy), which only the curvature form reads (zeros if absent)."""
    pre = np.ascontiguousarray(pre27, dtype=np.float64)
    st = np.zeros(10)
    st[:len(stencil)] = np.asarray(stencil, dtype=np.float64)
    out = np.zeros(27)
    aux = np.zeros(11)
    lib(variant).orc_collide_site(ctypes.byref(_make_params(p)), _ptr(pre), _ptr(st),
                           _ptr(out), _ptr(aux))
    keys = ("c", "T", "p", "mu", "Fx", "Fy", "ux", "uy", "wf", "wT", "wg")
    return out, dict(zip(keys, aux))


class Oracle:
    """A grid (or a window of one) advanced by the plain FP64 oracle.

    ``variant="fma"`` runs the build with fused multiply-adds (for round-off
floors only).  ``window=(x0, y0, wx, wy)`` holds only that part of the global domain;
    values whose dependence leaves the window come out as NaN.  Field arrays
    are (wy, wx) float64, x fastest.  The state is (27, wy, wx): f, g, hbar.
    """

    def __init__(self, params: dict, Twall_bot=None, Twall_top=None,
                 window=None, variant: str = ""):
        self.params = dict(params)
        self._lib = lib(variant)
        self.P = _make_params(params, window)
        self.wx, self.wy = self.P.wx, self.P.wy
        nx = self.P.NX
        tb = np.ascontiguousarray(
            np.zeros(nx) if Twall_bot is None else Twall_bot, dtype=np.float64)
        tt = np.ascontiguousarray(
            np.zeros(nx) if Twall_top is None else Twall_top, dtype=np.float64)
        assert tb.shape == (nx,) and tt.shape == (nx,)
        self._h = self._lib.orc_create(ctypes.byref(self.P), _ptr(tb), _ptr(tt))
        if not self._h:
            raise ValueError("oracle: invalid grid")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def _field(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape == (self.wy, self.wx), a.shape
        return a

    def init(self, phi0, T0):
        self._lib.orc_init(self._h, _ptr(self._field(phi0)), _ptr(self._field(T0)))
        return self

    def set_state(self, F):
        F = np.ascontiguousarray(F, dtype=np.float64)
        assert F.shape == (27, self.wy, self.wx)
        self._lib.orc_set_state(self._h, _ptr(F))
        return self

    def state(self):
        F = np.zeros((27, self.wy, self.wx))
        self._lib.orc_get_state(self._h, _ptr(F))
        return F

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, int(n))
        return self

    def fields(self):
        out = [np.zeros((self.wy, self.wx)) for _ in range(5)]
        self._lib.orc_fields(self._h, *[_ptr(a) for a in out])
        return dict(zip(("phi", "ux", "uy", "p", "T"), out))

    def intermediates(self):
        out = np.zeros((len(INTERMEDIATE_KEYS), self.wy, self.wx))
        self._lib.orc_intermediates(self._h, _ptr(out))
        return dict(zip(INTERMEDIATE_KEYS, out))

    def diag(self):
        d = np.zeros(N_DIAG)
        self._lib.orc_diag(self._h, _ptr(d))
        out = dict(zip(DIAG_KEYS, d))
        out["n_nonfinite"] = int(out["n_nonfinite"])
        out["centroid_y"] = out["sum_cy"] / out["mass"] if out["mass"] else float("nan")
        out["u_r"] = (out["sum_cuy_thr"] / out["mass_thr"]
                      if out["mass_thr"] else float("nan"))
        return out
