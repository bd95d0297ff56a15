"""ctypes binding of liblbe_csf.so (the C ABI in include/lbe_csf.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory (the workspace and all input and
output arrays are torch tensors) and the HIP stream.  Importing this module
raises if the library has not been built (``python -m
paper_1412_6238_amd.build``); there is no fallback path.

The functions keep the C names (``lbe_csf_create``, ``lbe_csf_step``, ...);
``Simulation`` bundles a handle with the tensors it borrows.  Two
``torch.autograd.Function`` wrappers differentiate a recorded run through
lbe_csf_backward: ``CSFDroplet`` (the droplet migration J, Sec. IV C) and
``LbeRun`` (the final order-parameter field).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbe_csf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1412_6238_amd.build` "
        "(hipcc, gfx950).  There is no fallback implementation.")

# torch is imported first so that the library binds to the HIP runtime torch
# already loaded (same soname): one runtime per process, shared device memory
# and streams.  Loading the library first would pull in a second copy.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

LBE_CSF_OK, LBE_CSF_EINVAL, LBE_CSF_ENOMEM, LBE_CSF_EDEVICE = 0, -1, -2, -3
LBE_CSF_ENOTRECORDED, LBE_CSF_ENONFINITE = -4, -5
LBE_CSF_FP64, LBE_CSF_FP32_DEV = 0, 1
PRECISIONS = {"fp64": LBE_CSF_FP64, "fp32_dev": LBE_CSF_FP32_DEV}

EXPORTED = ("lbe_csf_workspace_size", "lbe_csf_create", "lbe_csf_step", "lbe_csf_fields",
            "lbe_csf_diagnostics", "lbe_csf_diagnostics_noalloc", "lbe_csf_diag_history",
            "lbe_csf_get_state",
            "lbe_csf_set_state", "lbe_csf_step_count", "lbe_csf_backward", "lbe_csf_destroy",
            "lbe_csf_strerror", "lbe_csf_last_error")


class lbe_csf_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("walls_y", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("rho", ctypes.c_double), ("cv", ctypes.c_double),
        ("tau_f", ctypes.c_double * 2), ("tau_T", ctypes.c_double * 2),
        ("tau_g", ctypes.c_double), ("mobility", ctypes.c_double),
        ("width", ctypes.c_double), ("beta", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("sigmaT", ctypes.c_double), ("Tref", ctypes.c_double),
        ("force", ctypes.c_double * 2),
        ("p0", ctypes.c_double), ("T_shift", ctypes.c_double), ("T_grad", ctypes.c_double),
        ("diag_every", ctypes.c_int32), ("csf_form", ctypes.c_int32),
        ("rho2", ctypes.c_double),
    ]


class lbe_csf_diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("mass", ctypes.c_double), ("energy", ctypes.c_double),
        ("sum_cy", ctypes.c_double), ("sum_cx", ctypes.c_double),
        ("mass_thr", ctypes.c_double), ("sum_cuy_thr", ctypes.c_double),
        ("centroid_y", ctypes.c_double), ("u_r", ctypes.c_double),
        ("n_nonfinite", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
_P = ctypes.POINTER(lbe_csf_params)
_sig = {
    "lbe_csf_workspace_size": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "lbe_csf_create": (ctypes.c_int, [_P, _vp, ctypes.c_size_t, ctypes.c_int64, _vp, _vp, _vp,
                                      _vp, _vp, ctypes.POINTER(_vp)]),
    "lbe_csf_step": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int32]),
    "lbe_csf_fields": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "lbe_csf_diagnostics": (ctypes.c_int, [_vp, ctypes.POINTER(lbe_csf_diag)]),
    "lbe_csf_diagnostics_noalloc": (ctypes.c_int, [_vp, ctypes.POINTER(lbe_csf_diag)]),
    "lbe_csf_diag_history": (ctypes.c_int, [_vp, ctypes.POINTER(lbe_csf_diag), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32)]),
    "lbe_csf_get_state": (ctypes.c_int, [_vp, _vp]),
    "lbe_csf_set_state": (ctypes.c_int, [_vp, _vp]),
    "lbe_csf_step_count": (ctypes.c_int64, [_vp]),
    "lbe_csf_backward": (ctypes.c_int, [_vp, _vp, _dp, _vp, _vp, _vp]),
    "lbe_csf_destroy": (None, [_vp]),
    "lbe_csf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lbe_csf_last_error": (ctypes.c_char_p, [_vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype, _f.argtypes = _res, _args
    globals()[_name] = _f


class LbeCsfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lbe_csf_strerror(status).decode()} ({status}): {msg}")
        self.status = status


def _check(rc, handle=None):
    if rc != LBE_CSF_OK:
        raise LbeCsfError(rc, (lbe_csf_last_error(handle) or b"").decode())
    return rc


def make_params(p: dict, precision="fp64", diag_every=0) -> lbe_csf_params:
    """lbe_csf_params from a workload parameter dict."""
    P = lbe_csf_params()
    P.nx, P.ny = int(p["nx"]), int(p["ny"])
    P.walls_y = int(p.get("walls_y", 1))
    P.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    P.rho, P.cv = float(p["rho"]), float(p["cv"])
    P.tau_f[0], P.tau_f[1] = map(float, p["tau_f"])
    P.tau_T[0], P.tau_T[1] = map(float, p["tau_T"])
    P.tau_g, P.mobility = float(p["tau_g"]), float(p["mobility"])
    P.width, P.beta = float(p["width"]), float(p["beta"])
    P.sigma0, P.sigmaT, P.Tref = float(p["sigma0"]), float(p["sigmaT"]), float(p["Tref"])
    P.force[0], P.force[1] = map(float, p["force"])
    P.p0, P.T_shift = float(p["p0"]), float(p.get("T_shift", 0.0))
    P.T_grad = float(p.get("T_grad", 0.0))
    P.diag_every, P.csf_form = int(diag_every), int(p.get("csf_form", 0))
    P.rho2 = float(p.get("rho2", 0.0))
    return P


def workspace_bytes(params: lbe_csf_params, record_steps: int = 0) -> int:
    n = ctypes.c_size_t()
    _check(lbe_csf_workspace_size(ctypes.byref(params), int(record_steps), ctypes.byref(n)))
    return n.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Simulation:
    """A handle plus the torch tensors it borrows (workspace, outputs).

    Inputs may be numpy arrays or tensors; they are copied to the device as
    float64.  All work goes to ``stream`` (default: torch's current stream).
    """

    def __init__(self, params: dict, phi0, T0, Twall_bot=None, Twall_top=None,
                 precision="fp64", diag_every=0, record_steps=0, device="cuda:0",
                 stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.P = make_params(params, precision, diag_every)
        self.nx, self.ny = self.P.nx, self.P.ny
        self.record_steps = int(record_steps)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = workspace_bytes(self.P, self.record_steps)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        dev = lambda a: None if a is None else torch.as_tensor(
            np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a,
            dtype=torch.float64).to(self.device).contiguous()
        phi0_t, T0_t = dev(phi0), dev(T0)
        tb, tt = dev(Twall_bot), dev(Twall_top)
        assert phi0_t.shape == (self.ny, self.nx) and T0_t.shape == (self.ny, self.nx)
        h = ctypes.c_void_p()
        rc = lbe_csf_create(ctypes.byref(self.P), _ptr(self.workspace), nbytes,
                            self.record_steps, ctypes.c_void_p(self.stream.cuda_stream),
                            _ptr(phi0_t), _ptr(T0_t), _ptr(tb), _ptr(tt), ctypes.byref(h))
        _check(rc, None)
        self.h = h
        self._destroy = lbe_csf_destroy   # still reachable during interpreter shutdown
        # the init kernel reads these; keep them until the stream has run it
        self._keep = (phi0_t, T0_t, tb, tt)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self._destroy(h)
            self.h = None

    @property
    def step_count(self):
        return lbe_csf_step_count(self.h)

    def step(self, n=1, record=False):
        _check(lbe_csf_step(self.h, int(n), int(bool(record))), self.h)
        return self

    def fields(self, names=("phi", "ux", "uy", "p", "T")):
        torch = self.torch
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for k in names}
        _check(lbe_csf_fields(self.h, *[_ptr(out.get(k)) for k in ("phi", "ux", "uy", "p", "T")]),
               self.h)
        return out

    def diagnostics(self):
        d = lbe_csf_diag()
        _check(lbe_csf_diagnostics(self.h, ctypes.byref(d)), self.h)
        return d.as_dict()

    def diagnostics_noalloc(self):
        """lbe_csf_diagnostics_noalloc: the same values, scratch in the
        library's static device array."""
        d = lbe_csf_diag()
        _check(lbe_csf_diagnostics_noalloc(self.h, ctypes.byref(d)), self.h)
        return d.as_dict()

    def diag_history(self, max_records=4096):
        buf = (lbe_csf_diag * max_records)()
        cnt = ctypes.c_int32()
        _check(lbe_csf_diag_history(self.h, buf, max_records, ctypes.byref(cnt)), self.h)
        return [buf[k].as_dict() for k in range(cnt.value)]

    def get_state(self):
        F = self.torch.empty((27, self.ny, self.nx), dtype=self.torch.float64, device=self.device)
        _check(lbe_csf_get_state(self.h, _ptr(F)), self.h)
        return F

    def set_state(self, F):
        F = self.torch.as_tensor(F, dtype=self.torch.float64).to(self.device).contiguous()
        assert F.shape == (27, self.ny, self.nx)
        _check(lbe_csf_set_state(self.h, _ptr(F)), self.h)
        self._keep_state = F
        return self

    def backward(self, dJ_dc, want_F0=False, want_T0=True):
        """Adjoint of the recorded run: returns dict(sigmaT, Twall[2, nx], F0, T0)."""
        torch = self.torch
        seed = torch.as_tensor(dJ_dc, dtype=torch.float64).to(self.device).contiguous()
        assert seed.shape == (self.ny, self.nx)
        s = ctypes.c_double()
        tw = torch.zeros((2, self.nx), dtype=torch.float64, device=self.device)
        f0 = (torch.zeros((27, self.ny, self.nx), dtype=torch.float64, device=self.device)
              if want_F0 else None)
        t0 = (torch.zeros((self.ny, self.nx), dtype=torch.float64, device=self.device)
              if want_T0 else None)
        _check(lbe_csf_backward(self.h, _ptr(seed), ctypes.byref(s), _ptr(tw), _ptr(f0),
                                _ptr(t0)), self.h)
        return dict(sigmaT=s.value, Twall=tw, F0=f0, T0=t0)


class LbeRun(torch.autograd.Function):
    """phi_N of an N-step run as a differentiable function of sigmaT, the wall
    temperatures and the initial temperature field.

    Forward: one recorded run (sqrt(N)-spaced checkpoints) in the library.
    Backward: lbe_csf_backward with the seed dJ/dc = 2 dJ/dphi (phi = 2c - 1).
    ``apply(sigmaT, Twall_bot, Twall_top, T0, params, phi0, nsteps, precision)``;
    sigmaT is a 0-d tensor, Twall_* are (nx,) tensors (None with periodic y),
    T0 is (ny, nx).  The handle stays with the graph until backward has run.
    """

    @staticmethod
    def forward(ctx, sigmaT, Twall_bot, Twall_top, T0, params, phi0, nsteps, precision):
        p = dict(params)
        p["sigmaT"] = float(sigmaT.detach().cpu())
        nsteps = int(nsteps)
        sim = Simulation(p, phi0, T0.detach(), None if Twall_bot is None else Twall_bot.detach(),
                         None if Twall_top is None else Twall_top.detach(), precision=precision,
                         record_steps=nsteps, device=T0.device if T0.is_cuda else "cuda:0")
        sim.step(nsteps, record=True)
        phi = sim.fields(("phi",))["phi"]
        ctx.sim = sim
        ctx.has_walls = Twall_bot is not None
        ctx.sT_device = sigmaT.device
        return phi

    @staticmethod
    def backward(ctx, dphi):
        sim = ctx.sim
        g = sim.backward(2.0 * dphi.detach().to(torch.float64), want_F0=False, want_T0=True)
        ctx.sim = None
        dsT = torch.tensor(g["sigmaT"], dtype=torch.float64, device=ctx.sT_device)
        dtb = g["Twall"][0] if ctx.has_walls else None
        dtt = g["Twall"][1] if ctx.has_walls else None
        return dsT, dtb, dtt, g["T0"], None, None, None, None


class CSFDroplet(torch.autograd.Function):
    """Droplet migration J = y_c(N) - y_c(0) of an N-step run, y_c = sum c y /
    sum c the centroid of the order parameter (Sec. IV C, unthresholded so
    that J is differentiable), as a differentiable function of sigmaT, the
    wall temperatures and the initial temperature field.

    ``apply(sigmaT, Twall_bot, Twall_top, T0, params, phi0, nsteps, precision)``
    returns a 0-d FP64 tensor on the device of T0.  Forward: a recorded run in
    the library; the centroids are the library's FP64 diagnostics.  Backward:
    lbe_csf_backward with the seed dJ/dc_N = (y - y_c(N)) / sum c_N, giving
    dJ/dsigmaT, the direct wall derivatives and dJ/dT0.  When T0 is itself a
    function of the walls (a conduction profile computed with torch ops),
    autograd adds the path through T0 to the wall gradients.
    """

    @staticmethod
    def forward(ctx, sigmaT, Twall_bot, Twall_top, T0, params, phi0, nsteps, precision):
        p = dict(params)
        p["sigmaT"] = float(sigmaT.detach().cpu())
        nsteps = int(nsteps)
        dev = T0.device if T0.is_cuda else torch.device("cuda:0")
        sim = Simulation(p, phi0, T0.detach(), None if Twall_bot is None else Twall_bot.detach(),
                         None if Twall_top is None else Twall_top.detach(), precision=precision,
                         record_steps=nsteps, device=dev)
        y0 = sim.diagnostics()["centroid_y"]
        sim.step(nsteps, record=True)
        d = sim.diagnostics()
        ctx.sim, ctx.yN, ctx.mass = sim, d["centroid_y"], d["mass"]
        ctx.has_walls = Twall_bot is not None
        ctx.sT_device = sigmaT.device
        return torch.tensor(d["centroid_y"] - y0, dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, dJ):
        sim = ctx.sim
        y = torch.arange(sim.ny, dtype=torch.float64, device=sim.device)[:, None] + 0.5
        seed = ((y - ctx.yN) / ctx.mass).expand(sim.ny, sim.nx) * dJ.to(sim.device)
        # the seed carries the incoming gradient, so every output does too
        g = sim.backward(seed.contiguous(), want_F0=False, want_T0=True)
        ctx.sim = None
        dsT = torch.tensor(g["sigmaT"], dtype=torch.float64, device=ctx.sT_device)
        dtb = g["Twall"][0] if ctx.has_walls else None
        dtt = g["Twall"][1] if ctx.has_walls else None
        return dsT, dtb, dtt, g["T0"], None, None, None, None


def run_phi(params, phi0, T0, Twall_bot, Twall_top, nsteps, sigmaT, precision="fp32_dev"):
    """phi after nsteps steps, differentiable w.r.t. sigmaT, Twall_* and T0."""
    return LbeRun.apply(sigmaT, Twall_bot, Twall_top, T0, params, phi0, nsteps, precision)
