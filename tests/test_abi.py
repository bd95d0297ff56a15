"""Host-side checks of liblbe_csf.so: it loads, exports every function the
header declares, and rejects bad arguments before touching a device.
No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbe_csf.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"LBE_CSF_API\s+[\w\s\*]*?\b(lbe_csf_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def binding():
    from paper_1412_6238_amd import lbe_csf
    return lbe_csf


def test_every_declared_symbol_is_exported(binding):
    names = _declared()
    assert len(names) == 14, names
    lib = ctypes.CDLL(binding.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(binding.EXPORTED) == names


def test_struct_layouts_match_header(binding, tmp_path):
    """ctypes mirrors of the two structs match the C compiler's layout."""
    import subprocess
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbe_csf.h"', "int main(void){"]
    for cname, py in (("lbe_csf_params", binding.lbe_csf_params), ("lbe_csf_diag", binding.lbe_csf_diag)):
        prog.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            prog.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    prog.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for cname, py in (("lbe_csf_params", binding.lbe_csf_params), ("lbe_csf_diag", binding.lbe_csf_diag)):
        assert got[(cname, "size")] == ctypes.sizeof(py)
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_workspace_size_and_validation(binding):
    from paper_1412_6238_amd import workloads as wl
    p = wl.make("planar_marangoni")["params"]
    P64 = binding.make_params(p, "fp64")
    P32 = binding.make_params(p, "fp32_dev")
    n64, n32 = binding.workspace_bytes(P64), binding.workspace_bytes(P32)
    n = p["nx"] * p["ny"]
    # a state: 25 planes of the storage type, then g_0 in FP64 and hbar_0 in
    # the storage type (FP64, or the FP32 deviation)
    s64, s32 = 25 * n * 8 + 16 * n, 25 * n * 4 + 12 * n
    assert n64 >= 2 * s64 and n32 >= 2 * s32
    # the same bookkeeping regions but for the diagnostic partials, 7 FP64
    # sums per block of the step launch, whose block count depends on each
    # form's launch shape (planar 256 x 128: 128 blocks in FP64, 256 in FP32)
    d = (n64 - 2 * s64) - (n32 - 2 * s32)
    assert d % 8 == 0 and abs(d) <= 7 * 8 * n
    rec = binding.workspace_bytes(P32, 4000)
    # sqrt(N) checkpoints (63) + one replayed segment (64) + 2 adjoint states
    # (27 planes of FP32 each)
    assert rec - n32 >= (63 + 64) * s32 + 2 * 27 * n * 4
    for bad in (dict(nx=2), dict(tau_f=(0.5, 1.0)), dict(tau_T=(1.0, 0.4)), dict(tau_g=0.5),
                dict(mobility=0.0), dict(width=-1.0), dict(beta=0.0), dict(rho=0.0),
                dict(sigmaT=float("nan"))):
        Pb = binding.make_params(dict(p, **bad), "fp64")
        with pytest.raises(binding.LbeCsfError) as e:
            binding.workspace_bytes(Pb)
        assert e.value.status == binding.LBE_CSF_EINVAL
    Pb = binding.make_params(p, 7)
    with pytest.raises(binding.LbeCsfError):
        binding.workspace_bytes(Pb)


def test_create_rejects_before_device_work(binding):
    """Argument errors are detected on the host: small workspace -> ENOMEM,
    misaligned workspace / NULL inputs -> EINVAL (fake pointers are never
    dereferenced on these paths)."""
    from paper_1412_6238_amd import workloads as wl
    p = wl.make("poiseuille")["params"]
    P = binding.make_params(p, "fp64")
    need = binding.workspace_bytes(P)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)
    rc = binding.lbe_csf_create(ctypes.byref(P), fake, need - 1, 0, None, fake, fake, fake, fake,
                                ctypes.byref(h))
    assert rc == binding.LBE_CSF_ENOMEM and not h.value
    assert b"workspace too small" in binding.lbe_csf_last_error(None)
    rc = binding.lbe_csf_create(ctypes.byref(P), ctypes.c_void_p((1 << 20) + 8), need, 0, None,
                                fake, fake, fake, fake, ctypes.byref(h))
    assert rc == binding.LBE_CSF_EINVAL
    rc = binding.lbe_csf_create(ctypes.byref(P), fake, need, 0, None, None, fake, fake, fake,
                                ctypes.byref(h))
    assert rc == binding.LBE_CSF_EINVAL
    rc = binding.lbe_csf_create(ctypes.byref(P), fake, need, 0, None, fake, fake, None, None,
                                ctypes.byref(h))
    assert rc == binding.LBE_CSF_EINVAL       # walls need wall temperatures
    for s in range(-5, 1):
        assert binding.lbe_csf_strerror(s)


def test_force_form_and_density_parameters(binding):
    """csf_form must be 0 or 1; rho2 >= 0 (0: one density); two densities
    add one FP64 plane (the pressure of Eq. 9) to the workspace in either
    form; a grid whose state would pass 4 GiB is refused, and so is a linear
    thermal reference (T_grad) in the FP32 form with periodic y."""
    from paper_1412_6238_amd import workloads as wl
    p = wl.make("planar_marangoni")["params"]
    n = p["nx"] * p["ny"]
    base = binding.workspace_bytes(binding.make_params(p, "fp64"))
    assert binding.workspace_bytes(binding.make_params(dict(p, csf_form=1), "fp64")) == base
    assert binding.workspace_bytes(binding.make_params(dict(p, rho2=p["rho"]), "fp64")) == base
    two = binding.workspace_bytes(binding.make_params(dict(p, rho2=2.0), "fp64"))
    assert two - base == (n * 8 + 255) // 256 * 256
    base32 = binding.workspace_bytes(binding.make_params(p, "fp32_dev"))
    two32 = binding.workspace_bytes(binding.make_params(dict(p, rho2=2.0), "fp32_dev"))
    assert two32 - base32 == (n * 8 + 255) // 256 * 256
    for bad, prec in ((dict(csf_form=2), "fp64"), (dict(csf_form=-1), "fp32_dev"),
                      (dict(rho2=-1.0), "fp64"), (dict(rho2=float("inf")), "fp64"),
                      (dict(nx=8192, ny=8192), "fp32_dev"),
                      (dict(walls_y=0, T_grad=0.01), "fp32_dev"),
                      (dict(nx=4096, ny=8192), "fp64")):
        with pytest.raises(binding.LbeCsfError) as e:
            binding.workspace_bytes(binding.make_params(dict(p, **bad), prec))
        assert e.value.status == binding.LBE_CSF_EINVAL, bad
    # the largest FP32 state below 4 GiB is accepted
    binding.workspace_bytes(binding.make_params(dict(p, nx=6000, ny=6000), "fp32_dev"))
