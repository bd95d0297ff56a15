"""CPU checks under AddressSanitizer and UndefinedBehaviorSanitizer.

* The library's host-side logic (host_layout.h: state sizes, workspace
  layout, launch shapes, parameter checks) built into a C++ driver with
  -fsanitize=address,undefined and run over about a million parameter cases
  (tests/host_layout_check.cpp).
* The oracle (oracle/lbe_oracle.c) built with the same sanitizers and
  driven through every entry point -- walls and periodic y, both capillary
  forms, two densities, a window with undefined edges, single-site
  collisions, state get/set, intermediates and diagnostics -- in a child
  process with the ASan runtime preloaded (Python itself is not
  instrumented).  Any sanitizer report aborts the child.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_lib(name):
    return subprocess.check_output(["gcc", f"-print-file-name={name}"]).decode().strip()


def test_host_layout_under_sanitizers(tmp_path):
    exe = tmp_path / "host_layout_check"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1412_6238_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host_layout_check.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.startswith("ok ") and int(r.stdout.split()[1]) > 100000


_ORACLE_RUN = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
from oracle import oracle
from paper_1412_6238_amd import workloads as wl
V = "asan"
for walls, form, rho2 in ((1, 0, 0.0), (0, 1, 0.0), (1, 1, 2.0), (1, 0, 0.5)):
    case = wl.random_case(23, 17, seed=3 + walls + form, walls_y=walls, csf_form=form,
                          **({{"rho2": rho2}} if rho2 else {{}}))
    p = case["params"]
    o = oracle.Oracle(p, case["Twall_bot"], case["Twall_top"], variant=V)
    o.init(case["phi0"], case["T0"]).step(3)
    f, st, d = o.fields(), o.state(), o.diag()
    im = o.intermediates()
    o.set_state(st).step(1)
    assert all(np.isfinite(v).all() for v in f.values()), (walls, form, rho2)
    x0, y0, wx, wy = 3, 1, 17, 15
    win = oracle.Oracle(p, case["Twall_bot"], case["Twall_top"], window=(x0, y0, wx, wy),
                        variant=V)
    win.init(np.ascontiguousarray(case["phi0"][y0:y0 + wy, x0:x0 + wx]),
             np.ascontiguousarray(case["T0"][y0:y0 + wy, x0:x0 + wx])).step(2)
    wf = win.fields()
    assert np.isfinite(wf["phi"][7, 8]) and np.isnan(wf["phi"][0, 0])
    rng = np.random.default_rng(1)
    post, aux = oracle.collide_site(p, 0.1 + 0.01 * rng.random(27), rng.random(10) * 1e-3,
                                    variant=V)
    assert np.isfinite(post).all()
    oracle.derived(p, variant=V)
print("oracle under sanitizers ok", flush=True)
"""


def test_oracle_under_sanitizers():
    from oracle import oracle
    oracle.build(variant="asan")
    env = dict(os.environ, LD_PRELOAD=_gcc_lib("libasan.so"),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", _ORACLE_RUN.format(root=ROOT)],
                       capture_output=True, text=True, timeout=600, env=env, cwd=ROOT)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "oracle under sanitizers ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
