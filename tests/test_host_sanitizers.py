"""The host half of libsrp under AddressSanitizer and UndefinedBehaviorSanitizer.

plan.cpp (geometry, eigensolvers, SLRI/SSPI fits, window selection) and
api.cpp (argument checks, exports) are compiled with g++ and the sanitizers,
linked with host-only stand-ins for the device entry points
(tests/native/device_stubs.cpp) and driven through the C ABI with host-only
plans on four geometries (tests/native/host_plan_driver.cpp).  Any sanitizer
report, unexpected status or non-finite export fails the test.  The driver's
export sums are then compared with the same plans built by the hipcc library,
so the sanitized code is the code that ships.
"""

import math
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_08514_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


@pytest.fixture(scope="module")
def driver_output(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("asan") / "host_plan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"),
           os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "api.cpp"),
           os.path.join(NATIVE, "device_stubs.cpp"), os.path.join(NATIVE, "host_plan_driver.cpp"),
           "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    return r.returncode, out


def test_host_plan_code_is_clean_under_asan_and_ubsan(driver_output):
    rc, out = driver_output
    assert "AddressSanitizer" not in out, out[-6000:]
    assert "runtime error" not in out, out[-6000:]
    assert "LeakSanitizer" not in out, out[-6000:]
    assert rc == 0, out[-6000:]
    assert "failures 0" in out
    # every planned case ran
    assert len(re.findall(r"^case ", out, re.M)) >= 30


def _driver_geometry(name):
    """The geometries host_plan_driver.cpp builds, in the same order."""
    def circle(M, radius, z):
        a = 2.0 * math.pi * np.arange(M) / M
        return np.stack([radius * np.cos(a), radius * np.sin(a), np.full(M, z)], axis=1)

    def box(nx, ny, nz, x0, x1, y0, y1, z0, z1):
        pts = []
        for i in range(nx):
            for j in range(ny):
                for k in range(nz):
                    pts.append([x0 + (x1 - x0) * i / (nx - 1) if nx > 1 else x0,
                                y0 + (y1 - y0) * j / (ny - 1) if ny > 1 else y0,
                                z0 + (z1 - z0) * k / (nz - 1) if nz > 1 else z0])
        return np.array(pts)

    if name == "uca8":
        return circle(8, 0.15, 1.2), box(12, 12, 6, 0.0, 5.0, 0.0, 5.0, 0.0, 2.5), 1024
    if name == "square4":
        return circle(4, 0.1 * math.sqrt(2.0), 0.0), box(30, 30, 1, -1.5, 1.5, -1.5, 1.5, 1.0, 1.0), 512
    raise KeyError(name)


@pytest.mark.parametrize("case", [("uca8", "slri8", "slri", 8, False, "bf16"),
                                  ("uca8", "sspi4", "sspi", 4, False, "bf16"),
                                  ("uca8", "sspi_global3", "sspi", 3, True, "bf16"),
                                  ("square4", "slri_global20", "slri", 20, True, "f32")])
def test_sanitized_build_computes_the_shipped_plans(driver_output, case):
    from paper_2306_08514_amd import native
    try:
        native.lib()
    except Exception as e:  # the library is built by build(); without it only the sanitizer run counts
        pytest.skip(f"libsrp not built: {e}")
    geo, label, variant, rq, glob, dt = case
    _, out = driver_output
    line = next(ln for ln in out.splitlines() if ln.startswith(f"case {geo}/{label} "))
    sums = {k: float(v) for k, v in re.findall(r"(\w+)=([-0-9.e+]+)", line)
            if k not in ("P", "K", "PN", "max_np", "rq", "macs")}
    mics, grid, N = _driver_geometry(geo)
    kw = {"global_fit": True} if glob else {}
    p = native.Plan(mics, grid, 16000.0, N, variant, rq, dtype=dt, device=-1, **kw)
    for what, s in sums.items():
        got = float(np.abs(p.export(what).astype(np.float64)).sum())
        assert got == pytest.approx(s, rel=1e-9, abs=1e-9), (geo, label, what)
    p.close()
