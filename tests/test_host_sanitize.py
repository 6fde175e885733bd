"""The setup's host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU: the
library's sources built with the sanitizers on their host side (tests/sanitize/host_check.cpp
drives the host stages: element order, geometry and interpolation factors, the exact polynomial
potentials by Green's identity with host threads, the interpolation solves, and the sparsifying
preconditioner's stencils, threaded block LU and host sweeps).  Any sanitizer report fails the
run.  The build is kept under _build/ and redone when a source changes."""
import hashlib
import os
import subprocess

import numpy as np
import pytest

import paper_2608_17615_amd as lsg
from workloads import problems as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_17615_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_check.cpp")
OUT = os.path.join(ROOT, "_build", "sanitize")


def _build():
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    hdrs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h"))
    h = hashlib.sha256()
    for f in [DRIVER, *srcs, *hdrs, os.path.join(ROOT, "include", "ls.h")]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    exe = os.path.join(OUT, "host_check_" + h.hexdigest()[:16])
    if os.path.exists(exe):
        return exe
    os.makedirs(OUT, exist_ok=True)
    # the sanitizers on the host side only (each -fsanitize= after -Xarch_host)
    cmd = ["/opt/rocm/bin/hipcc", "-std=c++17", "-O1", "-g", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, DRIVER, "-x", "hip", *srcs, "-o", exe + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    os.replace(exe + ".tmp", exe)
    return exe


def _write(prob, path):
    sc = lsg.Scatterer.from_mesh(prob.mesh, prob.m, prob.k)
    n = int(np.asarray(sc.x).size)
    kinds = {"circle": lsg.CIRCLE, "ellipse": lsg.ELLIPSE}
    with open(path, "wb") as f:
        np.array([n], np.int64).tofile(f)
        np.array([n // 10, len(sc.curves)], np.int32).tofile(f)
        np.array([sc.k], np.float64).tofile(f)
        for a in (sc.x, sc.y, sc.w):
            np.ascontiguousarray(a, np.float64).tofile(f)
        np.ascontiguousarray(np.asarray(sc.m, np.complex128)).view(np.float64).tofile(f)
        np.ascontiguousarray(sc.elem_subdomain, np.int32).tofile(f)
        for c in sc.curves:
            kind = c.kind if isinstance(c.kind, int) else kinds[c.kind]
            np.array([kind, int(c.orientation), int(c.subdomain), 0], np.int32).tofile(f)
            np.array([c.cx, c.cy, c.a, c.b], np.float64).tofile(f)


@pytest.mark.parametrize("name", ["disk", "two-material"])
def test_setup_host_code_is_clean_under_asan_and_ubsan(name, tmp_path):
    exe = _build()
    prob = P.disk_problem(3, 6.0, 2.0) if name == "disk" else P.graded_two_material(2, 8.0)
    path = str(tmp_path / "scatterer.bin")
    _write(prob, path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, path, "4"], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout.strip())
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "host_check:" in r.stdout
