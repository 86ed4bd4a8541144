"""AddressSanitizer + UndefinedBehaviorSanitizer runs on the CPU (no GPU).

tests/sanitize_driver.c runs every oracle routine on small inputs (degenerate shapes
included) and, linked with the library's entry-point sources (wf_api.hip, tri.hip), the
argument checks of every entry point of include/wf.h and include/tri.h on invalid
arguments.  The sanitizers instrument host code only (device code is not instrumented); the
sweep kernels' launchers are replaced by stubs (tests/sanitize_stubs.hip), since no call
here reaches a kernel.  A sanitizer report or a wrong return code fails the test.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]
ORACLE = [os.path.join(ROOT, "oracle", f) for f in ("wf_oracle.c", "tridiag.c", "softmin.c")]
LIB = [os.path.join(ROOT, "paper_2510_27351_amd", "csrc", f + ".hip") for f in ("wf_api", "tri")]
LIB.append(os.path.join(HERE, "sanitize_stubs.hip"))
DRIVER = os.path.join(HERE, "sanitize_driver.c")


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-4000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "drv")
    _run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", DRIVER, *ORACLE, "-lm", "-o", exe])
    out = _run([exe])
    assert "sanitized run ok" in out


def test_library_argument_checks_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    objs = []
    procs = []
    for src in LIB:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        procs.append(subprocess.Popen([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", *SAN,
                                       "-c", src, "-o", obj], stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out.decode()[-4000:]
    for src in [DRIVER, *ORACLE]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, "-O1", "-g", "-x", "c", "-std=c11", "-ffp-contract=off", "-DWITH_LIB", *SAN, "-c", src,
              "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "drvlib")
    _run([HIPCC, *SAN, "--offload-arch=gfx950", *objs, "-lm", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    out = _run([exe], env=env, timeout=120)
    assert "sanitized run ok" in out
