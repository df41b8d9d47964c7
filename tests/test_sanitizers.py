"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the oracle (g++) driven through every code path on small seeded graphs, and
the GPU library's host code (hipcc, sanitizers on the host pass only) driven
through its planning, partial-order checks, exact standard error, batch
options and argument checks.  A sanitizer finding aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    run(["g++", "-std=c++17", "-O1", "-g"] + SAN + ["-I" + os.path.join(ROOT, "oracle"),
        os.path.join(ROOT, "tests", "sanitize", "oracle_driver.cpp"), os.path.join(ROOT, "oracle", "oracle.cpp"),
        os.path.join(ROOT, "oracle", "brute.cpp"), "-o", exe])
    r = run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert "oracle driver ok" in r.stdout


def test_library_host_code_under_sanitizers(tmp_path):
    objdir = os.path.join(ROOT, "_build", "timest")
    kernels = [os.path.join(objdir, f + ".o") for f in ("csr.hip", "weights.hip", "sample.hip", "scan.hip")]
    if shutil.which("hipcc") is None or not all(os.path.exists(k) for k in kernels):
        pytest.skip("needs hipcc and the library's kernel objects (run the build first)")
    inc = "-I" + os.path.join(ROOT, "include")
    drv = str(tmp_path / "host_driver.o")
    run(["g++", "-std=c++17", "-O1", "-g"] + SAN + [inc, "-c",
        os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", drv])
    host = []
    for f in ("api.cpp", "mem.cpp", "serve.cpp"):
        o = str(tmp_path / (f + ".o"))
        run(["hipcc", "-x", "hip", "-c", os.path.join(ROOT, "paper_2507_20441_amd", "csrc", f), "-o", o, "-O1", "-g",
             "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", inc, "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all"])
        host.append(o)
    exe = str(tmp_path / "host_san")
    run(["hipcc", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
         "-fsanitize=undefined", drv] + host + kernels + ["-o", exe])
    # the HIP runtime's own allocations at exit are not this code's: no leak check
    r = run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1"))
    assert "host driver ok" in r.stdout
