"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the FP64 oracle over every boundary rule on small and ragged grids, and the
GPU-free entry points of the C ABI (validation, sizes, the model, status
strings, NULL handling).  Each driver is built in a temporary folder and
must print "ok" with no sanitizer report."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _have(tool):
    return shutil.which(tool) is not None


def _run(cmd, cwd, timeout=600):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=timeout, env=ENV)
    assert r.returncode == 0, (cmd, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(not _have("gcc"), reason="gcc missing")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_driver")
        _run(["gcc", "-std=c11", "-O1", "-g", *SAN, "-Wno-unknown-pragmas",
              os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", exe], d)
        assert _run([exe], d).strip() == "ok"


@pytest.mark.skipif(not (_have("gcc") and _have("g++") and os.path.exists("/opt/rocm/bin/hipcc")),
                    reason="toolchain missing")
def test_abi_host_code_under_sanitizers():
    from paper_0908_3749_amd import _abi, build_lib
    if not os.path.exists(_abi.LIB_PATH):
        build_lib.build()
    libdir = os.path.dirname(_abi.LIB_PATH)
    with tempfile.TemporaryDirectory() as d:
        host = os.path.join(d, "host_san.o")
        # sanitizers on the host side only
        _run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-ffp-contract=off", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
              "-Wno-unused-command-line-argument", "-c",
              os.path.join(ROOT, "paper_0908_3749_amd", "csrc", "mrtfd_host.cpp"), "-o", host], d)
        drv = os.path.join(d, "drv.o")
        _run(["gcc", "-std=c11", "-O1", "-g", *SAN, "-c", os.path.join(HERE, "abi_driver.c"), "-o", drv], d)
        exe = os.path.join(d, "abi_driver")
        # the driver's entry points come from the sanitized object; the
        # kernel launchers it references from the built library
        _run(["g++", "-fsanitize=address,undefined", drv, host, f"-L{libdir}", "-lmrtfd",
              "-L/opt/rocm/lib", "-lamdhip64", f"-Wl,-rpath,{libdir}", "-Wl,-rpath,/opt/rocm/lib",
              "-o", exe], d)
        assert _run([exe], d).strip() == "ok"
