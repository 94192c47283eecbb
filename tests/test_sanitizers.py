"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code.

* The CPU oracle's C part, built with gcc and both sanitizers, runs a driver
  that checks it against naive loops on small and degenerate inputs.
* The host side of libqbsm's C ABI: every source compiled with the
  sanitizers on the host pass only (the device code is built normally and
  never runs here: there is no GPU), linked with a C driver that exercises
  argument validation, status mapping, handle lifetimes and the error path of
  a failing allocator.

Both builds go to a scratch directory; a sanitizer report fails the test
through the driver's exit status (halt_on_error, no recovery).
"""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout[-3000:]}\n{res.stderr[-3000:]}"
    return res


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("sanitize"))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_c_under_asan_ubsan(workdir):
    exe = os.path.join(workdir, "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(ROOT, "oracle", "qbsm_oracle.c"), os.path.join(HERE, "oracle_driver.c"),
          "-o", exe, "-lm"])
    res = _run([exe], env=ENV)
    assert "oracle driver ok" in res.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_abi_host_side_under_asan_ubsan(workdir):
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2011_11762_amd", "csrc", "*.hip")))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
             "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

    def compile_one(src):
        obj = os.path.join(workdir, os.path.basename(src) + ".o")
        _run([HIPCC, *flags, "-c", src, "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv_o = os.path.join(workdir, "abi_host_driver.o")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-c", os.path.join(HERE, "abi_host_driver.c"), "-o", drv_o])
    exe = os.path.join(workdir, "abi_host_driver")
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address,undefined", drv_o, *objs,
          "-o", exe])
    res = _run([exe], env=ENV)
    assert "abi host driver ok" in res.stdout
