"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The host runtime of the library (sst_host.cpp, with host stand-ins for the
device launchers) and the float64 oracle (sst_oracle.c) are compiled by a plain
host compiler with -fsanitize=address,undefined and run through their host
paths: plans of every size and tier, invalid parameters, batches, the tuning
cache; the oracle's whole pipeline and its mirror ABI on a small signal.  Any sanitizer report
fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang++"
CC = "/opt/rocm/llvm/bin/clang"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
ENV.pop("LD_PRELOAD", None)


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    assert r.returncode == 0, (cmd[0], r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not installed")
def test_host_runtime_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    _run([CLANG, "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
          "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2003_07065_amd", "csrc"),
          os.path.join(ROOT, "paper_2003_07065_amd", "csrc", "sst_host.cpp"),
          os.path.join(HERE, "host_stubs.cpp"), os.path.join(HERE, "host_driver.cpp"),
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe, str(tmp_path / "tune.json")], env=ENV)
    assert "0 failure(s)" in r.stdout


@pytest.mark.skipif(not os.path.exists(CC), reason="ROCm clang not installed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run([CC, "-std=c11", "-D_GNU_SOURCE", *SAN, "-I" + os.path.join(ROOT, "oracle"),
          os.path.join(ROOT, "oracle", "sst_oracle.c"), os.path.join(ROOT, "oracle", "sst_oracle_abi.c"),
          os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV)
    assert "synthesis max err" in r.stdout
    assert "mirror ABI ok" in r.stdout
