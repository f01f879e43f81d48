"""CPU-side hardening: the oracle and the host runtime code of libqtm (circuit
validation, planner, program encoding, specialised-kernel source generation,
uneven-batch schedule) built with AddressSanitizer and
UndefinedBehaviorSanitizer and driven through their entry points.  Only host
code is built here (gcc / g++, no device code)."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HERE = Path(__file__).resolve().parent / "sanitize"
CSRC = ROOT / "paper_2404_06314_amd" / "csrc"
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(map(str, cmd[:3]))} ...: rc {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-6000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_driver"
    run(["gcc", "-std=c11", *SAN, "-fopenmp", "-fcx-limited-range", str(HERE / "oracle_driver.c"),
         str(ROOT / "oracle" / "qtm_oracle.c"), "-lm", "-o", str(exe)])
    r = run([str(exe)], env=ENV, timeout=300)
    assert "oracle driver ok" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not Path("/opt/rocm/lib/libamdhip64.so").exists(),
                    reason="needs g++ and the HIP runtime library to link against")
def test_host_runtime_under_sanitizers(tmp_path):
    from paper_2404_06314_amd import build as qb
    qb.write_jit_headers(tmp_path)
    exe = tmp_path / "host_driver"
    run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{ROOT / 'include'}",
         f"-I{CSRC}", f"-I{tmp_path}", str(HERE / "host_driver.cpp"), str(CSRC / "circuit.cpp"),
         str(CSRC / "schedule.cpp"), str(CSRC / "jit.cpp"), "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib",
         "-lamdhip64", "-ldl", "-lpthread", "-o", str(exe)])
    r = run([str(exe)], env=ENV, timeout=300)
    assert "host driver ok" in r.stdout
