"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code.

* The FP64 oracle (oracle/lbmref.c), built with gcc and both sanitizers,
  driven through every option on tiny lattices (tests/sanitize/oracle_driver.c).
* The host side of the C-ABI library (validation, node classification, wall,
  ghost and sub-voxel tables, tile tables, arena layout, the server's entry
  points), built host-only with the sanitizers on its host code and with the
  kernel launchers replaced by stand-ins that report no device
  (tests/sanitize/launch_stubs.cpp), driven through lbm_footprint and
  lbm_create on valid and invalid lattices (tests/sanitize/host_driver.c).
  Without a GPU lbm_create stops at its first device call after the layout.

A sanitizer report or a non-zero exit fails the test.  CPU only.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2512_01032_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    print(r.stdout[-3000:])
    print(r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-2000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    assert r.stdout.strip().endswith("OK")


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), "-o", exe,
           os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "lbmref.c"), "-lm"]
    subprocess.check_call(cmd)
    _run(exe)


def _hip_compiler():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        pytest.skip("hipcc not found")
    return exe


def test_library_host_code_under_asan_ubsan(tmp_path):
    hc = _hip_compiler()
    # host-only compilation; each sanitizer flag applies to the host pass only
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in (os.path.join(CSRC, "lattice_host.hip"), os.path.join(CSRC, "lbm_api.hip"),
                os.path.join(CSRC, "serve.hip"), os.path.join(SAN, "launch_stubs.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.check_call([hc, "-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17",
                               "-fPIC", "-w"] + san + ["-c", src, "-o", obj])
        objs.append(obj)
    drv = str(tmp_path / "driver.o")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-c",
                           os.path.join(SAN, "host_driver.c"), "-o", drv])
    exe = str(tmp_path / "host_driver")
    subprocess.check_call([hc, "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                           "-fsanitize=undefined", "-o", exe, drv] + objs)
    _run(exe)
