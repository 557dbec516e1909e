"""The host-side netlist builder and lowering, compiled with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer (no HIP, no device), build,
share, hash and lower several FFT shapes and evaluate the schedules on
plaintext bits against the netlist (csrc/host_check.cpp).  A planted wrong
epilogue coefficient must be caught."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1611_08769_amd", "csrc")


@pytest.fixture(scope="module")
def host_check(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("hc") / "host_check")
    srcs = [os.path.join(CSRC, f) for f in ("host_check.cpp", "netlist.cpp", "schedule.cpp")]
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer"] + srcs + ["-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([exe, *args], capture_output=True, text=True, timeout=600, env=env)


def test_host_code_clean_under_sanitizers(host_check):
    r = _run(host_check)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "host check passed" in r.stdout
    assert "runtime error" not in r.stderr


def test_host_check_catches_planted_mistake(host_check):
    r = _run(host_check, "plant")
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "host check failed" in r.stderr
