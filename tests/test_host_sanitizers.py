"""The library's host-only parts under sanitizers (CPU, no GPU): the delay
table builder, the sigproc header parser and the threaded host search, built
from their sources with g++ together with tests/host_sanitize.cpp, once with
AddressSanitizer + UndefinedBehaviorSanitizer (every vector path of the host
search, capped through DEDISP_CPU_ISA) and once with ThreadSanitizer (the
search's worker threads); and the streaming server's bookkeeping (admission,
tickets, completion callbacks on stream threads, ring positions), built with
tests/host_server.cpp, which stands in for the HIP runtime calls it makes,
under the same two.  A sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1111_6399_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "host_sanitize.cpp")] + [
    os.path.join(CSRC, f) for f in ("cpu_kernel.cpp", "shift_table.cpp", "sigproc.cpp")]
SERVER_SOURCES = [os.path.join(ROOT, "tests", "host_server.cpp")] + [
    os.path.join(CSRC, f) for f in ("server.cpp", "shift_table.cpp")]
ROCM_INCLUDE = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                                reason="needs g++ and the ROCm headers")


def build(tmp_path, name, flags, sources=SOURCES):
    exe = str(tmp_path / name)
    # host code only (g++, no device pass): the HIP headers give the types
    # the internal header declares
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
           "-I" + ROCM_INCLUDE, "-I" + CSRC] + flags + sources + ["-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def run(exe, env_extra, level=None, passed="host checks passed"):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-4000:]
    for marker in ("AddressSanitizer", "runtime error:", "ThreadSanitizer", "LeakSanitizer"):
        assert marker not in text, text[-4000:]
    assert passed in text
    if level is not None:  # the cap took effect (a host without the wider paths runs a lower level)
        assert "vector level %d" % level in text or int(text.split("vector level ")[1][0]) < level


def test_address_and_undefined(tmp_path):
    exe = build(tmp_path, "host_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])
    for isa in ("0", "1", "2"):
        run(exe, {"DEDISP_CPU_ISA": isa, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                  "UBSAN_OPTIONS": "print_stacktrace=1"}, level=int(isa))


def test_threads(tmp_path):
    exe = build(tmp_path, "host_tsan", ["-fsanitize=thread"])
    run(exe, {"TSAN_OPTIONS": "halt_on_error=1"})


def test_server_address_and_undefined(tmp_path):
    exe = build(tmp_path, "server_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                SERVER_SOURCES)
    run(exe, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"},
        passed="server checks passed")


def test_server_threads(tmp_path):
    exe = build(tmp_path, "server_tsan", ["-fsanitize=thread"], SERVER_SOURCES)
    run(exe, {"TSAN_OPTIONS": "halt_on_error=1"}, passed="server checks passed")
