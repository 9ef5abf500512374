"""The library's host code (plans, grouped steps with their cached step graphs, batches, the
allocation-free solve's bookkeeping) built for the CPU with AddressSanitizer and
UndefinedBehaviorSanitizer against a HIP stand-in that checks every API use
(tests/host_mock), then driven through served streams of the kind the GPU server runs: long
streams whose active set changes at almost every tick (thousands of distinct grouped steps), and
one that fills the server. No sanitizer report, no API misuse, nothing left allocated; the same
with every k-th fallible runtime call failing (the library's error paths)."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2209_08437_amd", "csrc")
MOCK = os.path.join(HERE, "host_mock")


def _runtime(name):
    out = subprocess.run(["g++", f"-print-file-name={name}"], stdout=subprocess.PIPE, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ is not available")
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("the sanitizer runtimes are not installed")
    lib = str(tmp_path_factory.mktemp("host_build") / "libsfac_host.so")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-I", os.path.join(MOCK, "inc"), "-I", CSRC,
           os.path.join(CSRC, "sfac_runtime.cpp"), os.path.join(CSRC, "sfac_tables.cpp"),
           os.path.join(MOCK, "mock_hip.cpp"), os.path.join(MOCK, "mock_kernels.cpp"), "-o", lib]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-4000:]
    return lib, f"{asan}:{ubsan}"


def test_served_streams_under_sanitizers(sanitized_lib):
    lib, preload = sanitized_lib
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    streams = ["150:6.32:51", "120:20:50", "200:200:5", "60:20:7:200"]   # the last: ticks of 8-step graphs
    r = subprocess.run([sys.executable, os.path.join(MOCK, "replay_served.py"), lib] + streams,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=900)
    assert r.returncode == 0, r.stdout[-6000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("stream ")]
    assert len(lines) == len(streams), r.stdout[-3000:]
    for spec, line in zip(streams, lines):
        count = spec.split(":")[0]
        assert f"completed {count} " in line, line
        assert line.endswith("allocations 0 streams 0 graphs 0"), line


@pytest.mark.parametrize("every", [7, 29])
def test_served_streams_with_failing_runtime_calls(sanitized_lib, every):
    """Every k-th allocation, stream or event creation, copy, capture, instantiation, launch or
    synchronisation fails: each failure comes back as a library error, the server goes on, and the
    error paths leave no sanitizer report, no API misuse and nothing allocated."""
    lib, preload = sanitized_lib
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", MOCK_FAIL_EVERY=str(every))
    streams = ["120:20:50", "150:200:5"]
    r = subprocess.run([sys.executable, os.path.join(MOCK, "replay_served.py"), lib] + streams,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=900)
    assert r.returncode == 0, r.stdout[-6000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("stream ")]
    assert len(lines) == len(streams), r.stdout[-3000:]
    for spec, line in zip(streams, lines):
        count = spec.split(":")[0]
        assert f"completed {count} " in line, line
        injected = int(line.split(" injected ")[1].split()[0])
        errors = int(line.split(" errors ")[1].split()[0])
        assert injected > 0 and errors > 0, line
        assert line.endswith("allocations 0 streams 0 graphs 0"), line
