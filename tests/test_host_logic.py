"""Host-only builds of the C ABI's device-free logic (pvfind_params.cpp,
pvfind_server.cpp) against a CPU stand-in of the server's device side
(tests/host/fake_server_device.cpp), under AddressSanitizer with
UndefinedBehaviorSanitizer (and leak checking), and under ThreadSanitizer.
The driver, tests/host/server_logic_test.cpp, checks parameter and schedule
validation and the server's admission, batch sealing, completions, second
copy of vertex records, back-pressure, replay, concurrent callers, device
errors and shutdown."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_14966_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
SOURCES = [os.path.join(CSRC, "pvfind_params.cpp"), os.path.join(CSRC, "pvfind_server.cpp"),
           os.path.join(HOST, "fake_server_device.cpp"), os.path.join(HOST, "server_logic_test.cpp")]
COMMON = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-Werror",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", HOST, "-pthread"]
# ThreadSanitizer of GCC 11 misses pthread_cond_clockwait (std::condition_variable
# waits with a timeout) and reports false double locks; clang's does not.
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build_and_run(cxx, sanitize, tmp_path, env_extra):
    exe = str(tmp_path / "server_logic_test")
    subprocess.run([cxx, *COMMON, *sanitize, *SOURCES, "-o", exe], check=True, timeout=300,
                   capture_output=True, text=True)
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("all ok"), r.stdout[-2000:] + r.stderr[-4000:]


def test_server_logic_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    _build_and_run(cxx, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"], tmp_path,
                   {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})


def test_server_logic_under_thread_sanitizer(tmp_path):
    if not os.path.exists(CLANG):
        pytest.skip("no clang++ with the ThreadSanitizer runtime")
    _build_and_run(CLANG, ["-fsanitize=thread"], tmp_path, {"TSAN_OPTIONS": "halt_on_error=1"})
