"""The fit server's host logic under the thread and address/undefined-behaviour sanitizers (CPU
only): tests/host/server_stress.cpp drives the real scheduler (sb_server.cpp), with a host stand-in
for the HIP runtime and a fake fit launch, from four submitting threads, a canceller and a
statistics reader.  Every ticket must end exactly once, a completed fit must carry the chi-square
of its own observations (so admissions, the inbox and the arena never mix requests), the
statistics must balance, and the sanitizers must report nothing.  Built with clang, whose thread
sanitizer intercepts the clock waits that std::condition_variable uses."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build_and_run(tmp_path, sanitize, extra_env=None):
    cxx = CLANG if os.path.exists(CLANG) else shutil.which("clang++")
    if cxx is None:
        pytest.skip("no clang++")
    exe = tmp_path / f"stress_{sanitize.replace(',', '_')}"
    cmd = [cxx, "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "tests", "host", "fake_hip"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2504_08081_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "server_stress.cpp"),
           os.path.join(ROOT, "paper_2504_08081_amd", "csrc", "sb_server.cpp"), "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, **(extra_env or {}))
    r = subprocess.run([str(exe), "300"], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-500:], r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "WARNING" not in r.stderr and "ERROR" not in r.stderr
    assert "failures 0 consistent 1" in r.stdout


def test_server_under_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, "thread", {"TSAN_OPTIONS": "halt_on_error=1"})


def test_server_under_address_and_ub_sanitizers(tmp_path):
    _build_and_run(tmp_path, "address,undefined", {"ASAN_OPTIONS": "detect_leaks=1"})
