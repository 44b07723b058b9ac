"""The host side of batches and servers (api.cpp: the hub, its scheduler thread, worker threads, the
server's queue and the RR-pool admission) built on the CPU against a stand-in HIP runtime and stand-in
kernels (tests/host_stub), and driven from many threads under ThreadSanitizer and under
AddressSanitizer with UndefinedBehaviorSanitizer: no data race, memory error, leak or undefined
behaviour may be reported, and every batched or served query must equal the same query alone.

clang's sanitizer runtimes are used: GCC 11's ThreadSanitizer does not intercept
pthread_cond_clockwait, which std::condition_variable::wait_until calls, and so reports accesses made
under the hub's mutex across such a wait as races."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
SOURCES = ["paper_1404_0900_amd/csrc/api.cpp", "tests/host_stub/hip_stub.cpp", "tests/host_stub/launch_stub.cpp",
           "tests/host_stub/driver.cpp"]


def _build(tmp_path, flags):
    exe = str(tmp_path / "driver")
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-I", "tests/host_stub", "-I",
           "include", "-I", "paper_1404_0900_amd/csrc", *SOURCES, "-o", exe, "-lpthread"]
    subprocess.run(cmd, cwd=ROOT, check=True, capture_output=True, text=True)
    return exe


def _run(exe, args, env_extra):
    env = dict(os.environ, **env_extra)
    p = subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=600)
    return p.returncode, p.stdout + p.stderr


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of the ROCm toolchain not found")
def test_batches_and_servers_under_thread_sanitizer(tmp_path):
    exe = _build(tmp_path, ["-fsanitize=thread"])
    rc, out = _run(exe, ["1", "0", "12"], {"TSAN_OPTIONS": "halt_on_error=1"})
    assert rc == 0 and "WARNING: ThreadSanitizer" not in out, out[-4000:]
    assert "round 0: batch and server ok" in out
    # a 1 GB budget and a 2 MB RR pool: NodeSelections wait for memory
    rc, out = _run(exe, ["1", str(1 << 30), "12"], {"TSAN_OPTIONS": "halt_on_error=1",
                                                    "TIM_RR_POOL_BYTES": str(2 << 20)})
    assert rc == 0 and "WARNING: ThreadSanitizer" not in out, out[-4000:]
    held = int(out.split("(held ")[1].split(")")[0])
    assert held > 0


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of the ROCm toolchain not found")
def test_batches_and_servers_under_address_sanitizer(tmp_path):
    exe = _build(tmp_path, ["-fsanitize=address,undefined"])
    rc, out = _run(exe, ["2", "0", "12"], {"ASAN_OPTIONS": "detect_leaks=1",
                                           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert rc == 0 and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "round 1: batch and server ok" in out
