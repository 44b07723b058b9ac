"""Device-memory budgets on the host side of tim_run (api.cpp built on the CPU against the stand-in
runtime and kernels of tests/host_stub): the same queries on contexts with budgets from a geometric
sweep.  More memory must never turn a success into a failure, and every success must give the results
of the run without a budget.

The stand-in sets grow with the KptEstimation round (TIM_STUB_GROWTH=1), so that the round kept in
device memory for RefineKPT (R' of Algorithm 3) comes out larger than the previous round predicts.
RefineKPT then has to fall back to generating R' again from its keys where the inverted index does
not fit beside the kept sets.  With TIM_STUB_GROWTH=2 the sets of RefineKPT and NodeSelection are
larger still, so that the buffers one query leaves behind fill most of the budget when the next
query's KptEstimation starts: those have to make room instead of failing the query."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
SOURCES = ["paper_1404_0900_amd/csrc/api.cpp", "tests/host_stub/hip_stub.cpp", "tests/host_stub/launch_stub.cpp",
           "tests/host_stub/budget_driver.cpp"]


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of the ROCm toolchain not found")
@pytest.mark.parametrize("growth", ["1", "2"])
def test_larger_budgets_never_fail(tmp_path, growth):
    exe = str(tmp_path / "budget_driver")
    cmd = [CLANG, "-std=c++17", "-O2", "-I", "tests/host_stub", "-I", "include", "-I", "paper_1404_0900_amd/csrc",
           *SOURCES, "-o", exe, "-lpthread"]
    subprocess.run(cmd, cwd=ROOT, check=True, capture_output=True, text=True)
    # budgets from 256 KiB to 256 MiB in steps of 1.2x
    p = subprocess.run([exe, str(1 << 18), str(1 << 28), "1.2"], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, TIM_STUB_GROWTH=growth))
    out = p.stdout + p.stderr
    assert p.returncode == 0 and out.rstrip().endswith("done"), out[-4000:]
    # the sweep spans the budgets too small for any query and those that run every one
    assert ": 0 of 4 ok" in out and ": 4 of 4 ok, 0 differ" in out, out[-4000:]


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of the ROCm toolchain not found")
def test_batch_and_server_under_budget_after_queries_alone(tmp_path):
    """A batch and a server on a context whose own queries (run alone first, with the larger stand-in
    sets of growth mode 2) left their work buffers behind: a 150 MB budget holds 12 queries at once
    only if those buffers make room, and every batched or served query must equal its run alone."""
    exe = str(tmp_path / "driver")
    cmd = [CLANG, "-std=c++17", "-O2", "-I", "tests/host_stub", "-I", "include", "-I", "paper_1404_0900_amd/csrc",
           "paper_1404_0900_amd/csrc/api.cpp", "tests/host_stub/hip_stub.cpp", "tests/host_stub/launch_stub.cpp",
           "tests/host_stub/driver.cpp", "-o", exe, "-lpthread"]
    subprocess.run(cmd, cwd=ROOT, check=True, capture_output=True, text=True)
    p = subprocess.run([exe, "1", str(150_000_000), "12"], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, TIM_STUB_GROWTH="2", TIM_RR_POOL_BYTES=str(4 << 20)))
    out = p.stdout + p.stderr
    assert p.returncode == 0 and "round 0: batch and server ok" in out, out[-4000:]
