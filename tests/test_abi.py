"""The C ABI library loads and exports every entry point include/tim.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "tim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tim_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_phase_calls():
    names = _declared()
    for n in ("tim_graph_upload", "tim_sample_rr", "tim_kpt_estimate", "tim_refine_kpt", "tim_node_select", "tim_run"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1404_0900_amd as tim
    if not os.path.exists(tim.LIB_PATH):
        pytest.skip("libtim.so not built")
    lib = ctypes.CDLL(tim.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert missing == []
    assert sorted(_declared()) == sorted(tim.EXPORTED)


def test_struct_layouts_match_header():
    import subprocess
    import tempfile

    import paper_1404_0900_amd as tim
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "tim.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(tim_report), sizeof(tim_kpt_result),
         sizeof(tim_batch_stats), sizeof(tim_refine_result), sizeof(tim_select_result), offsetof(tim_report, s_prime),
         offsetof(tim_report, ms_kpt), offsetof(tim_report, sets_total), sizeof(tim_query),
         offsetof(tim_query, status), sizeof(tim_batch_info), offsetof(tim_batch_info, ms_wall));
  printf("%zu %zu %zu\n", sizeof(tim_tune_result), offsetof(tim_tune_result, ms_emit),
         offsetof(tim_tune_result, ms_lanes_emit));
  printf("%zu %zu %zu %zu\n", sizeof(tim_profile), offsetof(tim_profile, greedy_ms), offsetof(tim_profile, ic_wide),
         offsetof(tim_profile, grouped));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "sz.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "sz")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(x) for x in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(tim.Report), ctypes.sizeof(tim.KptResult), ctypes.sizeof(tim.BatchStats),
            ctypes.sizeof(tim.RefineResult), ctypes.sizeof(tim.SelectResult), tim.Report.s_prime.offset,
            tim.Report.ms_kpt.offset, tim.Report.sets_total.offset, ctypes.sizeof(tim.Query), tim.Query.status.offset,
            ctypes.sizeof(tim.BatchInfo), tim.BatchInfo.ms_wall.offset, ctypes.sizeof(tim.TuneResult),
            tim.TuneResult.ms_emit.offset, tim.TuneResult.ms_lanes_emit.offset,
            ctypes.sizeof(tim.Profile), tim.Profile.greedy_ms.offset, tim.Profile.ic_wide.offset,
            tim.Profile.grouped.offset]
    assert got == want


def test_engine_refuses_to_run_without_gpu():
    import torch

    import paper_1404_0900_amd as tim
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        tim.Engine(0)
