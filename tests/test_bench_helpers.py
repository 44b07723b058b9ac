"""bench.py's host-side helpers: the traffic key, the roofline and per-phase figures, kernel names and the
one-GPU guard (no GPU needed)."""
import os
import shutil
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _kp(launches=0, kernel_ms=0.0, sets=0, nodes=0, edges=0, nbytes=0, large_ms=0.0, deferred=0):
    return SimpleNamespace(launches=launches, kernel_ms=kernel_ms, sets=sets, nodes=nodes, edges=edges, bytes=nbytes,
                           large_launches=launches, large_ms=large_ms, deferred=deferred)


def _prof():
    s = [[_kp() for _ in range(3)] for _ in range(2)]
    s[0][0] = _kp(10, 8.0, 1000, 9000, 70000, 424000, 2.0, 10)
    s[0][1] = _kp(4, 12.0, 500, 5000, 40000, 30_000_000_000, 1.0, 5)
    s[1][0] = _kp(3, 1.0, 100, 300, 900, 6000)
    wide = [_kp() for _ in range(3)]
    wide[0] = _kp(5, 2.0, 400, 1000, 8000, 48000, 0.5, 0)
    grouped = [_kp(2, 1.0, 300, 600, 5000, 29600, 0.5, 0), _kp()]
    return SimpleNamespace(sampler=s, ic_wide=wide, grouped=grouped, index_ms=0.0, greedy_ms=0.0, index_calls=0)


def test_dominant_roofline_takes_the_longest_kernel():
    # the 64-lane launches of few sets (ic_wide) and the multi-job launches of the early rounds (grouped) are
    # other kernels: never the roofline's
    r = bench.dominant_roofline(_prof(), lambda model, mode: f"k{model}{mode}", lambda model, mode: 123)
    assert r["kernel"] == "k01" and r["launches"] == 4
    assert r["achieved"] == pytest.approx(30e9 / 12e-3 / 1e9, rel=1e-6)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    assert r["bytes_per_launch"] == 7_500_000_000 and r["avg_launch_us"] == pytest.approx(3000.0)
    assert r["traffic"] == 123 and r["bound"] == "hbm" and r["unit"] == "GB/s"


def test_sampler_by_mode_counts_every_tier():
    out = bench.sampler_by_mode(_prof(), 0)
    assert set(out) == {"kpt_widths", "stored_sets"}  # no coverage launches in this profile
    w = out["kpt_widths"]  # the 8-lane launches, the 64-lane ones of few sets and the grouped rounds together
    assert w["sets"] == 1010 + 400 + 300 and w["gpu_ms"] == pytest.approx(14.0) and w["launches"] == 17
    assert w["sets_per_s"] == pytest.approx(1710 / 14.0e-3)
    assert w["tier0_edges_per_s"] == pytest.approx(83000 / 11e-3)
    assert w["wide_launches"] == 5 and "wide_launches" not in out["stored_sets"]
    assert w["grouped_launches"] == 2 and "grouped_launches" not in out["stored_sets"]


def test_kernel_names_follow_the_shape_table():
    assert bench.kernel_name(0, 0, 8) == "ic_seg_kernel<0, true, 8, 128, 0, 512, 1> (widths)"
    assert bench.kernel_name(0, 1, 16) == "ic_seg_kernel<1, true, 16, 128, 8, 512, 1> (store)"
    assert bench.kernel_name(1, 2) == "lt_lane_kernel<2> (cover)"
    # traffic is kept for weighted-cascade first-tier kernels, under the names kernel_name gives them
    names = {bench.kernel_name(0, mode, 8) for mode in (0, 1)}
    assert set(bench.TRAFFIC) == names


def test_traffic_key_ignores_comments_but_not_code(tmp_path, monkeypatch):
    for p in bench.KERNEL_SOURCES:
        dst = tmp_path / p
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, p), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.sources_sha()
    assert base == bench.sources_sha()
    src = tmp_path / bench.KERNEL_SOURCES[0]
    text = src.read_text()
    src.write_text("// a new comment line\n" + text.replace("\n", "  /* trailing block comment */\n", 1) + "\n\n")
    assert bench.sources_sha() == base
    src.write_text(text + "\nstatic int extra_code = 1;\n")
    assert bench.sources_sha() != base


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
