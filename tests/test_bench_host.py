"""Host logic of bench.py, on the CPU: the one-GPU guard, the roofline
arithmetic over the library's per-kernel counters, the gating of the measured
HBM traffic on the kernel sources it was taken on, and the whole-sort
algorithmic bytes."""
import hashlib
import json
import os
import subprocess
import sys
import types

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stats(ms, nbytes, launches, kind=3):
    st = types.SimpleNamespace(kernel_ms=[0.0] * 8, kernel_bytes=[0.0] * 8, kernel_launches=[0] * 8)
    st.kernel_ms[kind], st.kernel_bytes[kind], st.kernel_launches[kind] = ms, nbytes, launches
    return st


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_roofline_is_bytes_over_time_against_the_peak():
    # two sorts: 3 launches moving 6e9 B in 3 ms, 2 launches moving 4e9 B in 2 ms
    r = bench.roofline_from_stats([_stats(3.0, 6e9, 3), _stats(2.0, 4e9, 2)])
    assert r["launches"] == 5
    assert r["bytes_per_launch"] == pytest.approx(2e9)
    assert r["avg_launch_ms"] == pytest.approx(1.0)
    assert r["achieved"] == pytest.approx(2000.0)  # 1e10 B / 5 ms
    assert r["frac"] == pytest.approx(2000.0 / bench.HBM_PEAK_GBS)
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"


def test_roofline_without_launches_is_absent():
    assert bench.roofline_from_stats([_stats(0.0, 0.0, 0)]) is None


def test_traffic_counts_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    tr = json.load(open(bench.TRAFFIC_FILE))
    h = hashlib.sha256()
    for f in tr["kernel_sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    current = h.hexdigest()
    good = dict(tr, kernel_sources_sha256=current, k_scatter_bytes_per_launch=1.25e9)
    stale = dict(good, kernel_sources_sha256="0" * 64)
    for doc, expect in ((good, 1.25e9), (stale, None)):
        p = tmp_path / "traffic.json"
        p.write_text(json.dumps(doc))
        monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
        assert bench.roofline_from_stats([_stats(1.0, 1e9, 1)])["traffic"] == expect


def test_whole_sort_bytes():
    # 10 records of 4-byte keys distributed twice (20 distributions), 10 leaf
    # sorted, 4 pair-merged, 6 dovetail-merged, 2 copied: every one is read
    # and written once (2 x 4 B); the histogram reads the 20 distributed keys
    st = types.SimpleNamespace(records_distributed=20, records_leaf_sorted=10, records_pair_merged=4,
                               records_merged=6, records_copied=2)
    moved, hist = bench.algorithmic_bytes(st, 4, 4)
    assert moved == 8 * 42
    assert hist == 4 * 20
    # 16-byte pairs: the histogram still reads only the 8-byte keys
    moved, hist = bench.algorithmic_bytes(st, 8, 16)
    assert moved == 32 * 42 and hist == 8 * 20
