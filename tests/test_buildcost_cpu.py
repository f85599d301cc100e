"""The build-cost report (analogues of the paper's Tables II and III): medians
and per-set sums on small hand-made inputs, and the committed build's stats
file covering every variant of the manifest."""
import os

import pytest

from paper_2507_15277_amd import buildcost, tuned
from paper_2507_15277_amd.tune import read_manifest


def test_report_medians_and_set_sums(monkeypatch):
    monkeypatch.setattr(buildcost, "read_manifest", lambda with_prec=True: [(0, "a", 0), (1, "b", 0), (2, "c", 1)])
    stats = {0: ("a", 2.0, 2048), 1: ("b", 4.0, 4096), 2: ("c", 10.0, 10240)}
    rows = [{"prec": 0, "status": "ok", "data": "uniform", "ms": t} for t in (0.5, 1.0, 3.0)]
    rows += [{"prec": 0, "status": "wrong", "data": "uniform", "ms": 100.0},
             {"prec": 1, "status": "ok", "data": "lognormal", "ms": 100.0}]
    rep = buildcost.report(stats, rows, {"s": [0, 2]})
    t2, t3 = rep["table_ii"], rep["table_iii"]
    assert t2["median_run_ms"] == 1.0 and t2["median_compile_ms"] == 3000.0
    assert t2["compile_over_run"] == 3000.0 and t2["runs"] == 3 and t2["variants"] == 2
    assert t3["fp32_mean_kb"] == 3.0 and t3["all_mean_kb"] == pytest.approx(16.0 / 3)
    assert t3["all_family_compile_s"] == 16.0 and t3["variants"] == 3
    assert rep["sets"]["s"] == {"members": [0, 2], "kb": 12.0, "compile_s": 12.0}


def test_stats_cover_the_manifest():
    if not os.path.exists(buildcost.STATS):
        pytest.skip("variants not built")
    stats = buildcost.read_stats()
    man = read_manifest(with_prec=True)
    assert sorted(stats) == [vid for vid, _, _ in man]
    assert all(stats[vid][0] == name and stats[vid][1] > 0 and stats[vid][2] > 0 for vid, name, _ in man)
