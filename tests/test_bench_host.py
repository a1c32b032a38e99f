"""The measurement's host logic, on the CPU: the algorithmic flop count of a
launch (8 flops per kept term, 6 per complex multiplication of the 2 log2 l
squarings and products of z^l), and the committed counter summaries, which
bench.py reports only for the kernel sources they were taken from."""
from __future__ import annotations

import math
import os
import shutil

import numpy as np

import bench


def test_algorithmic_flops_by_hand():
    terms = np.array([0, 1, 5, 100], np.int32)
    window = np.array([[0, -1], [0, 0], [1, 5], [1000, 1099]], np.int64)
    # l = 0 and l = 1: no powering; l = 1000: ceil(2 log2 1000) = 20 multiplications
    want = 8.0 * (0 + 1 + 5 + 100) + 6.0 * math.ceil(2 * math.log2(1000))
    assert bench.algorithmic_flops(terms, window) == want
    # l = 2: two multiplications (one squaring, counted as 2 log2 2 = 2)
    assert bench.algorithmic_flops(np.array([1]), np.array([[2, 2]])) == 8.0 + 12.0


def test_recorded_figures_follow_the_sources(tmp_path, monkeypatch):
    # figures while the summaries match the sources, none otherwise
    sha = bench.window_sources_sha256()
    with open(bench.TRAFFIC_PROFILE) as fh:
        fresh = f"window_sources_sha256 = {sha}" in fh.read()
    t512 = bench.recorded_traffic("uniform_d1e6", 512)
    c512 = bench.recorded_counters("uniform_d1e6", 512)
    if fresh:
        assert t512 is not None and 56e6 <= t512 <= 1e9       # at least the algorithmic 56 MB
        assert c512 is not None and 0 < c512["executed_frac"] <= 1 and 0 < c512["l2_hit_rate"] < 1
    else:
        assert t512 is None and c512 is None
    assert bench.recorded_traffic("uniform_d1e6", 2048) is None        # a chunk not profiled
    assert bench.recorded_traffic("wide_d2p20", 512) is None           # another workload
    # a changed kernel source: no figure
    src = tmp_path / "fpe_eval.hip"
    shutil.copy(bench.WINDOW_SOURCES[0], src)
    with open(src, "a") as fh:
        fh.write("\n// changed\n")
    monkeypatch.setattr(bench, "WINDOW_SOURCES", [str(src)] + bench.WINDOW_SOURCES[1:])
    assert bench.recorded_traffic("uniform_d1e6", 512) is None
    assert bench.recorded_counters("uniform_d1e6", 512) is None


def test_more_than_one_gpu_is_refused(capsys, monkeypatch):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "single" in capsys.readouterr().err
    assert os.path.exists(bench.TRAFFIC_PROFILE)
