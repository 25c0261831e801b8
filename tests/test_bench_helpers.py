"""Host logic of bench.py: recall and list agreement against stored oracle
lists, and the source-hash gate on committed counter summaries."""
import json
import os

import numpy as np

import bench


def _stored():
    # a stored oracle list of 16 (ranked), with a tie between ranks 1 and 2
    idx = np.arange(100, 116)
    F = np.array([0.99, 0.8, 0.8, 0.7, 0.6, 0.5, 0.45, 0.4, 0.35, 0.3, 0.25, 0.2, 0.15, 0.1,
                  0.05, 0.01])
    return idx, F


def test_identical_list_is_exact():
    idx, F = _stored()
    rec, ex, err = bench.score_vs_stored(idx[:8], F[:8], idx, F, 8)
    assert rec == 1.0 and ex and err == 0.0


def test_swap_within_a_tie_is_still_exact_but_not_outside():
    idx, F = _stored()
    got = idx[:8].copy()
    got[[1, 2]] = got[[2, 1]]                      # tied scores: allowed
    rec, ex, _ = bench.score_vs_stored(got, F[[0, 2, 1, 3, 4, 5, 6, 7]], idx, F, 8)
    assert rec == 1.0 and ex
    got = idx[:8].copy()
    got[[0, 1]] = got[[1, 0]]                      # 0.99 vs 0.8: not a tie
    rec, ex, _ = bench.score_vs_stored(got, F[[1, 0, 2, 3, 4, 5, 6, 7]], idx, F, 8)
    assert rec == 1.0 and not ex


def test_window_outside_the_stored_list_is_a_miss():
    idx, F = _stored()
    got = idx[:8].copy()
    got[7] = 999
    rec, ex, _ = bench.score_vs_stored(got, F[:8], idx, F, 8)
    assert rec == 7 / 8 and not ex


def test_window_from_the_stored_tail_counts_only_within_the_tie_margin():
    idx, F = _stored()
    got = idx[:8].copy()
    got[7] = idx[12]                               # F = 0.15 < F_(8) = 0.4
    rec, _, err = bench.score_vs_stored(got, np.r_[F[:7], 0.15], idx, F, 8)
    assert rec == 7 / 8 and err == 0.0
    F2 = F.copy()
    F2[8] = F2[7] - 5e-6                            # within 1e-5 of the 8th
    got[7] = idx[8]
    rec, _, _ = bench.score_vs_stored(got, F2[:8], idx, F2, 8)
    assert rec == 1.0


def test_duplicates_are_not_exact():
    idx, F = _stored()
    got = idx[:8].copy()
    got[3] = got[2]
    _, ex, _ = bench.score_vs_stored(got, F[:8], idx, F, 8)
    assert not ex


def test_traffic_is_read_only_for_the_current_kernel_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    for f in bench.SCORE_SOURCES:
        d = tmp_path / os.path.dirname(f)
        d.mkdir(parents=True, exist_ok=True)
        (tmp_path / f).write_text("kernel v1")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("precision", "fp16") is None   # no summary
    digest = bench.score_source_digest()
    body = {"bytes_per_launch": 123, "source_sha256": digest}
    (prof / "score_topk_fp16_precision_traffic.txt").write_text(
        "# summary\n\n```json\n" + json.dumps(body) + "\n```\n")
    assert bench.measured_traffic("precision", "fp16") == 123
    assert bench.measured_traffic("scale", "fp16") is None       # another workload's summary
    assert bench.measured_traffic("precision", "fp8") is None    # another precision's
    assert bench.measured_traffic("precision", "fp16", row_reals=256) == 123  # summaries default to 256
    assert bench.measured_traffic("precision", "fp16", row_reals=192) is None  # another row form
    (tmp_path / bench.SCORE_SOURCES[0]).write_text("kernel v2")
    assert bench.measured_traffic("precision", "fp16") is None   # kernel changed


def test_location_clusters_join_overlapping_windows_only():
    assert bench.location_clusters([], 150) == 0
    assert bench.location_clusters([7], 150) == 1
    # 100..250 overlap one another (ids within 150); 401 is a new place
    assert bench.location_clusters([250, 100, 180, 401], 150) == 2
    assert bench.location_clusters([0, 150, 300], 150) == 1      # a chain of overlaps
    assert bench.location_clusters([0, 151], 150) == 2
