"""Host-side read bucketing (C ABI helper, no GPU needed)."""
import numpy as np
import pytest

from paper_2603_22245_amd import _lib as L


def test_bucket_reads_matches_definition():
    rng = np.random.default_rng(0)
    lens = rng.integers(50, 12_000, 500)
    off = np.zeros(501, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    buckets = (100, 200, 400, 800, 1600, 3200, 6400)
    b, cnt = L.rm_bucket_reads(off, buckets)
    for r in range(500):
        want = max([i for i, n in enumerate(buckets) if n <= lens[r]], default=-1)
        assert b[r] == want
    assert list(cnt) == [int(np.sum(b == i)) for i in range(len(buckets))]


def test_bucket_reads_validation():
    off = np.array([0, 10, 300], dtype=np.int64)
    with pytest.raises(L.RotorMapError):
        L.rm_bucket_reads(off, (200, 100))          # not increasing
    with pytest.raises(L.RotorMapError):
        L.rm_bucket_reads(off, (0, 100))            # non-positive length
