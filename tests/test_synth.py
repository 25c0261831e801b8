"""The seeded input generators produce what the workloads state."""
import numpy as np

import synth


def test_reads_without_errors_are_reference_substrings():
    ref = synth.make_reference(5000, seed=0, uniform=True)
    r = synth.simulate_reads(ref, np.full(50, 150), 0, 0, 0, seed=1)
    for i in range(r.n):
        s = r.truth[i]
        assert np.array_equal(r.read(i), ref[s:s + 150])


def test_read_lengths_and_error_rates():
    ref = synth.make_reference(200_000, gc=0.41, repeat_frac=0.05, seed=200)
    lengths = np.array([100, 150, 2000, 9999])
    r = synth.simulate_reads(ref, lengths, 0.02, 0.01, 0.01, seed=2)
    assert np.array_equal(r.lengths(), lengths)
    assert r.seq.max() <= 3


def test_reference_composition():
    ref = synth.make_reference(1_000_000, gc=0.41, repeat_frac=0.05, seed=200)
    gc = np.mean((ref == 1) | (ref == 2))
    assert abs(gc - 0.41) < 0.01
    u = synth.make_reference(20_000, seed=0, uniform=True)
    assert np.array_equal(u, np.random.default_rng(0).integers(0, 4, 20_000, dtype=np.uint8))


def test_pairs_shape():
    p = synth.mutate_pairs(1000, 150, 30, seed=402)
    assert p.n == 1000
    assert p.edits.min() >= 0 and p.edits.max() <= 30
    lb = np.diff(p.b_off)
    assert lb.min() >= 120 and lb.max() <= 180
    zero = np.nonzero(p.edits == 0)[0]
    for i in zero[:10]:
        a, b = p.pair(i)
        assert np.array_equal(a, b)


def test_lognormal_lengths():
    rng = np.random.default_rng(0)
    L = synth.lognormal_lengths(20_000, 2000, 0.8, 100, 10_000, rng)
    assert L.min() >= 100 and L.max() <= 10_000
    assert 1800 < np.median(L) < 2200
