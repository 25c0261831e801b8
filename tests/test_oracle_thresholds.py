"""Pins of the per-fragment threshold oracle (oracle.thresholds)."""
import numpy as np

from oracle import lev, mapping, rope
from oracle import thresholds as T


def test_philox_known_answers():
    """Philox4x32-10 known-answer vectors published with the generator
    (Random123): zero counter and key, all-ones, and the digits of pi."""
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF),
              (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        got = tuple(int(x) for x in T.philox4x32(ctr, key))
        assert got == want


def test_philox_vectorised_equals_one_by_one():
    ctr = (np.arange(5, dtype=np.uint64) * 977, np.full(5, 3), np.arange(5), np.arange(5) ** 2)
    many = T.philox4x32(ctr, (11, 12))
    for i in range(5):
        one = T.philox4x32(tuple(int(c[i]) for c in ctr), (11, 12))
        assert tuple(int(w[i]) for w in many) == tuple(int(x) for x in one)


def test_event_threshold_integer_rule():
    assert T.event_threshold(0.0) == 0
    # err = 0.75: each event type 1/4 of the 32-bit range
    assert T.event_threshold(0.75) == 1 << 30
    assert 3 * T.event_threshold(0.9999) < 1 << 32


def test_zero_rate_copies_are_the_window():
    rng = np.random.default_rng(70)
    ref = rng.integers(0, 4, 600).astype(np.uint8)
    for j in (0, 17, 450):
        for c in range(3):
            y, ev, used = T.mutate_window(ref, j, 150, 0.0, j, c, 5)
            np.testing.assert_array_equal(y, ref[j:j + 150])
            assert ev == (0, 0, 0) and used == 150
    assert T.window_threshold(ref, 17, 1, 150, 0.0, 8, 0, 5) == 1.0


def test_copies_are_within_their_edit_count_of_the_consumed_text():
    """Each insertion, deletion or substitution is one edit, so the edit
    distance between a copy and the reference text it consumed is at most the
    number of events; the copy has exactly N letters."""
    rng = np.random.default_rng(71)
    ref = rng.integers(0, 4, 2000).astype(np.uint8)
    for c in range(40):
        j = int(rng.integers(0, 1700))
        y, (ni, nd, ns), used = T.mutate_window(ref, j, 100, 0.2, j, c, 9)
        assert y.size == 100 and np.all(y < 4)
        assert used == 100 - ni + nd
        a = ref[j:j + used]
        d = lev.lev_many(a, np.array([0, a.size]), y, np.array([0, y.size]))[0]
        assert d <= ni + nd + ns


def test_event_frequencies_follow_the_rate():
    rng = np.random.default_rng(72)
    ref = rng.integers(0, 4, 5000).astype(np.uint8)
    tot = np.zeros(3)
    steps = 0
    for c in range(64):
        y, ev, used = T.mutate_window(ref, 100, 150, 0.3, 100, c, 3)
        tot += ev
        steps += 150 + ev[1]           # emitted letters plus deletions
    frac = tot / steps
    # 0.1 each, binomial standard error ~0.003 over ~10,000 steps
    assert np.all(np.abs(frac - 0.1) < 0.015), frac


def test_threshold_is_an_order_statistic_of_the_copy_fidelities():
    rng = np.random.default_rng(73)
    ref = rng.integers(0, 4, 1000).astype(np.uint8)
    F = T.window_copy_fidelities(ref, 7, 2, 150, 0.05, 16, 4)
    assert np.all((F > 0) & (F <= 1))
    assert T.window_threshold(ref, 7, 2, 150, 0.05, 16, 0, 4) == F.min()
    assert T.window_threshold(ref, 7, 2, 150, 0.05, 16, 15, 4) == F.max()
    # each copy's F is the direct F of the window and the copy's letters
    y, _, _ = T.mutate_window(ref, 14, 150, 0.05, 7, 3, 4)
    want = rope.fidelity(rope.encode_raw(ref[14:164], 150), rope.encode_raw(y, 150), 150)
    assert abs(F[3] - want) < 1e-15


def test_threshold_regime_hand_made():
    F = np.array([0.9, 0.2, 0.6, 0.6, 0.0, 0.35])
    thr = np.array([0.95, 0.1, 0.5, 0.6, 0.0, 0.3])
    ids, f = T.threshold_hits(F, thr)
    # 0 fails its threshold; 4 has F = 0 (no location) although 0 >= 0
    np.testing.assert_array_equal(ids, [2, 3, 5, 1])
    np.testing.assert_array_equal(f, [0.6, 0.6, 0.35, 0.2])
    ids, _ = T.threshold_hits(F, thr, floor=0.4)
    np.testing.assert_array_equal(ids, [2, 3])
    ids, _ = T.threshold_hits(F, np.ones(6))
    assert ids.size == 0
