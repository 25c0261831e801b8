"""Pins of the FP64 mapping oracle: brute force on tiny inputs, exact substrings,
tie order, recall metrics."""
import numpy as np
import pytest

from oracle import mapping, rope
from synth import make_reference, simulate_reads


def _brute_topk(ref, head, N, m, k, stride):
    # every window scored one pair at a time; ranked by F descending, scores
    # within RANK_EPS counting as equal and ordered by window id
    W = mapping.n_windows(ref.shape[0], N, stride)
    x = rope.encode_raw(head, N, m)
    F = np.array([rope.fidelity(x, rope.encode_raw(ref[j * stride:j * stride + N], N, m), N)
                  for j in range(W)])
    order = sorted(range(W), key=lambda j: -F[j])
    groups, cur = [], [order[0]]
    for a, b in zip(order, order[1:]):
        if F[a] - F[b] > mapping.RANK_EPS:
            groups.append(cur)
            cur = []
        cur.append(b)
    groups.append(cur)
    ranked = [j for g in groups for j in sorted(g)][:k]
    return ranked, [F[j] for j in ranked]


def test_rank_order_ties_by_index():
    F = np.array([0.5, 0.9, 0.5 + 1e-14, 0.7, 0.9 - 3e-13, 0.1])
    ids = np.array([10, 3, 2, 8, 5, 1])
    o = mapping.rank_order(F, ids)
    assert list(ids[o]) == [3, 5, 8, 2, 10, 1]
    F2 = np.array([0.5, 0.5 + 1e-9])                 # a real difference is kept
    assert list(mapping.rank_order(F2, np.array([0, 1]))) == [1, 0]


@pytest.mark.parametrize("stride", [1, 3])
def test_map_reads_matches_pairwise_brute_force(stride):
    rng = np.random.default_rng(10)
    ref = rng.integers(0, 4, 400).astype(np.uint8)
    # a repeated block makes exact ties between identical windows
    ref[300:340] = ref[100:140]
    N, m, k = 30, 8, 6
    heads = np.stack([ref[s:s + N] for s in (0, 100, 257)] + [rng.integers(0, 4, N).astype(np.uint8)])
    idx, F = mapping.map_reads(ref, heads, N, m, k, stride, chunk=7)
    for r in range(heads.shape[0]):
        bi, bf = _brute_topk(ref, heads[r], N, m, k, stride)
        assert list(idx[r]) == bi
        assert np.allclose(F[r], bf, atol=1e-12)


def test_exact_substring_scores_one_and_ties_order_by_index():
    rng = np.random.default_rng(11)
    ref = rng.integers(0, 4, 1000).astype(np.uint8)
    ref[600:700] = ref[200:300]          # window 200 == window 600 for N <= 100
    N = 80
    heads = np.stack([ref[200:200 + N], ref[33:33 + N]])
    idx, F = mapping.map_reads(ref, heads, N, 32, 4)
    assert idx[0, 0] == 200 and idx[0, 1] == 600
    assert abs(F[0, 0] - 1) < 1e-12 and abs(F[0, 1] - 1) < 1e-12
    assert idx[1, 0] == 33 and abs(F[1, 0] - 1) < 1e-12


def test_degenerate_window_scores_zero():
    ref = np.concatenate([np.zeros(150, np.uint8), np.arange(150, dtype=np.uint8) % 4])
    head = (np.arange(150) % 4).astype(np.uint8)
    F = mapping.pair_fidelities(ref, head[None], np.array([[0, 150]]), 150)
    assert F[0, 0] == 0.0 and abs(F[0, 1] - 1) < 1e-12


def test_no_location_when_every_fidelity_is_zero():
    """§3: a read's position is reported only if one exists.  Reference: 160
    A's then one C (N = 150, W = 12).  Windows 0..10 are all A, the zero
    vector (every factor sums a full turn of roots of unity), so every read
    scores 0 with them; only window 11 holds the C.  A read of 100 letters
    (shorter than N) and a read of 150 A's are zero vectors too."""
    ref = np.r_[np.zeros(160, np.uint8), np.ones(1, np.uint8)]
    rng = np.random.default_rng(12)
    reads = [rng.integers(0, 4, 150).astype(np.uint8), rng.integers(0, 4, 100).astype(np.uint8),
             np.zeros(150, np.uint8), ref[11:161].copy()]
    off = np.r_[0, np.cumsum([len(x) for x in reads])]
    heads = mapping.read_heads(np.concatenate(reads), off, 150)
    assert np.all(heads[1] == mapping.NO_LETTER)
    np.testing.assert_array_equal(heads[0], reads[0])
    idx, F = mapping.map_reads(ref, heads, 150, 32, 8)
    # brute force, pair by pair: only (read 0, window 11) and (read 3, window 11) are > 0
    for r in range(4):
        for j in range(12):
            f = mapping.pair_fidelity(ref, heads[r], j, 150)
            assert (f > 0) == (r in (0, 3) and j == 11), (r, j, f)
    assert idx[0, 0] == 11 and F[0, 0] > 0 and idx[3, 0] == 11 and abs(F[3, 0] - 1) < 1e-12
    assert np.all(idx[:, 1:] == -1) and np.all(F[:, 1:] == 0)
    assert np.all(idx[1:3] == -1) and np.all(F[1:3] == 0)


def test_pair_fidelities_match_full_scan():
    ref = make_reference(3000, seed=0, uniform=True)
    reads = simulate_reads(ref, np.full(5, 150), 0.01, 0.005, 0.005, seed=3)
    heads = mapping.read_heads(reads.seq, reads.offsets, 150)
    idx, F = mapping.map_reads(ref, heads, 150, 32, 8, chunk=1000)
    F2 = mapping.pair_fidelities(ref, heads, idx, 150)
    assert np.allclose(F, F2, atol=1e-12)
    for r in range(5):
        assert abs(mapping.pair_fidelity(ref, heads[r], int(idx[r, 0]), 150) - F[r, 0]) < 1e-12


def test_true_location_is_found_for_low_error_reads():
    # Qualitative: on a uniform random reference reads at 2% error map to their
    # true start (the paper reports all true matches on a random reference).
    ref = make_reference(20_000, seed=0, uniform=True)
    reads = simulate_reads(ref, np.full(40, 150), 0.01, 0.005, 0.005, seed=101)
    heads = mapping.read_heads(reads.seq, reads.offsets, 150)
    idx, _ = mapping.map_reads(ref, heads, 150, 32, 8)
    assert np.mean(np.abs(idx[:, 0] - reads.truth) <= 3) >= 0.95


def test_recall_and_tie_metrics():
    ref_idx = np.array([[5, 7, 9]])
    ref_F = np.array([[0.9, 0.5, 0.3]])
    # exact
    assert mapping.recall_at_k(ref_idx, ref_idx, ref_F, ref_F) == 1.0
    # a tie member (F within tau of the 3rd) replacing the 3rd counts as correct
    got = np.array([[5, 7, 11]])
    assert mapping.recall_at_k(got, ref_idx, ref_F, np.array([[0.9, 0.5, 0.3 - 1e-6]])) == 1.0
    assert mapping.same_up_to_ties(got, ref_F, np.array([[0.9, 0.5, 0.3 - 1e-6]]))[0]
    # a clearly worse window does not
    assert abs(mapping.recall_at_k(got, ref_idx, ref_F, np.array([[0.9, 0.5, 0.2]])) - 2 / 3) < 1e-12
    assert not mapping.same_up_to_ties(got, ref_F, np.array([[0.9, 0.5, 0.2]]))[0]
    # duplicates count once
    dup = np.array([[5, 5, 7]])
    assert abs(mapping.recall_at_k(dup, ref_idx, ref_F, np.array([[0.9, 0.9, 0.5]])) - 2 / 3) < 1e-12
    # swapped order is not "same", unless tied
    sw = np.array([[7, 5, 9]])
    assert not mapping.same_up_to_ties(sw, ref_F, np.array([[0.5, 0.9, 0.3]]))[0]


def test_window_count():
    assert mapping.n_windows(20_000, 150, 1) == 19_851
    assert mapping.n_windows(10_000_000, 150, 1) == 9_999_851
    assert mapping.n_windows(1000, 100, 7) == 129
    assert mapping.n_windows(99, 100, 1) == 0


def test_refine_pool_clamps_and_deduplicates():
    # coarse stride 4, radius 3, 50 step-1 windows: neighbourhoods of ids 0, 1
    # overlap, id 12 (start 48) is clamped at the last start 49, -1 is skipped
    pool = mapping.refine_pool([0, 1, 12, -1], 4, 3, 50)
    assert list(pool) == [0, 1, 2, 3, 4, 5, 6, 7] + [45, 46, 47, 48, 49]
    assert list(mapping.refine_pool([5], 4, 0, 50)) == [20]
    assert mapping.refine_pool([-1, -3], 4, 3, 50).size == 0


@pytest.mark.parametrize("stride", [2, 5])
def test_refine_with_full_coverage_is_the_step1_brute_force(stride):
    """Every coarse window with radius stride-1 covers every step-1 start, so
    the refined top-k must be the brute-force top-k over all step-1 windows."""
    rng = np.random.default_rng(12 + stride)
    ref = rng.integers(0, 4, 300).astype(np.uint8)
    ref[200:240] = ref[50:90]
    N, m, k = 30, 8, 6
    heads = np.stack([ref[s:s + N] for s in (0, 51, 203)] + [rng.integers(0, 4, N).astype(np.uint8)])
    W1 = mapping.n_windows(ref.shape[0], N, 1)
    Wc = mapping.n_windows(ref.shape[0], N, stride)
    x = np.stack([rope.encode_raw(h, N, m) for h in heads])
    C = np.stack([rope.encode_raw(ref[s:s + N], N, m) for s in range(W1)])
    F1 = np.array([[rope.fidelity(x[r], C[s], N) for s in range(W1)] for r in range(len(heads))])
    for r in range(len(heads)):
        got_i, got_f = mapping.refine_topk(F1[r], np.arange(Wc), stride, stride - 1, k)
        bi, bf = _brute_topk(ref, heads[r], N, m, k, 1)
        assert list(got_i) == bi
        assert np.allclose(got_f, bf, atol=1e-12)


def test_refine_radius_zero_is_the_coarse_scan_and_finds_off_grid_substrings():
    rng = np.random.default_rng(14)
    ref = rng.integers(0, 4, 400).astype(np.uint8)
    N, m, k, stride = 40, 8, 5, 4
    W1 = mapping.n_windows(ref.shape[0], N, 1)
    Wc = mapping.n_windows(ref.shape[0], N, stride)
    head = ref[101:101 + N]               # start 101: not on the stride-4 grid
    x = rope.encode_raw(head, N, m)
    F1 = np.array([rope.fidelity(x, rope.encode_raw(ref[s:s + N], N, m), N) for s in range(W1)])
    # radius 0: the coarse windows' own scores, ids mapped to their starts
    got_i, got_f = mapping.refine_topk(F1, np.arange(Wc), stride, 0, k)
    ci, cf = _brute_topk(ref, head, N, m, k, stride)
    assert list(got_i) == [stride * j for j in ci]
    assert np.allclose(got_f, cf, atol=1e-12)
    # around the nearest coarse window (start 100) radius 2 reaches start 101,
    # an exact copy of the head: self-fidelity 1, ranked first
    got_i, got_f = mapping.refine_topk(F1, [25], stride, 2, 3)
    assert got_i[0] == 101 and abs(got_f[0] - 1.0) < 1e-12


def test_reverse_complement_definition():
    s = np.array([0, 0, 1, 2, 3, 1], dtype=np.uint8)          # AACGTC
    assert list(mapping.reverse_complement(s)) == [2, 0, 1, 2, 3, 3]   # GACGTT
    rng = np.random.default_rng(15)
    x = rng.integers(0, 4, 200).astype(np.uint8)
    assert np.array_equal(mapping.reverse_complement(mapping.reverse_complement(x)), x)


def test_reverse_strand_read_maps_back_with_fidelity_one():
    """A read taken from the other strand (the reverse complement of a
    reference substring) is found by mapping its reverse complement: F = 1 at
    the substring's start on strand 1, while its forward head scores low."""
    rng = np.random.default_rng(16)
    ref = rng.integers(0, 4, 600).astype(np.uint8)
    N, m, k = 40, 8, 4
    read = mapping.reverse_complement(ref[250:250 + 60])      # other strand, longer than N
    fwd_head = read[:N]
    rev_head = mapping.reverse_complement(read)[:N]          # = ref[250:290]
    fi, ff = mapping.map_reads(ref, fwd_head[None], N, m, k)
    ri, rf = mapping.map_reads(ref, rev_head[None], N, m, k)
    ids, F, strands = mapping.merge_strands(fi[0], ff[0], ri[0], rf[0], k)
    assert ids[0] == 250 and strands[0] == 1 and abs(F[0] - 1.0) < 1e-12
    assert ff[0, 0] < 0.5


def test_merge_strands_order_ties_and_threshold():
    ids, F, st = mapping.merge_strands([5, 9, -1], [0.9, 0.4, 0.0], [7, 5], [0.9, 0.6], 4)
    # equal F: lower id first, then forward before reverse on the same id
    assert list(ids) == [5, 7, 5, 9] and list(st) == [0, 1, 1, 0]
    ids, F, st = mapping.merge_strands([5, 9], [0.9, 0.4], [5, 2], [0.9, 0.3], 3)
    assert list(ids) == [5, 5, 9] and list(st) == [0, 1, 0]
    ids, F, st = mapping.merge_strands([5, 9], [0.9, 0.4], [7, 2], [0.6, 0.3], 4, min_fidelity=0.5)
    assert list(ids) == [5, 7] and list(st) == [0, 1]
    ids, F, st = mapping.merge_strands([5], [0.2], [7], [0.1], 4, min_fidelity=0.5)
    assert ids.size == 0                                      # unmapped
