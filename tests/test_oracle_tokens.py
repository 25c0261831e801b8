"""Pins of the s-mer token oracle (oracle.tokens) against what the paper and
the mathematics fix: the s = 1 case of §2.1-§2.3 (oracle.rope, pinned on its
own), the §2.10 matrix-power formulation, a closed-form geometric sum, brute
force over token locations found by string slicing, the §3.4 slide and the
rolling inner product against direct encoding, linearity of the compact map (§2.6) and exact-substring
mapping (§3.1)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import mapping, rope, tokens

RNG = np.random.default_rng(11)


def _rand(n, rng=RNG):
    return rng.integers(0, 4, n).astype(np.uint8)


@pytest.mark.parametrize("schedule", ["default", "finetuned"])
def test_single_letters_reduce_to_the_letter_encoding(schedule):
    w = _rand(150)
    got = tokens.encode_raw(w, 150, 1, 32, 4, schedule=schedule)
    want = rope.encode_raw(w, 150, 32, schedule)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("s,m,C,with_map", [(2, 8, 16, False), (3, 2, 64, False),
                                             (4, 8, 16, True), (5, 4, 8, True)])
def test_matrix_power_formulation(s, m, C, with_map):
    """§2.10: sum_loc D^loc (ones(m) (x) onehot(class)), with a letter outside
    0..3 in the string (its tokens add nothing) and, for the compact case, a
    map that leaves some s-mers out."""
    N = 40
    w = _rand(N)
    w[17] = 4
    tm = None
    if with_map:
        tm = synth.token_map(s, C).astype(np.int64)
        tm[::7] = tokens.SKIP
    a = tokens.encode_raw(w, N, s, m, C, tm)
    b = tokens.encode_dloc(w, N, s, m, C, tm)
    assert np.max(np.abs(a - b)) < 1e-11 * N


@pytest.mark.parametrize("s,m,n", [(2, 8, 150), (3, 2, 150), (6, 5, 97), (8, 3, 8)])
def test_sum_over_classes_is_a_geometric_series(s, m, n):
    """With every s-mer its own class, summing a factor's components over the
    classes gives sum_{p=0}^{n-s} omega^(k p) = (1 - omega^(k (n-s+1))) / (1 - omega^k):
    one term per location 0..n-s (§2.1)."""
    N = 150
    w = _rand(n)
    c = tokens.encode_raw(w, N, s, m, 4 ** s).reshape(m, 4 ** s)
    k = np.arange(1, m + 1)
    om = np.exp(2j * np.pi * k / N)
    want = (1 - om ** (n - s + 1)) / (1 - om)
    assert np.max(np.abs(c.sum(axis=1) - want)) < 1e-11 * n


@pytest.mark.parametrize("s", [1, 2, 3])
def test_brute_force_over_token_locations(s):
    """Component (k, mer) = sum of omega^(k loc) over the locations where the
    string, sliced as text, reads `mer`; mers enumerated in lexicographic order
    over A,C,G,T (the code reading: first letter most significant)."""
    N, m = 23, 3
    w = _rand(N)
    text = synth.to_string(w)
    c = tokens.encode_raw(w, N, s, m, 4 ** s).reshape(m, 4 ** s)
    for code, mer in enumerate(itertools.product("ACGT", repeat=s)):
        mer = "".join(mer)
        locs = [p for p in range(N - s + 1) if text[p:p + s] == mer]
        for k in range(1, m + 1):
            want = sum(np.exp(2j * np.pi * k * p / N) for p in locs)
            assert abs(c[k - 1, code] - want) < 1e-12


@pytest.mark.parametrize("s,m,C,schedule,with_map", [(2, 8, 16, "default", False),
                                                      (3, 2, 64, "finetuned", False),
                                                      (5, 4, 8, "default", True),
                                                      (8, 8, 16, "finetuned", True)])
def test_slide_matches_direct_encoding(s, m, C, schedule, with_map):
    """§3.4 with s-mers: the slid state equals the direct encoding of every
    window, including slides whose outgoing and incoming tokens coincide
    (a run of one letter) and slides over a letter outside 0..3."""
    N = 31
    ref = _rand(260)
    ref[100:140] = 2                      # a run: old and new tokens coincide
    ref[200] = 4
    tm = synth.token_map(s, C).astype(np.int64) if with_map else None
    if with_map:
        tm[1::5] = tokens.SKIP
    count = ref.size - N + 1
    roll = tokens.sliding_encodings(ref, N, count, s, m, C, tm, schedule)
    direct = np.stack([tokens.encode_raw(ref[j:j + N], N, s, m, C, tm, schedule)
                       for j in range(count)])
    assert np.max(np.abs(roll - direct)) < 1e-10
    cls = tokens.token_classes(ref, s, tm)
    coincide = [j for j in range(1, count) if cls[j - 1] == cls[j + N - s] >= 0]
    assert coincide


def test_compact_map_sums_the_codes_it_merges():
    """A 4^s-to-C map (§2.6) adds the components of the s-mers it merges:
    c_map[k, q] = sum over codes with map[code] = q of c_identity[k, code]."""
    s, m, C, N = 4, 8, 16, 150
    w = _rand(N)
    tm = synth.token_map(s, C).astype(np.int64)
    tm[3] = tokens.SKIP
    a = tokens.encode_raw(w, N, s, m, C, tm).reshape(m, C)
    ident = tokens.encode_raw(w, N, s, m, 4 ** s).reshape(m, 4 ** s)
    want = np.zeros((m, C), dtype=np.complex128)
    for code in range(4 ** s):
        if tm[code] >= 0:
            want[:, tm[code]] += ident[:, code]
    assert np.max(np.abs(a - want)) < 1e-11


def test_fidelity_invariants():
    """Self fidelity 1; relabelling classes by a bijection changes no fidelity
    (a permutation of components); fidelity lies in [0, 1]."""
    s, m, C, N = 2, 8, 16, 150
    a, b = _rand(N), _rand(N)
    perm = RNG.permutation(C)
    for tm in (None, perm):
        x = tokens.encode_raw(a, N, s, m, C, tm)
        assert abs(rope.fidelity(x, x, N) - 1.0) < 1e-12
    f0 = rope.fidelity(tokens.encode_raw(a, N, s, m, C), tokens.encode_raw(b, N, s, m, C), N)
    f1 = rope.fidelity(tokens.encode_raw(a, N, s, m, C, perm),
                       tokens.encode_raw(b, N, s, m, C, perm), N)
    assert abs(f0 - f1) < 1e-12 and 0.0 <= f0 <= 1.0


def test_encode_many_matches_encode_raw():
    s, m, C, N = 3, 2, 64, 150
    strings = np.stack([_rand(N) for _ in range(5)])
    strings[2, 40] = 7
    many = tokens.encode_many(strings, N, s, m, C)
    one = np.stack([tokens.encode_raw(w, N, s, m, C) for w in strings])
    assert np.max(np.abs(many - one)) < 1e-11


@pytest.mark.parametrize("s,m,C,with_map", [(2, 8, 16, False), (8, 8, 16, True)])
def test_exact_substring_reads_map_to_their_window(s, m, C, with_map):
    """§3.1: a read head equal to the reference window at j has F = 1 there,
    and every top-1 window reads the same letters (up to identical windows)."""
    N, stride = 150, 1
    ref = _rand(3000)
    tm = synth.token_map(s, C) if with_map else None
    starts = np.array([0, 17, 1234, 3000 - N])
    heads = np.stack([ref[j:j + N] for j in starts])
    idx, F = tokens.map_reads(ref, heads, N, s, m, C, tm, k=4, stride=stride, chunk=700)
    assert np.all(np.abs(F[:, 0] - 1.0) < 1e-12)
    assert list(idx[:, 0]) == list(starts)
    # the same, one pair at a time
    Fp = tokens.pair_fidelities(ref, heads, idx, N, s, m, C, tm, stride)
    assert np.max(np.abs(Fp - F)) < 1e-12
    # and the brute force agrees with encoding every window one by one
    W = mapping.n_windows(ref.size, N, stride)
    x = tokens.encode(heads[1], N, s, m, C, tm)
    allF = np.array([abs(np.vdot(x, tokens.encode(ref[j:j + N], N, s, m, C, tm))) ** 2
                     for j in range(0, W, 37)])
    assert np.max(allF) <= F[1, 0] + 1e-12


@pytest.mark.parametrize("name", sorted(synth.TOKEN_ENCODINGS))
def test_window_encodings_gathered_from_the_reference(name):
    """encode_windows (the reference's tokens found once, gathered per window)
    equals encoding each window's letters, unknown letters included."""
    s, m, C, tm, sched = synth.token_encoding(name)
    ref = _rand(2_000)
    ref[[10, 500, 501, 1999]] = 4
    N, stride = 60, 3
    starts = mapping.window_starts(ref.size, N, stride)
    a = tokens.encode_windows(ref, starts, N, s, m, C, tm, sched)
    b = tokens.encode_many(mapping.window_letters(ref, starts, N), N, s, m, C, tm, sched)
    assert np.max(np.abs(a - b)) < 1e-12


def test_mer_counts_by_slicing_text():
    """Counts of every s-mer found by sliding over the text, letter code 4
    breaking the s-mers that contain it."""
    ref = _rand(300)
    ref[[40, 41, 200]] = 4
    text = "".join("ACGTN"[v] for v in ref)
    for s in (1, 2, 3):
        got = tokens.mer_counts(ref, s)
        for code, mer in enumerate(itertools.product("ACGT", repeat=s)):
            mer = "".join(mer)
            want = sum(1 for p in range(len(text) - s + 1) if text[p:p + s] == mer)
            assert got[code] == want, (s, mer)


def test_frequent_map_by_hand():
    """A reference whose 2-mer counts are known: the kept 2-mers are the most
    frequent, ties broken by the lower code, classes in code order."""
    # AAAAA: AA x4; then CACACA: AC x1, CA x3, AC x2 (total AC 3); GT once
    ref = synth.to_codes("AAAAACACACAGT")
    counts = tokens.mer_counts(ref, 2)
    code = lambda m: 4 * "ACGT".index(m[0]) + "ACGT".index(m[1])
    assert counts[code("AA")] == 4 and counts[code("AC")] == 3 and counts[code("CA")] == 3
    assert counts[code("AG")] == 1 and counts[code("GT")] == 1
    mp = tokens.frequent_map(ref, 2, 4)
    # AA (4), AC (3), CA (3), then the lowest code among the count-1 2-mers: AG
    kept = {m: mp[code(m)] for m in ("AA", "AC", "AG", "CA")}
    assert kept == {"AA": 0, "AC": 1, "AG": 2, "CA": 3}
    assert np.sum(mp >= 0) == 4 and mp[code("GT")] == tokens.SKIP
    # more classes than distinct 2-mers present: unseen codes fill by code order
    mp = tokens.frequent_map(ref, 2, 8)
    assert np.sum(mp >= 0) == 8 and sorted(mp[mp >= 0].tolist()) == list(range(8))


@pytest.mark.parametrize("name", ["s8c256", "s4m4"])
def test_rolling_inner_product_over_slides(name):
    """§3.4's rolling inner product, the form the 1,024-component refinement
    uses: with u the first window's components (locations counted from its
    start), u losing omega^(f i) at the class of each token that leaves and
    gaining omega^(f (i + T)) at the class of each token that enters, window i
    is omega^(-f i) u, so <x|c_i> = sum_k omega^(-f_k i) P_k with P_k the
    factor-k part of <x|u>, and |c_i|^2 = |u|^2.  Checked against the direct
    encodings of every window for 14 slides."""
    s, m, C, tm, sched = synth.token_encoding(name)
    N = 150
    T = N - s + 1
    rng = np.random.default_rng(21)
    ref = _rand(600, rng)
    x = tokens.encode_raw(_rand(N, rng), N, s, m, C, tm, sched).reshape(m, C)
    lo = 200
    u = tokens.encode_raw(ref[lo:lo + N], N, s, m, C, tm, sched).reshape(m, C)
    cls = tokens.token_classes(ref, s, tm)
    step = rope.unit_phases(N, m, np.array([1]), sched)[0]      # omega^(f_k)
    for i in range(15):
        c = tokens.encode_raw(ref[lo + i:lo + i + N], N, s, m, C, tm, sched).reshape(m, C)
        wt = step ** i
        P = np.sum(np.conj(x) * u, axis=1)
        assert np.isclose(np.sum(np.conj(wt) * P), np.vdot(x, c), rtol=0, atol=1e-9)
        assert np.isclose(np.sum(np.abs(u) ** 2), np.sum(np.abs(c) ** 2), rtol=1e-12)
        o, n = cls[lo + i], cls[lo + i + T]
        if 0 <= o < C:
            u[:, o] -= wt
        if 0 <= n < C:
            u[:, n] += wt * step ** T
