"""Pins of the FP64 oracle of the §2.4 correlation score (oracle.correlation)."""
import numpy as np

import synth
from oracle import correlation as C
from oracle import rope


def test_hand_worked_two_rates():
    """Rates 0.1 and 0.3 with fidelities (0.8, 0.6) and (0.3, 0.1): E_fid =
    0.7 and 0.2, so the curve joins (0.2, 0.3) and (0.7, 0.1).  Rate 0.1:
    fid 0.8 lies past the last point (err 0.1, distance 0); fid 0.6 lies 0.8
    of the way along the segment, err 0.3 - 0.8 * 0.2 = 0.14, distance 0.04:
    RMSE = sqrt(0.04^2 / 2) = 0.0282843.  Rate 0.3: fid 0.3 gives err 0.26
    (distance 0.04), fid 0.1 lies before the first point (err 0.3, distance 0):
    the same RMSE."""
    E, curve, rmse = C.score([0.1, 0.3], [[0.8, 0.6], [0.3, 0.1]])
    np.testing.assert_allclose(E, [0.7, 0.2], atol=1e-15)
    np.testing.assert_allclose(curve[0], [0.2, 0.7], atol=1e-15)
    np.testing.assert_allclose(curve[1], [0.3, 0.1], atol=1e-15)
    assert abs(C.curve_err(curve, 0.6) - 0.14) < 1e-15
    assert abs(C.curve_err(curve, 0.3) - 0.26) < 1e-15
    np.testing.assert_allclose(rmse, [0.028284271247461901] * 2, rtol=1e-12)


def test_points_are_ordered_by_expected_fidelity():
    """E_fid need not fall monotonically with err: rates 0.1, 0.2, 0.3 with
    E_fid 0.5, 0.6, 0.1 give the curve (0.1, 0.3) - (0.5, 0.1) - (0.6, 0.2), so
    fid 0.55 maps to 0.15 and fid 0.3 to 0.2."""
    curve = C.fitting_curve([0.1, 0.2, 0.3], [0.5, 0.6, 0.1])
    assert abs(C.curve_err(curve, 0.55) - 0.15) < 1e-15
    assert abs(C.curve_err(curve, 0.3) - 0.2) < 1e-15
    assert C.curve_err(curve, 0.05) == 0.3 and C.curve_err(curve, 0.9) == 0.2


def test_exact_function_of_the_rate_has_zero_rmse():
    err = (np.arange(25) + 0.5) * 0.5 / 25
    fids = [np.full(7, (1 - e) ** 3) for e in err]
    E, _, rmse = C.score(err, fids)
    np.testing.assert_allclose(E, (1 - err) ** 3, rtol=1e-15)
    assert np.max(rmse) < 1e-15


def test_plain_pair_fidelity_of_substitutions_is_the_hamming_closed_form():
    """With m = N factors the plain fidelity of two equal-length strings at
    Hamming distance d is ((N - d) / N)^2 (§1)."""
    rng = np.random.default_rng(50)
    N = 24
    pairs, want = [], []
    for d in range(0, 13, 3):
        a = rng.integers(0, 4, N)
        b = a.copy()
        pos = rng.choice(N, d, replace=False)
        b[pos] = (b[pos] + rng.integers(1, 4, d)) % 4
        pairs.append((a, b))
        want.append(((N - d) / N) ** 2)
    np.testing.assert_allclose(C.plain_pair_fidelities(pairs, N, m=N), want, atol=1e-12)


def test_plain_pair_fidelity_matches_encodings_of_unequal_strings():
    """Pairs of the §2.4 protocol have unequal lengths after insertions and
    deletions: F is taken between the whole strings' encodings at the nominal
    N (the direct sum of §2.1 and the §2.10 matrix-power form agree)."""
    P = synth.mutate_pairs(3, 20, 10, seed=51)
    pairs = [P.pair(i) for i in range(P.n)]
    got = C.plain_pair_fidelities(pairs, 20, m=8)
    for (a, b), f in zip(pairs, got):
        ca, cb = rope.encode_dloc(a, 20, 8), rope.encode_dloc(b, 20, 8)
        assert abs(f - abs(np.vdot(ca, cb)) ** 2 / (rope.sq_norm(ca) * rope.sq_norm(cb))) < 1e-12
        assert 0.0 <= f <= 1.0 + 1e-12
