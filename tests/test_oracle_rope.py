"""Pins of the FP64 encoding oracle against what the paper and mathematics fix."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import rope
from synth import to_codes

GOLDEN = __file__.rsplit("/", 1)[0] + "/golden/"


def _rows(name):
    with open(GOLDEN + name) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def test_single_letters_small_exact():
    # N = 4: omega = i exactly; letter L at location L with factor 1 gives i^L;
    # with factor 2 gives (-1)^L (§2.1, §2.2).  Order is (k-1)*4 + letter (§2.10).
    c = rope.encode_raw([0, 1, 2, 3], N=4, m=2)
    want = np.array([1, 1j, -1, -1j, 1, -1, 1, -1])
    assert np.allclose(c, want, atol=1e-15)


def test_hamming_closed_form_golden():
    # §1: fidelity of quantum fingerprints is ((n-d)/n)^2; RoPE with s = 1 and
    # m = N integer factors equals it exactly.
    for a, b, d, frac in _rows("hamming_closed_form.txt"):
        a, b = to_codes(a), to_codes(b)
        n = len(a)
        assert int(d) == int(np.sum(a != b))
        want = float(Fraction(frac))
        got = rope.fidelity(rope.encode_raw(a, n, m=n), rope.encode_raw(b, n, m=n), n)
        assert abs(got - want) < 1e-12, (a, b, got, want)


@pytest.mark.parametrize("seed", range(5))
def test_hamming_closed_form_random_at_production_width(seed):
    # N = m = 32 gives 128 complex components, the production width.
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 4, 32)
    b = a.copy()
    d = int(rng.integers(0, 33))
    pos = rng.choice(32, d, replace=False)
    b[pos] = (b[pos] + rng.integers(1, 4, d)) % 4
    got = rope.fidelity(rope.encode_raw(a, 32, 32), rope.encode_raw(b, 32, 32), 32)
    assert abs(got - ((32 - d) / 32) ** 2) < 1e-12


def test_dimension():
    # §2.3: dimension m*4^s; 2s+q qubits when m = 2^q -> 128 components, 7 qubits.
    c = rope.encode(np.zeros(150, dtype=np.uint8) + np.arange(150) % 4, 150, 32)
    assert c.shape == (128,)
    assert 2 * 1 + int(math.log2(32)) == int(math.log2(c.shape[0]))


@pytest.mark.parametrize("schedule", ["default", "finetuned"])
def test_self_fidelity_is_one(schedule):
    rng = np.random.default_rng(1)
    for _ in range(20):
        w = rng.integers(0, 4, 150)
        c = rope.encode_raw(w, 150, 32, schedule)
        assert abs(rope.fidelity(c, c, 150) - 1.0) < 1e-13


@pytest.mark.parametrize("schedule", ["default", "finetuned"])
def test_two_formulations_agree(schedule):
    # §2.1/§2.2 location sums == §2.10 sum of D^loc applied to stretched one-hots.
    rng = np.random.default_rng(2)
    for N, m in [(10, 3), (37, 8), (150, 32)]:
        w = rng.integers(0, 4, N)
        a = rope.encode_raw(w, N, m, schedule)
        if schedule == "default":
            b = rope.encode_dloc(w, N, m)
        else:  # D built from the fine-tuned factors
            f = rope.frequencies(m, schedule)
            D = np.diag(np.kron(np.exp(2j * np.pi * f / N), np.ones(4)))
            b = np.zeros(4 * m, dtype=complex)
            Dp = np.eye(4 * m, dtype=complex)
            for L in w:
                b = b + Dp @ np.kron(np.ones(m), np.eye(4)[L])
                Dp = Dp @ D
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a)) + 1e-12


def test_finetuned_factors_span_one_to_three():
    # §3.3: the fine-tuned factor runs evenly from 1 (k = 1) to 3 (k = m).
    for m in (2, 4, 32):
        f = rope.frequencies(m, "finetuned")
        assert f[0] == 1.0 and abs(f[-1] - 3.0) < 1e-15
        assert np.allclose(np.diff(f), 2.0 / (m - 1))
    assert np.array_equal(rope.frequencies(32), np.arange(1, 33))


@pytest.mark.parametrize("schedule", ["default", "finetuned"])
def test_common_position_shift_leaves_inner_product(schedule):
    # Adding l to every location of both strings multiplies component (k, .) of
    # both by the same unit phase, so <x|c> is unchanged.
    rng = np.random.default_rng(3)
    a = rng.integers(0, 4, 150)
    b = a.copy()
    b[rng.choice(150, 20, replace=False)] = rng.integers(0, 4, 20)
    pos = np.arange(150)
    ip0 = np.vdot(rope.encode_raw(a, 150, 32, schedule), rope.encode_raw(b, 150, 32, schedule))
    for l in (1, 77, 12345):
        ip1 = np.vdot(rope.encode_raw(a, 150, 32, schedule, pos + l),
                      rope.encode_raw(b, 150, 32, schedule, pos + l))
        assert abs(ip1 - ip0) < 1e-9 * abs(ip0)


def test_cyclic_shift():
    # §2.5 with s = 1 and integer factors: c^(k)(dna_l) = c^(k)(dna) omega^(k l)
    # exactly, so m = 1 gives fidelity 1, and for m > 1 the mean over k of the
    # separately normalised per-factor fidelities is 1, while the concatenated
    # fidelity is not.
    rng = np.random.default_rng(4)
    N, m = 60, 8
    w = rng.integers(0, 4, N)
    for l in (1, 5, 17):
        wl = np.roll(w, l)
        assert abs(rope.fidelity(rope.encode_raw(w, N, 1), rope.encode_raw(wl, N, 1), N) - 1) < 1e-12
        a = rope.encode_raw(w, N, m).reshape(m, 4)
        b = rope.encode_raw(wl, N, m).reshape(m, 4)
        per_k = [rope.fidelity(a[k], b[k], N) for k in range(m)]
        assert abs(np.mean(per_k) - 1) < 1e-12
        assert rope.fidelity(a.reshape(-1), b.reshape(-1), N) < 0.99


def test_periodic_windows_are_zero_golden():
    for unit, reps, N, m in _rows("periodic_zero.txt"):
        w = np.tile(to_codes(unit), int(reps))
        N, m = int(N), int(m)
        assert w.shape[0] == N
        c = rope.encode_raw(w, N, m)
        assert np.max(np.abs(c)) < 1e-12
        assert rope.is_degenerate(c, N)
        x = rope.encode_raw(np.arange(N) % 4, N, m)
        assert rope.fidelity(x, c, N) == 0.0
        # one factor more than the bound makes it non-zero
        if m + 1 <= N and N % len(unit) == 0 and (m + 1) % (N // len(unit)) == 0:
            assert np.max(np.abs(rope.encode_raw(w, N, m + 1))) > 0.5


def test_letter_sum_identity():
    # For integer k not a multiple of N: sum_L c_{k,L} = sum_p omega^(k p) = 0.
    rng = np.random.default_rng(5)
    for _ in range(10):
        w = rng.integers(0, 4, 150)
        c = rope.encode_raw(w, 150, 32).reshape(32, 4)
        assert np.max(np.abs(c.sum(axis=1))) < 1e-12


@pytest.mark.parametrize("schedule", ["default", "finetuned"])
def test_sliding_rule_matches_direct(schedule):
    # §3.4: one-letter slides (including the matched case, outgoing == incoming
    # letter) reproduce the direct encoding of every window.
    rng = np.random.default_rng(6)
    ref = rng.integers(0, 4, 420)
    N, m = 60, 16
    count = ref.shape[0] - N + 1
    roll = rope.sliding_encodings(ref, N, count, m, schedule)
    direct = rope.encode_many(np.stack([ref[j:j + N] for j in range(count)]), N, m, schedule)
    matched = sum(1 for j in range(1, count) if ref[j - 1] == ref[j + N - 1])
    assert matched > 10
    assert np.max(np.abs(roll - direct)) < 1e-10


def test_sliding_inner_product_rule():
    # §3.4: ip_new = ip omega^-1 - conj(x_old) omega^-1 + conj(x_new) omega^(N-s), per k.
    rng = np.random.default_rng(7)
    ref = rng.integers(0, 4, 300)
    N, m = 50, 8
    x = rope.encode_raw(rng.integers(0, 4, N), N, m)
    ipk = rope.ip_per_factor(x, rope.encode_raw(ref[:N], N, m), m)
    for j in range(1, ref.shape[0] - N + 1):
        ipk = rope.slide_ip(ipk, x, int(ref[j - 1]), int(ref[j + N - 1]), N, m)
        direct = np.vdot(x, rope.encode_raw(ref[j:j + N], N, m))
        assert abs(ipk.sum() - direct) < 1e-9


def test_encode_many_matches_encode_raw():
    rng = np.random.default_rng(8)
    S = rng.integers(0, 4, (7, 150))
    many = rope.encode_many(S, 150, 32)
    for i in range(7):
        assert np.max(np.abs(many[i] - rope.encode_raw(S[i], 150, 32))) < 1e-11


def test_unrelated_strings_mean_fidelity():
    # Statistical check: unrelated uniform strings have mean fidelity close to
    # 1/(3m) (the four letter components of one factor are tied by the letter-sum
    # identity, leaving 3m effective complex dimensions).  Loose: 10%.
    rng = np.random.default_rng(9)
    A = rope.encode_many(rng.integers(0, 4, (1500, 150)), 150, 32)
    B = rope.encode_many(rng.integers(0, 4, (1500, 150)), 150, 32)
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    B /= np.linalg.norm(B, axis=1, keepdims=True)
    F = np.abs(np.sum(np.conj(A) * B, axis=1)) ** 2
    assert abs(F.mean() * 96 - 1) < 0.1
