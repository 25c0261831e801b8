"""Pins of the FP64 learned-offset oracle."""
import numpy as np
import pytest

import synth
from oracle import learned, lev, rope, stats


def test_parameter_count():
    assert learned.N_PARAMS == 10_432


def test_zero_output_layer_is_plain_encoding_of_trimmed_string():
    rng = np.random.default_rng(0)
    params = learned.init_params(1)                 # W2 = b2 = 0
    for n in (9, 40, 150, 173):
        w = rng.integers(0, 4, n)
        c, _ = learned.forward_string(params, w, 150)
        plain = rope.encode_raw(w[4:n - 4], 150, 32)
        assert np.max(np.abs(c - plain)) < 1e-12


def test_constant_offset_cancels_in_fidelity():
    # An offset that depends only on (letter, factor) multiplies component (k, L)
    # of both strings by the same unit number, leaving |<a|b>| unchanged.
    rng = np.random.default_rng(1)
    W1, b1, W2, b2 = learned.unpack(learned.init_params(2))
    b2 = rng.normal(0, 1, 128)
    params = learned.pack(W1, b1, W2, b2)
    plain = learned.init_params(2)
    a = rng.integers(0, 4, 150)
    b = a.copy()
    b[rng.choice(150, 15, replace=False)] = rng.integers(0, 4, 15)
    f1 = learned.pair_fidelities(params, [(a, b)], 150)
    f0 = learned.pair_fidelities(plain, [(a, b)], 150)
    assert abs(f1[0] - f0[0]) < 1e-12


def test_self_fidelity_one():
    rng = np.random.default_rng(3)
    params = learned.init_params(4)
    params[-200:] = rng.normal(0, 0.5, 200)
    w = rng.integers(0, 4, 150)
    assert abs(learned.pair_fidelities(params, [(w, w)], 150)[0] - 1) < 1e-12


def test_fidelity_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    ca = rng.normal(size=128) + 1j * rng.normal(size=128)
    cb = ca + 0.5 * (rng.normal(size=128) + 1j * rng.normal(size=128))
    F, Ga, Gb = learned.fidelity_and_grads(ca, cb)
    eps = 1e-6
    for vec, G, which in ((ca, Ga, 0), (cb, Gb, 1)):
        for m in rng.choice(128, 6, replace=False):
            for d in (1.0, 1j):
                v = vec.copy(); v[m] += eps * d
                fp = learned.fidelity_and_grads(v, cb)[0] if which == 0 else learned.fidelity_and_grads(ca, v)[0]
                v = vec.copy(); v[m] -= eps * d
                fm = learned.fidelity_and_grads(v, cb)[0] if which == 0 else learned.fidelity_and_grads(ca, v)[0]
                num = (fp - fm) / (2 * eps)
                ana = np.real(np.conj(G[m]) * d)
                assert abs(num - ana) < 1e-6


def test_ranking_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(6)
    F = rng.uniform(0, 1, 12)
    ld = rng.integers(0, 6, 12)
    loss, dF = learned.ranking_loss(F, ld)
    for i in range(12):
        e = np.zeros(12); e[i] = 1e-6
        num = (learned.ranking_loss(F + e, ld)[0] - learned.ranking_loss(F - e, ld)[0]) / 2e-6
        assert abs(num - dF[i]) < 1e-6


def test_parameter_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    params = learned.init_params(8)
    params[learned.N_HID * 33:] += rng.normal(0, 0.3, learned.N_PARAMS - learned.N_HID * 33)
    p = synth.mutate_pairs(6, 40, 8, seed=9)
    pairs = [p.pair(i) for i in range(p.n)]
    ld = lev.lev_many(p.a, p.a_off, p.b, p.b_off)
    loss, grad, _ = learned.batch_loss_and_grad(params, pairs, ld, 40)
    eps = 1e-5
    idx = np.concatenate([rng.choice(2048, 6, replace=False),            # W1
                          2048 + rng.choice(64, 3, replace=False),        # b1
                          2112 + rng.choice(8192, 8, replace=False),      # W2
                          10304 + rng.choice(128, 4, replace=False)])     # b2
    for i in idx:
        e = np.zeros(learned.N_PARAMS); e[i] = eps
        num = (learned.batch_loss(params + e, pairs, ld, 40) -
               learned.batch_loss(params - e, pairs, ld, 40)) / (2 * eps)
        assert abs(num - grad[i]) <= 1e-6 + 1e-4 * abs(num), (i, num, grad[i])


# ---- inference arithmetic and learned mapping -------------------------------

def test_bf16_round_matches_library_conversion_and_ties_to_even():
    import torch
    rng = np.random.default_rng(30)
    x = rng.normal(size=20000) * np.exp(rng.uniform(-30, 30, 20000))
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(learned.bf16_round(x), want)
    assert learned.bf16_round(1 + 2.0 ** -8) == 1.0                  # tie -> even (down)
    assert learned.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6    # tie -> even (up)
    assert learned.bf16_round(-(1 + 2.0 ** -7)) == -(1 + 2.0 ** -7)  # representable


def test_token_offsets_read_the_eight_flanks_in_order():
    # Identity first layer (hidden c = input c), output k of every letter block =
    # hidden k: delta_(p,k) is 1 exactly when flank k//4 of token p is letter k%4,
    # flanks being w[p], .., w[p+3], w[p+5], .., w[p+8].
    W1 = np.zeros((64, 32)); W1[np.arange(32), np.arange(32)] = 1.0
    W2 = np.zeros((128, 64))
    for L in range(4):
        W2[L * 32 + np.arange(32), np.arange(32)] = 1.0
    params = learned.pack(W1, np.zeros(64), W2, np.zeros(128))
    rng = np.random.default_rng(31)
    w = rng.integers(0, 4, 60)
    for bf16 in (False, True):
        mid, delta = learned.token_offsets(params, w, bf16)
        np.testing.assert_array_equal(mid, w[4:56])
        flank = [0, 1, 2, 3, 5, 6, 7, 8]
        for p in range(52):
            want = np.zeros(32)
            for i, o in enumerate(flank):
                want[4 * i + w[p + o]] = 1.0
            np.testing.assert_array_equal(delta[p], want)


def _trained_like_params(seed):
    rng = np.random.default_rng(seed)
    W1, b1, W2, b2 = learned.unpack(learned.init_params(seed))
    return learned.pack(W1, b1, rng.normal(0, 0.05, W2.shape), rng.normal(0, 0.4, 128))


def test_bf16_offsets_within_error_bound():
    params = _trained_like_params(32)
    w = np.random.default_rng(33).integers(0, 4, 3000)
    _, exact = learned.token_offsets(params, w, False)
    _, low = learned.token_offsets(params, w, True)
    bound = learned.offset_error_bound(params, w)
    assert np.all(np.abs(low - exact) <= bound)
    assert np.max(bound) < 0.05            # the bound is not vacuous
    assert np.max(np.abs(low - exact)) > 0  # and bf16 really rounds


def test_window_encodings_equal_whole_window_forward():
    params = _trained_like_params(34)
    ref = np.random.default_rng(35).integers(0, 4, 700)
    N = 150
    starts = np.array([0, 1, 77, 300, 550])
    C = learned.window_encodings(params, ref, starts, N, bf16=False)
    for i, s in enumerate(starts):
        c, _ = learned.forward_string(params, ref[s:s + N], N)
        assert np.max(np.abs(C[i] - c)) < 1e-11
    # zero output layer: the plain encoding of the window's token middles
    plain = learned.init_params(3)
    C0 = learned.window_encodings(plain, ref, starts, N, bf16=True)
    for i, s in enumerate(starts):
        assert np.max(np.abs(C0[i] - rope.encode_raw(ref[s + 4:s + N - 4], N, 32))) < 1e-11


def test_learned_mapping_finds_error_free_reads_with_fidelity_one():
    params = _trained_like_params(36)
    rng = np.random.default_rng(37)
    N = 150
    ref = rng.integers(0, 4, 3000)
    W = ref.shape[0] - N + 1
    true = rng.choice(W, 6, replace=False)
    heads = np.stack([ref[j:j + N] for j in true])
    idx, F = learned.map_reads(params, ref, heads, N, k=4, chunk=1000)
    np.testing.assert_array_equal(idx[:, 0], true)
    assert np.max(np.abs(F[:, 0] - 1.0)) < 1e-12
    assert np.all(F[:, 1] < 0.9)
    idx2, F2 = learned.map_reads(params, ref, heads, N, k=4, chunk=W)
    np.testing.assert_array_equal(idx, idx2)
    G = learned.head_window_fidelities(params, ref, heads, idx, N)
    assert np.max(np.abs(G - F)) < 1e-12


def test_token_offsets_blocking_changes_nothing():
    params = _trained_like_params(38)
    w = np.random.default_rng(39).integers(0, 4, 5000)
    for bf16 in (False, True):
        m1, d1 = learned.token_offsets(params, w, bf16)
        m2, d2 = learned.token_offsets(params, w, bf16, block=333)
        np.testing.assert_array_equal(m1, m2)
        np.testing.assert_array_equal(d1, d2)
