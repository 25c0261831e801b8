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


# ---- hand-worked values of the loss and of the optimiser ----------------------

def test_ranking_loss_hand_worked_four_pairs():
    """F = (0.9, 0.5, 0.4, 0.6), labels (1, 3, 2, 3).  The ordered pairs with
    d_i < d_j are (0,1), (0,2), (0,3), (2,1), (2,3); (1,3) is a label tie and
    does not count, and (2,1) is ranked the wrong way (F_2 < F_1 although
    d_2 < d_1).  F_i - F_j = 0.4, 0.5, 0.3, -0.1, -0.2, so with tau = 0.05 the
    softplus arguments -(F_i - F_j)/tau are -8, -10, -6, 2, 4 and
      loss = (ln(1+e^-8) + ln(1+e^-10) + ln(1+e^-6) + ln(1+e^2) + ln(1+e^4)) / 5
           = (0.000335406 + 0.0000453989 + 0.00247569 + 2.12692801 + 4.01814993) / 5
           = 1.22958688587.
    dloss/dF_i sums sigma(z)/(tau * 5) with sign -1 where i is the lower-label
    member of a pair and +1 where it is the higher one:
      dF_0 = -(sigma(-8) + sigma(-10) + sigma(-6)) / 0.25 = -0.0114134846
      dF_1 = (sigma(-8) + sigma(2)) / 0.25             =  3.52452971
      dF_2 = (sigma(-10) - sigma(2) - sigma(4)) / 0.25  = -7.45106188
      dF_3 = (sigma(-6) + sigma(4)) / 0.25             =  3.93794565
    A flipped sign or a reversed label mask gives 4.83; counting the tie adds
    a sixth pair."""
    loss, dF = learned.ranking_loss(np.array([0.9, 0.5, 0.4, 0.6]), np.array([1, 3, 2, 3]))
    assert abs(loss - 1.2295868858741251) < 1e-13
    np.testing.assert_allclose(dF, [-0.011413484623214747, 3.5245297124333957,
                                    -7.451061880588354, 3.9379456527781729],
                               rtol=1e-12, atol=1e-15)


def test_ranking_loss_no_ordered_pair_is_zero():
    loss, dF = learned.ranking_loss(np.array([0.3, 0.8, 0.1]), np.array([2, 2, 2]))
    assert loss == 0.0 and np.all(dF == 0.0)


def test_adam_two_steps_hand_worked_default_constants():
    """theta_0 = 1, lr = 0.1, gradients 0.5 then -1 (beta 0.9 / 0.999, eps 1e-8).
    Step 1: m = 0.05, v = 0.00025, m_hat = 0.05/0.1 = 0.5, v_hat =
    0.00025/0.001 = 0.25, theta_1 = 1 - 0.1 * 0.5 / (0.5 + 1e-8) = 0.900000002.
    Step 2: m = 0.045 - 0.1 = -0.055, v = 0.00024975 + 0.001 = 0.00124975,
    m_hat = -0.055/0.19 = -0.289473684, v_hat = 0.00124975/0.001999 =
    0.625187594, theta_2 = theta_1 + 0.1 * 0.289473684 / 0.790688 = 0.936610354."""
    th, m, v, t = learned.adam_step(np.array([1.0]), np.zeros(1), np.zeros(1), 0,
                                    np.array([0.5]), 0.1)
    assert t == 1 and abs(m[0] - 0.05) < 1e-16 and abs(v[0] - 0.00025) < 1e-18
    assert abs(th[0] - 0.90000000199999996) < 1e-15
    th, m, v, t = learned.adam_step(th, m, v, t, np.array([-1.0]), 0.1)
    assert t == 2 and abs(m[0] + 0.055) < 1e-16 and abs(v[0] - 0.00124975) < 1e-17
    assert abs(th[0] - 0.93661035424056560) < 1e-14


def test_adam_two_steps_hand_worked_closed_form():
    """beta1 = beta2 = 0.5, eps = 0, lr = 1, theta_0 = 0, gradients 2 then 4.
    Step 1: m = 1, v = 2, m_hat = 2, v_hat = 4: theta_1 = -2/2 = -1.
    Step 2: m = 0.5 + 2 = 2.5, v = 1 + 8 = 9, m_hat = 2.5/0.75 = 10/3,
    v_hat = 9/0.75 = 12: theta_2 = -1 - (10/3)/sqrt(12) = -1 - 5 sqrt(3)/9.
    Without the bias corrections step 2 would move by 2.5/3 instead."""
    kw = dict(beta1=0.5, beta2=0.5, eps=0.0)
    th, m, v, t = learned.adam_step(np.zeros(1), np.zeros(1), np.zeros(1), 0, np.array([2.0]),
                                    1.0, **kw)
    assert th[0] == -1.0 and m[0] == 1.0 and v[0] == 2.0
    th, m, v, t = learned.adam_step(th, m, v, t, np.array([4.0]), 1.0, **kw)
    assert m[0] == 2.5 and v[0] == 9.0 and t == 2
    assert abs(th[0] - (-1.0 - 5.0 * np.sqrt(3.0) / 9.0)) < 1e-15


def test_adam_constant_gradient_moves_lr_per_step():
    """With the same gradient g at every step the bias-corrected moments are
    exactly m_hat = g and v_hat = g^2, so each step moves every parameter by
    lr * g / (|g| + eps), whatever the step count."""
    rng = np.random.default_rng(40)
    g = rng.normal(size=50) * np.exp(rng.uniform(-5, 5, 50))
    th = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    t = 0
    for step in range(1, 8):
        prev = th
        th, m, v, t = learned.adam_step(th, m, v, t, g, 0.01)
        np.testing.assert_allclose(prev - th, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        assert t == step
