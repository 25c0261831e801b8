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
