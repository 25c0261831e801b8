"""GPU parity of the learned-offset kernels against the FP64 oracle, and of the
edit-distance kernel against the oracle's dynamic programme (bit-exact).

Tolerances (FP32 kernels vs FP64 oracle): an encoding component is a sum of at
most n unit terms, each with a phase error of a few FP32 ulps of an argument
below 2 pi plus the offset; the summation adds at most n * 2^-24 relative per
term, so |dc| <= 1e-5 * n bounds both with room.  Fidelities are ratios of such
sums: 1e-4 absolute.  Gradients: every parameter's gradient is a sum over
~10^4 token terms with cancellation, computed in FP32; the bound is relative to
the largest component, 2e-3 (elementwise) and 1e-3 (2-norm).
"""
import numpy as np
import pytest

import synth
from oracle import learned as OL
from oracle import lev, rope, stats

from gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu

N = 150


def _mod():
    from paper_2603_22245_amd import learned
    return learned


def _pack(seqs):
    off = np.zeros(len(seqs) + 1, np.int64)
    off[1:] = np.cumsum([len(s) for s in seqs])
    cat = np.concatenate(seqs).astype(np.uint8) if off[-1] else np.zeros(1, np.uint8)
    return cat, off


def _strings(rng, lengths):
    seqs = [rng.integers(0, 4, n).astype(np.uint8) for n in lengths]
    cat, off = _pack(seqs)
    return seqs, cat, off


def _to_complex(c):
    c = c.astype(np.float64)
    return c[:, 0::2] + 1j * c[:, 1::2]


def _random_params(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    W1, b1, W2, b2 = OL.unpack(OL.init_params(seed))
    W2 = rng.normal(0, scale / 8, W2.shape)
    b2 = rng.normal(0, scale, b2.shape)
    return OL.pack(W1, b1, W2, b2)


def test_levenshtein_bit_exact():
    torch = torch_cuda()
    M = _mod()
    P = synth.mutate_pairs(3000, 150, 30, seed=7)
    rng = np.random.default_rng(8)
    # edge cases: empty strings, single letters, word boundaries of the
    # bit-parallel pattern (63..65, 127..129, 255, 256), unrelated strings
    extra_a, extra_b = [], []
    for la, lb in [(0, 0), (0, 5), (5, 0), (1, 1), (1, 7), (63, 70), (64, 64), (65, 64),
                   (127, 140), (128, 128), (129, 200), (255, 256), (256, 256), (256, 300),
                   (300, 256), (20, 256), (200, 17)]:
        extra_a.append(rng.integers(0, 4, la).astype(np.uint8))
        b = rng.integers(0, 4, lb).astype(np.uint8)
        if lb and la:  # share a prefix so that distances are not trivial
            q = min(la, lb) // 2
            b[:q] = extra_a[-1][:q]
        extra_b.append(b)
    a = [P.pair(i)[0] for i in range(P.n)] + extra_a
    b = [P.pair(i)[1] for i in range(P.n)] + extra_b
    acat, aoff = _pack(a)
    bcat, boff = _pack(b)
    want = lev.lev_many(acat, aoff, bcat, boff)
    ps = M.upload_pairs(acat, aoff, bcat, boff)
    got = M.levenshtein(ps).cpu().numpy()
    np.testing.assert_array_equal(got, want)


def test_levenshtein_pattern_too_long_is_minus_one():
    torch = torch_cuda()
    M = _mod()
    rng = np.random.default_rng(9)
    a = rng.integers(0, 4, 300).astype(np.uint8)
    b = rng.integers(0, 4, 257).astype(np.uint8)
    ps = M.upload_pairs(a, np.array([0, 300]), b, np.array([0, 257]))
    assert int(M.levenshtein(ps).cpu()[0]) == -1


def test_plain_encoding_matches_oracle():
    torch = torch_cuda()
    M = _mod()
    rng = np.random.default_rng(10)
    lengths = [0, 1, 9, 64, 150, 151, 180, 400, 1000]
    seqs, cat, off = _strings(rng, lengths)
    c = M.encode(None, torch.from_numpy(cat).cuda(), torch.from_numpy(off).cuda(), len(seqs), N)
    got = _to_complex(c.cpu().numpy())
    for i, w in enumerate(seqs):
        want = rope.encode_raw(w, N, 32) if len(w) else np.zeros(128, complex)
        assert np.max(np.abs(got[i] - want)) <= 1e-5 * max(len(w), 1), i


def test_learned_encoding_matches_oracle():
    torch = torch_cuda()
    M = _mod()
    rng = np.random.default_rng(11)
    lengths = [0, 8, 9, 10, 120, 150, 173, 256, 300]
    seqs, cat, off = _strings(rng, lengths)
    params = _random_params(12)
    p = torch.from_numpy(params.astype(np.float32)).cuda()
    c = M.encode(p, torch.from_numpy(cat).cuda(), torch.from_numpy(off).cuda(), len(seqs), N)
    got = _to_complex(c.cpu().numpy())
    p32 = params.astype(np.float32).astype(np.float64)  # the kernel sees FP32 parameters
    for i, w in enumerate(seqs):
        w = w[:256]  # strings are cut at the kernel's maximum length
        want, _ = OL.forward_string(p32, w, N)
        assert np.max(np.abs(got[i] - want)) <= 1e-5 * max(len(w), 1), i


def test_zero_output_layer_is_plain_encoding_of_token_middles():
    torch = torch_cuda()
    M = _mod()
    rng = np.random.default_rng(13)
    seqs, cat, off = _strings(rng, [9, 40, 150, 177])
    params = torch.from_numpy(OL.init_params(3).astype(np.float32)).cuda()
    c = M.encode(params, torch.from_numpy(cat).cuda(), torch.from_numpy(off).cuda(), len(seqs), N)
    mids = [w[4:len(w) - 4] for w in seqs]
    mcat, moff = _pack(mids)
    cp = M.encode(None, torch.from_numpy(mcat).cuda(), torch.from_numpy(moff).cuda(), len(mids), N)
    assert torch.max(torch.abs(c - cp)).item() <= 1e-5 * 177


def test_pair_fidelity_matches_oracle():
    torch = torch_cuda()
    M = _mod()
    P = synth.mutate_pairs(200, 150, 30, seed=14)
    params = _random_params(15)
    ps = M.upload_pairs(P.a, P.a_off, P.b, P.b_off)
    p = torch.from_numpy(params.astype(np.float32)).cuda()
    F = M.pair_fidelity(p, ps, N).cpu().numpy()
    pairs = [P.pair(i) for i in range(P.n)]
    want = OL.pair_fidelities(params.astype(np.float32).astype(np.float64), pairs, N)
    assert np.max(np.abs(F - want)) <= 1e-4
    Fp = M.pair_fidelity(None, ps, N).cpu().numpy()
    want_p = np.array([abs(np.vdot(rope.encode_raw(a, N, 32), rope.encode_raw(b, N, 32))) ** 2 /
                       (np.sum(np.abs(rope.encode_raw(a, N, 32)) ** 2) *
                        np.sum(np.abs(rope.encode_raw(b, N, 32)) ** 2)) for a, b in pairs])
    assert np.max(np.abs(Fp - want_p)) <= 1e-4


@pytest.mark.parametrize("n_pairs", [2, 96, 1024])
def test_gradient_matches_oracle(n_pairs):
    torch = torch_cuda()
    M = _mod()
    P = synth.mutate_pairs(n_pairs, 150, 30, seed=16 + n_pairs)
    ld = lev.lev_many(P.a, P.a_off, P.b, P.b_off)
    if n_pairs == 2 and ld[0] == ld[1]:
        ld = np.array([ld[0], ld[0] + 1])
    params = _random_params(17).astype(np.float32)
    tr = M.Trainer(params=params, batch=max(n_pairs, 2))
    ps = M.upload_pairs(P.a, P.a_off, P.b, P.b_off, ld)
    loss, grad = tr.gradient(ps)
    loss = float(loss.cpu()[0]); grad = grad.cpu().numpy().astype(np.float64)
    pairs = [P.pair(i) for i in range(P.n)]
    want_loss, want_grad, _ = OL.batch_loss_and_grad(params.astype(np.float64), pairs, ld, N)
    assert abs(loss - want_loss) <= 1e-4 * max(1.0, abs(want_loss))
    scale = np.max(np.abs(want_grad))
    assert scale > 0
    assert np.max(np.abs(grad - want_grad)) <= 2e-3 * scale
    assert np.linalg.norm(grad - want_grad) <= 1e-3 * np.linalg.norm(want_grad)


def test_three_adam_steps_match_oracle():
    """Three device training steps (rm_learned_train_step: loss, gradient and
    Adam update on the GPU) on three consecutive batches, against three steps
    of the FP64 oracle (oracle.learned.batch_loss_and_grad, then
    oracle.learned.adam_step) from the same parameters on the same batches.
    The device keeps [params | m | v | step] in FP32; each is compared with
    the oracle's.  Tolerances: the gradients agree to 2e-3 of their largest
    component (the gradient test's bound), so m (a weighted sum of the three
    gradients with weights summing below 1) agrees to 2e-3 of the largest
    gradient component and v (weights summing below 0.003, squares) to
    1.2e-5 of the largest squared component; the update lr * m_hat /
    (sqrt(v_hat) + eps) is checked elementwise to 1e-4 * lr per step wherever
    every step's gradient component exceeds 1e-3 of that step's largest (a
    smaller component's direction is rounding noise), and every parameter's
    move is bounded by the largest Adam can make in three steps."""
    torch = torch_cuda()
    M = _mod()
    steps, batch, lr = 3, 128, 1e-2
    P = synth.mutate_pairs(steps * batch, 150, 30, seed=20)
    ld = lev.lev_many(P.a, P.a_off, P.b, P.b_off)
    params = _random_params(21).astype(np.float32)
    tr = M.Trainer(params=params, batch=batch, lr=lr)
    ps = M.upload_pairs(P.a, P.a_off, P.b, P.b_off, ld)
    losses = tr.epoch(ps).cpu().numpy()
    torch.cuda.synchronize()
    state = tr.state.cpu().numpy().astype(np.float64)
    n = OL.N_PARAMS
    th, m, v, t = params.astype(np.float64), np.zeros(n), np.zeros(n), 0
    big = np.ones(n, dtype=bool)
    gmax = 0.0
    for s in range(steps):
        pairs = [P.pair(i) for i in range(s * batch, (s + 1) * batch)]
        want_loss, g, _ = OL.batch_loss_and_grad(th, pairs, ld[s * batch:(s + 1) * batch], N)
        assert abs(float(losses[s]) - want_loss) <= 1e-4 * max(1.0, want_loss), s
        big &= np.abs(g) > 1e-3 * np.max(np.abs(g))
        gmax = max(gmax, float(np.max(np.abs(g))))
        th, m, v, t = OL.adam_step(th, m, v, t, g, lr)
    assert state[-1] == float(t) == 3.0
    assert big.mean() > 0.5
    assert np.max(np.abs(state[n:2 * n] - m)) <= 2e-3 * gmax
    assert np.max(np.abs(state[2 * n:3 * n] - v)) <= 1.2e-5 * gmax ** 2
    d = np.abs(state[:n] - th)
    assert np.max(d[big]) <= steps * 1e-4 * lr + 1e-7
    # m_hat = sum_s a_s g_s and v_hat = sum_s b_s g_s^2 with bias-corrected weights, so by
    # Cauchy-Schwarz |m_hat| / sqrt(v_hat) <= sqrt(sum_s a_s^2 / b_s): 1, 1.0014 and 1.0036
    # at steps 1, 2, 3, and no parameter moves more than 3.006 lr in three steps
    assert np.max(np.abs(state[:n] - params)) <= 3.006 * lr + 1e-6


def test_graph_epoch_equals_eager_epoch():
    torch = torch_cuda()
    M = _mod()
    P = synth.mutate_pairs(1024, 150, 30, seed=22)
    ld = lev.lev_many(P.a, P.a_off, P.b, P.b_off)
    ps = M.upload_pairs(P.a, P.a_off, P.b, P.b_off, ld)
    eager = M.Trainer(seed=5, batch=256)
    graph = M.Trainer(seed=5, batch=256)
    for rep in range(3):
        le = eager.epoch(ps).clone()
        lg = graph.epoch(ps, graph=True).clone()
        torch.cuda.synchronize()
        # every kernel of a step is deterministic: replays equal eager runs bit for bit
        assert torch.equal(eager.state, graph.state), rep
        assert torch.equal(le, lg), rep
    assert float(graph.state[-1].cpu()) == 12.0
    graph.close()


def test_training_lowers_loss_and_beats_plain_spearman():
    """The learned encoding's gain over the plain one has no value in the paper
    (parity unpinned); the test asks only that training lowers the loss and
    that held-out Spearman correlation with -LD exceeds the plain encoding's."""
    torch = torch_cuda()
    M = _mod()
    P = synth.mutate_pairs(24576, 150, 30, seed=23)
    ld = lev.lev_many(P.a, P.a_off, P.b, P.b_off)
    tr_set = M.upload_pairs(P.a, P.a_off, P.b, P.b_off, ld)
    ho = synth.mutate_pairs(4096, 150, 30, seed=24)
    ho_ld = lev.lev_many(ho.a, ho.a_off, ho.b, ho.b_off)
    ho_set = M.upload_pairs(ho.a, ho.a_off, ho.b, ho.b_off)
    # GPU labels agree with the oracle's
    np.testing.assert_array_equal(M.levenshtein(ho_set).cpu().numpy(), ho_ld)
    t = M.Trainer(seed=1, batch=512, lr=3e-3)
    first = None
    for ep in range(4):
        losses = t.epoch(tr_set, graph=True).cpu().numpy()
        if first is None:
            first = losses[:8].mean()
    last = losses[-8:].mean()
    assert last < 0.8 * first
    F_l = M.pair_fidelity(t.params, ho_set, N).cpu().numpy()
    F_p = M.pair_fidelity(None, ho_set, N).cpu().numpy()
    rho_l = -stats.spearman(F_l, ho_ld)
    rho_p = -stats.spearman(F_p, ho_ld)
    print(f"held-out Spearman: learned {rho_l:.4f}, plain {rho_p:.4f}")
    assert rho_l > rho_p + 0.02
    t.close()
