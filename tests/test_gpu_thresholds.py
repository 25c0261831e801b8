"""Per-fragment thresholds (§3.3) and the threshold regime (§3.5) on the GPU
against the FP64 oracle (oracle.thresholds).

Tolerances: a threshold is one window-copy fidelity (an order statistic), an
FP32 ratio of direct sums of at most N unit terms: 1e-5.  Regime decisions
F >= cut are taken in FP32 on the GPU and in FP64 by the oracle, so windows
whose oracle F lies within 1e-5 of the cut may fall either way; every other
decision must agree, the hits must be ranked as the oracle ranks them (up to
ties within 1e-5) and their FP32 scores lie within 2e-6 of the oracle's."""
import numpy as np
import pytest

import synth
from oracle import mapping, rope
from oracle import thresholds as OT

from gpu_helpers import oracle_heads, oracle_windows, torch_cuda

pytestmark = pytest.mark.gpu

TAU = 1e-5


@pytest.fixture(scope="module")
def plain_data():
    w = synth.WORKLOADS["plain"]
    ref = w.reference()
    reads = w.reads(ref)
    return ref, reads, mapping.read_heads(reads.seq, reads.offsets, 150)


def _index(ref, precision="fp32", N=150, stride=1, reduced=None):
    from paper_2603_22245_amd import mapper
    return mapper.build_index(ref, window_len=N, stride=stride, precision=precision,
                              reduced=reduced)


@pytest.mark.parametrize("N,stride,err,copies,rank", [(150, 1, 0.05, 16, 1), (150, 3, 0.3, 8, 0),
                                                      (64, 1, 0.0, 4, 3), (150, 1, 0.5, 64, 63),
                                                      (37, 2, 0.1, 1, 0)])
def test_window_thresholds_match_oracle(N, stride, err, copies, rank):
    """Sampled windows, the reference's last windows included (deletions there
    run past its end, where the mutator inserts)."""
    torch = torch_cuda()
    from paper_2603_22245_amd import mapper
    ref = synth.make_reference(20_000, seed=0, uniform=True)
    index = _index(ref, "fp16", N, stride)
    W = index.n_windows
    seed = 1000 + N + copies
    thr = mapper.window_thresholds(index, err, copies, rank, seed).cpu().numpy()
    rng = np.random.default_rng(80)
    pick = np.unique(np.concatenate([[0, 1, W // 2, W - 3, W - 2, W - 1],
                                     rng.choice(W, 40, replace=False)]))
    want = np.array([OT.window_threshold(ref, int(j), stride, N, err, copies, rank, seed)
                     for j in pick])
    print(f"N={N} stride={stride} err={err}: thresholds {want.min():.4f}..{want.max():.4f}, "
          f"max |d| {np.max(np.abs(thr[pick] - want)):.2e}")
    assert np.max(np.abs(thr[pick] - want)) <= TAU
    assert np.all((thr > 0) & (thr <= 1 + 1e-6))
    if err == 0.0:
        assert np.all(np.abs(thr - 1) <= 1e-5)


def _check_regime(hits, F, cut):
    """hits: per read (ids, F) from the GPU; F [R, W] oracle fidelities; cut [W]."""
    n_hits = 0
    for r, (ids, sc) in enumerate(hits):
        ids = ids.astype(np.int64)
        sure = set(np.nonzero((F[r] >= cut + TAU) & (F[r] > 0))[0].tolist())
        maybe = set(np.nonzero((F[r] >= cut - TAU) & (F[r] > 0))[0].tolist())
        got = set(ids.tolist())
        assert len(got) == ids.size, r                          # distinct
        assert sure <= got <= maybe, (r, sorted(sure - got)[:5], sorted(got - maybe)[:5])
        if ids.size:
            f = F[r, ids]
            assert np.all(np.diff(f) <= TAU), r                 # ranked by F (up to ties)
            assert np.max(np.abs(sc - f)) <= 2e-6, r
        n_hits += ids.size
    return n_hits


@pytest.mark.parametrize("precision,reduced", [("fp32", None), ("fp16", None), ("fp8", None),
                                               ("fp32", True), ("fp16", False), ("fp8", True)])
def test_threshold_regime_matches_oracle(precision, reduced, plain_data):
    """The plain workload (200 reads, 19,851 windows) with seeded synthetic
    thresholds: most windows cut at 0.3-0.9, 1 % at 0.005 (so that every read
    passes about 200 windows: lists far longer than any top-k), a floor of
    0.004; reads 0-2 cut to 100 letters (no head) and a run of one letter (zero
    windows) in the reference."""
    torch = torch_cuda()
    from paper_2603_22245_amd import mapper
    ref, reads, heads = plain_data
    ref = ref.copy()
    ref[5000:5400] = 2                                      # windows 5000..5250 are zero vectors
    seq, off = reads.seq.copy(), reads.offsets.copy()
    keep = np.ones(seq.size, bool)
    lens = np.diff(off)
    for r in (0, 1, 2):
        keep[off[r] + 100:off[r + 1]] = False
        lens[r] = 100
    seq = seq[keep]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    heads = mapping.read_heads(seq, off, 150)
    index = _index(ref, precision, reduced=reduced)
    W = index.n_windows
    rng = np.random.default_rng(81)
    thr = rng.uniform(0.3, 0.9, W).astype(np.float32)
    thr[rng.random(W) < 0.01] = 0.005
    floor = 0.004
    rb = mapper.upload_reads(index, seq, off)
    mapper.encode_reads(index, rb)
    h = mapper.score_threshold(index, rb, torch.from_numpy(thr).cuda(), floor)
    torch.cuda.synchronize()
    hits = h.lists()
    Cn, _ = oracle_windows(ref, 150)
    Xn, _ = oracle_heads(heads, 150)
    F = np.abs(np.conj(Xn) @ Cn.T) ** 2
    cut = np.maximum(thr.astype(np.float64), floor)
    n = _check_regime(hits, F, cut)
    for r in (0, 1, 2):
        assert hits[r][0].size == 0
    for r in range(reads.n):
        assert not np.any((hits[r][0] >= 5000) & (hits[r][0] <= 5250)), r
    total = int(h.total.cpu()[0])
    print(f"{precision}: {n} hits ({n / reads.n:.1f} per read), {total} proposals")
    assert n / reads.n > 100
    # want_ids from the oracle's own regime agree where decisions are clear
    for r in (3, 50, 199):
        wi, _ = OT.threshold_hits(F[r], cut)
        clear = np.abs(F[r, wi] - cut[wi]) > TAU
        assert set(wi[clear].tolist()) <= set(hits[r][0].tolist())


def test_threshold_regime_capacity():
    """A capacity below the proposals found: *total reports how many there were
    (the lists are then incomplete); the mapper's second pass with that
    capacity returns the same lists as a large first capacity."""
    torch = torch_cuda()
    from paper_2603_22245_amd import mapper
    ref = synth.make_reference(8_000, seed=5, uniform=True)
    reads = synth.simulate_reads(ref, np.full(30, 150), 0.01, 0.005, 0.005, seed=6)
    index = _index(ref, "fp16")
    thr = torch.full((index.n_windows,), 0.001, dtype=torch.float32, device="cuda")
    rb = mapper.upload_reads(index, reads.seq, reads.offsets)
    mapper.encode_reads(index, rb)
    small = mapper.score_threshold(index, rb, thr, capacity=100)
    big = mapper.score_threshold(index, rb, thr, capacity=1 << 20)
    auto = mapper.score_threshold(index, rb, thr)
    torch.cuda.synchronize()
    total = int(small.total.cpu()[0])
    assert total > 100 and int(big.total.cpu()[0]) == total
    assert int(small.hit_off.cpu()[-1]) == 100              # only what fitted was grouped
    for (bi, bs), (ai, asc) in zip(big.lists(), auto.lists()):
        np.testing.assert_array_equal(bi, ai)
        np.testing.assert_array_equal(bs, asc)


def test_threshold_regime_with_estimated_thresholds():
    """Thresholds estimated at the reads' own error rate (2 %, 16 copies, the
    second smallest), the regime with them, against the oracle's thresholds and
    regime over every window of a 3,000-letter reference: locations per read
    and the fraction of reads whose hits contain their true window (§3.5
    reports both for its human reads)."""
    torch = torch_cuda()
    from paper_2603_22245_amd import mapper
    ref = synth.make_reference(3_000, gc=0.41, repeat_frac=0.05, seed=7)
    reads = synth.simulate_reads(ref, np.full(60, 150), 0.02 / 3, 0.02 / 3, 0.02 / 3, seed=8)
    index = _index(ref, "fp16")
    W = index.n_windows
    thr = mapper.window_thresholds(index, 0.02, 16, 1, 9)
    rb = mapper.upload_reads(index, reads.seq, reads.offsets)
    mapper.encode_reads(index, rb)
    h = mapper.score_threshold(index, rb, thr)
    torch.cuda.synchronize()
    hits = h.lists()
    want_thr = np.array([OT.window_threshold(ref, j, 1, 150, 0.02, 16, 1, 9) for j in range(W)])
    assert np.max(np.abs(thr.cpu().numpy() - want_thr)) <= TAU
    heads = mapping.read_heads(reads.seq, reads.offsets, 150)
    Cn, _ = oracle_windows(ref, 150)
    Xn, _ = oracle_heads(heads, 150)
    F = np.abs(np.conj(Xn) @ Cn.T) ** 2
    n = _check_regime(hits, F, want_thr)
    found = np.mean([int(t) in set(ids.tolist()) for t, (ids, _) in zip(reads.truth, hits)])
    print(f"estimated thresholds: {n / reads.n:.2f} locations per read, true window among "
          f"them for {found:.3f} of reads, unmapped {np.mean([i.size == 0 for i, _ in hits]):.3f}")
    assert found >= 0.5
