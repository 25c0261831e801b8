"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Sizes: the plain workload (20,000 bp uniform reference, 200 reads of 150 bp)
spans many 32-window tiles, several window chunks and a ragged tail
(W = 19,851); other cases cover strides, the fine-tuned schedule, long
re-anchor segments and the edge cases."""
import numpy as np
import pytest

import synth
from oracle import mapping, rope
from tests.gpu_helpers import (assert_lists_exact, emb_to_complex, fp8_bound, interleave,
                               oracle_heads, oracle_windows, read_rows, stored_form, torch_cuda)

pytestmark = pytest.mark.gpu

PLAIN = synth.WORKLOADS["plain"]
# Score tolerance of the low-precision product against the FP64 oracle.
# FP32/FP16: |dF| <= tol * max(F, best F of the read).  FP8: |dF| <= 1e-2 in
# fidelity units (F lies in [0, 1]); e4m3's 3 mantissa bits leave an absolute
# error floor of a few 1e-3 on every score, which the relative form cannot
# meet for reads whose best score is low.  The fraction of FP8 scores inside
# the relative form is printed.
TOL = {"fp32": 1e-5, "fp16": 1e-3, "fp8": 1e-2}


@pytest.fixture(scope="module")
def plain_data():
    ref = PLAIN.reference()
    reads = PLAIN.reads(ref)
    heads = mapping.read_heads(reads.seq, reads.offsets, 150)
    return ref, reads, heads


@pytest.fixture(scope="module")
def plain_oracle(plain_data):
    ref, reads, heads = plain_data
    Cn, n2 = oracle_windows(ref, 150)
    Xn, _ = oracle_heads(heads, 150)
    F = np.abs(np.conj(Xn) @ Cn.T) ** 2          # [200, 19851]
    return Cn, n2, Xn, F


def _build(ref, precision, **kw):
    from paper_2603_22245_amd import mapper
    torch_cuda()
    return mapper.build_index(ref, precision=precision, **kw)


def _map(index, reads, k, k_fetch):
    from paper_2603_22245_amd import mapper
    torch = torch_cuda()
    rb = mapper.upload_reads(index, reads.seq, reads.offsets)
    bufs = mapper.map_buffers(index, reads.n, k, k_fetch)
    mapper.map_reads(index, rb, bufs)
    torch.cuda.synchronize()
    return rb, bufs


def test_angle_tables_fp64():
    torch = torch_cuda()
    ref = synth.make_reference(1000, seed=1, uniform=True)
    for sched in ("default", "finetuned"):
        for N in (150, 37):
            index = _build(ref, "fp32", window_len=N, schedule=sched)
            torch.cuda.synchronize()
            off = index.idx.d_phase64 - index.buf.data_ptr()
            ph = index.buf[off: off + N * 32 * 16].view(torch.float64).cpu().numpy()
            ph = ph[0::2] + 1j * ph[1::2]
            want = rope.unit_phases(N, 32, np.arange(N), sched).reshape(-1)
            assert np.max(np.abs(ph - want)) < 1e-14


@pytest.mark.parametrize("N,stride,sched", [(150, 1, "default"), (150, 3, "default"),
                                            (150, 1, "finetuned"), (32, 1, "default"),
                                            (1000, 7, "default"),
                                            # block rolling with omega^(f N) != 1, the
                                            # largest block, a block of N letters, and
                                            # strides rolled letter by letter (above
                                            # the largest block, and above N)
                                            (150, 3, "finetuned"), (150, 64, "default"),
                                            (40, 40, "default"), (150, 100, "default"),
                                            (32, 48, "finetuned")])
def test_rolling_encoder_fp32(N, stride, sched):
    torch = torch_cuda()
    ref = synth.make_reference(30_000, gc=0.45, repeat_frac=0.05, seed=7)
    index = _build(ref, "fp32", window_len=N, stride=stride, schedule=sched)
    torch.cuda.synchronize()
    got = emb_to_complex(index, torch)
    Cn, n2 = oracle_windows(ref, N, stride, schedule=sched)
    assert got.shape == Cn.shape
    ok = n2 >= 1e-3 * N                                   # far from degenerate
    err = np.max(np.abs(got[ok] - Cn[ok]))
    assert err < 5e-5, err
    gn2 = index.norms2().cpu().numpy()
    assert np.max(np.abs(gn2[ok] - n2[ok]) / n2[ok]) < 1e-4


@pytest.mark.parametrize("N,stride,reanchor", [(100, 4, 0), (150, 16, 300), (300, 17, 0),
                                               (400, 32, 77), (500, 33, 0), (6400, 64, 0),
                                               (64, 64, 5), (200, 5, 9)])
def test_block_rolling_on_matrix_cores_fp32(N, stride, reanchor):
    """Strides 4..64 with integer factors roll on the matrix cores (block
    sums as signed one-hot rows times the phase table, 16 positions per step:
    one, two and four steps); segments of lengths that are not multiples of
    the eight windows per product, a block of N letters, and codes other than
    A, C, G, T (4 and 255) in the reference, which add nothing."""
    torch = torch_cuda()
    ref = synth.make_reference(60_000, gc=0.45, repeat_frac=0.05, seed=17)
    rng = np.random.default_rng(17)
    pos = rng.choice(ref.shape[0], 400, replace=False)
    ref[pos[:200]] = 4
    ref[pos[200:]] = 255
    index = _build(ref, "fp32", window_len=N, stride=stride, reanchor=reanchor)
    torch.cuda.synchronize()
    got = emb_to_complex(index, torch)
    Cn, n2 = oracle_windows(ref, N, stride)
    assert got.shape == Cn.shape
    ok = n2 >= 1e-3 * N
    err = np.max(np.abs(got[ok] - Cn[ok]))
    print(f"N={N} stride={stride} reanchor={reanchor}: W={got.shape[0]}, max |d| {err:.2e}")
    assert err < 5e-5, err
    gn2 = index.norms2().cpu().numpy()
    assert np.max(np.abs(gn2[ok] - n2[ok]) / n2[ok]) < 1e-4


@pytest.mark.parametrize("precision,reduced,N,stride", [("fp16", True, 400, 4), ("fp16", True, 1600, 16),
                                                        ("fp8", False, 3200, 32), ("fp8", True, 6400, 64)])
def test_block_rolling_on_matrix_cores_quantised(precision, reduced, N, stride):
    """The batching buckets' shapes (N = 100 stride) in FP16 and FP8 rows, both
    forms: stored rows within the rounding bounds of the oracle's vectors."""
    torch = torch_cuda()
    ref = synth.make_reference(80_000, gc=0.45, repeat_frac=0.08, seed=18)
    index = _build(ref, precision, window_len=N, stride=stride, reduced=reduced)
    torch.cuda.synchronize()
    assert bool(index.params.reduced) == reduced
    got = emb_to_complex(index, torch)
    Cn, _ = oracle_windows(ref, N, stride)
    Cn = stored_form(Cn, index)
    assert got.shape == Cn.shape
    if precision == "fp16":
        bound_re = 2.0 ** -11 * np.abs(Cn.real) + 2e-5
        bound_im = 2.0 ** -11 * np.abs(Cn.imag) + 2e-5
    else:
        scale = index.scales().cpu().numpy()
        sc = np.exp2(np.round(np.log2(scale)))[:, None]
        bound_re = fp8_bound(np.abs(Cn.real), sc) + 0.05 * np.abs(Cn.real)
        bound_im = fp8_bound(np.abs(Cn.imag), sc) + 0.05 * np.abs(Cn.imag)
        nz = np.abs(got).sum(axis=1) > 0
        assert np.max(np.abs(np.linalg.norm(got[nz], axis=1) - 1)) < 1e-5
    assert np.all(np.abs(got.real - Cn.real) <= bound_re)
    assert np.all(np.abs(got.imag - Cn.imag) <= bound_im)


def test_rolling_drift_over_long_segments():
    # 65,536 starts per FP64 re-anchor: the FP32 recurrence's error after the
    # longest segment stays far below FP16 rounding of a unit vector.
    torch = torch_cuda()
    ref = synth.make_reference(140_000, seed=8, uniform=True)
    index = _build(ref, "fp32", reanchor=65_536)
    torch.cuda.synchronize()
    got = emb_to_complex(index, torch)
    Cn, n2 = oracle_windows(ref, 150)
    err = np.abs(got - Cn).max(axis=1)
    first = err[:1000].max()
    last = err[64_000:65_536].max()
    print(f"drift: max |d| first 1000 starts {first:.2e}, starts 64000-65535 {last:.2e}")
    assert last < 2e-4
    assert err[65_536] < 1e-5                               # re-anchored


def test_fp32_letter_sum_rows(plain_data, plain_oracle):
    """FP32 windows in the letter-sum form: the oracle's normalised vectors
    projected on the letter-sum basis, to the FP32 rolling error."""
    torch = torch_cuda()
    ref, _, _ = plain_data
    Cn, n2, _, _ = plain_oracle
    index = _build(ref, "fp32", reduced=True)
    torch.cuda.synchronize()
    got = emb_to_complex(index, torch)
    want = stored_form(Cn, index)
    assert got.shape == want.shape == (Cn.shape[0], 96)
    ok = n2 >= 1e-3 * 150
    assert np.max(np.abs(got[ok] - want[ok])) < 5e-5
    # the projection keeps the norm: letter-only windows stay unit vectors
    assert np.max(np.abs(np.linalg.norm(got[ok], axis=1) - 1)) < 1e-5


def test_letter_sum_identity_on_device():
    # For integer factors sum_L c_{k,L} = 0 in every full window.
    torch = torch_cuda()
    ref = synth.make_reference(20_000, seed=9, uniform=True)
    index = _build(ref, "fp32")
    torch.cuda.synchronize()
    got = emb_to_complex(index, torch).reshape(-1, 32, 4)
    assert np.max(np.abs(got.sum(axis=2))) < 5e-5


@pytest.mark.parametrize("precision,reduced", [("fp16", False), ("fp16", True), ("fp8", False),
                                               ("fp8", True)])
def test_quantised_encodings(precision, reduced, plain_data, plain_oracle):
    """Stored FP16/FP8 window rows against the oracle's vectors, in the full
    form and in the letter-sum form (the oracle's vectors projected on the
    letter-sum basis)."""
    torch = torch_cuda()
    ref, _, _ = plain_data
    Cn, n2, _, _ = plain_oracle
    index = _build(ref, precision, reduced=reduced)
    torch.cuda.synchronize()
    assert bool(index.params.reduced) == reduced
    got = emb_to_complex(index, torch)
    Cn = stored_form(Cn, index)
    assert got.shape == Cn.shape
    if precision == "fp16":
        # half an FP16 ulp (2^-11 relative) plus the FP32 rolling error
        assert np.all(np.abs(got.real - Cn.real) <= 2.0 ** -11 * np.abs(Cn.real) + 2e-5)
        assert np.all(np.abs(got.imag - Cn.imag) <= 2.0 ** -11 * np.abs(Cn.imag) + 2e-5)
    else:
        scale = index.scales().cpu().numpy()
        s = np.exp2(np.round(np.log2(scale)))[:, None]    # the power of two of the codes
        nz = np.abs(got).sum(axis=1) > 0
        # dequantised rows are unit length (norm folded into the FP32 scale)
        assert np.max(np.abs(np.linalg.norm(got[nz], axis=1) - 1)) < 1e-5
        assert np.max(np.abs(scale[nz] / s[nz, 0] - 1)) < 0.05
        corr = 0.05
        assert np.all(np.abs(got.real - Cn.real) <= fp8_bound(np.abs(Cn.real), s) + corr * np.abs(Cn.real))
        assert np.all(np.abs(got.imag - Cn.imag) <= fp8_bound(np.abs(Cn.imag), s) + corr * np.abs(Cn.imag))
        # window codes share the power of two 2^-8 (a unit vector's reals are at most
        # 1, so codes stay below 448); the index records the largest (256 s_j)^2,
        # which the e4m3 rounding bounds by 1.138
        assert np.all(s[:, 0] == 2.0 ** -8)
        W = scale.shape[0]
        off = index.idx.d_scale - index.buf.data_ptr()
        rec = float(index.buf[off + 4 * W: off + 4 * W + 4].view(torch.float32).cpu()[0])
        assert np.max((256.0 * scale.astype(np.float32)) ** 2) == np.float32(rec)
        assert 1.0 <= rec <= 1.138
        print(f"largest (256 s_j)^2 over the index: {rec:.5f}")
        # bytes equal torch's RNE cast of the oracle value, up to one code where
        # the FP32 rolling value and the FP64 value straddle a rounding boundary
        q = index.embeddings().cpu().numpy().astype(np.int32)
        inter = interleave(Cn)
        import torch as T
        want = T.from_numpy(np.clip(inter / s, -448, 448)).to(T.float8_e4m3fn).view(T.uint8)
        want = want.numpy().astype(np.int32)
        # signed ordinal of a code: codes adjacent in value differ by one
        ord_g = np.where(q >> 7, -(q & 127), q & 127)
        ord_w = np.where(want >> 7, -(want & 127), want & 127)
        diff = np.abs(ord_g - ord_w)
        print(f"fp8 codes: {np.mean(diff == 0):.6f} equal, {np.mean(diff == 1):.2e} one apart, "
              f"max {diff.max()}")
        assert diff.max() <= 1
        assert np.mean(diff == 0) > 0.999


@pytest.mark.parametrize("precision,reduced", [("fp32", False), ("fp32", True), ("fp16", False),
                                               ("fp16", True), ("fp8", False), ("fp8", True)])
def test_read_encoder(precision, reduced, plain_data):
    from paper_2603_22245_amd import mapper
    torch = torch_cuda()
    ref, reads, heads = plain_data
    index = _build(ref, precision, reduced=reduced)
    rb = mapper.upload_reads(index, reads.seq, reads.offsets)
    mapper.encode_reads(index, rb)
    torch.cuda.synchronize()
    re_row, im_row = read_rows(rb, precision, torch)
    Xn, _ = oracle_heads(heads, 150)
    Xn = stored_form(Xn, index)
    want_re = interleave(Xn)
    want_im = interleave(1j * Xn)           # (-Im x, Re x) per component
    assert re_row.shape == want_re.shape
    s = np.exp2(np.round(np.log2(rb.scale.cpu().numpy())))[:, None]

    def bound(w):
        if precision == "fp32":
            return 1e-6
        if precision == "fp16":
            return 2.0 ** -11 * np.abs(w) + 1e-7
        return fp8_bound(np.abs(w), s) + 0.05 * np.abs(w)   # plus the norm correction

    assert np.all(np.abs(re_row - want_re) <= bound(want_re))
    assert np.all(np.abs(im_row - want_im) <= bound(want_im))


def _check_candidates(idx, score, F, tol, absolute=False):
    R, kf = idx.shape
    best = F.max(axis=1)
    inside = []
    for r in range(R):
        ids = idx[r]
        assert len(set(ids.tolist())) == kf and ids.min() >= 0
        assert np.all(np.diff(score[r]) <= 0)             # sorted by the path's score
        f_or = F[r, ids]
        err = np.abs(score[r] - f_or)
        rel_ok = err <= tol * np.maximum(f_or, best[r]) + 1e-7
        inside.append(rel_ok)
        assert np.all(err <= tol + 1e-7) if absolute else np.all(rel_ok), r
    frac = float(np.mean(inside))
    print(f"scores within {tol} x max(F, best F): {frac:.5f}; max |dF| "
          f"{np.max(np.abs(score - np.take_along_axis(F, idx, 1))):.2e}")
    return frac


@pytest.mark.parametrize("reduced", [False, True])
def test_block_rolling_drift_over_long_segments(reduced):
    """65,536 starts per FP64 re-anchor at stride 4 (block sums on the matrix
    cores, in the letter basis or the letter-sum basis): the FP32 recurrence's
    error after the longest segment stays far below FP16 rounding of a unit
    vector, and the next segment starts re-anchored."""
    torch = torch_cuda()
    N, stride = 150, 4
    ref = synth.make_reference(4 * 70_000 + N, seed=9, uniform=True)
    index = _build(ref, "fp32", window_len=N, stride=stride, reanchor=65_536, reduced=reduced)
    torch.cuda.synchronize()
    got = emb_to_complex(index, torch)
    Cn, _ = oracle_windows(ref, N, stride)
    Cn = stored_form(Cn, index)
    err = np.abs(got - Cn).max(axis=1)
    first, last = err[:1000].max(), err[64_000:65_536].max()
    print(f"stride {stride} reduced={reduced}: max |d| first 1000 starts {first:.2e}, "
          f"starts 64000-65535 {last:.2e}, start 65536 {err[65_536]:.2e}")
    assert last < 2e-4
    assert err[65_536] < 1e-5                               # re-anchored


@pytest.mark.parametrize("precision,k_fetch,reduced", [
    ("fp32", 8, None), ("fp16", 8, None), ("fp16", 16, None), ("fp16", 32, None), ("fp8", 16, None),
    ("fp8", 32, None), ("fp32", 32, None), ("fp16", 16, False), ("fp16", 32, False),
    ("fp8", 16, True), ("fp8", 32, True), ("fp16", 64, None), ("fp8", 64, None),
    ("fp32", 64, None), ("fp16", 48, False), ("fp8", 64, True), ("fp32", 16, True),
    ("fp32", 64, True)])
def test_score_topk_and_rescore(precision, k_fetch, reduced, plain_data, plain_oracle):
    """The product's candidates and the rescored lists against the oracle; FP16
    and FP8 indexes in the letter-sum form (FP16's default for letters) and in
    the full form (FP8's default)."""
    torch = torch_cuda()
    ref, reads, heads = plain_data
    _, _, _, F = plain_oracle
    index = _build(ref, precision, reduced=reduced)
    assert bool(index.params.reduced) == (reduced is True or (reduced is None and precision == "fp16"))
    k = 8
    rb, bufs = _map(index, reads, k, k_fetch)
    cidx = bufs.cand_idx.cpu().numpy()
    csc = bufs.cand_score.cpu().numpy()
    _check_candidates(cidx, csc, F, TOL[precision], absolute=precision == "fp8")
    # oracle top-k_fetch and top-k with ties ordered by index
    W = F.shape[1]
    order = np.lexsort((np.broadcast_to(np.arange(W), F.shape), -F), axis=1)
    o_idx = order[:, :k]
    o_F = np.take_along_axis(F, o_idx, 1)
    cand_F = np.take_along_axis(F, cidx, 1)
    rec_c = mapping.recall_at_k(cidx[:, :k], o_idx, o_F, cand_F[:, :k])
    tidx = bufs.top_idx.cpu().numpy()
    tsc = bufs.top_score.cpu().numpy()
    top_F = np.take_along_axis(F, tidx, 1)
    rec = mapping.recall_at_k(tidx, o_idx, o_F, top_F)
    exact = mapping.same_up_to_ties(tidx, o_F, top_F)
    print(f"{precision} k_fetch={k_fetch}: candidate recall@8 {rec_c:.4f}, "
          f"rescored recall@8 {rec:.4f}, exact lists {exact.mean():.4f}")
    assert np.max(np.abs(tsc - top_F)) < 2e-6            # FP32 rescore vs FP64
    assert_lists_exact(exact, rec, k_fetch, k, precision)


@pytest.mark.parametrize("precision,n_reads", [("fp16", 40), ("fp8", 40), ("fp16", 300),
                                               ("fp8", 300)])
def test_thin_read_tiles(precision, n_reads, plain_data, plain_oracle):
    """Batches that would leave a quarter or more of their 256-read tiles empty
    (40 reads: one tile; 300 reads: two) run with 128-read tiles in the
    256-read launch: candidates within the product's tolerance, rescored lists
    equal to the oracle's up to ties."""
    torch = torch_cuda()
    ref, reads, heads = plain_data
    _, _, _, F = plain_oracle
    n = min(n_reads, reads.n)
    sub = synth.Reads(reads.seq[:reads.offsets[n]], reads.offsets[:n + 1], reads.truth[:n])
    F = F[:n]
    if n_reads > reads.n:  # repeat the plain reads to reach the batch size
        reps = -(-n_reads // reads.n)
        seq = np.concatenate([reads.seq] * reps)
        lens = np.tile(np.diff(reads.offsets), reps)[:n_reads]
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        sub = synth.Reads(seq[:off[-1]], off, np.tile(reads.truth, reps)[:n_reads])
        F = np.tile(plain_oracle[3], (reps, 1))[:n_reads]
    index = _build(ref, precision)
    k, k_fetch = 8, 16
    rb, bufs = _map(index, sub, k, k_fetch)
    cidx = bufs.cand_idx.cpu().numpy()
    csc = bufs.cand_score.cpu().numpy()
    _check_candidates(cidx, csc, F, TOL[precision], absolute=precision == "fp8")
    W = F.shape[1]
    order = np.lexsort((np.broadcast_to(np.arange(W), F.shape), -F), axis=1)
    o_idx = order[:, :k]
    o_F = np.take_along_axis(F, o_idx, 1)
    tidx = bufs.top_idx.cpu().numpy()
    top_F = np.take_along_axis(F, tidx, 1)
    rec = mapping.recall_at_k(tidx, o_idx, o_F, top_F)
    exact = mapping.same_up_to_ties(tidx, o_F, top_F)
    print(f"{precision} {n_reads} reads: rescored recall@8 {rec:.4f}, exact lists {exact.mean():.4f}")
    assert_lists_exact(exact, rec, k_fetch, k, precision)


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp8"])
def test_sixty_four_candidates_and_long_lists(precision, plain_data, plain_oracle):
    """64 product candidates (lists of 64 keys per chunk, merged two keys per
    lane) rescored into top-48 lists (top-32 for FP8, whose product error needs
    the usual two-fold over-fetch: with 48 of 64, 5 of the 200 lists missed a
    window near rank 48): candidates are the product's own top-64, rescored
    lists equal the oracle's up to ties."""
    torch = torch_cuda()
    ref, reads, heads = plain_data
    _, _, _, F = plain_oracle
    index = _build(ref, precision)
    k, k_fetch = (32 if precision == "fp8" else 48), 64
    rb, bufs = _map(index, reads, k, k_fetch)
    cidx = bufs.cand_idx.cpu().numpy()
    csc = bufs.cand_score.cpu().numpy()
    _check_candidates(cidx, csc, F, TOL[precision], absolute=precision == "fp8")
    # every window the oracle scores clearly above the product's 64th entry is
    # in the list (clearly: by more than twice the product's error)
    f_c = np.take_along_axis(F, cidx, 1)
    margin = {"fp32": 2e-5, "fp16": 2e-3, "fp8": 3e-2}[precision]
    for r in range(F.shape[0]):
        above = np.nonzero(F[r] > f_c[r].min() + margin)[0]
        assert set(above.tolist()) <= set(cidx[r].tolist()), r
    W = F.shape[1]
    order = np.lexsort((np.broadcast_to(np.arange(W), F.shape), -F), axis=1)
    o_idx = order[:, :k]
    o_F = np.take_along_axis(F, o_idx, 1)
    tidx = bufs.top_idx.cpu().numpy()
    top_F = np.take_along_axis(F, tidx, 1)
    rec = mapping.recall_at_k(tidx, o_idx, o_F, top_F)
    exact = mapping.same_up_to_ties(tidx, o_F, top_F)
    print(f"{precision} top-{k} of {k_fetch}: recall {rec:.4f}, exact lists {exact.mean():.4f}")
    assert np.max(np.abs(bufs.top_score.cpu().numpy() - top_F)) < 2e-6
    assert_lists_exact(exact, rec, k_fetch, k, precision)


def test_more_reads_than_one_tile_and_many_chunks():
    torch = torch_cuda()
    ref = synth.make_reference(60_000, gc=0.41, repeat_frac=0.05, seed=11)
    reads = synth.simulate_reads(ref, np.full(700, 150), 0.01, 0.005, 0.005, seed=12)
    heads = mapping.read_heads(reads.seq, reads.offsets, 150)
    index = _build(ref, "fp16")
    rb, bufs = _map(index, reads, 8, 16)
    Cn, _ = oracle_windows(ref, 150)
    Xn, _ = oracle_heads(heads, 150)
    F = np.abs(np.conj(Xn) @ Cn.T) ** 2
    _check_candidates(bufs.cand_idx.cpu().numpy(), bufs.cand_score.cpu().numpy(), F, TOL["fp16"])
    W = F.shape[1]
    order = np.lexsort((np.broadcast_to(np.arange(W), F.shape), -F), axis=1)
    o_idx = order[:, :8]
    tidx = bufs.top_idx.cpu().numpy()
    rec = mapping.recall_at_k(tidx, o_idx, np.take_along_axis(F, o_idx, 1),
                              np.take_along_axis(F, tidx, 1))
    assert rec >= 0.999


def test_hamming_closed_form_on_device():
    # N = m = 32 integer factors: the fidelity of equal-length strings is
    # ((N - d)/N)^2 with d the Hamming distance (§1), exactly.
    torch = torch_cuda()
    rng = np.random.default_rng(13)
    ref = rng.integers(0, 4, 4000).astype(np.uint8)
    starts = rng.integers(0, 4000 - 32, 64)
    ds = rng.integers(0, 12, 64)
    seqs = []
    for s, d in zip(starts, ds):
        w = ref[s:s + 32].copy()
        pos = rng.choice(32, d, replace=False)
        w[pos] = (w[pos] + rng.integers(1, 4, d)) % 4
        seqs.append(w)
    reads = synth.Reads(np.concatenate(seqs), np.arange(65, dtype=np.int64) * 32, starts)
    index = _build(ref, "fp32", window_len=32)
    rb, bufs = _map(index, reads, 8, 8)
    tidx = bufs.top_idx.cpu().numpy()
    tsc = bufs.top_score.cpu().numpy()
    for r in range(64):
        w = seqs[r]
        for i in range(8):
            j = int(tidx[r, i])
            d = int(np.sum(ref[j:j + 32] != w))
            assert abs(tsc[r, i] - ((32 - d) / 32) ** 2) < 2e-6


def test_edge_cases():
    torch = torch_cuda()
    rng = np.random.default_rng(14)
    # tiny reference: fewer windows (6) than k_fetch (8)
    ref = rng.integers(0, 4, 155).astype(np.uint8)
    reads = synth.Reads(ref[:150].copy(), np.array([0, 150], dtype=np.int64), np.array([0]))
    index = _build(ref, "fp16")
    rb, bufs = _map(index, reads, 8, 8)
    tidx = bufs.top_idx.cpu().numpy()[0]
    assert tidx[0] == 0 and list(tidx[6:]) == [-1, -1]
    assert sorted(tidx[:6].tolist()) == list(range(6))
    assert np.all(bufs.top_score.cpu().numpy()[0][6:] == 0)
    # degenerate windows (a run of one letter), an exact duplicate block, a
    # degenerate read and a read shorter than N: the last two are zero vectors,
    # every window scores 0 and the read has no location (id -1, score 0), as
    # in the oracle
    ref = rng.integers(0, 4, 5000).astype(np.uint8)
    ref[1000:1400] = 0
    ref[3000:3300] = ref[2000:2300]
    good = ref[2050:2200].copy()
    seq = np.concatenate([good, ref[1100:1250], rng.integers(0, 4, 100).astype(np.uint8)])
    off = np.array([0, 150, 300, 400], dtype=np.int64)
    reads = synth.Reads(seq, off, np.array([2050, 1100, 0]))
    o_idx, o_F = mapping.map_reads(ref, mapping.read_heads(seq, off, 150), 150, 32, 8)
    assert np.all(o_idx[1:] == -1) and np.all(o_F[1:] == 0)
    for prec in ("fp32", "fp16", "fp8"):
        index = _build(ref, prec)
        rb, bufs = _map(index, reads, 8, 16)
        tidx = bufs.top_idx.cpu().numpy()
        tsc = bufs.top_score.cpu().numpy()
        assert tidx[0, 0] == 2050 and tidx[0, 1] == 3050, prec   # tie: lower id first
        assert abs(tsc[0, 0] - 1) < 1e-5 and abs(tsc[0, 1] - 1) < 1e-5
        np.testing.assert_array_equal(tidx[1:], o_idx[1:], err_msg=prec)  # no location
        assert np.all(tsc[1:] == 0.0), prec
        cidx = bufs.cand_idx.cpu().numpy()
        assert np.all(cidx[1:] == -1) and np.all(bufs.cand_score.cpu().numpy()[1:] == 0), prec
        e = emb_to_complex(index, torch)
        assert np.all(e[1000:1251] == 0)                   # windows inside the run


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_largest_window_length(precision):
    """N = RM_MAX_WINDOW: sampled index rows and squared norms against the
    oracle one window at a time; exact and mutated reads of that length."""
    from paper_2603_22245_amd import _lib as L
    torch = torch_cuda()
    N = L.RM_MAX_WINDOW
    rng = np.random.default_rng(15)
    ref = rng.integers(0, 4, 20_000).astype(np.uint8)
    index = _build(ref, precision, window_len=N)
    W = index.n_windows
    assert W == 20_000 - N + 1
    rows = np.unique(np.r_[0, 1, 255, 256, 257, W // 2, W - 2, W - 1, rng.choice(W, 12)])
    got = emb_to_complex(index, torch)[rows]
    want = np.stack([rope.encode_raw(ref[j:j + N], N, 32) for j in rows])
    wn, n2 = mapping.normalized_rows(want, N)
    wn = stored_form(wn, index)
    # FP32 rolling error; FP16 adds half an ulp (2^-11 relative)
    rel = 1e-5 if precision == "fp32" else 2.0 ** -11
    for part in (np.real, np.imag):
        assert np.all(np.abs(part(got) - part(wn)) <= rel * np.abs(part(wn)) + 2e-5)
    norms = index.norms2().cpu().numpy()[rows]
    assert np.max(np.abs(norms / n2 - 1)) <= 2e-4
    # reads: exact copies of windows 0, 1234 and W-1, and a mutated copy of 2000
    mut = ref[2000:2000 + N].copy()
    pos = rng.choice(N, N // 100, replace=False)
    mut[pos] = (mut[pos] + rng.integers(1, 4, pos.size)) % 4
    heads = [ref[0:N], ref[1234:1234 + N], ref[W - 1:W - 1 + N], mut]
    seq = np.concatenate(heads)
    off = np.arange(5, dtype=np.int64) * N
    reads = synth.Reads(seq, off, np.array([0, 1234, W - 1, 2000]))
    rb, bufs = _map(index, reads, 4, 8)
    tidx = bufs.top_idx.cpu().numpy()
    tsc = bufs.top_score.cpu().numpy().astype(np.float64)
    assert list(tidx[:3, 0]) == [0, 1234, W - 1]
    assert np.all(np.abs(tsc[:3, 0] - 1) < 1e-5)
    F = mapping.pair_fidelities(ref, np.stack(heads), tidx.astype(np.int64), N)
    assert np.max(np.abs(tsc - F)) <= 1e-4
    # with 32 frequencies over 16,384 letters neighbouring windows score almost
    # alike: the mutated read's best must be the oracle's best near its origin
    near = np.arange(1900, 2101, dtype=np.int64)[None, :]
    Fn = mapping.pair_fidelities(ref, mut[None, :], near, N)[0]
    assert abs(int(tidx[3, 0]) - 2000) <= 100
    assert tsc[3, 0] >= Fn.max() - 1e-4


def test_one_letter_windows():
    """N = 1: a window is one letter (phase 1), so every window holding the
    read's letter scores 1 and the list is the first k such windows."""
    torch = torch_cuda()
    rng = np.random.default_rng(16)
    ref = rng.integers(0, 4, 3000).astype(np.uint8)
    index = _build(ref, "fp16", window_len=1)
    assert index.n_windows == 3000
    seq = np.array([0, 1, 2, 3], dtype=np.uint8)
    reads = synth.Reads(seq, np.arange(5, dtype=np.int64), np.zeros(4, np.int64))
    rb, bufs = _map(index, reads, 8, 16)
    tidx = bufs.top_idx.cpu().numpy()
    tsc = bufs.top_score.cpu().numpy()
    for L in range(4):
        want = np.nonzero(ref == L)[0][:8]
        assert list(tidx[L]) == list(want), L
        assert np.all(np.abs(tsc[L] - 1) < 1e-6)


@pytest.mark.parametrize("k_fetch,k", [(1, 1), (5, 3), (9, 9), (20, 8), (27, 16), (32, 32)])
def test_rescore_given_candidates(k_fetch, k, plain_data, plain_oracle):
    """The FP32 rescore alone, on candidate pools that the product did not
    choose: random windows with some invalid entries (-1 and >= W), every
    pool-size class of the kernel (1 to 5 blocks of 32 one-hot rows), and a
    few reads shorter than the window (no head: F = 0 for every candidate).
    The top-k must be the FP64 oracle's order of the same pool, up to ties."""
    from paper_2603_22245_amd import mapper
    torch = torch_cuda()
    ref, reads, heads = plain_data
    _, _, _, F = plain_oracle
    R, W = F.shape
    index = _build(ref, "fp32")
    # reads 0..2 cut to 100 letters: heads shorter than N = 150
    seq, off = reads.seq.copy(), reads.offsets.copy()
    short = [0, 1, 2]
    keep = np.ones(seq.size, bool)
    for r in short:
        keep[off[r] + 100:off[r + 1]] = False
    lens = np.diff(off)
    lens[short] = 100
    seq = seq[keep]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    rng = np.random.default_rng(7 + k_fetch)
    pool = np.stack([rng.choice(W, k_fetch, replace=False) for _ in range(R)]).astype(np.int32)
    bad = rng.random(pool.shape) < 0.1
    pool[bad] = np.where(rng.random(bad.sum()) < 0.5, -1, W + 5)
    rb = mapper.upload_reads(index, seq, off)
    bufs = mapper.map_buffers(index, R, k, k_fetch)
    bufs.cand_idx.copy_(torch.from_numpy(pool).cuda())
    mapper.rescore(index, rb, bufs)
    torch.cuda.synchronize()
    tidx = bufs.top_idx.cpu().numpy()
    tsc = bufs.top_score.cpu().numpy()
    for r in range(R):
        valid = [int(j) for j in pool[r] if 0 <= j < W]
        if r in short or not valid:           # no head, or every candidate invalid:
            assert np.all(tidx[r] == -1) and np.all(tsc[r] == 0.0), r   # no location
            continue
        n = min(k, len(valid))
        fv = np.array([F[r, j] for j in valid])
        order = np.lexsort((np.array(valid), -fv))
        want_F = fv[order[:n]]
        got_ids = tidx[r, :n]
        assert np.all(got_ids >= 0) and np.all(tidx[r, n:] == -1) and np.all(tsc[r, n:] == 0), r
        assert len(set(got_ids.tolist())) == n and set(got_ids.tolist()) <= set(valid), r
        got_true = F[r, got_ids]
        assert np.all(np.abs(got_true - want_F) <= mapping.TIE_TAU), r
        assert np.max(np.abs(tsc[r, :n] - got_true)) < 2e-6, r
