"""GPU parity of mapping with the learned encoding: BF16 token offsets, the
learned rolling index, read heads, and the FP32 rescore, against the FP64
oracle (whose offsets use the same bfloat16 rounding of weights and hidden
values).

Tolerances.  Offsets: every value within the derived bfloat16 error bound of
the exact offsets (oracle.learned.offset_error_bound); against the oracle's
bfloat16 offsets, 99% within 1e-5 (FP32 vs FP64 sums) -- the rest are hidden
values whose rounding flips between the two, bounded by twice the bound.
Encodings: a flipped hidden value moves one token's phase by at most ~1e-3,
a normalised component by well under 1e-3; the rolling FP32 update adds
~1e-5; FP16 storage adds 2^-11 relative.  Fidelities after the FP32 rescore:
2e-4 absolute.
"""
import numpy as np
import pytest

import synth
from oracle import learned as OL
from oracle import mapping

from gpu_helpers import assert_lists_exact, torch_cuda, emb_to_complex, read_rows

pytestmark = pytest.mark.gpu

N = 150


def _params(seed):
    rng = np.random.default_rng(seed)
    W1, b1, W2, b2 = OL.unpack(OL.init_params(seed))
    return OL.pack(W1, b1, rng.normal(0, 0.05, W2.shape), rng.normal(0, 0.4, 128)).astype(
        np.float32).astype(np.float64)


def _infer(torch, params, w):
    from paper_2603_22245_amd import _lib as L
    d_p = torch.from_numpy(params.astype(np.float32)).cuda()
    d_w = torch.from_numpy(np.ascontiguousarray(w, dtype=np.uint8)).cuda()
    out = torch.full((len(w) - 8, 32), float("nan"), dtype=torch.float32, device="cuda")
    L.rm_mlp_infer(d_p, d_w, len(w), out)
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("n", [9, 40, 41, 72, 5003])
def test_mlp_infer_matches_oracle(n):
    torch = torch_cuda()
    params = _params(40)
    w = np.random.default_rng(41 + n).integers(0, 4, n)
    got = _infer(torch, params, w)
    _, exact = OL.token_offsets(params, w, bf16=False)
    _, low = OL.token_offsets(params, w, bf16=True)
    bound = OL.offset_error_bound(params, w)
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - exact) <= bound)
    d = np.abs(got - low)
    assert np.all(d <= 2 * bound)
    assert np.mean(d <= 1e-5) >= 0.99


def test_mlp_infer_zero_output_layer_gives_b2():
    torch = torch_cuda()
    rng = np.random.default_rng(42)
    W1, b1, W2, b2 = OL.unpack(OL.init_params(5))
    b2 = rng.normal(0, 1, 128)
    params = OL.pack(W1, b1, W2, b2).astype(np.float32).astype(np.float64)
    w = rng.integers(0, 4, 300)
    got = _infer(torch, params, w)
    mid = w[4:296]
    want = OL.unpack(params)[3].reshape(4, 32)[mid]   # b2 as the kernel sees it (FP32)
    assert np.max(np.abs(got - want)) == 0.0


def _index(torch, ref, params, precision, stride=1, reanchor=0):
    from paper_2603_22245_amd import mapper
    return mapper.build_index(ref, N, stride, precision, reanchor=reanchor, learned=params)


@pytest.mark.parametrize("precision,stride,reanchor", [("fp32", 1, 300), ("fp32", 3, 0),
                                                        ("fp16", 1, 0), ("fp8", 2, 500)])
def test_learned_index_matches_oracle(precision, stride, reanchor):
    torch = torch_cuda()
    params = _params(43)
    ref = np.random.default_rng(44).integers(0, 4, 4000).astype(np.uint8)
    idx = _index(torch, ref, params, precision, stride, reanchor)
    torch.cuda.synchronize()
    got = emb_to_complex(idx, torch)
    starts = mapping.window_starts(len(ref), N, stride)
    assert got.shape[0] == starts.shape[0]
    C = OL.window_encodings(params, ref, starts, N, bf16=True)
    Cn, _ = mapping.normalized_rows(C, N)
    tol = {"fp32": 1e-3, "fp16": 1.5e-3, "fp8": 0.0}[precision]
    if precision == "fp8":
        # e4m3 codes: 3 mantissa bits, relative 2^-4 of the row's largest value
        tol = 2.0 ** -4 * np.max(np.abs(Cn), axis=1, keepdims=True) + 1e-3
    err = np.abs(got - Cn)
    assert np.all(err <= tol), float(np.max(err - tol))


def test_learned_read_heads_match_oracle():
    torch = torch_cuda()
    from paper_2603_22245_amd import mapper
    params = _params(45)
    rng = np.random.default_rng(46)
    ref = rng.integers(0, 4, 3000).astype(np.uint8)
    idx = _index(torch, ref, params, "fp32")
    lens = [150, 151, 200, 149, 150, 400]
    seqs = [rng.integers(0, 4, n).astype(np.uint8) for n in lens]
    off = np.zeros(len(seqs) + 1, np.int64); off[1:] = np.cumsum(lens)
    reads = mapper.upload_reads(idx, np.concatenate(seqs), off)
    mapper.encode_reads(idx, reads)
    torch.cuda.synchronize()
    re, im = read_rows(reads, "fp32", torch)
    got = re[:, 0::2] + 1j * re[:, 1::2]
    np.testing.assert_allclose(im[:, 1::2], re[:, 0::2], atol=0)   # row 2r+1 = i * row 2r
    for r, w in enumerate(seqs):
        if len(w) < N:
            assert np.all(got[r] == 0)
            continue
        X = OL.head_encodings(params, w[None, :N], N)
        Xn, _ = mapping.normalized_rows(X, N)
        assert np.max(np.abs(got[r] - Xn[0])) <= 1e-3


@pytest.mark.parametrize("precision", ["fp16", "fp8"])
def test_learned_mapping_matches_oracle(precision):
    torch = torch_cuda()
    from paper_2603_22245_amd import mapper
    params = _params(47)
    ref = synth.make_reference(20000, 0.45, 0.05, seed=48)
    reads = synth.simulate_reads(ref, np.full(48, 150), 0.01, 0.005, 0.005, seed=49)
    idx = _index(torch, ref, params, precision)
    rb = mapper.upload_reads(idx, reads.seq, reads.offsets)
    k, k_fetch = 8, 16
    bufs = mapper.map_buffers(idx, rb.n, k, k_fetch)
    mapper.map_reads(idx, rb, bufs)
    torch.cuda.synchronize()
    got_i = bufs.top_idx.cpu().numpy().astype(np.int64)
    got_f = bufs.top_score.cpu().numpy().astype(np.float64)
    heads = mapping.read_heads(reads.seq, reads.offsets, N)
    want_i, want_f = OL.map_reads(params, ref, heads, N, k=k)
    true_f = OL.head_window_fidelities(params, ref, heads, got_i, N)
    assert np.max(np.abs(got_f - true_f)) <= 2e-4
    ok = mapping.same_up_to_ties(got_i, want_f, true_f, tau=2e-4)
    rec = mapping.recall_at_k(got_i, want_i, want_f, true_f, tau=2e-4)
    assert_lists_exact(ok, rec, k_fetch, k, precision)
