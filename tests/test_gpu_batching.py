"""Batching: several bucket indexes scored in one persistent launch, HIP graph
replay, tile-shape tuning and the autotuner, against the FP64 oracle."""
import os

import numpy as np
import pytest

import synth
from oracle import mapping
from tests.gpu_helpers import assert_lists_exact, torch_cuda

pytestmark = pytest.mark.gpu

BUCKETS = (100, 200, 400, 800)


@pytest.fixture(scope="module")
def batch_data():
    ref = synth.make_reference(150_000, gc=0.45, repeat_frac=0.08, seed=31)
    rng = np.random.default_rng(32)
    lengths = np.clip(np.rint(np.exp(rng.normal(np.log(350), 0.7, 160))), 60, 1000).astype(np.int64)
    e = rng.uniform(0.05, 0.10, size=lengths.shape[0])
    reads = synth.simulate_reads(ref, lengths, 0.2 * e, 0.4 * e, 0.4 * e, seed=33)
    return ref, reads


def _mapper(ref, reads, precision="fp16", k=8, k_fetch=16):
    from paper_2603_22245_amd import mapper
    torch_cuda()
    return mapper.BatchMapper(ref, reads.seq, reads.offsets, k=k, k_fetch=k_fetch,
                              precision=precision, buckets=BUCKETS)


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp8"])
def test_batched_matches_oracle_per_bucket(batch_data, precision):
    torch = torch_cuda()
    ref, reads = batch_data
    bm = _mapper(ref, reads, precision)
    bm.run()
    torch.cuda.synchronize()
    ids, sc = bm.results()
    assert np.all(ids[bm.bucket_of < 0] == -1)              # shorter than every bucket
    assert len(bm.buckets) >= 3
    for b in bm.buckets:
        heads = np.stack([reads.read(i)[:b.length] for i in b.read_ids])
        o_idx, o_F = mapping.map_reads(ref, heads, b.length, 32, 8, b.stride)
        got = ids[b.read_ids]
        got_F = mapping.pair_fidelities(ref, heads, got, b.length, 32, b.stride)
        ok = mapping.same_up_to_ties(got, o_F, got_F)
        rec = mapping.recall_at_k(got, o_idx, o_F, got_F)
        print(f"{precision} bucket N={b.length} stride={b.stride}: {b.read_ids.size} reads, "
              f"exact {ok.mean():.3f}, recall {rec:.4f}")
        assert_lists_exact(ok, rec, 16, 8, precision)
        assert np.max(np.abs(sc[b.read_ids] - got_F)) < 2e-6
    bm.close()


def test_graph_replay_matches_eager(batch_data):
    torch = torch_cuda()
    ref, reads = batch_data
    bm = _mapper(ref, reads, "fp16")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bm.run(stream)
    stream.synchronize()
    eager = [(b.bufs.top_idx.clone(), b.bufs.top_score.clone(), b.bufs.cand_idx.clone())
             for b in bm.buckets]
    bm.capture(stream)
    for rep in range(3):
        for b in bm.buckets:                                 # scribble over the outputs
            b.bufs.top_idx.fill_(-7)
            b.bufs.cand_idx.fill_(-7)
        torch.cuda.synchronize()
        bm.replay(stream)
        stream.synchronize()
        x = torch.ones(1 << 20, device="cuda").sum()         # eager work between replays
        torch.cuda.synchronize()
        for b, (ti, ts, ci) in zip(bm.buckets, eager):
            assert torch.equal(b.bufs.top_idx, ti), rep
            assert torch.equal(b.bufs.top_score, ts), rep
            assert torch.equal(b.bufs.cand_idx, ci), rep
    bm.close()


@pytest.mark.parametrize("precision", ["fp16", "fp8"])
def test_every_tuning_gives_identical_lists(batch_data, precision, tmp_path):
    from paper_2603_22245_amd import _lib as L
    torch = torch_cuda()
    ref, reads = batch_data
    bm = _mapper(ref, reads, precision)
    bm.encode()
    bm.score()
    torch.cuda.synchronize()
    base = [(b.bufs.cand_idx.clone(), b.bufs.cand_score.clone()) for b in bm.buckets]
    for rt in (128, 256):
        for ct in (0, 1, 7, 128, 4096):
            bm.tune = L.rm_tuning(rt, ct)
            bm.ws_bytes = bm._ws_bytes(bm.tune)
            if bm.ws_bytes > bm.ws.numel():
                bm.ws = torch.empty(bm.ws_bytes, dtype=torch.uint8, device="cuda")
            bm.score()
            torch.cuda.synchronize()
            for b, (ci, cs) in zip(bm.buckets, base):
                assert torch.equal(b.bufs.cand_idx, ci), (rt, ct, b.length)
                assert torch.equal(b.bufs.cand_score, cs), (rt, ct, b.length)
    cache = str(tmp_path / "tune.jsonl")
    best, ms = bm.autotune(cache)
    assert best.read_tile in (128, 256) and ms > 0
    assert os.path.exists(cache)
    best2, ms2 = bm.autotune(cache)                           # from the cache, no timing
    assert (best2.read_tile, best2.chunk_tiles) == (best.read_tile, best.chunk_tiles)
    assert abs(ms2 - ms) < 1e-3
    bm.close()


def test_grouped_launch_equals_separate_launches(batch_data):
    from paper_2603_22245_amd import mapper
    torch = torch_cuda()
    ref, reads = batch_data
    bm = _mapper(ref, reads, "fp16")
    bm.encode()
    bm.score()
    torch.cuda.synchronize()
    for b in bm.buckets:
        solo = mapper.map_buffers(b.index, b.reads.n, 8, 16)
        mapper.score_topk(b.index, b.reads, solo)
        torch.cuda.synchronize()
        assert torch.equal(solo.cand_idx, b.bufs.cand_idx)
        assert torch.equal(solo.cand_score, b.bufs.cand_score)
    bm.close()
