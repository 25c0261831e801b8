"""rm_score_topk_noalloc (the product + top-k with the library's own device
scratch) against rm_score_topk with a caller workspace, through the C ABI:
identical candidate lists on two calls in a row, the second with fewer reads
(the scratch keeps the first call's contents), plus the size limit."""
import ctypes

import numpy as np
import pytest

import synth
from paper_2603_22245_amd import _lib as L

from gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,k_fetch", [("fp16", 16), ("fp8", 32), ("fp32", 8)])
def test_noalloc_equals_workspace_call(precision, k_fetch):
    torch = torch_cuda()
    from paper_2603_22245_amd import mapper
    ref = synth.make_reference(60_000, gc=0.41, repeat_frac=0.05, seed=90)
    reads = synth.simulate_reads(ref, np.full(700, 150), 0.01, 0.005, 0.005, seed=91)
    index = mapper.build_index(ref, precision=precision)
    rb = mapper.upload_reads(index, reads.seq, reads.offsets)
    mapper.encode_reads(index, rb)
    for n in (700, 123):                       # second call: a smaller input
        bufs = mapper.map_buffers(index, n, min(8, k_fetch), k_fetch)
        L.rm_score_topk(index.idx, rb.emb, rb.scale, n, k_fetch, bufs.cand_idx, bufs.cand_score,
                        bufs.ws, bufs.ws_bytes)
        ci = torch.full((n, k_fetch), -7, dtype=torch.int32, device="cuda")
        cs = torch.full((n, k_fetch), -7.0, dtype=torch.float32, device="cuda")
        L.rm_score_topk_noalloc(index.idx, rb.emb, rb.scale, n, k_fetch, ci, cs)
        torch.cuda.synchronize()
        assert torch.equal(ci, bufs.cand_idx), (precision, n)
        assert torch.equal(cs, bufs.cand_score), (precision, n)
        assert int((ci >= 0).sum()) == n * k_fetch


def test_noalloc_rejects_workspace_above_its_scratch():
    torch = torch_cuda()
    from paper_2603_22245_amd import mapper
    ref = synth.make_reference(20_000, seed=92, uniform=True)
    index = mapper.build_index(ref, precision="fp16")
    n = 3_000_000                               # its workspace exceeds the scratch
    assert L.rm_score_workspace_bytes(index.idx, n, 32) > L.RM_NOALLOC_SCRATCH_BYTES
    st = L.lib().rm_score_topk_noalloc(ctypes.byref(index.idx), 256, 256, n, 32, 256, 256, None)
    assert st == L.RM_ESIZE
    st = L.lib().rm_score_topk_noalloc(ctypes.byref(index.idx), None, 256, 10, 32, 256, 256, None)
    assert st == L.RM_EINVAL
