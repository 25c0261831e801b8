"""Device-buffer plumbing around the C ABI: allocate with torch, call the
library in order (index -> read heads -> product + top-k -> FP32 rescore).

Every step of the method runs inside librotormap's HIP kernels; this module
only owns the torch tensors that hold their inputs and outputs.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import _lib as L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a ROCm GPU is required (torch.cuda.is_available() is False)")
    return torch


@dataclasses.dataclass
class Index:
    params: L.rm_params
    idx: L.rm_index
    buf: object      # torch uint8 tensor owning the index memory
    ref: object      # torch uint8 tensor, the reference letters on the device

    @property
    def n_windows(self) -> int:
        return int(self.idx.n_windows)

    def embeddings(self):
        """The stored [W, 256] embeddings as a torch view (float32/float16/uint8)."""
        torch = _torch()
        W = self.n_windows
        dt = {L.RM_FP32: torch.float32, L.RM_FP16: torch.float16, L.RM_FP8_E4M3: torch.uint8}
        dtype = dt[self.params.precision]
        esz = torch.tensor([], dtype=dtype).element_size()
        return self.buf[: W * 256 * esz].view(dtype).view(W, 256)

    def scales(self):
        off = self.idx.d_scale - self.buf.data_ptr()
        return self.buf[off: off + 4 * self.n_windows].view(_torch().float32)

    def norms2(self):
        off = self.idx.d_norm2 - self.buf.data_ptr()
        return self.buf[off: off + 4 * self.n_windows].view(_torch().float32)


def build_index(ref: np.ndarray, window_len=150, stride=1, precision="fp16", schedule="default",
                reanchor=0, stream=None, device="cuda") -> Index:
    torch = _torch()
    p = L.make_params(window_len, stride, L.RM_DIM, schedule, precision, reanchor)
    d_ref = torch.from_numpy(np.ascontiguousarray(ref, dtype=np.uint8)).to(device)
    nbytes = L.rm_index_bytes(int(ref.shape[0]), p)
    if nbytes == 0:
        raise L.RotorMapError(L.RM_ESIZE, "rm_index_bytes")
    buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
    idx = L.rm_encode_reference(d_ref, int(ref.shape[0]), p, buf, nbytes, stream)
    return Index(p, idx, buf, d_ref)


@dataclasses.dataclass
class ReadBatch:
    n: int
    seq: object
    off: object
    emb: object
    scale: object


def upload_reads(index: Index, seq: np.ndarray, offsets: np.ndarray, device="cuda") -> ReadBatch:
    torch = _torch()
    n = int(offsets.shape[0] - 1)
    d_seq = torch.from_numpy(np.ascontiguousarray(seq, dtype=np.uint8)).to(device)
    d_off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(device)
    emb = torch.empty(L.rm_read_emb_bytes(n, index.params), dtype=torch.uint8, device=device)
    scale = torch.empty(n, dtype=torch.float32, device=device)
    return ReadBatch(n, d_seq, d_off, emb, scale)


@dataclasses.dataclass
class MapBuffers:
    k: int
    k_fetch: int
    ws: object
    ws_bytes: int
    cand_idx: object
    cand_score: object
    top_idx: object
    top_score: object


def map_buffers(index: Index, n_reads: int, k: int, k_fetch: Optional[int] = None,
                device="cuda") -> MapBuffers:
    torch = _torch()
    k_fetch = k if k_fetch is None else k_fetch
    ws_bytes = L.rm_score_workspace_bytes(index.idx, n_reads, k_fetch)
    if ws_bytes == 0:
        raise L.RotorMapError(L.RM_ESIZE, "rm_score_workspace_bytes")
    return MapBuffers(
        k, k_fetch,
        torch.empty(ws_bytes, dtype=torch.uint8, device=device), ws_bytes,
        torch.empty((n_reads, k_fetch), dtype=torch.int32, device=device),
        torch.empty((n_reads, k_fetch), dtype=torch.float32, device=device),
        torch.empty((n_reads, k), dtype=torch.int32, device=device),
        torch.empty((n_reads, k), dtype=torch.float32, device=device))


def encode_reads(index: Index, reads: ReadBatch, stream=None):
    L.rm_encode_reads(index.idx, reads.seq, reads.off, reads.n, reads.emb, reads.scale, stream)


def score_topk(index: Index, reads: ReadBatch, bufs: MapBuffers, stream=None):
    L.rm_score_topk(index.idx, reads.emb, reads.scale, reads.n, bufs.k_fetch, bufs.cand_idx,
                    bufs.cand_score, bufs.ws, bufs.ws_bytes, stream)


def rescore(index: Index, reads: ReadBatch, bufs: MapBuffers, stream=None):
    L.rm_rescore(index.idx, index.ref, reads.seq, reads.off, reads.n, bufs.k_fetch,
                 bufs.cand_idx, bufs.k, bufs.top_idx, bufs.top_score, stream)


def map_reads(index: Index, reads: ReadBatch, bufs: MapBuffers, stream=None):
    """encode heads -> product + top-k_fetch -> FP32 rescore to top-k."""
    encode_reads(index, reads, stream)
    score_topk(index, reads, bufs, stream)
    rescore(index, reads, bufs, stream)
