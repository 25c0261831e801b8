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
    learned: object = None  # FP32 network parameters (device) of a learned index
    delta: object = None    # token offsets of the reference [G-8, 32] (learned index)
    token_map: object = None  # device copy of the caller's s-mer class table (token index)

    @property
    def n_windows(self) -> int:
        return int(self.idx.n_windows)

    @property
    def real_dim(self) -> int:
        """Reals per stored row: 256 (192 in the letter-sum form), or
        2 n_class m for a token encoding."""
        p = self.params
        return 2 * p.n_class * p.n_freq if p.n_class else (192 if p.reduced else 256)

    def embeddings(self):
        """The stored [W, real_dim] embeddings as a torch view (float32/float16/uint8)."""
        torch = _torch()
        W, D = self.n_windows, self.real_dim
        dt = {L.RM_FP32: torch.float32, L.RM_FP16: torch.float16, L.RM_FP8_E4M3: torch.uint8}
        dtype = dt[self.params.precision]
        esz = torch.tensor([], dtype=dtype).element_size()
        return self.buf[: W * D * esz].view(dtype).view(W, D)

    def scales(self):
        off = self.idx.d_scale - self.buf.data_ptr()
        return self.buf[off: off + 4 * self.n_windows].view(_torch().float32)

    def norms2(self):
        off = self.idx.d_norm2 - self.buf.data_ptr()
        return self.buf[off: off + 4 * self.n_windows].view(_torch().float32)


def _delta_buffer(n_letters: int, device):
    torch = _torch()
    nbytes = L.rm_delta_bytes(n_letters)
    if nbytes == 0:
        raise L.RotorMapError(L.RM_ESIZE, "rm_delta_bytes")
    return torch.empty((nbytes // 128, 32), dtype=torch.float32, device=device)


def letter_sum_applies(ref, window_len, precision, schedule="default", token=False,
                       learned=None) -> bool:
    """Whether build_index stores an index in the letter-sum form
    (rm_params.reduced) by default: the plain letter encoding with integer
    factors, windows longer than m, an FP16 index and a reference of letters
    only (codes 0..3).  FP8 indexes can take the form too (reduced=True), but
    not by default: in it e4m3's error per score grows by about sqrt(4/3)
    (fewer, larger components of the same unit vector)."""
    if token or learned is not None or schedule != "default" or window_len <= L.RM_DIM:
        return False
    if precision not in ("fp16", L.RM_FP16):
        return False
    if isinstance(ref, np.ndarray):
        return ref.size == 0 or int(ref.max()) < 4
    return ref.numel() == 0 or int(ref.max().item()) < 4


def build_index(ref: np.ndarray, window_len=150, stride=1, precision="fp16", schedule="default",
                reanchor=0, stream=None, device="cuda", learned=None, mer_len=1,
                n_freq=None, token_map=None, n_class=None, reduced=None) -> Index:
    """Encode the reference's windows.  learned: network parameters (10,432
    FP32 values, numpy or device tensor) for the learned encoding, else plain.
    reduced: store the letter-sum form (192 reals per row); None chooses it
    wherever it applies (letter_sum_applies).

    Token encodings (s-mers): mer_len = s, token_map = None (class = s-mer
    code, n_class = 4^s) or a table of 4^s classes (uint8; a value >= n_class
    leaves an s-mer out), n_class (default 4^s without a map, 128 / n_freq
    with one) and n_freq = m (default 128 / n_class, or 1024 / n_class for
    n_class above 64).  n_class * n_freq is 128 (every precision) or 1,024
    (FP16 or FP8)."""
    torch = _torch()
    d_map = None
    token = mer_len > 1 or token_map is not None or n_class is not None
    if token_map is not None:
        if isinstance(token_map, np.ndarray) or not hasattr(token_map, "data_ptr"):
            d_map = torch.as_tensor(np.ascontiguousarray(token_map, dtype=np.uint8)).to(device)
        else:  # already a device tensor (e.g. frequent_token_map's)
            d_map = token_map
        if d_map.numel() != 4 ** mer_len:
            raise ValueError(f"token_map must have 4^{mer_len} entries")
        if n_freq is None and n_class is None:
            raise ValueError("n_freq or n_class is required with a token map")
    if not token:
        n_class, n_freq = 0, L.RM_DIM if n_freq is None else n_freq
    else:
        if n_class is None:
            n_class = 4 ** mer_len if token_map is None else 128 // n_freq
        if n_freq is None:
            n_freq = max(1, (128 if n_class <= 64 else 1024) // n_class)
    if reduced is None:
        reduced = letter_sum_applies(ref, window_len, precision, schedule, token, learned)
    p = L.make_params(window_len, stride, n_freq, schedule, precision, reanchor, mer_len, n_class,
                      d_map, reduced)
    if isinstance(ref, np.ndarray):
        d_ref = torch.from_numpy(np.ascontiguousarray(ref, dtype=np.uint8)).to(device)
    else:  # already a device tensor
        d_ref = ref
    nbytes = L.rm_index_bytes(int(d_ref.numel()), p)
    if nbytes == 0:
        raise L.RotorMapError(L.RM_ESIZE, "rm_index_bytes")
    buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
    if learned is None:
        idx = L.rm_encode_reference(d_ref, int(d_ref.numel()), p, buf, nbytes, stream)
        return Index(p, idx, buf, d_ref, token_map=d_map)
    params = torch.as_tensor(learned, dtype=torch.float32).to(device).contiguous()
    if params.numel() != L.RM_LEARNED_PARAMS:
        raise ValueError(f"learned parameters must have {L.RM_LEARNED_PARAMS} values")
    delta = _delta_buffer(int(d_ref.numel()), device)
    L.rm_mlp_infer(params, d_ref, int(d_ref.numel()), delta, stream)
    idx = L.rm_encode_reference_learned(d_ref, int(d_ref.numel()), p, delta, buf, nbytes, stream)
    return Index(p, idx, buf, d_ref, params, delta)


def frequent_token_map(ref, mer_len: int, n_class: int, stream=None, device="cuda"):
    """The compact context-aware map of §2.6 on the device: the n_class most
    frequent s-mers of `ref` (numpy or device uint8) as classes in code order,
    the others RM_TOKEN_SKIP.  Returns (map [4^s] uint8, counts [4^s] int32 view
    of the uint32 counts) as device tensors."""
    torch = _torch()
    d_ref = ref if hasattr(ref, "data_ptr") else \
        torch.from_numpy(np.ascontiguousarray(ref, dtype=np.uint8)).to(device)
    nbytes = L.rm_token_counts_bytes(mer_len)
    if nbytes == 0:
        raise L.RotorMapError(L.RM_ESIZE, "rm_token_counts_bytes")
    counts = torch.empty(nbytes // 4, dtype=torch.int32, device=device)
    d_map = torch.empty(4 ** mer_len, dtype=torch.uint8, device=device)
    L.rm_token_counts(d_ref, int(d_ref.numel()), mer_len, counts, stream)
    L.rm_token_map_frequent(counts, mer_len, n_class, d_map, stream)
    return d_map, counts


@dataclasses.dataclass
class ReadBatch:
    n: int
    seq: object
    off: object
    emb: object
    scale: object
    delta: object = None  # token offsets of seq (learned index)


def upload_reads(index: Index, seq: np.ndarray, offsets: np.ndarray, device="cuda") -> ReadBatch:
    torch = _torch()
    n = int(offsets.shape[0] - 1)
    d_seq = torch.from_numpy(np.ascontiguousarray(seq, dtype=np.uint8)).to(device)
    d_off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(device)
    emb = torch.empty(L.rm_read_emb_bytes(n, index.params), dtype=torch.uint8, device=device)
    scale = torch.empty(n, dtype=torch.float32, device=device)
    delta = None if index.learned is None else _delta_buffer(int(d_seq.numel()), device)
    return ReadBatch(n, d_seq, d_off, emb, scale, delta)


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
    if index.learned is None:
        L.rm_encode_reads(index.idx, reads.seq, reads.off, reads.n, reads.emb, reads.scale, stream)
        return
    L.rm_mlp_infer(index.learned, reads.seq, int(reads.seq.numel()), reads.delta, stream)
    L.rm_encode_reads_learned(index.idx, reads.seq, reads.off, reads.n, reads.delta, reads.emb,
                              reads.scale, stream)


def score_topk(index: Index, reads: ReadBatch, bufs: MapBuffers, stream=None):
    L.rm_score_topk(index.idx, reads.emb, reads.scale, reads.n, bufs.k_fetch, bufs.cand_idx,
                    bufs.cand_score, bufs.ws, bufs.ws_bytes, stream)


def rescore(index: Index, reads: ReadBatch, bufs: MapBuffers, stream=None):
    if index.learned is None:
        L.rm_rescore(index.idx, index.ref, reads.seq, reads.off, reads.n, bufs.k_fetch,
                     bufs.cand_idx, bufs.k, bufs.top_idx, bufs.top_score, stream)
        return
    L.rm_rescore_learned(index.idx, index.ref, index.delta, reads.seq, reads.off, reads.delta,
                         reads.n, bufs.k_fetch, bufs.cand_idx, bufs.k, bufs.top_idx,
                         bufs.top_score, stream)


def map_reads(index: Index, reads: ReadBatch, bufs: MapBuffers, stream=None):
    """encode heads -> product + top-k_fetch -> FP32 rescore to top-k."""
    encode_reads(index, reads, stream)
    score_topk(index, reads, bufs, stream)
    rescore(index, reads, bufs, stream)


def window_thresholds(index: Index, err: float, copies: int = 16, rank: int = 1, seed: int = 1,
                      stream=None):
    """Per-window cutting thresholds at a target mutation rate (§3.3): the
    rank-th smallest fidelity of each window with `copies` mutated copies of
    itself.  Returns a device float32 tensor [W]."""
    torch = _torch()
    thr = torch.empty(index.n_windows, dtype=torch.float32, device=index.buf.device)
    L.rm_window_thresholds(index.idx, index.ref, err, copies, rank, seed, thr, stream)
    return thr


@dataclasses.dataclass
class ThresholdHits:
    hit_off: object    # [R+1] int64: read r's span is hit_idx[hit_off[r] : hit_off[r+1]]
    n_found: object    # [R] int32: hits of read r, ranked at the start of its span
    hit_idx: object    # [capacity] int32 window ids (-1 past n_found)
    hit_score: object  # [capacity] FP32 fidelities
    total: object      # [1] int64: proposals found (> capacity: incomplete)
    capacity: int

    def lists(self):
        """Per read, (window ids, F) of its hits as numpy arrays (host)."""
        off = self.hit_off.cpu().numpy()
        n = self.n_found.cpu().numpy()
        idx = self.hit_idx.cpu().numpy()
        sc = self.hit_score.cpu().numpy()
        return [(idx[off[r]:off[r] + n[r]], sc[off[r]:off[r] + n[r]]) for r in range(n.size)]


def score_threshold(index: Index, reads: ReadBatch, thr, floor: float = 0.0,
                    capacity: Optional[int] = None, stream=None) -> ThresholdHits:
    """The threshold regime (§3.5): every window whose FP32 fidelity with the
    read passes max(its threshold, floor).  The read heads must have been
    encoded (encode_reads).  If the proposals exceed `capacity` the call is
    repeated once with the capacity the first pass reported."""
    torch = _torch()
    dev = index.buf.device
    cap = capacity if capacity is not None else max(1024, 64 * reads.n)
    while True:
        ws_bytes = L.rm_threshold_workspace_bytes(reads.n, cap)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        h = ThresholdHits(torch.empty(reads.n + 1, dtype=torch.int64, device=dev),
                          torch.empty(reads.n, dtype=torch.int32, device=dev),
                          torch.empty(cap, dtype=torch.int32, device=dev),
                          torch.empty(cap, dtype=torch.float32, device=dev),
                          torch.empty(1, dtype=torch.int64, device=dev), cap)
        L.rm_score_threshold(index.idx, index.ref, reads.emb, reads.scale, reads.seq, reads.off,
                             reads.n, thr, floor, cap, h.hit_off, h.n_found, h.hit_idx,
                             h.hit_score, h.total, ws, ws_bytes, stream)
        total = int(h.total.cpu()[0])
        if total <= cap or capacity is not None:
            return h
        cap = total


@dataclasses.dataclass
class StrandResult:
    top_idx: object      # [R][k] window ids
    top_score: object    # [R][k] FP32 fidelities
    top_strand: object   # [R][k] int8: 0 forward, 1 reverse complement, -1 empty
    n_found: object      # [R] entries kept (0 = unmapped)


def upload_reads_both_strands(index: Index, seq: np.ndarray, offsets: np.ndarray,
                              device="cuda", stream=None) -> ReadBatch:
    """A batch of 2R reads: the R reads, then their reverse complements
    (computed on the GPU by rm_reverse_complement) with the same lengths."""
    torch = _torch()
    n = int(offsets.shape[0] - 1)
    nl = int(offsets[-1] - offsets[0])
    off = np.ascontiguousarray(offsets, dtype=np.int64) - int(offsets[0])
    d_seq = torch.empty(2 * nl, dtype=torch.uint8, device=device)
    d_seq[:nl].copy_(torch.from_numpy(np.ascontiguousarray(seq[offsets[0]:offsets[-1]],
                                                           dtype=np.uint8)))
    off2 = np.concatenate([off, off[1:] + nl])
    d_off = torch.from_numpy(off2).to(device)
    L.rm_reverse_complement(d_seq[:nl], d_off[:n + 1], n, nl, d_seq[nl:], stream)
    emb = torch.empty(L.rm_read_emb_bytes(2 * n, index.params), dtype=torch.uint8, device=device)
    scale = torch.empty(2 * n, dtype=torch.float32, device=device)
    delta = None if index.learned is None else _delta_buffer(int(d_seq.numel()), device)
    return ReadBatch(2 * n, d_seq, d_off, emb, scale, delta)


def map_reads_both_strands(index: Index, reads2: ReadBatch, bufs2: MapBuffers,
                           min_fidelity: float = 0.0, stream=None) -> StrandResult:
    """Map the 2R-read batch of upload_reads_both_strands (bufs2 sized for 2R
    reads) and combine each read's forward and reverse-complement lists with
    rm_merge_strands, keeping entries with F >= min_fidelity."""
    torch = _torch()
    map_reads(index, reads2, bufs2, stream)
    n, k = reads2.n // 2, bufs2.k
    dev = bufs2.top_idx.device
    out = StrandResult(torch.empty((n, k), dtype=torch.int32, device=dev),
                       torch.empty((n, k), dtype=torch.float32, device=dev),
                       torch.empty((n, k), dtype=torch.int8, device=dev),
                       torch.empty(n, dtype=torch.int32, device=dev))
    L.rm_merge_strands(bufs2.top_idx[:n], bufs2.top_score[:n], bufs2.top_idx[n:],
                       bufs2.top_score[n:], n, k, min_fidelity, out.top_idx, out.top_score,
                       out.top_strand, out.n_found, stream)
    return out


def refine(index: Index, reads: ReadBatch, bufs: MapBuffers, radius: int, ws=None, stream=None):
    """Step-1 refinement around the coarse candidates in bufs.cand_idx (§3.4):
    writes the k best step-1 window starts and their FP32 fidelities into
    bufs.top_idx / bufs.top_score.  `index` is the coarse (stride > 1) index;
    `ws` a device workspace of rm_refine_workspace_bytes (allocated if None)."""
    if index.learned is not None:
        raise ValueError("refinement is implemented for the plain and token encodings")
    torch = _torch()
    need = L.rm_refine_workspace_bytes(reads.n, bufs.k_fetch, radius)
    if ws is None:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=bufs.cand_idx.device)
    L.rm_refine(index.idx, index.ref, reads.seq, reads.off, reads.n, bufs.k_fetch, bufs.cand_idx,
                radius, bufs.k, bufs.top_idx, bufs.top_score, ws, ws.numel(), stream)
    return ws


def map_reads_coarse(index: Index, reads: ReadBatch, bufs: MapBuffers, radius: int, ws=None,
                     stream=None):
    """encode heads -> product over the coarse windows -> step-1 refinement."""
    encode_reads(index, reads, stream)
    score_topk(index, reads, bufs, stream)
    return refine(index, reads, bufs, radius, ws, stream)


# ---------------------------------------------------------------- batching

BUCKETS = (100, 200, 400, 800, 1600, 3200, 6400)


@dataclasses.dataclass
class Bucket:
    length: int            # head length N_b (the bucket's window length)
    stride: int
    read_ids: np.ndarray   # indices of the batch's reads in this bucket
    index: Index
    reads: ReadBatch
    bufs: MapBuffers


class BatchMapper:
    """Reads of uneven length: one index per head length (bucket), every bucket's
    reads scored against its index in one persistent launch (rm_score_topk_groups),
    then FP32 rescore per bucket.  Buckets without reads are skipped; reads shorter
    than the smallest bucket are left unmapped (id -1).  `reduced` picks the row
    form of the indexes as in build_index (None: the precision's default)."""

    def __init__(self, ref: np.ndarray, seq: np.ndarray, offsets: np.ndarray, k: int = 8,
                 k_fetch: int = 16, precision: str = "fp16", buckets=BUCKETS,
                 stride_div: int = 100, device="cuda", reduced=None):
        torch = _torch()
        self.k, self.k_fetch, self.precision = k, k_fetch, precision
        self.n_reads = int(offsets.shape[0] - 1)
        bucket_of, count = L.rm_bucket_reads(offsets, buckets)
        self.bucket_of = bucket_of
        self.buckets = []
        d_ref = torch.from_numpy(np.ascontiguousarray(ref, dtype=np.uint8)).to(device)
        for b, n_b in enumerate(buckets):
            ids = np.nonzero(bucket_of == b)[0]
            if ids.size == 0:
                continue
            stride = max(1, n_b // stride_div)
            index = build_index(d_ref, window_len=n_b, stride=stride, precision=precision,
                                device=device, reduced=reduced)
            # this bucket's reads, concatenated (each keeps all its letters)
            lens = offsets[ids + 1] - offsets[ids]
            off = np.zeros(ids.size + 1, dtype=np.int64)
            np.cumsum(lens, out=off[1:])
            parts = [seq[offsets[i]:offsets[i + 1]] for i in ids]
            bseq = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
            rb = upload_reads(index, bseq, off, device)
            bufs = map_buffers(index, ids.size, k, k_fetch, device)
            self.buckets.append(Bucket(n_b, stride, ids, index, rb, bufs))
        self.tune = None
        self.ws_bytes = self._ws_bytes(None)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.graph = None

    def _ws_bytes(self, tune):
        return L.rm_score_groups_workspace_bytes([b.index.idx for b in self.buckets],
                                                 [b.reads.n for b in self.buckets],
                                                 self.k_fetch, tune)

    def _group_args(self):
        bs = self.buckets
        return ([b.index.idx for b in bs], [b.reads.emb for b in bs],
                [b.reads.scale for b in bs], [b.reads.n for b in bs], self.k_fetch,
                [b.bufs.cand_idx for b in bs], [b.bufs.cand_score for b in bs])

    def autotune(self, cache_path=None, stream=None):
        """Pick the scoring launch's tile shape by timing candidates on these inputs
        (reads must be encoded first)."""
        torch = _torch()
        # the largest candidate workspace: 128-read tiles and the smallest chunks
        need = max(self._ws_bytes(L.rm_tuning(rt, ct)) for rt in (128, 256)
                   for ct in (0, 128, 512, 2048, 8192))
        if need > self.ws.numel():
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.ws.device)
        idxs, emb, scale, nr, kf, ci, cs = self._group_args()
        best, ms = L.rm_autotune_score(idxs, emb, scale, nr, kf, ci, cs, self.ws, self.ws.numel(),
                                       cache_path, stream)
        self.tune = best
        self.ws_bytes = self._ws_bytes(best)
        return best, ms

    def rebuild_indexes(self, stream=None):
        """Re-encode every bucket's index in place (same buffers)."""
        for b in self.buckets:
            idx = L.rm_encode_reference(b.index.ref, int(b.index.ref.numel()), b.index.params,
                                        b.index.buf, b.index.buf.numel(), stream)
            b.index.idx = idx

    def encode(self, stream=None):
        for b in self.buckets:
            encode_reads(b.index, b.reads, stream)

    def score(self, stream=None):
        idxs, emb, scale, nr, kf, ci, cs = self._group_args()
        L.rm_score_topk_groups(idxs, emb, scale, nr, kf, ci, cs, self.ws, self.ws_bytes, self.tune,
                               stream)

    def rescore(self, stream=None):
        for b in self.buckets:
            rescore(b.index, b.reads, b.bufs, stream)

    def run(self, stream=None):
        self.encode(stream)
        self.score(stream)
        self.rescore(stream)

    def capture(self, stream, with_index=False):
        """Record run() (preceded by the index builds if with_index) on `stream`
        (not the null stream) into a HIP graph."""
        if self.graph is not None:
            L.rm_graph_destroy(self.graph)
        L.rm_capture_begin(stream)
        try:
            if with_index:
                self.rebuild_indexes(stream)
            self.run(stream)
        finally:
            self.graph = L.rm_capture_end(stream)
        return self.graph

    def replay(self, stream):
        L.rm_graph_launch(self.graph, stream)

    def results(self):
        """Top-k window ids and FP32 scores of every read (id -1, score 0 for no location),
        and each read's bucket index."""
        ids = np.full((self.n_reads, self.k), -1, dtype=np.int32)
        sc = np.zeros((self.n_reads, self.k), dtype=np.float32)
        for b in self.buckets:
            ids[b.read_ids] = b.bufs.top_idx.cpu().numpy()
            sc[b.read_ids] = b.bufs.top_score.cpu().numpy()
        return ids, sc

    def close(self):
        if self.graph is not None:
            L.rm_graph_destroy(self.graph)
            self.graph = None
