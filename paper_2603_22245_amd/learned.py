"""Learned angle offsets: device-side training and evaluation.

Thin wrapper over the C-ABI (argument marshalling and buffer ownership only;
every step runs in the library's kernels).  The encoding: 9-mer tokens at
locations p = 0..n-9 (the s-mer locations of §2.1 with s = 9); the middle
letter picks the component, the 8 flanking letters feed a 32-64-128 network
whose output gives the token's phase offset per factor; the token adds
exp(i (theta_k p + delta)) (§2.2 phases plus the offset).  Training minimises a
pairwise logistic ranking loss between the fidelities (§2.4) of string pairs
and their edit distances.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import _lib as L

N_PARAMS = L.RM_LEARNED_PARAMS
N_IN, N_HID, N_OUT = 32, 64, 128


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2603_22245_amd.learned needs a ROCm GPU")
    return torch


def init_params(seed: int = 0) -> np.ndarray:
    """First layer ~ U(-1/sqrt(32), 1/sqrt(32)); output layer zero, so training
    starts from the plain encoding of the token middles."""
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(-1, 1, (N_HID, N_IN)) / np.sqrt(N_IN)
    b1 = rng.uniform(-1, 1, N_HID) / np.sqrt(N_IN)
    return np.concatenate([w1.ravel(), b1, np.zeros(N_OUT * N_HID), np.zeros(N_OUT)]).astype(
        np.float32)


@dataclasses.dataclass
class PairSet:
    """Device copies of string pairs (a_i, b_i) and, optionally, their labels."""
    a: object
    a_off: object
    b: object
    b_off: object
    n: int
    ld: Optional[object] = None


def upload_pairs(a, a_off, b, b_off, ld=None, device="cuda") -> PairSet:
    torch = _torch()
    t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt).to(device)
    n = int(np.asarray(a_off).shape[0] - 1)
    return PairSet(a=t(a, torch.uint8), a_off=t(a_off, torch.int64), b=t(b, torch.uint8),
                   b_off=t(b_off, torch.int64), n=n,
                   ld=None if ld is None else t(ld, torch.int32))


def levenshtein(ps: PairSet, stream=None):
    """Exact edit distances of the pairs (int32 device tensor)."""
    torch = _torch()
    out = torch.empty(ps.n, dtype=torch.int32, device=ps.a.device)
    L.rm_levenshtein(ps.a, ps.a_off, ps.b, ps.b_off, ps.n, out, stream)
    return out


def encode(params, seq, off, n_strings: int, nominal_len: int, stream=None):
    """Encodings [n_strings, 256] (FP32); params None gives the plain encoding."""
    torch = _torch()
    out = torch.empty((n_strings, 256), dtype=torch.float32, device=seq.device)
    L.rm_learned_encode(params, seq, off, n_strings, nominal_len, out, stream)
    return out


def pair_fidelity(params, ps: PairSet, nominal_len: int, stream=None):
    """F(a_i, b_i) under the learned (params) or plain (None) encoding."""
    torch = _torch()
    ca = encode(params, ps.a, ps.a_off, ps.n, nominal_len, stream)
    cb = encode(params, ps.b, ps.b_off, ps.n, nominal_len, stream)
    F = torch.empty(ps.n, dtype=torch.float32, device=ps.a.device)
    L.rm_pair_fidelity(ca, cb, ps.n, F, stream)
    return F


def _slice(ps: PairSet, i0: int, i1: int):
    """Pointers of pairs i0..i1-1 (offsets stay absolute, so the offset arrays
    are simply advanced)."""
    es = ps.a_off.element_size()
    return (ps.a.data_ptr(), ps.a_off.data_ptr() + i0 * es, ps.b.data_ptr(),
            ps.b_off.data_ptr() + i0 * es, ps.ld.data_ptr() + i0 * ps.ld.element_size())


class Trainer:
    """Adam training of the offset network on device; the state vector is
    [params | m | v | step] (FP32)."""

    def __init__(self, params=None, nominal_len: int = 150, batch: int = 1024, lr: float = 3e-3,
                 seed: int = 0, device="cuda"):
        torch = _torch()
        if not 2 <= batch <= L.RM_LEARNED_MAX_PAIRS:
            raise ValueError(f"batch must lie in 2..{L.RM_LEARNED_MAX_PAIRS}")
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        if p.shape != (N_PARAMS,):
            raise ValueError(f"params must have {N_PARAMS} values")
        self.N, self.batch, self.lr = nominal_len, batch, lr
        self.state = torch.zeros(3 * N_PARAMS + 1, dtype=torch.float32, device=device)
        self.state[:N_PARAMS] = torch.from_numpy(p).to(device)
        self.ws_bytes = L.rm_learned_workspace_bytes(batch)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1 << 16, dtype=torch.float32, device=device)
        self.grad = torch.empty(N_PARAMS, dtype=torch.float32, device=device)
        self._graphs = {}

    @property
    def params(self):
        return self.state[:N_PARAMS]

    def gradient(self, ps: PairSet, i0: int = 0, n: Optional[int] = None, stream=None):
        """Loss and gradient on pairs i0..i0+n-1 (no update)."""
        n = ps.n - i0 if n is None else n
        if n > self.batch:
            raise ValueError("more pairs than the workspace was sized for")
        a, ao, b, bo, ld = _slice(ps, i0, i0 + n)
        L.rm_learned_gradient(self.params, a, ao, b, bo, ld, n, self.N, self.ws, self.ws_bytes,
                              self.grad, self.loss, stream)
        return self.loss[0:1], self.grad

    def _steps(self, ps: PairSet, lr: float, stream):
        n_steps = ps.n // self.batch
        if n_steps > self.loss.shape[0]:
            raise ValueError("too many steps per epoch for the loss buffer")
        for s in range(n_steps):
            a, ao, b, bo, ld = _slice(ps, s * self.batch, (s + 1) * self.batch)
            L.rm_learned_train_step(self.state, lr, a, ao, b, bo, ld, self.batch, self.N, self.ws,
                                    self.ws_bytes, self.loss.data_ptr() + 4 * s, stream)
        return n_steps

    def epoch(self, ps: PairSet, lr: Optional[float] = None, graph: bool = False, stream=None):
        """One pass over the pair set in consecutive batches (the last partial
        batch is dropped); returns the per-step losses (device tensor).  With
        graph=True the epoch's launches are captured once per (pair set, lr) and
        replayed."""
        torch = _torch()
        if ps.ld is None:
            raise ValueError("the pair set has no labels")
        lr = self.lr if lr is None else lr
        if not graph:
            n = self._steps(ps, lr, stream)
            return self.loss[:n]
        key = (id(ps), lr)
        if key not in self._graphs:
            s = torch.cuda.Stream() if stream is None else stream
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                L.rm_capture_begin(s)
                n = self._steps(ps, lr, s)
                g = L.rm_capture_end(s)
            self._graphs[key] = (g, n, s)
        g, n, s = self._graphs[key]
        s.wait_stream(torch.cuda.current_stream())
        L.rm_graph_launch(g, s)
        torch.cuda.current_stream().wait_stream(s)
        return self.loss[:n]

    def close(self):
        for g, _, _ in self._graphs.values():
            L.rm_graph_destroy(g)
        self._graphs.clear()
