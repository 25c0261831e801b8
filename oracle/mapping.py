"""FP64 oracle: RotorMap's brute-force mapping (§3.1) and its metrics.

TEST INFRASTRUCTURE ONLY (see the package docstring).

§3.1: windows of length N slide over the reference with a step; each window
is encoded, forming the index.  A read's head (its first N letters) is
encoded and its fidelity with every window is computed; the best-scoring
windows are the candidate locations.

Here: window starts j = 0, sigma, 2 sigma, ... up to G-N, so there are
W = floor((G-N)/sigma) + 1 windows; F(r, j) = |<x_r|c_j>|^2 / (X_r C_j) with
F = 0 when either vector is degenerate; the top-k list of a read is ordered by
F descending, then by the window's position in the index ascending, and an
entry with F = 0 is no location (id -1, score 0).

Windows are processed in chunks to bound memory.  The top-k of a union of
chunks is the top-k of the union of the chunks' top-k lists, so merging the
per-chunk lists is the same selection as one pass over all windows.
"""
from __future__ import annotations

import numpy as np

from . import rope

TIE_TAU = 1e-5  # fidelity gap under which two candidates count as tied in metrics
# Scores closer than this are equal for ranking: FP64 summation order (which
# a matrix product may vary with a row's position in a batch) moves F by
# ~1e-16, so equal windows must not be ordered by rounding noise.
RANK_EPS = 1e-12


def n_windows(G: int, N: int, stride: int = 1) -> int:
    if G < N:
        return 0
    return (G - N) // stride + 1


def window_starts(G: int, N: int, stride: int = 1) -> np.ndarray:
    return np.arange(n_windows(G, N, stride), dtype=np.int64) * stride


def window_letters(ref: np.ndarray, starts: np.ndarray, N: int) -> np.ndarray:
    return ref[starts[:, None] + np.arange(N)[None, :]]


NO_LETTER = 4  # a code outside A,C,G,T: it adds nothing to any encoding


def read_heads(seq: np.ndarray, offsets: np.ndarray, N: int) -> np.ndarray:
    """First N letters of every read, [R, N] (§3.1 encodes a read's head).  A
    read shorter than N has no head of length N: its row is all NO_LETTER,
    which encodes as the zero vector, so it scores 0 with every window and has
    no location."""
    offsets = np.asarray(offsets, dtype=np.int64)
    short = np.diff(offsets) < N
    pos = np.where(short[:, None], 0, offsets[:-1, None] + np.arange(N)[None, :])
    heads = np.asarray(seq)[pos].astype(np.uint8)
    heads[short] = NO_LETTER
    return heads


def no_location(ids: np.ndarray, F: np.ndarray) -> np.ndarray:
    """§3 asks for a read's position only if one exists.  A fidelity of exactly
    0 means the read head or the window is the zero vector (degenerate, or a
    read shorter than N), so that window is no location: its id becomes -1
    (its score stays 0).  Returns the new ids."""
    ids = np.array(ids, copy=True)
    ids[np.asarray(F) == 0] = -1
    return ids


def normalized_rows(C: np.ndarray, N: int):
    """Normalise each row; degenerate rows become zero.  Returns (rows, sq_norms)."""
    n2 = np.sum(C.real ** 2 + C.imag ** 2, axis=1)
    ok = n2 >= rope.DEGENERATE_REL * N
    out = np.zeros_like(C)
    out[ok] = C[ok] / np.sqrt(n2[ok])[:, None]
    return out, n2


def fidelity_matrix(Xn: np.ndarray, Cn: np.ndarray) -> np.ndarray:
    """F[r, j] = |<x_r|c_j>|^2 for unit (or zero) rows."""
    return np.abs(np.conj(Xn) @ Cn.T) ** 2


def rank_order(F: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """Order of candidates by F descending, then id ascending, where scores that
    differ by at most RANK_EPS from their neighbour in F order form one tie group."""
    o = np.argsort(-F, kind="stable")
    Fs = F[o]
    group = np.cumsum(np.r_[True, (Fs[:-1] - Fs[1:]) > RANK_EPS])
    return o[np.lexsort((ids[o], group))]


def topk_rows(F: np.ndarray, ids: np.ndarray, k: int):
    """Per row, the k best by `rank_order`; returns (ids [R,k], F [R,k]).

    Every entry within RANK_EPS of the row's k-th largest F or above is a
    candidate, so all members of a boundary tie group take part."""
    R, n = F.shape
    ids = np.broadcast_to(ids, F.shape)
    kk = min(k, n)
    kth = -np.partition(-F, kk - 1, axis=1)[:, kk - 1]
    out_i = np.empty((R, kk), dtype=np.int64)
    out_f = np.empty((R, kk))
    for r in range(R):
        cand = np.nonzero(F[r] >= kth[r] - RANK_EPS)[0]
        order = rank_order(F[r, cand], ids[r, cand])[:kk]
        out_i[r] = ids[r, cand[order]]
        out_f[r] = F[r, cand[order]]
    return out_i, out_f


def map_reads(ref: np.ndarray, heads: np.ndarray, N: int, m: int = 32, k: int = 8,
              stride: int = 1, schedule: str = "default", chunk: int = 65536,
              window_range=None):
    """Exact top-k windows of every read head by brute force over all windows.

    Returns (idx [R,k] int64 window ids, F [R,k] float64).  `window_range`
    restricts the scan to window ids [lo, hi) (used to time a bounded sample)."""
    W = n_windows(ref.shape[0], N, stride)
    lo, hi = (0, W) if window_range is None else window_range
    Xn, _ = normalized_rows(rope.encode_many(heads, N, m, schedule), N)
    R = Xn.shape[0]
    best_i = np.full((R, 0), -1, dtype=np.int64)
    best_f = np.zeros((R, 0))
    for a in range(lo, hi, chunk):
        b = min(hi, a + chunk)
        ids = np.arange(a, b, dtype=np.int64)
        Cn, _ = normalized_rows(rope.encode_many(window_letters(ref, ids * stride, N), N, m, schedule), N)
        F = fidelity_matrix(Xn, Cn)
        allF = np.concatenate([best_f, F], axis=1)
        allI = np.concatenate([best_i, np.broadcast_to(ids, F.shape)], axis=1)
        best_i, best_f = topk_rows(allF, allI, k)
    return no_location(best_i, best_f), best_f


def pair_fidelity(ref: np.ndarray, head: np.ndarray, j: int, N: int, m: int = 32,
                  stride: int = 1, schedule: str = "default") -> float:
    """F(read head, window j), one pair at a time."""
    s = j * stride
    return rope.fidelity(rope.encode_raw(head, N, m, schedule),
                         rope.encode_raw(ref[s:s + N], N, m, schedule), N)


def pair_fidelities(ref: np.ndarray, heads: np.ndarray, idx: np.ndarray, N: int, m: int = 32,
                    stride: int = 1, schedule: str = "default") -> np.ndarray:
    """F(head r, window idx[r, i]) for every entry of idx [R, c] (entries < 0 give nan)."""
    R, c = idx.shape
    Xn, _ = normalized_rows(rope.encode_many(heads, N, m, schedule), N)
    safe = np.clip(idx, 0, None).reshape(-1)
    Cn, _ = normalized_rows(rope.encode_many(window_letters(ref, safe * stride, N), N, m, schedule), N)
    F = np.abs(np.sum(np.conj(np.repeat(Xn, c, axis=0)) * Cn, axis=1)) ** 2
    F = F.reshape(R, c)
    F[idx < 0] = np.nan
    return F


def refine_pool(coarse_ids, stride: int, radius: int, W1: int) -> np.ndarray:
    """§3.4, refinement around found locations: the step-1 window starts within
    `radius` of a found coarse window's start (coarse id j starts at j*stride),
    clamped to 0 .. W1-1, each start once.  Negative ids are skipped."""
    starts = set()
    for j in coarse_ids:
        j = int(j)
        if j < 0:
            continue
        c = j * stride
        for s in range(max(0, c - radius), min(W1 - 1, c + radius) + 1):
            starts.add(s)
    return np.array(sorted(starts), dtype=np.int64)


def refine_topk(F1_row: np.ndarray, coarse_ids, stride: int, radius: int, k: int):
    """The k best of the refinement pool of one read, ranked like every list
    here: F1_row holds the read's fidelities with ALL step-1 windows (an oracle
    F row); returns (starts, F) of length min(k, pool size)."""
    pool = refine_pool(coarse_ids, stride, radius, F1_row.shape[0])
    if pool.size == 0:
        return np.zeros(0, dtype=np.int64), np.zeros(0)
    i, f = topk_rows(F1_row[pool][None, :], pool[None, :], k)
    return no_location(i[0], f[0]), f[0]


def reverse_complement(seq: np.ndarray) -> np.ndarray:
    """The other strand read 5'->3': reverse the letters and complement them
    (A=0 <-> T=3, C=1 <-> G=2, i.e. L -> 3 - L)."""
    return (3 - seq[::-1]).astype(np.uint8)


def merge_strands(fwd_idx, fwd_F, rev_idx, rev_F, k: int, min_fidelity: float = 0.0):
    """Both mapping directions (the paper maps reads in both directions): the k
    best of a read's forward-strand list and its reverse-complement list, each
    already ranked (F desc, id asc), ranked the same way with the forward entry
    first on a full tie; entries with F below min_fidelity are dropped (the
    threshold regime: only locations whose fidelity passes the threshold are
    reported; none passing = unmapped).  Returns (ids, F, strands), strand 0 =
    forward, 1 = reverse; negative ids are skipped."""
    entries = [(-float(f), int(j), 0) for j, f in zip(fwd_idx, fwd_F) if j >= 0]
    entries += [(-float(f), int(j), 1) for j, f in zip(rev_idx, rev_F) if j >= 0]
    entries = sorted(e for e in entries if -e[0] >= min_fidelity)[:k]
    return (np.array([e[1] for e in entries], dtype=np.int64),
            np.array([-e[0] for e in entries]),
            np.array([e[2] for e in entries], dtype=np.int64))


def recall_at_k(got: np.ndarray, ref_idx: np.ndarray, ref_F: np.ndarray, got_true_F: np.ndarray,
                tau: float = TIE_TAU) -> float:
    """Mean over reads of |{j in got_r : j in oracle top-k or F(j) >= F_(k) - tau}| / k.

    got [R,k] are a path's window ids; ref_idx/ref_F the oracle's top-k;
    got_true_F the oracle's fidelity of each of `got`'s entries.  Duplicate ids
    count once."""
    R, k = ref_idx.shape
    total = 0.0
    for r in range(R):
        seen = set()
        hits = 0
        kth = ref_F[r, k - 1]
        oracle = set(int(v) for v in ref_idx[r])
        for i in range(k):
            j = int(got[r, i])
            if j in seen or j < 0:
                continue
            seen.add(j)
            if j in oracle or got_true_F[r, i] >= kth - tau:
                hits += 1
        total += hits / k
    return total / R


def same_up_to_ties(got: np.ndarray, ref_F: np.ndarray, got_true_F: np.ndarray,
                    tau: float = TIE_TAU) -> np.ndarray:
    """Per read: the path's list equals the oracle's rank by rank, up to swaps among
    candidates whose oracle fidelities differ by at most tau, with no duplicates."""
    R, k = got.shape
    ok = np.ones(R, dtype=bool)
    for r in range(R):
        if len(set(int(v) for v in got[r])) != k or np.any(got[r] < 0):
            ok[r] = False
            continue
        ok[r] = bool(np.all(np.abs(got_true_F[r] - ref_F[r]) <= tau))
    return ok
