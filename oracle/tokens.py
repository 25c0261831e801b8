"""FP64 oracle: the RoPE-DNA encoding with s-mer tokens and compact token maps.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, FP64 /
complex128 throughout.

Definitions followed (RotorMap paper, arXiv 2603.22245):

* §2.1, main feature vector: a string of nominal length N has N-s+1 token
  locations 0..N-s; the token at location loc is the s-mer w[loc .. loc+s);
  the feature of an s-mer is the sum over its locations of omega^loc,
  omega = exp(2 pi i / N).
* §2.2 / §3.3: factor k uses omega^(f_k loc) with f_k = k (default) or
  2(k-1)/(m-1)+1 (fine-tuned).
* §2.3: the default version concatenates the m feature vectors, each indexed
  by the 4^s s-mers, and normalises.
* §2.6 (compact versions): a 4^s-to-4^t mapping of the s-mers lowers the
  dimension; the tokens are then counted by their mapped value (their class).
  Here the mapping is any table `token_map` from s-mer code to class in
  0..C-1, or -1 for an s-mer left out (the variant that keeps only selected
  s-mers, e.g. the reference's most frequent ones: `frequent_map`).  With no
  table the class is the s-mer code and C = 4^s.
* §2.10: the same vector is sum_loc D^loc (ones(m) (x) onehot(class(loc))),
  D = Diag((omega^1..omega^m) (x) ones(C)): component index (k-1)*C + class.
* §3.4: one slide of a window multiplies every component by omega^-f_k,
  removes omega^-f_k from the outgoing token's component (location 0) and adds
  omega^(f_k (N-s)) to the incoming token's (location N-s); both apply when
  the two tokens coincide.

Readings where the paper is silent (listed in the design notes): the code of
an s-mer is sum_i w[loc+i] 4^(s-1-i) (first letter most significant, letters
A,C,G,T = 0..3); an s-mer containing a code outside 0..3 is no token; the
fidelity and degeneracy rules are those of `oracle.rope`.
"""
from __future__ import annotations

import numpy as np

from . import mapping, rope

SKIP = -1  # class of an s-mer that adds nothing


def mer_codes(w, s: int) -> np.ndarray:
    """Code of the s-mer at every location 0..n-s, -1 where it holds a letter
    outside 0..3; int64 [n-s+1] (empty when n < s)."""
    w = np.asarray(w, dtype=np.int64)
    n = w.shape[0]
    if n < s:
        return np.zeros(0, dtype=np.int64)
    codes = np.zeros(n - s + 1, dtype=np.int64)
    bad = np.zeros(n - s + 1, dtype=bool)
    for i in range(s):
        letters = w[i:i + n - s + 1]
        codes = codes * 4 + np.where((letters >= 0) & (letters < 4), letters, 0)
        bad |= (letters < 0) | (letters > 3)
    codes[bad] = -1
    return codes


def token_classes(w, s: int, token_map=None) -> np.ndarray:
    """Class of the token at every location (SKIP for no token)."""
    codes = mer_codes(w, s)
    if token_map is None:
        return codes
    tm = np.asarray(token_map, dtype=np.int64)
    out = np.full(codes.shape, SKIP, dtype=np.int64)
    ok = codes >= 0
    out[ok] = tm[codes[ok]]
    return out


def mer_counts(ref, s: int) -> np.ndarray:
    """Occurrences of every s-mer code in `ref` (locations 0..G-s; s-mers with
    a letter outside 0..3 are not counted), int64 [4^s]."""
    codes = mer_codes(ref, s)
    return np.bincount(codes[codes >= 0], minlength=4 ** s).astype(np.int64)


def frequent_map(ref, s: int, n_class: int) -> np.ndarray:
    """The compact context-aware version of §2.6: only the n_class most
    frequent s-mers of the reference are tokens.  Reading: ranked by count
    descending, then by code ascending; the kept s-mers take classes 0..n_class-1
    in code order; every other s-mer maps to SKIP.  int64 [4^s]."""
    counts = mer_counts(ref, s)
    codes = np.arange(4 ** s)
    order = np.lexsort((codes, -counts))          # count desc, code asc
    keep = np.sort(order[:n_class])
    out = np.full(4 ** s, SKIP, dtype=np.int64)
    out[keep] = np.arange(keep.size)
    return out


def encode_raw(w, N: int, s: int, m: int, n_class: int, token_map=None,
               schedule: str = "default") -> np.ndarray:
    """Unnormalised vector c, complex128 [m * n_class]:
    c[(k-1) n_class + cls] = sum over locations loc whose token has class cls
    of omega^(f_k loc) (§2.1-§2.3, §2.6)."""
    cls = token_classes(w, s, token_map)
    E = rope.unit_phases(N, m, np.arange(cls.shape[0]), schedule)   # [n-s+1, m]
    c = np.zeros((m, n_class), dtype=np.complex128)
    for q in range(n_class):
        c[:, q] = E[cls == q].sum(axis=0)
    return c.reshape(-1)


def encode(w, N: int, s: int, m: int, n_class: int, token_map=None,
           schedule: str = "default") -> np.ndarray:
    return rope.normalize(encode_raw(w, N, s, m, n_class, token_map, schedule), N)


def encode_dloc(w, N: int, s: int, m: int, n_class: int, token_map=None) -> np.ndarray:
    """The §2.10 formulation with default factors, written out: a dense
    diagonal D, its powers by repeated products, one stretched one-hot vector
    per location.  The token at each location is read by slicing the string
    and comparing letter by letter, independently of `mer_codes`."""
    w = [int(v) for v in np.asarray(w).tolist()]
    omega = np.exp(2j * np.pi / N)
    D = np.diag(np.kron(omega ** np.arange(1, m + 1), np.ones(n_class)))
    acc = np.zeros(m * n_class, dtype=np.complex128)
    Dp = np.eye(m * n_class, dtype=np.complex128)
    for loc in range(len(w) - s + 1):
        mer = w[loc:loc + s]
        if all(0 <= v < 4 for v in mer):
            code = 0
            for v in mer:
                code = 4 * code + v
            q = code if token_map is None else int(token_map[code])
            if q >= 0:
                onehot = np.zeros(n_class)
                onehot[q] = 1.0
                acc = acc + Dp @ np.kron(np.ones(m), onehot)
        Dp = Dp @ D
    return acc


def encode_many(strings: np.ndarray, N: int, s: int, m: int, n_class: int, token_map=None,
                schedule: str = "default") -> np.ndarray:
    """Unnormalised encodings of equal-length strings, complex128 [B, m*n_class]:
    the sum of `encode_raw` as one matrix product per class."""
    strings = np.asarray(strings, dtype=np.int64)
    B, n = strings.shape
    T = n - s + 1
    cls = np.stack([token_classes(row, s, token_map) for row in strings]) if B else \
        np.zeros((0, max(T, 0)), dtype=np.int64)
    E = rope.unit_phases(N, m, np.arange(T), schedule)
    Er, Ei = np.ascontiguousarray(E.real), np.ascontiguousarray(E.imag)
    out = np.empty((B, m, n_class), dtype=np.complex128)
    for q in range(n_class):
        ind = (cls == q).astype(np.float64)
        out[:, :, q] = (ind @ Er) + 1j * (ind @ Ei)
    return out.reshape(B, m * n_class)


def encode_windows(ref: np.ndarray, starts: np.ndarray, N: int, s: int, m: int, n_class: int,
                   token_map=None, schedule: str = "default") -> np.ndarray:
    """Unnormalised encodings of the windows ref[j : j+N] for j in `starts`,
    complex128 [len(starts), m*n_class]: the token at location p of window j
    is the reference's token at position j+p, so the reference's token classes
    are found once and gathered per window (§2.1, §3.1)."""
    starts = np.asarray(starts, dtype=np.int64)
    T = N - s + 1
    if starts.size == 0:
        return np.zeros((0, m * n_class), dtype=np.complex128)
    lo, hi = int(starts.min()), int(starts.max()) + N       # the letters the windows cover
    cls_ref = token_classes(np.asarray(ref)[lo:hi], s, token_map)
    cls = cls_ref[(starts - lo)[:, None] + np.arange(T)[None, :]]
    E = rope.unit_phases(N, m, np.arange(T), schedule)
    # location by location: each window's token at p adds omega^(f_k p) to
    # its class's component of every factor k (one token per window and p)
    out = np.zeros((cls.shape[0], m, n_class), dtype=np.complex128)
    rows = np.arange(cls.shape[0])
    for p in range(T):
        c = cls[:, p]
        ok = (c >= 0) & (c < n_class)
        out[rows[ok], :, c[ok]] += E[p]
    return out.reshape(cls.shape[0], m * n_class)


def slide(c: np.ndarray, old: int, new: int, N: int, s: int, m: int, n_class: int,
          schedule: str = "default") -> np.ndarray:
    """One-letter slide (§3.4): rotate by omega^-f_k, the outgoing token's class
    `old` loses omega^-f_k, the incoming token's class `new` gains
    omega^(f_k (N-s)); a class of SKIP touches nothing."""
    f = rope.frequencies(m, schedule)
    back = np.exp(-2j * np.pi * f / N)
    front = np.exp(2j * np.pi * f * (N - s) / N)
    c = c.reshape(m, n_class) * back[:, None]
    if old >= 0:
        c[:, old] -= back
    if new >= 0:
        c[:, new] += front
    return c.reshape(-1)


def sliding_encodings(ref, N: int, count: int, s: int, m: int, n_class: int, token_map=None,
                      schedule: str = "default") -> np.ndarray:
    """Windows ref[j:j+N], j = 0..count-1: window 0 directly, then `slide`."""
    ref = np.asarray(ref, dtype=np.int64)
    cls = token_classes(ref, s, token_map)
    out = np.empty((count, m * n_class), dtype=np.complex128)
    c = encode_raw(ref[:N], N, s, m, n_class, token_map, schedule)
    out[0] = c
    for j in range(1, count):
        # outgoing: the token at reference position j-1; incoming: j+N-s
        c = slide(c, int(cls[j - 1]), int(cls[j + N - s]), N, s, m, n_class, schedule)
        out[j] = c
    return out


def map_reads(ref: np.ndarray, heads: np.ndarray, N: int, s: int, m: int, n_class: int,
              token_map=None, k: int = 8, stride: int = 1, schedule: str = "default",
              chunk: int = 32768, window_range=None):
    """Exact top-k windows of every head by brute force (§3.1) with the token
    encoding; ordered as in `oracle.mapping`.  Returns (idx [R,k], F [R,k]).
    `window_range` restricts the scan to window ids [lo, hi)."""
    W = mapping.n_windows(ref.shape[0], N, stride)
    lo, hi = (0, W) if window_range is None else window_range
    Xn, _ = mapping.normalized_rows(encode_many(heads, N, s, m, n_class, token_map, schedule), N)
    R = Xn.shape[0]
    best_i = np.full((R, 0), -1, dtype=np.int64)
    best_f = np.zeros((R, 0))
    for a in range(lo, hi, chunk):
        b = min(hi, a + chunk)
        ids = np.arange(a, b, dtype=np.int64)
        Cw = encode_windows(ref, ids * stride, N, s, m, n_class, token_map, schedule)
        Cn, _ = mapping.normalized_rows(Cw, N)
        F = mapping.fidelity_matrix(Xn, Cn)
        best_i, best_f = mapping.topk_rows(np.concatenate([best_f, F], axis=1),
                                           np.concatenate([best_i, np.broadcast_to(ids, F.shape)],
                                                          axis=1), k)
    return mapping.no_location(best_i, best_f), best_f


def pair_fidelities(ref: np.ndarray, heads: np.ndarray, idx: np.ndarray, N: int, s: int, m: int,
                    n_class: int, token_map=None, stride: int = 1,
                    schedule: str = "default") -> np.ndarray:
    """F(head r, window idx[r, i]) for every entry of idx [R, c] (entries < 0 give nan)."""
    R, c = idx.shape
    Xn, _ = mapping.normalized_rows(encode_many(heads, N, s, m, n_class, token_map, schedule), N)
    safe = np.clip(idx, 0, None).reshape(-1)
    Cn, _ = mapping.normalized_rows(
        encode_many(mapping.window_letters(ref, safe * stride, N), N, s, m, n_class, token_map,
                    schedule), N)
    F = np.abs(np.sum(np.conj(np.repeat(Xn, c, axis=0)) * Cn, axis=1)) ** 2
    F = F.reshape(R, c)
    F[idx < 0] = np.nan
    return F
