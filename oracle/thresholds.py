"""FP64 oracle of per-fragment fidelity thresholds and the threshold regime.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy / Python.

§3.3 (closing paragraph): for a target mutation rate, the fidelity expected
of each reference fragment can be estimated and used as that fragment's
cutting threshold.  §3.5 describes the regime that outputs every location
whose fidelity passes its fragment's precomputed threshold (many locations
for some reads, none for others).  The paper does not say how the estimate is
made; the reading taken here:

* window j (letters ref[j*stride, j*stride + N)) is mutated M times at the
  target rate err by the streaming mutator the reads are simulated with:
  walking the reference from the window's start, each step is an insertion,
  a deletion or a substitution with probability err/3 each, else a match,
  until N letters are out (§2.4 splits mutations evenly between the three);
* the fidelity F of the window with each mutated copy (§2.4, the plain
  encoding, §2.1-§2.3) is computed, and the window's threshold is the
  `rank`-th smallest of the M values (an order statistic: rank 0 is the
  smallest, so a read mutated at the target rate passes the threshold of its
  own window with probability about 1 - (rank + 1) / (M + 1));
* the regime reports, for a read, every window j with F >= max(thr_j, floor)
  and F > 0 (a window or read with F = 0 is no location), ranked by F
  descending, then window id.

The random draws come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011), a counter-based
generator: step t of copy c of window j draws the four words of
philox(counter = (j mod 2^32, j >> 32, c, t), key = (seed, 0)).  Word 0 picks
the event (integer comparisons with floor(err / 3 * 2^32) per event type,
so both sides take the same decision); word 1 & 3 is an inserted letter;
1 + word 2 mod 3 is a substitution's shift (the new letter is (old + shift)
mod 4).  A step that needs a reference letter past the reference's end is an
insertion.  A copy takes at most 8 N + 64 steps; letters still missing then
are left as "no letter" (code 4).

Pins (tests/test_oracle_thresholds.py): Philox against the generator's
published known-answer vectors; err = 0 gives the window itself (F = 1,
threshold 1); every copy's edit distance to the reference text it consumed is
at most its number of edit events; event frequencies near err/3 each; the
order statistic's extremes; hand-made threshold-regime lists.
"""
from __future__ import annotations

import numpy as np

from . import mapping, rope

M0, M1 = 0xD2511F53, 0xCD9E8D57      # Philox4x32 round multipliers
W0, W1 = 0x9E3779B9, 0xBB67AE85      # Philox key increments (Weyl sequence)
MASK = 0xFFFFFFFF
NO_LETTER = 4


def philox4x32(ctr, key, rounds: int = 10):
    """Philox4x32-R of counter words ctr (4 arrays of uint64 holding 32-bit
    values, or ints) with key (k0, k1); returns four arrays of 32-bit words.
    A round multiplies words 0 and 2 by M0 and M1 (64-bit products split into
    high and low halves) and mixes: (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
    the key advances by (W0, W1) between rounds."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK for x in ctr)
    k0, k1 = np.uint64(key[0] & MASK), np.uint64(key[1] & MASK)
    for r in range(rounds):
        if r:
            k0 = np.uint64((int(k0) + W0) & MASK)
            k1 = np.uint64((int(k1) + W1) & MASK)
        p0 = c0 * np.uint64(M0)
        p1 = c2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def event_threshold(err: float) -> int:
    """floor(err / 3 * 2^32): word 0 below 1x / 2x / 3x this value means an
    insertion / deletion / substitution.  err is taken as an FP32 value."""
    return int(np.floor(float(np.float32(err)) / 3.0 * 4294967296.0))


def max_steps(N: int) -> int:
    return 8 * N + 64


def mutate_window(ref: np.ndarray, start: int, N: int, err: float, j: int, c: int,
                  seed: int):
    """Copy c of window j: the N letters the streaming mutator emits from
    ref[start:], and the counts of (insertions, deletions, substitutions) and
    the number of reference letters consumed."""
    T = event_threshold(err)
    G = ref.shape[0]
    steps = max_steps(N)
    t = np.arange(steps, dtype=np.uint64)
    w0, w1, w2, _ = philox4x32((np.full(steps, j & MASK), np.full(steps, j >> 32),
                                np.full(steps, c), t), (seed, 0))
    out = np.full(N, NO_LETTER, dtype=np.uint8)
    pos, n = start, 0
    ins = dele = sub = 0
    for s in range(steps):
        if n == N:
            break
        u = int(w0[s])
        kind = "ins" if u < T else "del" if u < 2 * T else "sub" if u < 3 * T else "match"
        if kind != "ins" and pos >= G:
            kind = "ins"
        if kind == "ins":
            out[n] = int(w1[s]) & 3
            n += 1
            ins += 1
        elif kind == "del":
            pos += 1
            dele += 1
        elif kind == "sub":
            L = int(ref[pos])
            out[n] = (L + 1 + int(w2[s]) % 3) % 4 if L < 4 else L
            n += 1
            pos += 1
            sub += 1
        else:
            out[n] = ref[pos]
            n += 1
            pos += 1
    return out, (ins, dele, sub), pos - start


def window_copy_fidelities(ref: np.ndarray, j: int, stride: int, N: int, err: float,
                           copies: int, seed: int, m: int = 32,
                           schedule: str = "default") -> np.ndarray:
    """F(window j, copy c) for c = 0..copies-1 (FP64, plain encoding)."""
    s = j * stride
    cw = rope.encode_raw(ref[s:s + N], N, m, schedule)
    out = np.empty(copies)
    for c in range(copies):
        y, _, _ = mutate_window(ref, s, N, err, j, c, seed)
        out[c] = rope.fidelity(cw, rope.encode_raw(y, N, m, schedule), N)
    return out


def window_threshold(ref: np.ndarray, j: int, stride: int, N: int, err: float, copies: int,
                     rank: int, seed: int, m: int = 32, schedule: str = "default") -> float:
    """The window's cutting threshold: the rank-th smallest copy fidelity."""
    F = window_copy_fidelities(ref, j, stride, N, err, copies, seed, m, schedule)
    return float(np.sort(F)[rank])


def threshold_hits(F_row: np.ndarray, thr: np.ndarray, floor: float = 0.0):
    """The threshold regime for one read: every window j with F_row[j] >=
    max(thr[j], floor) and F_row[j] > 0, ranked (F desc, id asc).  Returns
    (ids, F)."""
    F_row = np.asarray(F_row, dtype=np.float64)
    cut = np.maximum(np.asarray(thr, dtype=np.float64), floor)
    ids = np.nonzero((F_row >= cut) & (F_row > 0))[0]
    if ids.size == 0:
        return ids.astype(np.int64), np.zeros(0)
    order = mapping.rank_order(F_row[ids], ids)
    return ids[order].astype(np.int64), F_row[ids[order]]
