"""Seeded synthetic inputs for RotorMap workloads.

This module produces letters only: references, reads and string pairs as
uint8 codes A,C,G,T = 0,1,2,3.  It holds none of the encoding or scoring
arithmetic, so both the FP64 oracle and the HIP path can take their inputs
from it without sharing any part of the method.

What is generated (RotorMap paper, §3 "RotorMap", the mapping problem; §3.5
describes the paper's own tests on real genomes, which are replaced here by
synthetic stand-ins of the same shape):

* references: i.i.d. background with a given GC content, overwritten by
  repeat families (tandem or interspersed copies of a consensus unit with
  per-copy substitutions), until a given fraction of the length is covered;
* reads: a streaming mutator walks the reference from a uniform start and
  applies per-base substitution / insertion / deletion until the read has
  its target length; the start is the read's true location;
* string pairs: a uniform string and a copy after a number of random edits
  (substitution, insertion or deletion, each at a uniform position).

All randomness comes from numpy's PCG64 generator seeded per workload and
per role (reference, reads, pairs, sampling).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

ALPHABET = "ACGT"  # code of a letter = its index here


def to_codes(s: str) -> np.ndarray:
    """Letters 'ACGT' -> uint8 codes 0..3."""
    table = {c: i for i, c in enumerate(ALPHABET)}
    return np.array([table[c] for c in s], dtype=np.uint8)


def to_string(codes) -> str:
    return "".join(ALPHABET[int(c)] for c in codes)


def background(n: int, gc: float, rng: np.random.Generator) -> np.ndarray:
    """n i.i.d. letters with P(C)=P(G)=gc/2 and P(A)=P(T)=(1-gc)/2."""
    p = np.array([(1 - gc) / 2, gc / 2, gc / 2, (1 - gc) / 2])
    return rng.choice(4, size=n, p=p).astype(np.uint8)


def substitute(seq: np.ndarray, rate: float, rng: np.random.Generator) -> np.ndarray:
    """Replace each letter with probability `rate` by one of the three others."""
    out = seq.copy()
    mask = rng.random(seq.shape) < rate
    shift = rng.integers(1, 4, size=seq.shape, dtype=np.uint8)
    out[mask] = (out[mask] + shift[mask]) % 4
    return out


def add_repeats(ref: np.ndarray, frac: float, gc: float, rng: np.random.Generator,
                unit: Tuple[int, int] = (2, 300), copies: Tuple[int, int] = (2, 50),
                divergence: float = 0.10) -> int:
    """Overwrite `ref` in place with repeat families until `frac` of it is covered.

    Unit length is log-uniform on `unit`, the number of copies uniform on
    `copies`, each copy carries `divergence` per-base substitutions; even
    families are tandem (consecutive copies at one locus), odd families are
    interspersed (each copy at its own uniform locus).  Returns the number of
    families written.
    """
    G = ref.shape[0]
    target = frac * G
    covered = 0
    fam = 0
    lo, hi = math.log(unit[0]), math.log(unit[1])
    while covered < target:
        U = int(round(math.exp(rng.uniform(lo, hi))))
        n = int(rng.integers(copies[0], copies[1] + 1))
        cons = background(U, gc, rng)
        block = substitute(np.tile(cons, (n, 1)), divergence, rng)  # [n, U]
        if fam % 2 == 0 and U * n < G:
            s = int(rng.integers(0, G - U * n + 1))
            ref[s:s + U * n] = block.reshape(-1)
        else:
            pos = rng.integers(0, G - U + 1, size=n)
            ref[pos[:, None] + np.arange(U)[None, :]] = block
        covered += U * n
        fam += 1
    return fam


def make_reference(G: int, gc: float = 0.5, repeat_frac: float = 0.0, seed: int = 0,
                   uniform: bool = False) -> np.ndarray:
    """A synthetic reference of G letters.  `uniform` draws rng.integers(0,4)."""
    rng = np.random.default_rng(seed)
    if uniform:
        return rng.integers(0, 4, size=G, dtype=np.uint8)
    ref = background(G, gc, rng)
    if repeat_frac > 0:
        add_repeats(ref, repeat_frac, gc, rng)
    return ref


@dataclasses.dataclass
class Reads:
    seq: np.ndarray      # uint8, all reads concatenated
    offsets: np.ndarray  # int64 [n+1]; read i is seq[offsets[i]:offsets[i+1]]
    truth: np.ndarray    # int64 [n]; reference start the read was sampled from

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def read(self, i: int) -> np.ndarray:
        return self.seq[self.offsets[i]:self.offsets[i + 1]]

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)


def simulate_reads(ref: np.ndarray, lengths: np.ndarray, p_sub, p_ins, p_del,
                   seed: int) -> Reads:
    """Streaming mutator: from a uniform start, copy the reference letter by letter,
    applying per-step insertion (random letter, reference not consumed), deletion
    (reference letter skipped), substitution (a different letter) or a match, until
    each read reaches its target length.  Rates may be scalars or per-read arrays."""
    rng = np.random.default_rng(seed)
    lengths = np.asarray(lengths, dtype=np.int64)
    n = lengths.shape[0]
    G = ref.shape[0]
    p_sub = np.broadcast_to(np.asarray(p_sub, dtype=np.float64), (n,))
    p_ins = np.broadcast_to(np.asarray(p_ins, dtype=np.float64), (n,))
    p_del = np.broadcast_to(np.asarray(p_del, dtype=np.float64), (n,))
    span = np.ceil(lengths * 1.5).astype(np.int64) + 16
    if np.any(span >= G):
        raise ValueError("reference too short for the requested read lengths")
    start = (rng.random(n) * (G - span)).astype(np.int64)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    out = np.zeros(int(offsets[-1]), dtype=np.uint8)
    pos = start.copy()
    cnt = np.zeros(n, dtype=np.int64)
    active = np.nonzero(cnt < lengths)[0]
    while active.size:
        u = rng.random(active.size)
        rb = rng.integers(0, 4, size=active.size, dtype=np.uint8)
        sh = rng.integers(1, 4, size=active.size, dtype=np.uint8)
        pa = pos[active]
        ins = u < p_ins[active]
        dele = (~ins) & (u < p_ins[active] + p_del[active])
        sub = (~ins) & (~dele) & (u < p_ins[active] + p_del[active] + p_sub[active])
        ins |= pa >= G  # never runs off the end (guarded by `span` anyway)
        refl = ref[np.minimum(pa, G - 1)]
        letter = np.where(ins, rb, np.where(sub, (refl + sh) % 4, refl)).astype(np.uint8)
        emit = ~dele
        w = active[emit]
        out[offsets[w] + cnt[w]] = letter[emit]
        cnt[w] += 1
        pos[active[~ins]] += 1
        active = active[cnt[active] < lengths[active]]
    return Reads(seq=out, offsets=offsets, truth=start)


def lognormal_lengths(n: int, median: float, sigma: float, lo: int, hi: int,
                      rng: np.random.Generator) -> np.ndarray:
    x = np.exp(rng.normal(math.log(median), sigma, size=n))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


@dataclasses.dataclass
class Pairs:
    a: np.ndarray       # uint8 concat
    a_off: np.ndarray   # int64 [n+1]
    b: np.ndarray
    b_off: np.ndarray
    edits: np.ndarray   # int64 [n] number of edits applied (not the distance)

    @property
    def n(self) -> int:
        return int(self.a_off.shape[0] - 1)

    def pair(self, i: int):
        return (self.a[self.a_off[i]:self.a_off[i + 1]],
                self.b[self.b_off[i]:self.b_off[i + 1]])


def mutate_pairs(n: int, length: int, max_edits: int, seed: int, edits=None) -> Pairs:
    """a uniform of `length`; b = a after e ~ U{0..max_edits} edits (or the given
    per-pair counts `edits`, each <= max_edits), each edit a substitution,
    insertion or deletion (uniform type) at a uniform position of the current
    string."""
    rng = np.random.default_rng(seed)
    width = length + max_edits + 1
    a = rng.integers(0, 4, size=(n, length), dtype=np.uint8)
    if edits is None:
        e = rng.integers(0, max_edits + 1, size=n)
    else:
        e = np.asarray(edits, dtype=np.int64)
        assert e.shape == (n,) and e.min() >= 0 and e.max() <= max_edits
    buf = np.zeros((n, width), dtype=np.uint8)
    buf[:, :length] = a
    cur = np.full(n, length, dtype=np.int64)
    col = np.arange(width)[None, :]
    for t in range(max_edits):
        act = np.nonzero(e > t)[0]
        if act.size == 0:
            break
        typ = rng.integers(0, 3, size=act.size)
        L = cur[act]
        # deletions need a non-empty string; insert positions range over 0..L
        q = (rng.random(act.size) * np.where(typ == 1, L + 1, np.maximum(L, 1))).astype(np.int64)
        base = rng.integers(0, 4, size=act.size, dtype=np.uint8)
        shift = rng.integers(1, 4, size=act.size, dtype=np.uint8)
        rows = buf[act]
        qq = q[:, None]
        # substitution
        s = typ == 0
        if s.any():
            r = np.nonzero(s)[0]
            rows[r, q[r]] = (rows[r, q[r]] + shift[r]) % 4
        # insertion
        i = typ == 1
        if i.any():
            r = np.nonzero(i)[0]
            left = np.roll(rows[r], 1, axis=1)
            rows[r] = np.where(col < qq[r], rows[r], np.where(col == qq[r], base[r, None], left))
        # deletion
        d = (typ == 2) & (L > 0)
        if d.any():
            r = np.nonzero(d)[0]
            right = np.roll(rows[r], -1, axis=1)
            rows[r] = np.where(col < qq[r], rows[r], right)
        buf[act] = rows
        cur[act] += np.where(i, 1, np.where(d, -1, 0))
    a_off = np.arange(n + 1, dtype=np.int64) * length
    b_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cur, out=b_off[1:])
    mask = col < cur[:, None]
    return Pairs(a=a.reshape(-1), a_off=a_off, b=buf[mask], b_off=b_off, edits=e.astype(np.int64))


# --------------------------------------------------------------------------
# The workloads.  Seeds: 100*config + role (0 reference, 1 reads, 2 pairs,
# 3 sampling); the plain FP64 case uses reference seed 0.


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    G: int
    gc: float
    repeat_frac: float
    ref_seed: int
    uniform_ref: bool
    n_reads: int
    read_len: int            # fixed length; 0 = lognormal (batching case)
    p_sub: float
    p_ins: float
    p_del: float
    read_seed: int
    window_len: int = 150
    stride: int = 1
    n_freq: int = 32
    k: int = 8
    precision: str = "fp16"
    reanchor: int = 0

    def reference(self) -> np.ndarray:
        return make_reference(self.G, self.gc, self.repeat_frac, self.ref_seed, self.uniform_ref)

    def reads(self, ref: Optional[np.ndarray] = None, n: Optional[int] = None) -> Reads:
        if ref is None:
            ref = self.reference()
        n = self.n_reads if n is None else n
        if self.read_len > 0:
            lengths = np.full(n, self.read_len, dtype=np.int64)
            return simulate_reads(ref, lengths, self.p_sub, self.p_ins, self.p_del, self.read_seed)
        rng = np.random.default_rng(self.read_seed + 10_000)
        lengths = lognormal_lengths(n, 2000.0, 0.8, 100, 10_000, rng)
        e = rng.uniform(0.05, 0.10, size=n)
        return simulate_reads(ref, lengths, 0.2 * e, 0.4 * e, 0.4 * e, self.read_seed)

    def scaled(self, G: int, n_reads: int) -> "Workload":
        return dataclasses.replace(self, name=f"{self.name}@G{G}R{n_reads}", G=G, n_reads=n_reads)


E2 = 0.02 / 3
WORKLOADS = {
    # uniform ACGT reference of 20,000 bp (seed 0); 200 reads of 150 bp with 1% sub,
    # 0.5% ins, 0.5% del; every stride-1 window scored; top-8
    "plain": Workload("plain", 20_000, 0.5, 0.0, 0, True, 200, 150, 0.01, 0.005, 0.005, 101,
                      k=8, precision="fp32"),
    # 10 Mbp, 41% GC, 5% repeats; 100,000 reads of 150 bp at 2% error; FP16, top-8
    "precision": Workload("precision", 10_000_000, 0.41, 0.05, 200, False, 100_000, 150,
                          E2, E2, E2, 201, k=8, precision="fp16"),
    # 64 Mbp, 45% GC, 8% repeats; 20,000 reads of lognormal length, 5-10% indel-heavy
    "batching": Workload("batching", 64_000_000, 0.45, 0.08, 300, False, 20_000, 0,
                         0.0, 0.0, 0.0, 301, k=8, precision="fp16"),
    # 256 Mbp, 43% GC, 10% repeats; 1,000,000 reads of 150 bp at 2%; FP8, top-16,
    # FP64 re-anchor every 65,536 starts
    "scale": Workload("scale", 256_000_000, 0.43, 0.10, 500, False, 1_000_000, 150,
                      E2, E2, E2, 501, k=16, precision="fp8", reanchor=65_536),
}

PAIRS_SEED = 402  # learned-offsets workload: 1,000,000 pairs of 150 bp, 0..30 edits


TOKEN_MAP_SEED = 604  # compact token maps: seed = this + s


def token_map(s: int, n_class: int, seed: Optional[int] = None) -> np.ndarray:
    """A seeded 4^s-to-n_class table for the compact token encodings: a
    uniformly random assignment of the 4^s s-mer codes to n_class classes in
    which every class receives the same number of s-mers (4^s / n_class, or
    one more for the first 4^s mod n_class classes).  uint8 [4^s]."""
    if not 1 <= n_class <= 256:
        raise ValueError("n_class must be in 1..256")
    rng = np.random.default_rng(TOKEN_MAP_SEED + s if seed is None else seed)
    n = 4 ** s
    return (rng.permutation(n) % n_class).astype(np.uint8)


# Token encodings used by the tests, the stored oracle samples and the
# benchmark: name -> (s, m, n_class, mapped, schedule).  mapped = True takes
# token_map(s, n_class) as its 4^s-to-n_class table; mapped = "frequent" keeps
# the reference's n_class most frequent s-mers, a table the method itself
# derives from the reference (the caller builds it; token_encoding returns
# None for it).
TOKEN_ENCODINGS = {
    "s2": (2, 8, 16, False, "default"),
    "s3": (3, 2, 64, False, "finetuned"),
    "s8c16": (8, 8, 16, True, "finetuned"),
    # 1,024 complex components (FP16): 4-mers with m = 4, and 8-mers mapped to
    # 256 classes with m = 4 and fine-tuned factors (the paper's s = 8, m = 4,
    # t = 4 shape)
    "s4m4": (4, 4, 256, False, "default"),
    "s8c256": (8, 4, 256, True, "finetuned"),
    # the reference's 128 most frequent 4-mers, m = 8 (1,024 components)
    "s4f128": (4, 8, 128, "frequent", "default"),
}


def token_encoding(name: str):
    """(s, m, n_class, table or None, schedule) of a named token encoding
    (None also for a frequent-s-mer encoding: see token_map_is_frequent)."""
    s, m, C, mapped, sched = TOKEN_ENCODINGS[name]
    return s, m, C, (token_map(s, C) if mapped is True else None), sched


def token_map_is_frequent(name: str) -> bool:
    return TOKEN_ENCODINGS[name][3] == "frequent"
