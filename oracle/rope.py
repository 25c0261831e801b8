"""FP64 oracle: the RoPE-DNA encoding with single-letter tokens (s = 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, FP64 /
complex128 throughout.

Definitions followed (RotorMap paper, arXiv 2603.22245):

* §2.1, main feature vector: for a string of nominal length N, a token at
  location loc contributes omega^loc with omega = exp(2*pi*i/N); the feature of
  a token value is the sum over its locations.  With s = 1 a token is one
  letter and locations run 0..n-1.
* §2.2, eq. (mult-factor): factor k stretches the locations, omega^(k*loc).
* §3.3, eq. (mult-factor-finetune): the fine-tuned factor replaces k by
  2(k-1)/(m-1)+1.
* §2.3, default version: concatenate the feature vectors for k = 1..m and
  normalise; the dimension is m*4^s (here 4m).
* §2.10: the same vector as a sum over locations of D^loc applied to
  ones(m) (x) onehot(token), D = Diag((omega^1..omega^m) (x) ones(4^s)); this fixes
  the component order: index (k-1)*4 + letter.
* §3.4: moving a window one letter to the right multiplies every component
  by omega^-k, removes the outgoing token (-omega^-k) and adds the incoming one
  (+omega^(k(N-s))); the inner product with a fixed read obeys the same rule.

Readings where the paper is silent (listed in the design notes): letters
A,C,G,T = 0..3; e^(+i theta p) for positions and the read conjugated in the
inner product; integer factors reduce the exponent exactly, r = (k*loc) mod N,
before taking FP64 cos/sin; a vector is degenerate (zero) when its squared
norm is below 1e-9*N, and its fidelity with anything is 0.
"""
from __future__ import annotations

import numpy as np

N_LETTERS = 4
DEGENERATE_REL = 1e-9  # squared norm below this times N counts as the zero vector


def frequencies(m: int, schedule: str = "default") -> np.ndarray:
    """Multiplicity factors f_1..f_m.

    default   (§2.2 eq. mult-factor):           f_k = k
    finetuned (§3.3 eq. mult-factor-finetune):  f_k = 2(k-1)/(m-1) + 1
    """
    k = np.arange(1, m + 1, dtype=np.float64)
    if schedule == "default":
        return k
    if schedule == "finetuned":
        if m == 1:
            return np.ones(1)
        return 2.0 * (k - 1.0) / (m - 1.0) + 1.0
    raise ValueError(f"unknown schedule {schedule!r}")


def unit_phases(N: int, m: int, positions, schedule: str = "default") -> np.ndarray:
    """omega^(f_k * loc) for each location and factor: complex128 [len(positions), m].

    omega = exp(2 pi i / N) (§2.1).  For integer f_k the exponent f_k*loc is
    reduced modulo N in exact integer arithmetic first, so the angle passed to
    cos/sin is 2 pi r / N with 0 <= r < N whatever the location.
    """
    pos = np.asarray(positions, dtype=np.int64)
    f = frequencies(m, schedule)
    if np.all(f == np.round(f)):
        r = (pos[:, None] * f.astype(np.int64)[None, :]) % N
        ang = 2.0 * np.pi * r.astype(np.float64) / N
    else:
        ang = 2.0 * np.pi * (pos[:, None].astype(np.float64) * f[None, :]) / N
    return np.cos(ang) + 1j * np.sin(ang)


def encode_raw(w, N: int, m: int = 32, schedule: str = "default", positions=None) -> np.ndarray:
    """Unnormalised RoPE vector c of a string (§2.1-§2.2, s = 1).

    c[(k-1)*4 + L] = sum over locations loc with w[loc] == L of omega^(f_k loc).
    `positions` gives each letter's location (default 0..n-1).
    """
    w = np.asarray(w, dtype=np.int64)
    if positions is None:
        positions = np.arange(w.shape[0])
    E = unit_phases(N, m, positions, schedule)          # [n, m]
    c = np.zeros((m, N_LETTERS), dtype=np.complex128)
    for L in range(N_LETTERS):
        c[:, L] = E[w == L].sum(axis=0)
    return c.reshape(-1)


def sq_norm(c: np.ndarray) -> float:
    return float(np.sum(np.abs(c) ** 2))


def is_degenerate(c: np.ndarray, N: int) -> bool:
    return sq_norm(c) < DEGENERATE_REL * N


def normalize(c: np.ndarray, N: int) -> np.ndarray:
    """The state |RoPE> = c / |c| (§2.3); the zero vector for degenerate c."""
    X = sq_norm(c)
    if X < DEGENERATE_REL * N:
        return np.zeros_like(c)
    return c / np.sqrt(X)


def encode(w, N: int, m: int = 32, schedule: str = "default") -> np.ndarray:
    """Normalised RoPE_{1,m}(w) (§2.3)."""
    return normalize(encode_raw(w, N, m, schedule), N)


def encode_dloc(w, N: int, m: int = 32) -> np.ndarray:
    """The §2.10 formulation, default factors: sum_loc D^loc (ones(m) (x) onehot(w_loc)).

    D is built as a dense diagonal matrix and its powers by repeated matrix
    products, independently of `unit_phases`."""
    omega = np.exp(2j * np.pi / N)
    D = np.diag(np.kron(omega ** np.arange(1, m + 1), np.ones(N_LETTERS)))
    acc = np.zeros(m * N_LETTERS, dtype=np.complex128)
    Dp = np.eye(m * N_LETTERS, dtype=np.complex128)
    for letter in np.asarray(w, dtype=np.int64):
        onehot = np.zeros(N_LETTERS)
        onehot[letter] = 1.0
        acc = acc + Dp @ np.kron(np.ones(m), onehot)
        Dp = Dp @ D
    return acc


def fidelity(a: np.ndarray, b: np.ndarray, N: int) -> float:
    """|<a|b>|^2 / (|a|^2 |b|^2) (§2.4); 0 if either vector is degenerate."""
    A, B = sq_norm(a), sq_norm(b)
    if A < DEGENERATE_REL * N or B < DEGENERATE_REL * N:
        return 0.0
    return float(abs(np.vdot(a, b)) ** 2 / (A * B))


def encode_many(strings: np.ndarray, N: int, m: int = 32, schedule: str = "default") -> np.ndarray:
    """Unnormalised encodings of equal-length strings, complex128 [B, 4m].

    The same sum as `encode_raw`, written as one matrix product per letter:
    c[b, k, L] = sum_loc [strings[b, loc] == L] * omega^(f_k loc)."""
    strings = np.asarray(strings)
    B, n = strings.shape
    E = unit_phases(N, m, np.arange(n), schedule)       # [n, m]
    Er, Ei = np.ascontiguousarray(E.real), np.ascontiguousarray(E.imag)
    out = np.empty((B, m, N_LETTERS), dtype=np.complex128)
    for L in range(N_LETTERS):
        ind = (strings == L).astype(np.float64)          # [B, n]
        out[:, :, L] = (ind @ Er) + 1j * (ind @ Ei)
    return out.reshape(B, m * N_LETTERS)


# ---------------------------------------------------------------- §3.4 rules

def slide(c: np.ndarray, old: int, new: int, N: int, m: int = 32,
          schedule: str = "default", s: int = 1) -> np.ndarray:
    """One-letter slide of a window encoding (§3.4): every component is multiplied
    by omega^-f_k, the outgoing token loses omega^-f_k, the incoming one gains
    omega^(f_k (N-s)); when the two tokens coincide both terms apply."""
    f = frequencies(m, schedule)
    back = np.exp(-2j * np.pi * f / N)
    front = np.exp(2j * np.pi * f * (N - s) / N)
    c = c.reshape(m, N_LETTERS) * back[:, None]
    c[:, old] -= back
    c[:, new] += front
    return c.reshape(-1)


def sliding_encodings(ref, N: int, count: int, m: int = 32, schedule: str = "default") -> np.ndarray:
    """Unnormalised encodings of windows ref[j:j+N], j = 0..count-1, obtained by
    encoding window 0 directly and applying `slide` count-1 times."""
    ref = np.asarray(ref, dtype=np.int64)
    out = np.empty((count, m * N_LETTERS), dtype=np.complex128)
    c = encode_raw(ref[:N], N, m, schedule)
    out[0] = c
    for j in range(1, count):
        c = slide(c, int(ref[j - 1]), int(ref[j + N - 1]), N, m, schedule)
        out[j] = c
    return out


def slide_ip(ip_k: np.ndarray, x: np.ndarray, old: int, new: int, N: int, m: int = 32,
             schedule: str = "default", s: int = 1) -> np.ndarray:
    """§3.4 inner-product rule, per factor k (the paper states it for one factor):
    ip_k <- ip_k omega^-f_k - conj(x_{k,old}) omega^-f_k + conj(x_{k,new}) omega^(f_k (N-s)).
    The total inner product is ip_k.sum()."""
    f = frequencies(m, schedule)
    back = np.exp(-2j * np.pi * f / N)
    front = np.exp(2j * np.pi * f * (N - s) / N)
    xk = x.reshape(m, N_LETTERS)
    return ip_k * back - np.conj(xk[:, old]) * back + np.conj(xk[:, new]) * front


def ip_per_factor(x: np.ndarray, c: np.ndarray, m: int = 32) -> np.ndarray:
    """sum_L conj(x_{k,L}) c_{k,L} for each factor k."""
    return np.sum(np.conj(x.reshape(m, N_LETTERS)) * c.reshape(m, N_LETTERS), axis=1)
