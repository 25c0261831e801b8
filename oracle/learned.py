"""FP64 oracle of the learned angle offsets: forward, loss, analytic backward.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, FP64.

The paper has no learned component.  It remarks that RoPE variants could alter
the token definitions, initial encodings or rotation (§2.10), and it defines
tokens as s-mers at locations 0..N-s (§2.1) and weights per location
(§2.7).  The learned encoding used here (the design notes' reading of
"per-letter / per-frequency angle offsets"):

* tokens are 9-mers at locations p = 0..n-9 of a string w (n >= 9); the
  token's middle letter L_p = w[p+4] selects the component, its 8 flanking
  letters (w[p..p+3], w[p+5..p+8]) are one-hot encoded into x_p (32 values;
  a letter that is not A,C,G,T gives zeros);
* a 2-layer network gives offsets o = W2 relu(W1 x + b1) + b2, 128 values =
  4 letters x 32 factors, and delta_{p,k} = o[L_p * 32 + k];
* the token contributes exp(i (theta_k p + delta_{p,k})) to component (k, L_p)
  (theta_k = 2 pi f_k / N, N the nominal length, §2.1-§2.2), so with W2 = 0 and
  b2 = 0 the encoding is the plain one of w[4 : n-4];
* fidelity F = |<c_a|c_b>|^2 / (|c_a|^2 |c_b|^2) (§2.4);
* loss over a batch of pairs with Levenshtein labels d: mean over pairs (i, j)
  with d_i < d_j of softplus(-(F_i - F_j) / tau), tau = 0.05.

Parameter vector layout (10,432 values): W1 [64][32], b1 [64], W2 [128][64],
b2 [128], row-major.

Pins: W2 = b2 = 0 reduces to the plain encoding (exact); the analytic gradient
equals central finite differences; the loss's gradient w.r.t. F matches finite
differences; the loss and its gradient on a hand-worked batch of four pairs
(one pair ranked the wrong way, one label tie); Adam on hand-worked two-step
scalar examples and its constant-gradient invariant (m_hat = g, v_hat = g^2).
The Spearman gain of a trained network over the plain encoding has no paper
value: parity unpinned.
"""
from __future__ import annotations

import numpy as np

from . import rope

CTX = 4                     # flanking letters on each side
TOKEN = 2 * CTX + 1         # 9-mer tokens
N_IN, N_HID, N_OUT = 32, 64, 128
N_PARAMS = N_HID * N_IN + N_HID + N_OUT * N_HID + N_OUT   # 10,432
TAU = 0.05


def unpack(params: np.ndarray):
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    o = 0
    W1 = p[o:o + N_HID * N_IN].reshape(N_HID, N_IN); o += N_HID * N_IN
    b1 = p[o:o + N_HID]; o += N_HID
    W2 = p[o:o + N_OUT * N_HID].reshape(N_OUT, N_HID); o += N_OUT * N_HID
    b2 = p[o:o + N_OUT]
    return W1, b1, W2, b2


def pack(W1, b1, W2, b2) -> np.ndarray:
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(np.float64)


def init_params(seed: int = 0) -> np.ndarray:
    """First layer ~ U(-1/sqrt(32), 1/sqrt(32)), second layer zero (so training
    starts from the plain encoding)."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (N_HID, N_IN)) / np.sqrt(N_IN)
    b1 = rng.uniform(-1, 1, N_HID) / np.sqrt(N_IN)
    return pack(W1, b1, np.zeros((N_OUT, N_HID)), np.zeros(N_OUT))


def tokens(w):
    """Middle letters [T] and flank one-hots [T, 32] of a string's 9-mer tokens."""
    w = np.asarray(w, dtype=np.int64)
    T = w.shape[0] - 2 * CTX
    if T <= 0:
        return np.zeros(0, np.int64), np.zeros((0, N_IN))
    mid = w[CTX:CTX + T]
    x = np.zeros((T, N_IN))
    flank_pos = list(range(CTX)) + list(range(CTX + 1, TOKEN))
    for i, o in enumerate(flank_pos):
        letter = w[o:o + T]
        ok = letter < 4
        x[np.nonzero(ok)[0], 4 * i + letter[ok]] = 1.0
    return mid, x


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significant bits, ties to even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _network(params, x, bf16: bool):
    """Pre-activations, hidden values and outputs of the network for inputs x [T, 32].
    bf16: the inference arithmetic -- both weight matrices and the hidden values
    rounded to bfloat16, biases and sums exact."""
    W1, b1, W2, b2 = unpack(params)
    if bf16:
        W1, W2 = bf16_round(W1), bf16_round(W2)
    pre = x @ W1.T + b1                      # [T, 64]
    h = np.maximum(pre, 0.0)
    if bf16:
        h = bf16_round(h)
    o = h @ W2.T + b2                        # [T, 128]
    return pre, h, o


def select_offsets(mid, o, m: int = 32) -> np.ndarray:
    """delta [T, m]: the middle letter's m outputs (zero where it is not A,C,G,T)."""
    T = mid.shape[0]
    ok = mid < 4
    rows = np.arange(T)
    delta = np.zeros((T, m))
    delta[ok] = o[rows[ok, None], (mid[ok] * m)[:, None] + np.arange(m)[None, :]]
    return delta


def token_offsets(params, w, bf16: bool = False, m: int = 32, block: int = 1 << 18):
    """Middle letters [T] and phase offsets delta [T, m] of the 9-mer tokens of w
    (tokens are independent: long strings are taken in blocks of tokens)."""
    w = np.asarray(w)
    T = max(w.shape[0] - 2 * CTX, 0)
    if T <= block:
        mid, x = tokens(w)
        _, _, o = _network(params, x, bf16)
        return mid, select_offsets(mid, o, m)
    mid = np.empty(T, dtype=np.int64)
    delta = np.empty((T, m))
    for a in range(0, T, block):
        b = min(T, a + block)
        mb, x = tokens(w[a:b + 2 * CTX])
        _, _, o = _network(params, x, bf16)
        mid[a:b] = mb
        delta[a:b] = select_offsets(mb, o, m)
    return mid, delta


def forward_string(params, w, N: int, m: int = 32):
    """Learned encoding c (complex [4m], order k*4 + letter) and the cache for backward."""
    mid, x = tokens(w)
    pre, h, o = _network(params, x, False)
    T = mid.shape[0]
    theta = 2 * np.pi * rope.frequencies(m) / N
    delta = select_offsets(mid, o, m)
    phi = np.arange(T)[:, None] * theta[None, :] + delta      # [T, m]
    u = np.exp(1j * phi)
    c = np.zeros((m, 4), dtype=np.complex128)
    for L in range(4):
        c[:, L] = u[mid == L].sum(axis=0)
    cache = dict(mid=mid, x=x, pre=pre, h=h, phi=phi)
    return c.reshape(-1), cache


def fidelity_and_grads(ca, cb):
    """F = |z|^2/(A B), z = <a|b>, and its gradients G_a, G_b, with the
    convention dF = Re(sum conj(G) dc) over the real and imaginary parts."""
    z = np.vdot(ca, cb)
    A = np.sum(np.abs(ca) ** 2)
    B = np.sum(np.abs(cb) ** 2)
    F = abs(z) ** 2 / (A * B)
    Ga = 2 * np.conj(z) * cb / (A * B) - 2 * F * ca / A
    Gb = 2 * z * ca / (A * B) - 2 * F * cb / B
    return F, Ga, Gb


def ranking_loss(F, ld, tau: float = TAU):
    """Mean softplus(-(F_i - F_j)/tau) over pairs with ld_i < ld_j, and dLoss/dF."""
    F = np.asarray(F, dtype=np.float64)
    ld = np.asarray(ld)
    D = F[:, None] - F[None, :]
    M = (ld[:, None] < ld[None, :]).astype(np.float64)
    cnt = M.sum()
    if cnt == 0:
        return 0.0, np.zeros_like(F)
    z = -D / tau
    sp = np.logaddexp(0.0, z)
    loss = float((sp * M).sum() / cnt)
    s = 1.0 / (1.0 + np.exp(-z))             # softplus'(z)
    W = s * M / (tau * cnt)                   # d loss / d D_ij = -W_ij
    dF = -W.sum(axis=1) + W.sum(axis=0)
    return loss, dF


ADAM_BETA1, ADAM_BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_step(params, m, v, t: int, grad, lr: float, beta1: float = ADAM_BETA1,
              beta2: float = ADAM_BETA2, eps: float = ADAM_EPS):
    """One Adam update (Kingma and Ba, "Adam: a method for stochastic
    optimization", ICLR 2015, Algorithm 1), the optimiser the training uses.

    t is the number of updates already applied (0 before the first).  The
    first and second moment estimates decay by beta1 and beta2, each is
    divided by its bias-correction factor 1 - beta^(t+1), and the parameters
    move by lr * m_hat / (sqrt(v_hat) + eps).  Returns (params, m, v, t + 1)
    as new arrays."""
    params = np.asarray(params, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    t = int(t) + 1
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return params - lr * m_hat / (np.sqrt(v_hat) + eps), m, v, t


def backward_string(params, cache, G, m: int = 32):
    """Gradient of a real function of c w.r.t. the parameters, given G = its gradient
    w.r.t. c (convention of `fidelity_and_grads`).  c_{k,L} gains i exp(i phi) per
    unit of delta_{p,k}, so dF/d delta_{p,k} = Re(conj(G_{k,L_p}) i exp(i phi))."""
    W1, b1, W2, b2 = unpack(params)
    mid, x, pre, h, phi = cache["mid"], cache["x"], cache["pre"], cache["h"], cache["phi"]
    T = mid.shape[0]
    G = G.reshape(m, 4)
    ok = mid < 4
    Gt = np.zeros((T, m), dtype=np.complex128)
    Gt[ok] = G[:, mid[ok]].T
    ddelta = np.real(np.conj(Gt) * 1j * np.exp(1j * phi))        # [T, m]
    do = np.zeros((T, N_OUT))
    rows = np.arange(T)
    do[rows[ok, None], (mid[ok] * m)[:, None] + np.arange(m)[None, :]] = ddelta[ok]
    dW2 = do.T @ h
    db2 = do.sum(axis=0)
    dh = do @ W2
    dpre = dh * (pre > 0)
    dW1 = dpre.T @ x
    db1 = dpre.sum(axis=0)
    return pack(dW1, db1, dW2, db2)


def batch_loss_and_grad(params, pairs, ld, N: int, m: int = 32):
    """Loss and parameter gradient over a batch of string pairs [(a, b), ...]."""
    fw = [(forward_string(params, a, N, m), forward_string(params, b, N, m)) for a, b in pairs]
    Fs, Gs = [], []
    for (ca, _), (cb, _) in fw:
        F, Ga, Gb = fidelity_and_grads(ca, cb)
        Fs.append(F)
        Gs.append((Ga, Gb))
    loss, dF = ranking_loss(np.array(Fs), ld)
    grad = np.zeros(N_PARAMS)
    for i, ((_, cache_a), (_, cache_b)) in enumerate(fw):
        Ga, Gb = Gs[i]
        grad += backward_string(params, cache_a, dF[i] * Ga, m)
        grad += backward_string(params, cache_b, dF[i] * Gb, m)
    return loss, grad, np.array(Fs)


def batch_loss(params, pairs, ld, N: int, m: int = 32) -> float:
    Fs = []
    for a, b in pairs:
        ca, _ = forward_string(params, a, N, m)
        cb, _ = forward_string(params, b, N, m)
        Fs.append(fidelity_and_grads(ca, cb)[0])
    return ranking_loss(np.array(Fs), ld)[0]


def pair_fidelities(params, pairs, N: int, m: int = 32) -> np.ndarray:
    out = np.empty(len(pairs))
    for i, (a, b) in enumerate(pairs):
        ca, _ = forward_string(params, a, N, m)
        cb, _ = forward_string(params, b, N, m)
        out[i] = fidelity_and_grads(ca, cb)[0]
    return out


# --------------------------------------------------------------------------
# Mapping with the learned encoding (inference arithmetic: bf16=True).  A
# token's offsets depend only on its 9 letters, so the reference's tokens are
# evaluated once and every window sums its own N-8 tokens: window j (start s)
# has c_(k,L) = sum over p = 0..N-9 with w[s+p+4] = L of
# exp(i (theta_k p + delta_(s+p,k))).  A read head is encoded the same way
# from its first N letters.


def window_encodings(params, ref, starts, N: int, bf16: bool = True, m: int = 32,
                     ref_offsets=None) -> np.ndarray:
    """Learned encodings [len(starts), 4m] of the windows w[s, s+N)."""
    mid, delta = ref_offsets if ref_offsets is not None else token_offsets(params, ref, bf16, m)
    starts = np.asarray(starts, dtype=np.int64)
    theta = 2 * np.pi * rope.frequencies(m) / N
    C = np.zeros((starts.shape[0], m, 4), dtype=np.complex128)
    rows = np.arange(starts.shape[0])
    for p in range(N - 2 * CTX):
        t = starts + p
        u = np.exp(1j * (p * theta[None, :] + delta[t]))          # [W, m]
        L = mid[t]
        for letter in range(4):
            sel = L == letter
            C[rows[sel], :, letter] += u[sel]
    return C.reshape(starts.shape[0], 4 * m)


def head_encodings(params, heads, N: int, bf16: bool = True, m: int = 32) -> np.ndarray:
    """Learned encodings [R, 4m] of read heads [R, N] (each its own string)."""
    out = np.zeros((heads.shape[0], 4 * m), dtype=np.complex128)
    for r in range(heads.shape[0]):
        out[r] = window_encodings(params, heads[r], [0], N, bf16, m)[0]
    return out


def map_reads(params, ref, heads, N: int, k: int = 8, bf16: bool = True, m: int = 32,
              chunk: int = 16384, window_range=None):
    """Exact top-k windows of every read head under the learned encoding, by
    brute force over all windows (ranking as in the plain mapping)."""
    from . import mapping
    W = mapping.n_windows(ref.shape[0], N)
    lo, hi = (0, W) if window_range is None else window_range
    offs = token_offsets(params, ref, bf16, m)
    Xn, _ = mapping.normalized_rows(head_encodings(params, heads, N, bf16, m), N)
    R = Xn.shape[0]
    best_i = np.full((R, 0), -1, dtype=np.int64)
    best_f = np.zeros((R, 0))
    for a in range(lo, hi, chunk):
        b = min(hi, a + chunk)
        ids = np.arange(a, b, dtype=np.int64)
        Cn, _ = mapping.normalized_rows(window_encodings(params, ref, ids, N, bf16, m, offs), N)
        F = mapping.fidelity_matrix(Xn, Cn)
        allF = np.concatenate([best_f, F], axis=1)
        allI = np.concatenate([best_i, np.broadcast_to(ids, F.shape)], axis=1)
        best_i, best_f = mapping.topk_rows(allF, allI, k)
    return mapping.no_location(best_i, best_f), best_f


def head_window_fidelities(params, ref, heads, idx, N: int, bf16: bool = True,
                           m: int = 32) -> np.ndarray:
    """F(head r, window idx[r, i]) under the learned encoding (entries < 0 give nan)."""
    from . import mapping
    offs = token_offsets(params, ref, bf16, m)
    Xn, _ = mapping.normalized_rows(head_encodings(params, heads, N, bf16, m), N)
    out = np.full(idx.shape, np.nan)
    for r in range(idx.shape[0]):
        ok = idx[r] >= 0
        if not ok.any():
            continue
        Cn, _ = mapping.normalized_rows(window_encodings(params, ref, idx[r][ok], N, bf16, m, offs), N)
        out[r, ok] = np.abs(Cn.conj() @ Xn[r]) ** 2
    return out


def offset_error_bound(params, w, u: float = 2.0 ** -8) -> np.ndarray:
    """Bound [T, 32] on |delta_bf16 - delta_exact| for the tokens of w: with weights
    and hidden values rounded to bfloat16 (unit roundoff u), the first layer's
    error is at most u sum_i |W1_ji| x_i per hidden unit, the hidden rounding
    adds u |h_j|, and the second layer's weight rounding u |W2_kj| |h_j|; relu is
    1-Lipschitz.  Summation in FP32 adds a relative 2^-20 of the absolute sums."""
    mid, x = tokens(w)
    W1, b1, W2, b2 = unpack(params)
    h = np.maximum(x @ W1.T + b1, 0.0)
    a = x @ np.abs(W1.T)                                    # sum_i |W1_ji| x_i
    dh = u * a + u * (h + u * a)                            # |error of bf16 hidden|
    bound = (np.abs(W2) @ (u * (h + dh) + dh).T).T          # [T, 128]
    bound += 2.0 ** -20 * ((np.abs(W2) @ (h + dh).T).T + np.abs(b2) + (np.abs(b1) + a) @ np.abs(W2.T))
    return select_offsets(mid, bound) + 1e-7
