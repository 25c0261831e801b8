"""Shared helpers of the GPU parity tests: conversions between the library's
device buffers and complex numpy arrays, and oracle references."""
import numpy as np

from oracle import mapping, rope


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def emb_to_complex(index, torch):
    """Stored window embeddings -> dequantised complex [W, components] (float64)."""
    e = index.embeddings()
    if e.dtype == torch.uint8:
        vals = e.cpu().view(torch.float8_e4m3fn).to(torch.float32).numpy().astype(np.float64)
        vals *= index.scales().cpu().numpy().astype(np.float64)[:, None]
    else:
        vals = e.float().cpu().numpy().astype(np.float64)
    return vals[:, 0::2] + 1j * vals[:, 1::2]


# The letter-sum form an FP16/FP8 letter index stores by default
# (rm_params.reduced): per factor, the coordinates y_m = sum_L LETTER_SUM[m, L]
# x_L on the three non-constant Walsh-Hadamard rows over the letters (A,C,G,T).
LETTER_SUM = np.array([[1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]], dtype=np.float64) / 2.0


def stored_form(C, index):
    """Oracle vectors C [n, 128] (component (k-1)*4 + letter) in the form the
    index stores them: C itself, or [n, 96] letter-sum coordinates (component
    (k-1)*3 + m) when the index is in the letter-sum form."""
    C = np.asarray(C)
    if not index.params.reduced:
        return C
    return np.einsum("nkl,ml->nkm", C.reshape(C.shape[0], -1, 4), LETTER_SUM).reshape(C.shape[0], -1)


def interleave(C):
    """Complex [n, c] -> reals [n, 2c] (re, im interleaved per component)."""
    out = np.empty((C.shape[0], 2 * C.shape[1]))
    out[:, 0::2], out[:, 1::2] = C.real, C.imag
    return out


def read_rows(reads, precision, torch):
    """Read-embedding buffer -> (row Re, row Im) as float64 [R, reals per row] each, dequantised."""
    n = reads.n
    if precision == "fp32":
        v = reads.emb.view(torch.float32).view(n, 2, -1).cpu().numpy().astype(np.float64)
    elif precision == "fp16":
        v = reads.emb.view(torch.float16).view(n, 2, -1).float().cpu().numpy().astype(np.float64)
    else:
        v = reads.emb.view(n, 2, -1).cpu().view(torch.float8_e4m3fn).to(torch.float32).numpy()
        v = v.astype(np.float64) * reads.scale.cpu().numpy().astype(np.float64)[:, None, None]
    return v[:, 0], v[:, 1]


def oracle_windows(ref, N, stride=1, m=32, schedule="default"):
    starts = mapping.window_starts(ref.shape[0], N, stride)
    C = rope.encode_many(mapping.window_letters(ref, starts, N), N, m, schedule)
    Cn, n2 = mapping.normalized_rows(C, N)
    return Cn, n2


def oracle_heads(heads, N, m=32, schedule="default"):
    X = rope.encode_many(heads, N, m, schedule)
    return mapping.normalized_rows(X, N)


def fp8_bound(x_abs, scale):
    # half an e4m3 ulp relative (2^-4) for normal values, half the smallest
    # subnormal step (2^-10 * scale) near zero, plus FP32 rolling error
    return 2.0 ** -4 * x_abs + 2.0 ** -10 * scale + 2e-5


def check_refined_lists(tidx, tsc, cand, F1, stride, radius, k, tol):
    """Refined lists [R, k] against the oracle's refinement (mapping.refine_topk)
    of the same coarse candidates, F1 [R, W1] the oracle's fidelities with every
    step-1 window: distinct starts from the read's pool, the same ranking up to
    ties, scores within tol.  Returns the fraction of identical lists."""
    exact = 0
    for r in range(F1.shape[0]):
        want_i, want_f = mapping.refine_topk(F1[r], cand[r], stride, radius, k)
        n = int(np.sum(want_i >= 0))            # entries with F = 0 are no location
        want_i, want_f = want_i[:n], want_f[:n]
        got = tidx[r, :n]
        assert np.all(tidx[r, n:] == -1) and np.all(tsc[r, n:] == 0) and np.all(got >= 0), r
        assert len(set(got.tolist())) == n, r                       # distinct starts
        pool = set(mapping.refine_pool(cand[r], stride, radius, F1.shape[1]).tolist())
        assert set(got.tolist()) <= pool, r                           # only refined starts
        got_true = F1[r, got]
        assert np.all(np.abs(got_true - want_f) <= mapping.TIE_TAU), r  # same ranking up to ties
        assert np.max(np.abs(tsc[r, :n] - got_true)) < tol, r
        exact += int(np.array_equal(got, want_i))
    return exact / F1.shape[0]


def assert_lists_exact(exact, rec, k_fetch, k, precision):
    """Rescored lists against the oracle's.  When the product scores in FP32,
    or over-fetches (k_fetch > k), every list must equal the oracle's up to
    ties.  With k_fetch == k in FP16 or FP8, a window the product ranks just
    below the k-th best is never rescored, so a few lists may differ: recall
    >= 0.99 and at least 97 % identical lists."""
    bad = np.nonzero(~np.asarray(exact))[0]
    if precision == "fp32" or k_fetch > k:
        assert bad.size == 0, f"lists differing from the oracle's: reads {bad.tolist()}"
    else:
        assert rec >= 0.99 and np.mean(exact) >= 0.97, (rec, bad.tolist())
