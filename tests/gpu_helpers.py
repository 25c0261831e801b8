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
