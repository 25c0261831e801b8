"""The correlation score of §2.4 on the device (thin wrapper over the C ABI).

Pairs of a random string and a companion mutated at rate err, their
fidelities (rm_pair_fidelity, plain or learned encoding), then per rate the
expected fidelity, the fitting curve through the points (E_fid(err), err) and
the RMSE of predicting err from a pair's fidelity (rm_correlation_score).
"""
from __future__ import annotations

import numpy as np

from . import _lib as L
from . import learned


def score(F, err_rates, stream=None):
    """F: device float32 [n_rates * per_rate] (rate-major); err_rates: host
    sequence.  Returns device tensors (E_fid [n_rates], RMSE [n_rates])."""
    import torch
    err = torch.as_tensor(np.asarray(err_rates, dtype=np.float32)).to(F.device)
    n = int(err.numel())
    if F.numel() % n:
        raise ValueError("F must hold the same number of pairs for every rate")
    E = torch.empty(n, dtype=torch.float32, device=F.device)
    rmse = torch.empty(n, dtype=torch.float32, device=F.device)
    L.rm_correlation_score(F, err, n, F.numel() // n, E, rmse, stream)
    return E, rmse


def run(ps: learned.PairSet, err_rates, nominal_len: int, params=None, stream=None):
    """The protocol on a pair set ordered rate by rate: (F, E_fid, RMSE), device tensors."""
    F = learned.pair_fidelity(params, ps, nominal_len, stream)
    E, rmse = score(F, err_rates, stream)
    return F, E, rmse
