"""FP64 oracle of the correlation score of §2.4 (scoring the correlations).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, FP64.

§2.4 measures how well fidelity predicts the mutation rate between a random
string and a mutated companion:

1. for a string length N, a mutation rate err and an encoding, the expected
   fidelity E_fid(err) of pairs (dna, mut) sampled at that rate;
2. for rates err spread evenly over (0, 0.5), the points (E_fid(err), err)
   connected into a curve (the fitting curve);
3. for a rate err, the pairs' points (fid, err): the vertical distance of each
   to the fitting curve, squared, averaged, square-rooted (the RMSE of
   predicting err from an observed fidelity).

Readings where the paper is silent: the expectation is the sample mean of the
rate's pairs; "connect them" is straight segments between consecutive points
ordered by E_fid; a fidelity outside the range of the E_fid values takes the
err of the nearest end point (the curve is extended flat).

Pins (tests/test_oracle_correlation.py): a hand-worked two-rate example
(distances inside a segment and past both ends), fidelities that are an exact
decreasing function of err give RMSE 0 at every rate, and the plain fidelity
of substitution-only pairs with m = N equals the Hamming closed form.
"""
from __future__ import annotations

import numpy as np

from . import learned, rope


def expected_fidelity(fid_by_rate) -> np.ndarray:
    """E_fid per rate: the mean fidelity of that rate's pairs (step 1)."""
    return np.array([float(np.mean(np.asarray(f, dtype=np.float64))) for f in fid_by_rate])


def fitting_curve(err_rates, E):
    """The points (E_fid(err), err), ordered by E_fid ascending (step 2).
    Returns (E, err) arrays; the curve joins consecutive points."""
    E = np.asarray(E, dtype=np.float64)
    e = np.asarray(err_rates, dtype=np.float64)
    order = sorted(range(E.shape[0]), key=lambda i: (E[i], i))
    return E[order], e[order]


def curve_err(curve, fid: float) -> float:
    """The rate the fitting curve assigns to a fidelity: on the segment between
    the two consecutive points whose E_fid values enclose fid, linearly; the
    end point's rate below the first or above the last E_fid."""
    E, e = curve
    if fid <= E[0]:
        return float(e[0])
    if fid >= E[-1]:
        return float(e[-1])
    for i in range(E.shape[0] - 1):
        if E[i] <= fid <= E[i + 1]:
            if E[i + 1] == E[i]:
                return float(e[i])
            t = (fid - E[i]) / (E[i + 1] - E[i])
            return float(e[i] + t * (e[i + 1] - e[i]))
    raise AssertionError("unreachable")


def prediction_rmse(err_rates, fid_by_rate, curve) -> np.ndarray:
    """Per rate, sqrt(mean over its pairs of (curve_err(fid) - err)^2) (step 3)."""
    out = []
    for err, fids in zip(err_rates, fid_by_rate):
        d2 = [(curve_err(curve, float(f)) - float(err)) ** 2 for f in fids]
        out.append(float(np.sqrt(np.mean(d2))))
    return np.array(out)


def plain_pair_fidelities(pairs, N: int, m: int = 32) -> np.ndarray:
    """F = |<a|b>|^2 / (|a|^2 |b|^2) of the plain encodings (§2.1-§2.4, s = 1,
    f_k = k, nominal length N) of each pair's whole strings."""
    out = np.empty(len(pairs))
    for i, (a, b) in enumerate(pairs):
        ca = rope.encode_raw(a, N, m)
        cb = rope.encode_raw(b, N, m)
        out[i] = abs(np.vdot(ca, cb)) ** 2 / (rope.sq_norm(ca) * rope.sq_norm(cb))
    return out


def learned_pair_fidelities(params, pairs, N: int) -> np.ndarray:
    """The same with the learned encoding (FP64 network, oracle.learned)."""
    return learned.pair_fidelities(params, pairs, N)


def score(err_rates, fid_by_rate):
    """Steps 1-3: (E_fid per rate, the fitting curve, RMSE per rate)."""
    E = expected_fidelity(fid_by_rate)
    curve = fitting_curve(err_rates, E)
    return E, curve, prediction_rmse(err_rates, fid_by_rate, curve)
