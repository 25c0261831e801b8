"""The correlation score of §2.4 on the GPU (rm_correlation_score, fidelities
from rm_pair_fidelity) against the FP64 oracle (oracle.correlation).

Tolerances: pair fidelities are FP32 sums of at most a few hundred unit terms
(1e-4 absolute, as in the learned-encoding tests); E_fid is a mean of such
values (1e-5); the RMSE depends on the fidelities through the curve, whose
slope d err / d E_fid is large where E_fid flattens at high rates, so it is
compared to 1e-3 relative plus 1e-4.  On identical FP32 inputs the kernel's
E_fid and RMSE agree with the oracle's to FP32 summation error."""
import os

import numpy as np
import pytest

import synth
from oracle import correlation as OC

from gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
N = 150
RATES = (np.arange(25) + 0.5) * 0.5 / 25        # 25 rates evenly over (0, 0.5)


def _pairs(per, seed):
    edits = np.repeat(np.rint(RATES * N).astype(np.int64), per)
    return synth.mutate_pairs(edits.size, N, int(edits.max()), seed=seed, edits=edits)


def test_score_kernel_on_given_fidelities():
    """The kernel alone on fidelities the oracle also gets: random values
    (E_fid not monotone in the rate, fidelities past both ends of the curve),
    and an exact function of the rate (RMSE 0)."""
    torch = torch_cuda()
    from paper_2603_22245_amd import correlation as CR
    rng = np.random.default_rng(60)
    for n_rates, per in ((25, 40), (7, 1), (256, 3), (1, 5)):
        err = np.sort(rng.uniform(0, 0.5, n_rates)).astype(np.float32)
        F = rng.uniform(0, 1, (n_rates, per)).astype(np.float32)
        E, rmse = CR.score(torch.from_numpy(F.ravel()).cuda(), err)
        want_E, _, want_rmse = OC.score(err.astype(np.float64), F.astype(np.float64))
        np.testing.assert_allclose(E.cpu().numpy(), want_E, atol=1e-6)
        np.testing.assert_allclose(rmse.cpu().numpy(), want_rmse, rtol=1e-4, atol=1e-6)
    F = np.repeat(((1 - RATES) ** 2)[:, None], 9, axis=1).astype(np.float32)
    E, rmse = CR.score(torch.from_numpy(F.ravel()).cuda(), RATES)
    assert np.max(rmse.cpu().numpy()) < 1e-6


@pytest.mark.parametrize("encoding", ["plain", "learned"])
def test_correlation_protocol_matches_oracle(encoding):
    """The §2.4 protocol at all 25 rates (up to 74 edits of 150 letters, i.e.
    err up to 0.49): every pair's fidelity, E_fid and the RMSE per rate."""
    torch = torch_cuda()
    from paper_2603_22245_amd import correlation as CR, learned as LM
    per = 40
    P = _pairs(per, seed=61)
    pairs = [P.pair(i) for i in range(P.n)]
    ps = LM.upload_pairs(P.a, P.a_off, P.b, P.b_off)
    if encoding == "plain":
        params = None
        want_F = OC.plain_pair_fidelities(pairs, N)
    else:
        w = np.load(os.path.join(HERE, "golden", "learned_weights.npy"))
        params = torch.from_numpy(w).cuda()
        want_F = OC.learned_pair_fidelities(w.astype(np.float64), pairs, N)
    F, E, rmse = CR.run(ps, RATES, N, params)
    torch.cuda.synchronize()
    F = F.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(F - want_F)) <= 1e-4
    want_E, _, want_rmse = OC.score(RATES, want_F.reshape(25, per))
    E, rmse = E.cpu().numpy(), rmse.cpu().numpy()
    print(f"{encoding}: max |dF| {np.max(np.abs(F - want_F)):.2e}, max |dE| "
          f"{np.max(np.abs(E - want_E)):.2e}, max |dRMSE| {np.max(np.abs(rmse - want_rmse)):.2e}; "
          f"RMSE at 1/3/5 %: {want_rmse[0]:.4f} ...")
    assert np.max(np.abs(E - want_E)) <= 1e-5
    assert np.all(np.abs(rmse - want_rmse) <= 1e-3 * want_rmse + 1e-4)
