"""Train the offset network with the FP64 oracle on the CPU and write its weights.

Usage: python tests/golden/make_learned_weights.py 16384 3
Writes tests/golden/learned_weights.npy (10,432 float32 values, the layout of
oracle.learned) trained on the first n pairs of the learned-offsets workload
(synth.mutate_pairs, 150 bp, 0..30 edits, seed synth.PAIRS_SEED), labels by the
oracle's edit distance, loss and gradient by oracle.learned.batch_loss_and_grad,
oracle.learned.adam_step (beta 0.9 / 0.999, eps 1e-8, lr 3e-3), batches of 256 in order.  These
weights give the mapping tests and the learned-encoding mapping sample a
trained network that no GPU code produced.  Only the oracle and the seeded
input generators are used.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import learned, lev, stats  # noqa: E402

N = 150


def main(n: int, epochs: int, batch: int = 256, lr: float = 3e-3):
    P = synth.mutate_pairs(n + 2048, 150, 30, seed=synth.PAIRS_SEED)
    ld = lev.lev_many(P.a, P.a_off, P.b, P.b_off)
    pairs = [P.pair(i) for i in range(P.n)]
    params = learned.init_params(0)
    m = np.zeros_like(params)
    v = np.zeros_like(params)
    t = 0
    t0 = time.time()
    for ep in range(epochs):
        for i in range(0, n - batch + 1, batch):
            loss, g, _ = learned.batch_loss_and_grad(params, pairs[i:i + batch], ld[i:i + batch], N)
            params, m, v, t = learned.adam_step(params, m, v, t, g, lr)
        held = pairs[n:]
        Fl = learned.pair_fidelities(params, held, N)
        Fp = learned.pair_fidelities(learned.init_params(0), held, N)
        print(f"epoch {ep}: last batch loss {loss:.4f}, held-out Spearman learned "
              f"{-stats.spearman(Fl, ld[n:]):.4f} vs token-middle plain "
              f"{-stats.spearman(Fp, ld[n:]):.4f}, {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, "learned_weights.npy")
    np.save(out, params.astype(np.float32))
    print(out)


if __name__ == "__main__":
    main(int(sys.argv[1]), int(sys.argv[2]))
