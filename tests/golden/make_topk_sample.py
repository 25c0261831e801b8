"""Write the FP64 oracle's exact top-k for a seeded sample of a workload's reads.

Usage: python tests/golden/make_topk_sample.py precision 64 16
Writes tests/golden/<workload>_top<k>_sample<n>.npz with arrays
  reads  [n]    read indices of the sample (numpy PCG64, seed 100*config+3)
  idx    [n,k]  oracle window ids, ranked (F desc, ties within 1e-12 by id)
  F      [n,k]  oracle fidelities
computed by oracle.mapping.map_reads over every window of the workload.  Only
the oracle and the seeded input generators are used.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import mapping  # noqa: E402

CONFIG_NO = {"plain": 1, "precision": 2, "batching": 3, "scale": 5}


def sample_reads(name: str, n: int) -> np.ndarray:
    rng = np.random.default_rng(100 * CONFIG_NO[name] + 3)
    return np.sort(rng.choice(synth.WORKLOADS[name].n_reads, n, replace=False))


def main(name: str, n: int, k: int):
    w = synth.WORKLOADS[name]
    ref = w.reference()
    reads = w.reads(ref)
    pick = sample_reads(name, n)
    heads = mapping.read_heads(reads.seq, reads.offsets, w.window_len)[pick]
    t = time.time()
    idx, F = mapping.map_reads(ref, heads, w.window_len, w.n_freq, k, w.stride)
    dt = time.time() - t
    out = os.path.join(HERE, f"{name}_top{k}_sample{n}.npz")
    np.savez(out, reads=pick, idx=idx, F=F, seconds=np.array(dt))
    print(f"{out}: {n} reads x {mapping.n_windows(ref.shape[0], w.window_len, w.stride)} windows "
          f"in {dt:.1f} s")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), int(sys.argv[3]))
