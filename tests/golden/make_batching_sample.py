"""Write the FP64 oracle's exact top-k for a seeded sample of the batching
workload's reads, per bucket.

Usage: python tests/golden/make_batching_sample.py 4 16
Writes tests/golden/batching_top<k>_per_bucket<n>.npz with arrays
  reads   [m]      read indices (n per non-empty bucket, numpy PCG64 seed 303)
  bucket  [m]      bucket head length N_b of each read (stride N_b / 100)
  idx     [m, k]   oracle window ids (F desc, ties within 1e-12 by id)
  F       [m, k]   oracle fidelities
Only the oracle, the bucketing rule (longest bucket length not above the read
length) and the seeded input generators are used.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import mapping  # noqa: E402

BUCKETS = (100, 200, 400, 800, 1600, 3200, 6400)


def main(n: int, k: int):
    w = synth.WORKLOADS["batching"]
    ref = w.reference()
    reads = w.reads(ref)
    lens = reads.lengths()
    rng = np.random.default_rng(303)
    out_r, out_b, out_i, out_f = [], [], [], []
    t0 = time.time()
    for bi, nb in enumerate(BUCKETS):
        upper = BUCKETS[bi + 1] if bi + 1 < len(BUCKETS) else 1 << 62
        ids = np.nonzero((lens >= nb) & (lens < upper))[0]
        if ids.size == 0:
            continue
        pick = np.sort(rng.choice(ids, min(n, ids.size), replace=False))
        heads = np.stack([reads.read(i)[:nb] for i in pick])
        stride = max(1, nb // 100)
        idx, F = mapping.map_reads(ref, heads, nb, 32, k, stride)
        out_r.append(pick)
        out_b.append(np.full(pick.size, nb))
        out_i.append(idx)
        out_f.append(F)
        print(f"bucket {nb}: {pick.size} reads, {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(HERE, f"batching_top{k}_per_bucket{n}.npz")
    np.savez(path, reads=np.concatenate(out_r), bucket=np.concatenate(out_b),
             idx=np.concatenate(out_i), F=np.concatenate(out_f))
    print(path)


if __name__ == "__main__":
    main(int(sys.argv[1]), int(sys.argv[2]))
