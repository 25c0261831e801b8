"""Write the FP64 oracle's exact top-k under the learned encoding for the same
seeded read sample as make_topk_sample.py.

Usage: python tests/golden/make_learned_topk_sample.py precision 64 16
Reads tests/golden/learned_weights.npy (written by make_learned_weights.py from
the oracle alone) and writes tests/golden/<workload>_learned_top<k>_sample<n>.npz
with arrays reads [n], idx [n,k], F [n,k] from oracle.learned.map_reads with
the inference arithmetic (bfloat16 weights and hidden values).  Only the oracle
and the seeded input generators are used.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import synth  # noqa: E402
from make_topk_sample import sample_reads  # noqa: E402
from oracle import learned, mapping  # noqa: E402


def main(name: str, n: int, k: int):
    w = synth.WORKLOADS[name]
    params = np.load(os.path.join(HERE, "learned_weights.npy")).astype(np.float64)
    ref = w.reference()
    reads = w.reads(ref)
    pick = sample_reads(name, n)
    heads = mapping.read_heads(reads.seq, reads.offsets, w.window_len)[pick]
    t = time.time()
    idx, F = learned.map_reads(params, ref, heads, w.window_len, k, bf16=True)
    dt = time.time() - t
    out = os.path.join(HERE, f"{name}_learned_top{k}_sample{n}.npz")
    np.savez(out, reads=pick, idx=idx, F=F, seconds=np.array(dt))
    print(f"{out}: {n} reads in {dt:.1f} s")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), int(sys.argv[3]))
