"""Write the FP64 oracle's exact top-k under a token encoding (s-mers, §2.1;
compact maps, §2.6) for the same seeded read sample as make_topk_sample.py.

Usage: python tests/golden/make_token_topk_sample.py precision s2 64 16
Writes tests/golden/<workload>_<encoding>_top<k>_sample<n>.npz with arrays
  reads  [n]    read indices of the sample (numpy PCG64, seed 100*config+3)
  idx    [n,k]  oracle window ids, ranked (F desc, ties within 1e-12 by id)
  F      [n,k]  oracle fidelities
computed by oracle.tokens.map_reads over every window of the workload, with
the named encoding of synth.TOKEN_ENCODINGS (a frequent-s-mer map is the
oracle's own, oracle.tokens.frequent_map).  Only the oracle and the seeded
input generators are used.
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
from oracle import mapping, tokens  # noqa: E402


def main(name: str, enc: str, n: int, k: int):
    w = synth.WORKLOADS[name]
    s, m, C, tm, sched = synth.token_encoding(enc)
    ref = w.reference()
    if synth.token_map_is_frequent(enc):
        tm = tokens.frequent_map(ref, s, C)
    reads = w.reads(ref)
    pick = sample_reads(name, n)
    heads = mapping.read_heads(reads.seq, reads.offsets, w.window_len)[pick]
    t = time.time()
    idx, F = tokens.map_reads(ref, heads, w.window_len, s, m, C, tm, k, w.stride, sched)
    dt = time.time() - t
    out = os.path.join(HERE, f"{name}_{enc}_top{k}_sample{n}.npz")
    np.savez(out, reads=pick, idx=idx, F=F, seconds=np.array(dt))
    print(f"{out}: {n} reads x {mapping.n_windows(ref.shape[0], w.window_len, w.stride)} windows "
          f"in {dt:.1f} s")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2], int(sys.argv[3]), int(sys.argv[4]))
