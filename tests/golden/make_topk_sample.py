"""Write the FP64 oracle's exact top-k for a seeded sample of a workload's reads.

Usage: python tests/golden/make_topk_sample.py precision 64 16 [--parts P] [--threads T]
Writes tests/golden/<workload>_top<k>_sample<n>.npz with arrays
  reads  [n]    read indices of the sample (numpy PCG64, seed 100*config+3)
  idx    [n,k]  oracle window ids, ranked (F desc, ties within 1e-12 by id)
  F      [n,k]  oracle fidelities
computed by oracle.mapping.map_reads over every window of the workload.  Only
the oracle and the seeded input generators are used.

With --parts P the windows are split into P contiguous id ranges, each scanned
by oracle.mapping.map_reads in a child process (T BLAS threads each), and the
P partial top-k lists are combined with oracle.mapping.topk_rows: the top-k of
a union of ranges is the top-k of the union of the ranges' top-k lists (the
same argument the oracle uses for its own window chunks).
"""
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import mapping  # noqa: E402

CONFIG_NO = {"plain": 1, "precision": 2, "batching": 3, "scale": 5}


def sample_reads(name: str, n: int) -> np.ndarray:
    rng = np.random.default_rng(100 * CONFIG_NO[name] + 3)
    return np.sort(rng.choice(synth.WORKLOADS[name].n_reads, n, replace=False))


def _inputs(name: str, n: int):
    w = synth.WORKLOADS[name]
    ref = w.reference()
    pick = sample_reads(name, n)
    reads = w.reads(ref)
    heads = mapping.read_heads(reads.seq, reads.offsets, w.window_len)[pick]
    return w, ref, pick, heads


def _part(name: str, n: int, k: int, lo: int, hi: int, out: str):
    w, ref, pick, heads = _inputs(name, n)
    idx, F = mapping.map_reads(ref, heads, w.window_len, w.n_freq, k, w.stride,
                               window_range=(lo, hi))
    np.savez(out, idx=idx, F=F)


def main(name: str, n: int, k: int, parts: int = 1, threads: int = 0):
    w = synth.WORKLOADS[name]
    t = time.time()
    if parts <= 1:
        _, ref, pick, heads = _inputs(name, n)
        idx, F = mapping.map_reads(ref, heads, w.window_len, w.n_freq, k, w.stride)
        W = mapping.n_windows(ref.shape[0], w.window_len, w.stride)
    else:
        W = mapping.n_windows(w.G, w.window_len, w.stride)
        pick = sample_reads(name, n)
        cuts = np.linspace(0, W, parts + 1).astype(np.int64)
        env = dict(os.environ)
        if threads > 0:
            for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
                env[v] = str(threads)
        with tempfile.TemporaryDirectory() as tmp:
            files = [os.path.join(tmp, f"part{i}.npz") for i in range(parts)]
            procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--part", name,
                                       str(n), str(k), str(cuts[i]), str(cuts[i + 1]), files[i]],
                                      env=env) for i in range(parts)]
            for p in procs:
                if p.wait() != 0:
                    raise RuntimeError("an oracle part failed")
            got = [np.load(f) for f in files]
            allI = np.concatenate([g["idx"] for g in got], axis=1)
            allF = np.concatenate([g["F"] for g in got], axis=1)
        idx, F = mapping.topk_rows(allF, allI, k)
    dt = time.time() - t
    out = os.path.join(HERE, f"{name}_top{k}_sample{n}.npz")
    np.savez(out, reads=pick, idx=idx.astype(np.int32 if W < 2 ** 31 else np.int64), F=F,
             seconds=np.array(dt))
    print(f"{out}: {n} reads x {W} windows in {dt:.1f} s")


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "--part":
        _part(a[1], int(a[2]), int(a[3]), int(a[4]), int(a[5]), a[6])
        sys.exit(0)
    opts = {"--parts": 1, "--threads": 0}
    pos = []
    i = 0
    while i < len(a):
        if a[i] in opts:
            opts[a[i]] = int(a[i + 1])
            i += 2
        else:
            pos.append(a[i])
            i += 1
    main(pos[0], int(pos[1]), int(pos[2]), opts["--parts"], opts["--threads"])
