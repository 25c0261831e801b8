"""FP64 CPU oracle for RotorMap's hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
statement of what the HIP path computes, written from the paper (arXiv
2603.22245, "RotorMap and quantum fingerprints of DNA sequences via rotary
position embeddings").  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does,
and it shares no code with the HIP path.

Modules:
  rope     -- the RoPE-DNA encoding (s = 1), §2.1-§2.3 and §2.10, and the
              sliding-window update of §3.4
  tokens   -- the same with s-mer tokens and compact token maps (§2.1,
              §2.6, §2.10, §3.4)
  mapping  -- window index, read heads, fidelity, brute-force scoring and
              top-k (§3.1), recall metrics
  lev      -- textbook Levenshtein DP (§1) and a brute-force check
  stats    -- Spearman rank correlation
  learned  -- FP64 forward/backward of the angle-offset network

Parity status: every function here is pinned by a CPU test against an
identity or closed form the paper fixes (see tests/test_oracle_*.py), except
where a module header says "parity unpinned".
"""
