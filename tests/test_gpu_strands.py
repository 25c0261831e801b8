"""GPU parity of both-strand mapping and the fidelity-threshold regime against
the FP64 oracle (oracle.mapping.reverse_complement / merge_strands)."""
import numpy as np
import pytest

import synth
from oracle import mapping
from tests.gpu_helpers import oracle_heads, oracle_windows, torch_cuda

pytestmark = pytest.mark.gpu

PLAIN = synth.WORKLOADS["plain"]
N, K = 150, 8


def test_reverse_complement_kernel_bit_exact():
    from paper_2603_22245_amd import _lib as L
    torch = torch_cuda()
    rng = np.random.default_rng(21)
    lens = rng.integers(1, 300, 57)
    lens[3] = 1
    off = np.concatenate([[5], 5 + np.cumsum(lens)]).astype(np.int64)   # batch starts at 5
    seq = rng.integers(0, 4, int(off[-1])).astype(np.uint8)
    d_seq = torch.from_numpy(seq).cuda()
    d_off = torch.from_numpy(off).cuda()
    d_out = torch.full((seq.size,), 77, dtype=torch.uint8, device="cuda")
    L.rm_reverse_complement(d_seq, d_off, lens.size, int(off[-1] - off[0]), d_out)
    torch.cuda.synchronize()
    out = d_out.cpu().numpy()
    assert np.all(out[:5] == 77)                                        # outside the batch
    for r in range(lens.size):
        a, b = off[r], off[r + 1]
        assert np.array_equal(out[a:b], mapping.reverse_complement(seq[a:b])), r


@pytest.fixture(scope="module")
def strand_case():
    ref = PLAIN.reference()
    reads = PLAIN.reads(ref)
    seq, off = reads.seq.copy(), reads.offsets
    R = reads.n
    other = np.arange(R) % 2 == 1                 # odd reads come from the other strand
    for r in np.nonzero(other)[0]:
        seq[off[r]:off[r + 1]] = mapping.reverse_complement(seq[off[r]:off[r + 1]])
    fwd = np.stack([seq[off[r]:off[r] + N] for r in range(R)])
    rev = np.stack([mapping.reverse_complement(seq[off[r]:off[r + 1]])[:N] for r in range(R)])
    Cn, _ = oracle_windows(ref, N)
    Ff = np.abs(np.conj(oracle_heads(fwd, N)[0]) @ Cn.T) ** 2
    Fr = np.abs(np.conj(oracle_heads(rev, N)[0]) @ Cn.T) ** 2
    return ref, seq, off, other, Ff, Fr


@pytest.mark.parametrize("min_fidelity", [0.0, 0.5])
def test_both_strands_against_the_oracle(strand_case, min_fidelity):
    from paper_2603_22245_amd import mapper
    torch = torch_cuda()
    ref, seq, off, other, Ff, Fr = strand_case
    R, W = Ff.shape
    index = mapper.build_index(ref, precision="fp32")
    rb2 = mapper.upload_reads_both_strands(index, seq, off)
    bufs2 = mapper.map_buffers(index, 2 * R, K, 16)
    res = mapper.map_reads_both_strands(index, rb2, bufs2, min_fidelity)
    torch.cuda.synchronize()
    ti, ts = res.top_idx.cpu().numpy(), res.top_score.cpu().numpy()
    tst, nf = res.top_strand.cpu().numpy(), res.n_found.cpu().numpy()
    fi, ff = mapping.topk_rows(Ff, np.arange(W), K)
    ri, rf = mapping.topk_rows(Fr, np.arange(W), K)
    top1_strand_ok = 0
    for r in range(R):
        wi, wf, ws = mapping.merge_strands(fi[r], ff[r], ri[r], rf[r], K, min_fidelity)
        n = int(nf[r])
        # entries within TIE_TAU of the threshold may fall either side of it
        lo = sum(1 for f in wf if f >= min_fidelity + mapping.TIE_TAU)
        assert lo <= n <= wi.size + sum(1 for f in np.r_[ff[r], rf[r]]
                                        if min_fidelity - mapping.TIE_TAU <= f < min_fidelity), r
        assert np.all(ti[r, n:] == -1) and np.all(tst[r, n:] == -1) and np.all(ts[r, n:] == 0), r
        got_true = np.where(tst[r, :n] == 0, Ff[r, np.maximum(ti[r, :n], 0)],
                            Fr[r, np.maximum(ti[r, :n], 0)])
        m = min(n, wi.size)
        assert np.all(np.abs(got_true[:m] - wf[:m]) <= mapping.TIE_TAU), r
        assert np.all(got_true >= min_fidelity - mapping.TIE_TAU), r
        assert np.max(np.abs(ts[r, :n] - got_true), initial=0.0) < 2e-6, r
        if n:
            top1_strand_ok += int(tst[r, 0] == int(other[r]))
    mapped = int(np.sum(nf > 0))
    print(f"min_fidelity {min_fidelity}: mapped {mapped}/{R}, top-1 on the read's own strand "
          f"{top1_strand_ok}/{mapped}")
    assert top1_strand_ok >= 0.99 * mapped
    if min_fidelity == 0.0:
        assert mapped == R
