"""The C-ABI library loads, exports every declared entry point, and rejects bad
arguments on the host before enqueuing anything (no GPU needed)."""
import ctypes

import pytest

from paper_2603_22245_amd import _lib as L


def test_library_exports_every_declared_function():
    lib = L.lib()
    names = L.header_functions()
    assert {"rm_encode_reference", "rm_encode_reads", "rm_score_topk", "rm_rescore"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings_and_version():
    assert L.status_str(L.RM_OK) == "ok"
    for s in (L.RM_EINVAL, L.RM_ESIZE, L.RM_EUNSUPPORTED, L.RM_EHIP):
        assert L.status_str(s) not in ("ok", "unknown status")
    assert "gfx950" in L.rm_version()


def test_window_counts_and_sizes():
    p = L.make_params(150, 1, 32, "default", "fp16")
    assert L.rm_num_windows(20_000, p) == 19_851
    assert L.rm_num_windows(149, p) == -1
    assert L.rm_index_bytes(20_000, p) >= 19_851 * 256 * 2
    p8 = L.make_params(150, 1, 32, "default", "fp8")
    p32 = L.make_params(150, 1, 32, "default", "fp32")
    assert L.rm_index_bytes(10**7, p8) < L.rm_index_bytes(10**7, p) < L.rm_index_bytes(10**7, p32)
    assert L.rm_read_emb_bytes(10, p) == 10 * 2 * 256 * 2
    assert L.rm_read_emb_bytes(0, p) == 0
    p3 = L.make_params(150, 7, 32, "default", "fp16")
    assert L.rm_num_windows(1000, p3) == (1000 - 150) // 7 + 1


@pytest.mark.parametrize("field,value,status", [
    ("n_freq", 16, L.RM_EUNSUPPORTED),
    ("window_len", 0, L.RM_ESIZE),
    ("window_len", L.RM_MAX_WINDOW + 1, L.RM_ESIZE),
    ("stride", 0, L.RM_ESIZE),
    ("precision", 7, L.RM_EINVAL),
    ("schedule", 5, L.RM_EINVAL),
    ("reanchor", -1, L.RM_ESIZE),
])
def test_bad_params_rejected(field, value, status):
    p = L.make_params(150, 1, 32, "default", "fp16")
    setattr(p, field, value)
    assert L.rm_index_bytes(20_000, p) == 0
    out = L.rm_index()
    st = L.lib().rm_encode_reference(0x1000, 20_000, ctypes.byref(p), 0x10000, 1 << 30,
                                     ctypes.byref(out), None)
    assert st == status


def test_encode_reference_validation():
    lib = L.lib()
    p = L.make_params(150, 1, 32, "default", "fp16")
    out = L.rm_index()
    need = L.rm_index_bytes(20_000, p)
    enc = lambda ref, n, buf, nb: lib.rm_encode_reference(ref, n, ctypes.byref(p), buf, nb,
                                                          ctypes.byref(out), None)
    assert enc(None, 20_000, 0x10000, need) == L.RM_EINVAL
    assert enc(0x1000, 20_000, None, need) == L.RM_EINVAL
    assert enc(0x1000, 20_000, 0x10010, need) == L.RM_EINVAL      # misaligned buffer
    assert enc(0x1000, 20_000, 0x10000, need - 1) == L.RM_ESIZE
    assert enc(0x1000, 149, 0x10000, need) == L.RM_ESIZE           # shorter than a window
    assert lib.rm_encode_reference(0x1000, 20_000, None, 0x10000, need, ctypes.byref(out), None) \
        == L.RM_EINVAL
    huge = L.make_params(1, 1, 32, "default", "fp8")
    assert L.rm_index_bytes(2**31 + 5, huge) == 0                  # more than 2^31-1 windows


def _fake_index(precision="fp16", W_ref=20_000):
    p = L.make_params(150, 1, 32, "default", precision)
    idx = L.rm_index()
    idx.p = p
    idx.ref_len = W_ref
    idx.n_windows = L.rm_num_windows(W_ref, p)
    for f in ("d_emb", "d_scale", "d_norm2", "d_phase64", "d_phase32", "d_step32"):
        setattr(idx, f, 0x100000)
    return idx


def test_read_score_rescore_validation():
    lib = L.lib()
    idx = _fake_index()
    R = ctypes.byref
    # encode reads
    assert lib.rm_encode_reads(None, 1, 1, 10, 1, 1, None) == L.RM_EINVAL
    assert lib.rm_encode_reads(R(idx), None, 1, 10, 1, 1, None) == L.RM_EINVAL
    assert lib.rm_encode_reads(R(idx), 1, 1, 0, 1, 1, None) == L.RM_ESIZE
    bad = _fake_index()
    bad.n_windows += 1                                             # inconsistent descriptor
    assert lib.rm_encode_reads(R(bad), 1, 1, 10, 1, 1, None) == L.RM_EINVAL
    idx8 = _fake_index("fp8")
    assert lib.rm_encode_reads(R(idx8), 1, 1, 10, 1, None, None) == L.RM_EINVAL  # scale needed
    # score
    ws = L.rm_score_workspace_bytes(idx, 100, 8)
    assert ws > 0
    assert L.rm_score_workspace_bytes(idx, 100, 0) == 0
    assert L.rm_score_workspace_bytes(idx, 100, L.RM_MAX_KFETCH + 1) == 0
    sc = lambda i, n, kf, nb: lib.rm_score_topk(R(i), 1, 1, n, kf, 1, 1, 1, nb, None)
    assert sc(idx, 100, 8, ws - 1) == L.RM_ESIZE
    assert sc(idx, 100, 0, ws) == L.RM_ESIZE
    assert sc(idx, 100, L.RM_MAX_KFETCH + 1, 1 << 40) == L.RM_ESIZE
    assert L.rm_score_workspace_bytes(idx, 100, L.RM_MAX_KFETCH) > ws   # 64 candidates
    assert sc(idx, 0, 8, ws) == L.RM_ESIZE
    # 1,024-component token encodings keep at most RM_WIDE_MAX_KFETCH candidates
    wide = _fake_index()
    wide.p = L.make_params(150, 1, 4, "default", "fp16", 0, 8, 256, 0x2000)
    wide.d_token_class = 0x100000
    assert L.rm_score_workspace_bytes(wide, 100, L.RM_WIDE_MAX_KFETCH) > 0
    assert L.rm_score_workspace_bytes(wide, 100, L.RM_WIDE_MAX_KFETCH + 1) == 0
    assert sc(wide, 100, L.RM_WIDE_MAX_KFETCH + 1, 1 << 40) == L.RM_ESIZE
    assert lib.rm_score_topk(R(idx), None, 1, 100, 8, 1, 1, 1, ws, None) == L.RM_EINVAL
    assert lib.rm_score_topk(R(idx8), 1, None, 100, 8, 1, 1, 1, 1 << 30, None) == L.RM_EINVAL
    # rescore
    rs = lambda n, kf, k: lib.rm_rescore(R(idx), 1, 1, 1, n, kf, 1, k, 1, 1, None)
    assert rs(10, 8, 9) == L.RM_ESIZE                              # k > k_fetch
    assert rs(10, 8, 0) == L.RM_ESIZE
    assert rs(0, 8, 8) == L.RM_ESIZE
    assert lib.rm_rescore(R(idx), None, 1, 1, 10, 8, 1, 8, 1, 1, None) == L.RM_EINVAL


def test_learned_and_edit_distance_validation():
    """Argument checks of the learned and edit-distance entry points run on the
    host and return before anything is enqueued."""
    lib = L.lib()
    R = ctypes.byref
    assert L.rm_learned_workspace_bytes(1) == 0
    assert L.rm_learned_workspace_bytes(L.RM_LEARNED_MAX_PAIRS + 1) == 0
    ws = L.rm_learned_workspace_bytes(64)
    assert ws > 64 * 2 * 256 * 4
    assert L.rm_delta_bytes(8) == 0
    assert L.rm_delta_bytes(9) == 32 * 4
    # train step / gradient
    st = lambda n, ln, nb, loss=1: lib.rm_learned_train_step(1, 1e-3, 1, 1, 1, 1, 1, n, ln, 1, nb,
                                                             loss, None)
    assert st(64, 150, ws - 1) == L.RM_ESIZE        # (every call here fails validation)
    assert st(1, 150, ws) == L.RM_ESIZE
    assert st(L.RM_LEARNED_MAX_PAIRS + 1, 150, 1 << 40) == L.RM_ESIZE
    assert st(64, 0, ws) == L.RM_ESIZE
    assert st(64, 150, ws, loss=None) == L.RM_EINVAL
    assert lib.rm_learned_gradient(1, 1, 1, 1, 1, 1, 64, 150, 1, ws, None, 1, None) == L.RM_EINVAL
    # encode, fidelity, inference
    assert lib.rm_learned_encode(None, None, 1, 4, 150, 1, None) == L.RM_EINVAL
    assert lib.rm_learned_encode(None, 1, 1, 0, 150, 1, None) == L.RM_ESIZE
    assert lib.rm_pair_fidelity(1, None, 4, 1, None) == L.RM_EINVAL
    assert lib.rm_pair_fidelity(1, 1, 0, 1, None) == L.RM_ESIZE
    assert lib.rm_mlp_infer(1, 1, 8, 0x1000, None) == L.RM_ESIZE
    assert lib.rm_mlp_infer(1, 1, 100, 0x1004, None) == L.RM_EINVAL        # misaligned offsets
    assert lib.rm_mlp_infer(None, 1, 100, 0x1000, None) == L.RM_EINVAL
    # learned mapping calls
    idx = _fake_index()
    p = L.make_params(8, 1, 32, "default", "fp16")
    out = L.rm_index()
    assert lib.rm_encode_reference_learned(1, 1000, R(p), 1, 0x10000, 1 << 30, R(out), None) \
        == L.RM_ESIZE                                                       # N < 9
    p = L.make_params(150, 1, 32, "default", "fp16")
    assert lib.rm_encode_reference_learned(1, 1000, R(p), None, 0x10000, 1 << 30, R(out), None) \
        == L.RM_EINVAL
    assert lib.rm_encode_reads_learned(R(idx), 1, 1, 10, None, 1, 1, None) == L.RM_EINVAL
    assert lib.rm_rescore_learned(R(idx), 1, None, 1, 1, 1, 10, 8, 1, 8, 1, 1, None) == L.RM_EINVAL
    assert lib.rm_rescore_learned(R(idx), 1, 1, 1, 1, 1, 10, 8, 1, 9, 1, 1, None) == L.RM_ESIZE
    # edit distance
    assert lib.rm_levenshtein(None, 1, 1, 1, 10, 1, None) == L.RM_EINVAL
    assert lib.rm_levenshtein(1, 1, 1, 1, 0, 1, None) == L.RM_ESIZE
    assert lib.rm_levenshtein(1, 1, 1, 1, (2**31) * 256, 1, None) == L.RM_ESIZE


def test_refine_validation():
    """rm_refine rejects every bad argument before anything is launched."""
    lib = L.lib()
    idx = _fake_index()
    R = ctypes.byref
    assert L.rm_refine_workspace_bytes(10, 8, 3) == (10 * 8 * 7 * 8 + 255) // 256 * 256
    assert L.rm_refine_workspace_bytes(10, 8, L.RM_REFINE_MAX_RADIUS + 1) == 0
    assert L.rm_refine_workspace_bytes(10, 0, 3) == 0
    assert L.rm_refine_workspace_bytes(0, 8, 3) == 0
    ws = L.rm_refine_workspace_bytes(10, 8, 3)
    rf = lambda n, kf, rad, k, nb, i=idx: lib.rm_refine(R(i), 1, 1, 1, n, kf, 1, rad, k, 1, 1, 1,
                                                       nb, None)
    assert rf(10, 8, 3, 8, ws - 1) == L.RM_ESIZE                   # workspace too small
    assert rf(10, 8, -1, 8, ws) == L.RM_ESIZE
    assert rf(10, 8, L.RM_REFINE_MAX_RADIUS + 1, 8, 1 << 30) == L.RM_ESIZE
    assert rf(10, 0, 3, 1, ws) == L.RM_ESIZE
    assert rf(10, L.RM_MAX_KFETCH + 1, 3, 8, 1 << 30) == L.RM_ESIZE
    assert rf(0, 8, 3, 8, ws) == L.RM_ESIZE
    assert rf(10, 8, 3, 0, ws) == L.RM_ESIZE
    assert rf(10, 8, 3, L.RM_MAX_KFETCH + 1, ws) == L.RM_ESIZE     # k above the list limit
    assert rf(10, 2, 0, 3, ws) == L.RM_ESIZE                       # k > k_fetch (2 radius + 1)
    assert lib.rm_refine(None, 1, 1, 1, 10, 8, 1, 3, 8, 1, 1, 1, ws, None) == L.RM_EINVAL
    assert lib.rm_refine(R(idx), 1, 1, 1, 10, 8, 1, 3, 8, 1, 1, None, ws, None) == L.RM_EINVAL
    assert lib.rm_refine(R(idx), None, 1, 1, 10, 8, 1, 3, 8, 1, 1, 1, ws, None) == L.RM_EINVAL
    bad = _fake_index()
    bad.n_windows += 1
    assert rf(10, 8, 3, 8, ws, bad) == L.RM_EINVAL


def test_strand_calls_validation():
    lib = L.lib()
    assert lib.rm_reverse_complement(None, 1, 10, 100, 2, None) == L.RM_EINVAL
    assert lib.rm_reverse_complement(1, None, 10, 100, 2, None) == L.RM_EINVAL
    assert lib.rm_reverse_complement(1, 1, 10, 100, None, None) == L.RM_EINVAL
    assert lib.rm_reverse_complement(1, 1, 10, 100, 1, None) == L.RM_EINVAL    # in place
    assert lib.rm_reverse_complement(1, 1, 0, 100, 2, None) == L.RM_ESIZE
    assert lib.rm_reverse_complement(1, 1, 10, 0, 2, None) == L.RM_ESIZE
    ms = lambda n, k, *p: lib.rm_merge_strands(*(p or (1,) * 4), n, k, ctypes.c_float(0.0),
                                               1, 1, 1, 1, None)
    assert ms(10, 0) == L.RM_ESIZE
    assert ms(10, L.RM_MAX_KFETCH + 1) == L.RM_ESIZE
    assert ms(0, 8) == L.RM_ESIZE
    assert ms(10, 8, 1, 1, None, 1) == L.RM_EINVAL
    assert lib.rm_merge_strands(1, 1, 1, 1, 10, 8, ctypes.c_float(0.0), 1, 1, 1, None,
                                None) == L.RM_EINVAL


def test_token_params_validation():
    """Token encodings (s-mers): accepted shapes, rejected ones, the class-table
    region of the index buffer, and the calls that take letter indexes only."""
    lib = L.lib()
    R = ctypes.byref
    letters = L.make_params(150, 1, 32, "default", "fp16")
    ok = [L.make_params(150, 1, 8, "default", "fp16", 0, 2, 16),
          L.make_params(150, 1, 2, "finetuned", "fp8", 0, 3, 64),
          L.make_params(150, 1, 8, "default", "fp16", 0, 8, 16, 0x2000)]     # s = 8, a map
    for p in ok:
        assert L.rm_num_windows(20_000, p) == 19_851
    # the phase tables shrink with m; the class table adds 4^s bytes (256-byte aligned)
    assert L.rm_index_bytes(20_000, ok[0]) < L.rm_index_bytes(20_000, letters)
    assert L.rm_index_bytes(20_000, ok[2]) - L.rm_index_bytes(20_000, ok[0]) == 4 ** 8 - 256
    assert L.rm_index_bytes(20_000, ok[1]) > 19_851 * 256
    bad = [(L.make_params(150, 1, 32, "default", "fp16", 0, 2, 16), L.RM_EUNSUPPORTED),  # C m != 128
           (L.make_params(150, 1, 8, "default", "fp16", 0, 4, 16), L.RM_EUNSUPPORTED),   # no map, C != 4^s
           (L.make_params(150, 1, 2, "default", "fp16", 0, 4, 0), L.RM_EUNSUPPORTED),    # 4^4 * 2 != 128
           (L.make_params(150, 1, 1, "default", "fp16", 0, 2, 128, 0x2000), L.RM_OK),
           (L.make_params(150, 1, 128, "default", "fp16", 0, 2, 1, 0x2000), L.RM_EUNSUPPORTED),
           (L.make_params(150, 1, 8, "default", "fp16", 0, L.RM_MAX_MER + 1, 16, 0x2000),
            L.RM_ESIZE),
           (L.make_params(150, 1, 8, "default", "fp16", 0, -1, 16), L.RM_ESIZE),
           (L.make_params(7, 1, 8, "default", "fp16", 0, 8, 16, 0x2000), L.RM_ESIZE)]    # N < s
    out = L.rm_index()
    for p, status in bad:
        if status == L.RM_OK:
            assert L.rm_index_bytes(20_000, p) > 0
            continue
        assert L.rm_index_bytes(20_000, p) == 0
        assert lib.rm_encode_reference(0x1000, 20_000, R(p), 0x10000, 1 << 30, R(out), None) == status
    # 1,024 components (K = 2,048): FP16 and FP8 indexes, 4 KB / 2 KB rows; no FP32
    w16 = L.make_params(150, 1, 4, "default", "fp16", 0, 8, 256, 0x2000)
    w8 = L.make_params(150, 1, 4, "finetuned", "fp8", 0, 4, 0)      # 4-mers, no map
    assert L.rm_read_emb_bytes(10, w16) == 10 * 2 * 2048 * 2
    assert L.rm_read_emb_bytes(10, w8) == 10 * 2 * 2048
    assert L.rm_index_bytes(20_000, w16) > 19_851 * 4096 > L.rm_index_bytes(20_000, w8) > 19_851 * 2048
    for bad_p in (L.make_params(150, 1, 4, "default", "fp32", 0, 8, 256, 0x2000),
                  L.make_params(150, 1, 128, "default", "fp16", 0, 8, 8, 0x2000)):   # 8 classes: not a multiple of 16
        assert L.rm_index_bytes(20_000, bad_p) == 0
        assert lib.rm_encode_reference(0x1000, 20_000, R(bad_p), 0x10000, 1 << 30, R(out),
                                       None) == L.RM_EUNSUPPORTED
    # counts and the frequent-s-mer map (§2.6): sizes and validation
    assert L.rm_token_counts_bytes(8) == 4 ** 8 * 4 and L.rm_token_counts_bytes(9) == 0
    assert L.rm_token_counts_bytes(0) == 0
    assert lib.rm_token_counts(None, 100, 4, 1, None) == L.RM_EINVAL
    assert lib.rm_token_counts(1, 100, 4, None, None) == L.RM_EINVAL
    assert lib.rm_token_counts(1, 3, 4, 1, None) == L.RM_ESIZE                # shorter than s
    assert lib.rm_token_counts(1, 100, L.RM_MAX_MER + 1, 1, None) == L.RM_ESIZE
    assert lib.rm_token_map_frequent(None, 4, 8, 1, None) == L.RM_EINVAL
    assert lib.rm_token_map_frequent(1, 2, 17, 1, None) == L.RM_ESIZE         # more than 4^s
    assert lib.rm_token_map_frequent(1, 8, L.RM_MAX_FREQUENT + 1, 1, None) == L.RM_ESIZE
    assert lib.rm_token_map_frequent(1, 8, 0, 1, None) == L.RM_ESIZE
    # a token index descriptor needs its class table
    idx = _fake_index()
    idx.p = ok[0]
    assert lib.rm_encode_reads(R(idx), 1, 1, 10, 1, 1, None) == L.RM_EINVAL
    idx.d_token_class = 0x100000
    # the refinement takes token indexes with the same validation (every call
    # here fails before a launch); the learned calls take letter indexes only
    ws = L.rm_refine_workspace_bytes(10, 8, 3)
    assert lib.rm_refine(R(idx), 1, 1, 1, 10, 8, 1, 3, 8, 1, 1, 1, ws - 256, None) == L.RM_ESIZE
    assert lib.rm_refine(R(idx), 1, 1, 1, 10, 8, 1, 8, 8, 1, 1, 1, ws, None) == L.RM_ESIZE
    assert lib.rm_refine(R(idx), 1, 1, None, 10, 8, 1, 3, 8, 1, 1, 1, ws, None) == L.RM_EINVAL
    assert lib.rm_encode_reads_learned(R(idx), 1, 1, 10, 1, 1, 1, None) == L.RM_EUNSUPPORTED
    assert lib.rm_rescore_learned(R(idx), 1, 1, 1, 1, 1, 10, 8, 1, 8, 1, 1, None) \
        == L.RM_EUNSUPPORTED
    assert lib.rm_encode_reference_learned(0x1000, 20_000, R(ok[0]), 0x3000, 0x10000, 1 << 30,
                                           R(out), None) == L.RM_EUNSUPPORTED


def test_threshold_and_correlation_validation():
    """Argument checks of the threshold, threshold-regime and correlation
    entry points (host side, nothing enqueued)."""
    lib = L.lib()
    R = ctypes.byref
    idx = _fake_index()
    TP = L.rm_threshold_params
    th = lambda tp: lib.rm_window_thresholds(R(idx), 1, R(tp), 1, None)
    assert th(TP(1.0, 16, 1, 0)) == L.RM_EINVAL                    # err outside [0, 1)
    assert th(TP(-0.1, 16, 1, 0)) == L.RM_EINVAL
    assert th(TP(0.1, 0, 0, 0)) == L.RM_ESIZE
    assert th(TP(0.1, L.RM_THRESH_MAX_COPIES + 1, 0, 0)) == L.RM_ESIZE
    assert th(TP(0.1, 16, 16, 0)) == L.RM_ESIZE                    # rank >= copies
    assert lib.rm_window_thresholds(R(idx), None, R(TP(0.1, 16, 1, 0)), 1, None) == L.RM_EINVAL
    tok = _fake_index()
    tok.p.mer_len, tok.p.n_freq, tok.p.n_class, tok.d_token_class = 2, 8, 16, 0x100000
    assert lib.rm_window_thresholds(R(tok), 1, R(TP(0.1, 16, 1, 0)), 1, None) == L.RM_EUNSUPPORTED
    assert L.rm_threshold_workspace_bytes(0, 100) == 0
    assert L.rm_threshold_workspace_bytes(10, 0) == 0
    ws = L.rm_threshold_workspace_bytes(100, 1000)
    assert ws >= 1000 * 20 + 100 * 8
    st = lambda floor, cap, nb, n=100, i=idx, scale=1: lib.rm_score_threshold(
        R(i), 1, 1, scale, 1, 1, n, 1, floor, cap, 1, 1, 1, 1, 1, 1, nb, None)
    assert st(0.0, 1000, ws - 1) == L.RM_ESIZE
    assert st(0.0, 0, ws) == L.RM_ESIZE
    assert st(0.0, 1000, ws, n=0) == L.RM_ESIZE
    assert st(1.5, 1000, ws) == L.RM_EINVAL
    assert st(0.0, 1000, ws, i=_fake_index("fp8"), scale=None) == L.RM_EINVAL
    assert st(0.0, 1000, ws, i=tok) == L.RM_EUNSUPPORTED
    cs = lambda n, per: lib.rm_correlation_score(1, 1, n, per, 1, 1, None)
    assert cs(0, 10) == L.RM_ESIZE and cs(L.RM_CORR_MAX_RATES + 1, 10) == L.RM_ESIZE
    assert cs(5, 0) == L.RM_ESIZE
    assert lib.rm_correlation_score(None, 1, 5, 10, 1, 1, None) == L.RM_EINVAL


def test_noalloc_validation():
    """The entry point that allocates nothing validates like rm_score_topk and
    rejects workspaces above its scratch before touching the device."""
    lib = L.lib()
    R = ctypes.byref
    idx = _fake_index()
    assert lib.rm_score_topk_noalloc(None, 1, 1, 10, 8, 1, 1, None) == L.RM_EINVAL
    assert lib.rm_score_topk_noalloc(R(idx), None, 1, 10, 8, 1, 1, None) == L.RM_EINVAL
    assert lib.rm_score_topk_noalloc(R(idx), 1, 1, 0, 8, 1, 1, None) == L.RM_ESIZE
    assert lib.rm_score_topk_noalloc(R(idx), 1, 1, 10, L.RM_MAX_KFETCH + 1, 1, 1, None) == L.RM_ESIZE
    big = 4_000_000
    assert L.rm_score_workspace_bytes(idx, big, 32) > L.RM_NOALLOC_SCRATCH_BYTES
    assert lib.rm_score_topk_noalloc(R(idx), 1, 1, big, 32, 1, 1, None) == L.RM_ESIZE


def test_letter_sum_form_params():
    """The letter-sum form (rm_params.reduced): 192 reals per row for letter
    indexes with integer factors and N > m, in every precision; refused
    elsewhere."""
    lib = L.lib()
    R = ctypes.byref
    out = L.rm_index()
    for prec, esize in (("fp16", 2), ("fp8", 1)):
        full = L.make_params(150, 1, 32, "default", prec)
        red = L.make_params(150, 1, 32, "default", prec, reduced=True)
        assert L.rm_read_emb_bytes(10, red) == 10 * 2 * 192 * esize
        assert L.rm_read_emb_bytes(10, full) == 10 * 2 * 256 * esize
        # rows shrink by a quarter; the rest of the buffer is the same
        assert L.rm_index_bytes(20_000, full) - L.rm_index_bytes(20_000, red) >= \
            19_851 * 64 * esize - 256
    fp32 = L.make_params(150, 1, 32, "default", "fp32", reduced=True)
    assert L.rm_read_emb_bytes(10, fp32) == 10 * 2 * 192 * 4
    bad = [L.make_params(150, 1, 32, "finetuned", "fp16", reduced=True),        # non-integer factors
           L.make_params(32, 1, 32, "default", "fp16", reduced=True),           # N = m: f_m = N
           L.make_params(150, 1, 8, "default", "fp16", 0, 2, 16, reduced=True)]  # tokens
    for p in bad:
        assert L.rm_index_bytes(20_000, p) == 0
        assert lib.rm_encode_reference(0x1000, 20_000, R(p), 0x10000, 1 << 30, R(out), None) \
            == L.RM_EUNSUPPORTED
    p = L.make_params(150, 1, 32, "default", "fp16")
    p.reduced = 2
    assert lib.rm_encode_reference(0x1000, 20_000, R(p), 0x10000, 1 << 30, R(out), None) \
        == L.RM_EINVAL
    # the learned encoding has no letter-sum form
    red = L.make_params(150, 1, 32, "default", "fp16", reduced=True)
    assert lib.rm_encode_reference_learned(0x1000, 20_000, R(red), 0x3000, 0x10000, 1 << 30,
                                           R(out), None) == L.RM_EUNSUPPORTED
