"""ctypes binding of librotormap.so -- argument marshalling only.

Each function has the name of the C entry point it calls and takes device
buffers as torch tensors (or raw integer addresses).  Nothing here computes any
part of the method; if the library is not built the first call raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librotormap.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rotormap.h")

RM_OK, RM_EINVAL, RM_ESIZE, RM_EUNSUPPORTED, RM_EHIP = 0, -1, -2, -3, -4
RM_FP32, RM_FP16, RM_FP8_E4M3 = 0, 1, 2
RM_SCHED_DEFAULT, RM_SCHED_FINETUNED = 0, 1
RM_DIM, RM_MAX_WINDOW, RM_MAX_KFETCH, RM_WIDE_MAX_KFETCH = 32, 16384, 64, 32
RM_NOALLOC_SCRATCH_BYTES = 256 << 20
RM_MAX_MER, RM_TOKEN_SKIP, RM_MAX_FREQUENT = 8, 255, 128
PRECISIONS = {"fp32": RM_FP32, "fp16": RM_FP16, "fp8": RM_FP8_E4M3}
SCHEDULES = {"default": RM_SCHED_DEFAULT, "finetuned": RM_SCHED_FINETUNED}


class rm_params(ctypes.Structure):
    _fields_ = [("window_len", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("n_freq", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reanchor", ctypes.c_int32),
                ("mer_len", ctypes.c_int32), ("n_class", ctypes.c_int32),
                ("d_token_map", ctypes.c_void_p), ("reduced", ctypes.c_int32)]


class rm_index(ctypes.Structure):
    _fields_ = [("p", rm_params), ("ref_len", ctypes.c_int64), ("n_windows", ctypes.c_int64),
                ("d_emb", ctypes.c_void_p), ("d_scale", ctypes.c_void_p),
                ("d_norm2", ctypes.c_void_p), ("d_phase64", ctypes.c_void_p),
                ("d_phase32", ctypes.c_void_p), ("d_step32", ctypes.c_void_p),
                ("d_token_class", ctypes.c_void_p)]


class rm_threshold_params(ctypes.Structure):
    _fields_ = [("err", ctypes.c_float), ("copies", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("seed", ctypes.c_uint32)]


class rm_tuning(ctypes.Structure):
    _fields_ = [("read_tile", ctypes.c_int32), ("chunk_tiles", ctypes.c_int32)]


RM_MAX_GROUPS = 8
RM_LEARNED_PARAMS = 10432
RM_LEARNED_MAX_LEN = 256
RM_LEARNED_MAX_PAIRS = 1024
RM_REFINE_MAX_RADIUS = 31
RM_CORR_MAX_RATES = 256
RM_THRESH_MAX_COPIES = 64


class RotorMapError(RuntimeError):
    def __init__(self, status: int, call: str):
        self.status = status
        super().__init__(f"{call} failed: {status} ({status_str(status)})")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"librotormap.so is not built ({LIB_PATH}); run "
                               "__graft_entry__.build() or python paper_2603_22245_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        PP, IP = ctypes.POINTER(rm_params), ctypes.POINTER(rm_index)
        sig = {
            "rm_status_str": (ctypes.c_char_p, [ctypes.c_int]),
            "rm_version": (ctypes.c_char_p, []),
            "rm_num_windows": (I64, [I64, PP]),
            "rm_index_bytes": (SZ, [I64, PP]),
            "rm_encode_reference": (ctypes.c_int, [P, I64, PP, P, SZ, IP, P]),
            "rm_read_emb_bytes": (SZ, [I32, PP]),
            "rm_encode_reads": (ctypes.c_int, [IP, P, P, I32, P, P, P]),
            "rm_score_workspace_bytes": (SZ, [IP, I32, I32]),
            "rm_score_topk": (ctypes.c_int, [IP, P, P, I32, I32, P, P, P, SZ, P]),
            "rm_rescore": (ctypes.c_int, [IP, P, P, P, I32, I32, P, I32, P, P, P]),
            "rm_score_topk_noalloc": (ctypes.c_int, [IP, P, P, I32, I32, P, P, P]),
            "rm_refine_workspace_bytes": (SZ, [I32, I32, I32]),
            "rm_reverse_complement": (ctypes.c_int, [P, P, I32, I64, P, P]),
            "rm_token_counts_bytes": (ctypes.c_size_t, [I32]),
            "rm_token_counts": (ctypes.c_int, [P, I64, I32, P, P]),
            "rm_token_map_frequent": (ctypes.c_int, [P, I32, I32, P, P]),
            "rm_merge_strands": (ctypes.c_int, [P, P, P, P, I32, I32, ctypes.c_float, P, P, P, P,
                                                P]),
            "rm_refine": (ctypes.c_int, [IP, P, P, P, I32, I32, P, I32, I32, P, P, P, SZ, P]),
            "rm_bucket_reads": (ctypes.c_int, [P, I32, P, I32, P, P]),
            "rm_score_groups_workspace_bytes": (SZ, [IP, I32, P, I32, ctypes.POINTER(rm_tuning)]),
            "rm_score_topk_groups": (ctypes.c_int, [IP, I32, P, P, P, I32, P, P, P, SZ,
                                                    ctypes.POINTER(rm_tuning), P]),
            "rm_autotune_score": (ctypes.c_int, [IP, I32, P, P, P, I32, P, P, P, SZ,
                                                 ctypes.c_char_p, ctypes.POINTER(rm_tuning),
                                                 ctypes.POINTER(ctypes.c_float), P]),
            "rm_capture_begin": (ctypes.c_int, [P]),
            "rm_capture_end": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_void_p)]),
            "rm_graph_launch": (ctypes.c_int, [P, P]),
            "rm_graph_destroy": (ctypes.c_int, [P]),
            "rm_learned_workspace_bytes": (SZ, [I32]),
            "rm_learned_encode": (ctypes.c_int, [P, P, P, I32, I32, P, P]),
            "rm_pair_fidelity": (ctypes.c_int, [P, P, I32, P, P]),
            "rm_learned_train_step": (ctypes.c_int, [P, ctypes.c_float, P, P, P, P, P, I32, I32,
                                                     P, SZ, P, P]),
            "rm_learned_gradient": (ctypes.c_int, [P, P, P, P, P, P, I32, I32, P, SZ, P, P, P]),
            "rm_levenshtein": (ctypes.c_int, [P, P, P, P, I64, P, P]),
            "rm_correlation_score": (ctypes.c_int, [P, P, I32, I32, P, P, P]),
            "rm_window_thresholds": (ctypes.c_int, [IP, P, ctypes.POINTER(rm_threshold_params),
                                                    P, P]),
            "rm_threshold_workspace_bytes": (SZ, [I32, I64]),
            "rm_score_threshold": (ctypes.c_int, [IP, P, P, P, P, P, I32, P, ctypes.c_float, I64,
                                                  P, P, P, P, P, P, SZ, P]),
            "rm_delta_bytes": (SZ, [I64]),
            "rm_mlp_infer": (ctypes.c_int, [P, P, I64, P, P]),
            "rm_encode_reference_learned": (ctypes.c_int, [P, I64, PP, P, P, SZ, IP, P]),
            "rm_encode_reads_learned": (ctypes.c_int, [IP, P, P, I32, P, P, P, P]),
            "rm_rescore_learned": (ctypes.c_int, [IP, P, P, P, P, P, I32, I32, P, I32, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions include/rotormap.h declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rm_[a-z0-9_]+)\s*\(", text)))


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status: int, call: str):
    if status != RM_OK:
        raise RotorMapError(status, call)


def make_params(window_len=150, stride=1, n_freq=RM_DIM, schedule="default", precision="fp16",
                reanchor=0, mer_len=0, n_class=0, token_map=None, reduced=False) -> rm_params:
    """token_map: None or a device uint8 tensor of 4^mer_len classes (its
    address is stored; it must stay alive until rm_encode_reference returns).
    reduced: store the letter-sum form (rm_params.reduced)."""
    return rm_params(window_len, stride, n_freq,
                     SCHEDULES.get(schedule, schedule) if isinstance(schedule, str) else schedule,
                     PRECISIONS.get(precision, precision) if isinstance(precision, str) else precision,
                     reanchor, mer_len, n_class, None if token_map is None else _ptr(token_map),
                     int(bool(reduced)))


def status_str(status: int) -> str:
    return lib().rm_status_str(status).decode()


def rm_version() -> str:
    return lib().rm_version().decode()


def rm_num_windows(ref_len: int, p: rm_params) -> int:
    return int(lib().rm_num_windows(ref_len, ctypes.byref(p)))


def rm_index_bytes(ref_len: int, p: rm_params) -> int:
    return int(lib().rm_index_bytes(ref_len, ctypes.byref(p)))


def rm_encode_reference(d_ref, ref_len: int, p: rm_params, d_buf, buf_bytes: int,
                        stream=None) -> rm_index:
    out = rm_index()
    _check(lib().rm_encode_reference(_ptr(d_ref), ref_len, ctypes.byref(p), _ptr(d_buf), buf_bytes,
                                     ctypes.byref(out), _stream(stream)), "rm_encode_reference")
    return out


def rm_read_emb_bytes(n_reads: int, p: rm_params) -> int:
    return int(lib().rm_read_emb_bytes(n_reads, ctypes.byref(p)))


def rm_encode_reads(idx: rm_index, d_seq, d_off, n_reads: int, d_read_emb, d_read_scale=None,
                    stream=None) -> None:
    _check(lib().rm_encode_reads(ctypes.byref(idx), _ptr(d_seq), _ptr(d_off), n_reads,
                                 _ptr(d_read_emb), _ptr(d_read_scale), _stream(stream)),
           "rm_encode_reads")


def rm_score_workspace_bytes(idx: rm_index, n_reads: int, k_fetch: int) -> int:
    return int(lib().rm_score_workspace_bytes(ctypes.byref(idx), n_reads, k_fetch))


def rm_score_topk(idx: rm_index, d_read_emb, d_read_scale, n_reads: int, k_fetch: int,
                  d_cand_idx, d_cand_score, d_ws, ws_bytes: int, stream=None) -> None:
    _check(lib().rm_score_topk(ctypes.byref(idx), _ptr(d_read_emb), _ptr(d_read_scale), n_reads,
                               k_fetch, _ptr(d_cand_idx), _ptr(d_cand_score), _ptr(d_ws), ws_bytes,
                               _stream(stream)), "rm_score_topk")


def rm_score_topk_noalloc(idx: rm_index, d_read_emb, d_read_scale, n_reads: int, k_fetch: int,
                          d_cand_idx, d_cand_score, stream=None) -> None:
    _check(lib().rm_score_topk_noalloc(ctypes.byref(idx), _ptr(d_read_emb), _ptr(d_read_scale),
                                       n_reads, k_fetch, _ptr(d_cand_idx), _ptr(d_cand_score),
                                       _stream(stream)), "rm_score_topk_noalloc")


def rm_rescore(idx: rm_index, d_ref, d_seq, d_off, n_reads: int, k_fetch: int, d_cand_idx, k: int,
               d_top_idx, d_top_score, stream=None) -> None:
    _check(lib().rm_rescore(ctypes.byref(idx), _ptr(d_ref), _ptr(d_seq), _ptr(d_off), n_reads,
                            k_fetch, _ptr(d_cand_idx), k, _ptr(d_top_idx), _ptr(d_top_score),
                            _stream(stream)), "rm_rescore")


def rm_token_counts_bytes(mer_len: int) -> int:
    return int(lib().rm_token_counts_bytes(mer_len))


def rm_token_counts(d_ref, ref_len: int, mer_len: int, d_counts, stream=None) -> None:
    _check(lib().rm_token_counts(_ptr(d_ref), ref_len, mer_len, _ptr(d_counts), _stream(stream)),
           "rm_token_counts")


def rm_token_map_frequent(d_counts, mer_len: int, n_class: int, d_map, stream=None) -> None:
    _check(lib().rm_token_map_frequent(_ptr(d_counts), mer_len, n_class, _ptr(d_map),
                                       _stream(stream)), "rm_token_map_frequent")


def rm_reverse_complement(d_seq, d_off, n_reads: int, n_letters: int, d_out, stream=None) -> None:
    _check(lib().rm_reverse_complement(_ptr(d_seq), _ptr(d_off), n_reads, n_letters, _ptr(d_out),
                                       _stream(stream)), "rm_reverse_complement")


def rm_merge_strands(d_fwd_idx, d_fwd_score, d_rev_idx, d_rev_score, n_reads: int, k: int,
                     min_fidelity: float, d_top_idx, d_top_score, d_top_strand, d_n_found,
                     stream=None) -> None:
    _check(lib().rm_merge_strands(_ptr(d_fwd_idx), _ptr(d_fwd_score), _ptr(d_rev_idx),
                                  _ptr(d_rev_score), n_reads, k, min_fidelity, _ptr(d_top_idx),
                                  _ptr(d_top_score), _ptr(d_top_strand), _ptr(d_n_found),
                                  _stream(stream)), "rm_merge_strands")


def rm_refine_workspace_bytes(n_reads: int, k_fetch: int, radius: int) -> int:
    return lib().rm_refine_workspace_bytes(n_reads, k_fetch, radius)


def rm_refine(coarse: rm_index, d_ref, d_seq, d_off, n_reads: int, k_fetch: int, d_cand_idx,
              radius: int, k: int, d_top_idx, d_top_score, d_ws, ws_bytes: int,
              stream=None) -> None:
    _check(lib().rm_refine(ctypes.byref(coarse), _ptr(d_ref), _ptr(d_seq), _ptr(d_off), n_reads,
                           k_fetch, _ptr(d_cand_idx), radius, k, _ptr(d_top_idx),
                           _ptr(d_top_score), _ptr(d_ws), ws_bytes, _stream(stream)), "rm_refine")


# ---------------------------------------------------------------- batching

def rm_bucket_reads(offsets, bucket_len):
    """Host helper: bucket index per read (-1 if shorter than the first bucket) and
    per-bucket counts."""
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    bl = np.ascontiguousarray(bucket_len, dtype=np.int32)
    n = off.shape[0] - 1
    bucket = np.empty(n, dtype=np.int32)
    count = np.empty(bl.shape[0], dtype=np.int32)
    _check(lib().rm_bucket_reads(off.ctypes.data, n, bl.ctypes.data, bl.shape[0],
                                 bucket.ctypes.data, count.ctypes.data), "rm_bucket_reads")
    return bucket, count


def _groups(idxs, n_reads):
    n = len(idxs)
    arr = (rm_index * n)(*idxs)
    nr = (ctypes.c_int32 * n)(*[int(v) for v in n_reads])
    return n, arr, nr


def _ptrs(xs):
    return (ctypes.c_void_p * len(xs))(*[_ptr(x) for x in xs])


def rm_score_groups_workspace_bytes(idxs, n_reads, k_fetch, tune=None) -> int:
    n, arr, nr = _groups(idxs, n_reads)
    return int(lib().rm_score_groups_workspace_bytes(arr, n, nr, k_fetch,
                                                     ctypes.byref(tune) if tune else None))


def rm_score_topk_groups(idxs, d_read_emb, d_read_scale, n_reads, k_fetch, d_cand_idx,
                         d_cand_score, d_ws, ws_bytes, tune=None, stream=None) -> None:
    n, arr, nr = _groups(idxs, n_reads)
    scales = _ptrs(d_read_scale) if d_read_scale is not None else None
    _check(lib().rm_score_topk_groups(arr, n, _ptrs(d_read_emb), scales, nr, k_fetch,
                                      _ptrs(d_cand_idx), _ptrs(d_cand_score), _ptr(d_ws),
                                      ws_bytes, ctypes.byref(tune) if tune else None,
                                      _stream(stream)), "rm_score_topk_groups")


def rm_autotune_score(idxs, d_read_emb, d_read_scale, n_reads, k_fetch, d_cand_idx, d_cand_score,
                      d_ws, ws_bytes, cache_path=None, stream=None):
    n, arr, nr = _groups(idxs, n_reads)
    scales = _ptrs(d_read_scale) if d_read_scale is not None else None
    best = rm_tuning()
    ms = ctypes.c_float(0.0)
    _check(lib().rm_autotune_score(arr, n, _ptrs(d_read_emb), scales, nr, k_fetch,
                                   _ptrs(d_cand_idx), _ptrs(d_cand_score), _ptr(d_ws), ws_bytes,
                                   cache_path.encode() if cache_path else None,
                                   ctypes.byref(best), ctypes.byref(ms), _stream(stream)),
           "rm_autotune_score")
    return best, float(ms.value)


def rm_capture_begin(stream) -> None:
    _check(lib().rm_capture_begin(_stream(stream)), "rm_capture_begin")


def rm_capture_end(stream) -> int:
    g = ctypes.c_void_p()
    _check(lib().rm_capture_end(_stream(stream), ctypes.byref(g)), "rm_capture_end")
    return int(g.value)


def rm_graph_launch(graph: int, stream=None) -> None:
    _check(lib().rm_graph_launch(graph, _stream(stream)), "rm_graph_launch")


def rm_graph_destroy(graph: int) -> None:
    _check(lib().rm_graph_destroy(graph), "rm_graph_destroy")


def rm_learned_workspace_bytes(n_pairs: int) -> int:
    return int(lib().rm_learned_workspace_bytes(n_pairs))


def rm_learned_encode(d_params, d_seq, d_off, n_strings: int, nominal_len: int, d_c,
                      stream=None) -> None:
    _check(lib().rm_learned_encode(_ptr(d_params), _ptr(d_seq), _ptr(d_off), n_strings,
                                   nominal_len, _ptr(d_c), _stream(stream)), "rm_learned_encode")


def rm_pair_fidelity(d_ca, d_cb, n_pairs: int, d_F, stream=None) -> None:
    _check(lib().rm_pair_fidelity(_ptr(d_ca), _ptr(d_cb), n_pairs, _ptr(d_F), _stream(stream)),
           "rm_pair_fidelity")


def rm_learned_train_step(d_state, lr: float, d_a, d_aoff, d_b, d_boff, d_ld, n_pairs: int,
                          nominal_len: int, d_ws, ws_bytes: int, d_loss, stream=None) -> None:
    _check(lib().rm_learned_train_step(_ptr(d_state), lr, _ptr(d_a), _ptr(d_aoff), _ptr(d_b),
                                       _ptr(d_boff), _ptr(d_ld), n_pairs, nominal_len, _ptr(d_ws),
                                       ws_bytes, _ptr(d_loss), _stream(stream)),
           "rm_learned_train_step")


def rm_learned_gradient(d_params, d_a, d_aoff, d_b, d_boff, d_ld, n_pairs: int, nominal_len: int,
                        d_ws, ws_bytes: int, d_grad, d_loss, stream=None) -> None:
    _check(lib().rm_learned_gradient(_ptr(d_params), _ptr(d_a), _ptr(d_aoff), _ptr(d_b),
                                     _ptr(d_boff), _ptr(d_ld), n_pairs, nominal_len, _ptr(d_ws),
                                     ws_bytes, _ptr(d_grad), _ptr(d_loss), _stream(stream)),
           "rm_learned_gradient")


def rm_levenshtein(d_a, d_aoff, d_b, d_boff, n: int, d_out, stream=None) -> None:
    _check(lib().rm_levenshtein(_ptr(d_a), _ptr(d_aoff), _ptr(d_b), _ptr(d_boff), n, _ptr(d_out),
                                _stream(stream)), "rm_levenshtein")


def rm_delta_bytes(n_letters: int) -> int:
    return int(lib().rm_delta_bytes(n_letters))


def rm_mlp_infer(d_params, d_seq, n_letters: int, d_delta, stream=None) -> None:
    _check(lib().rm_mlp_infer(_ptr(d_params), _ptr(d_seq), n_letters, _ptr(d_delta),
                              _stream(stream)), "rm_mlp_infer")


def rm_encode_reference_learned(d_ref, ref_len: int, p: rm_params, d_ref_delta, d_buf,
                                buf_bytes: int, stream=None) -> rm_index:
    out = rm_index()
    _check(lib().rm_encode_reference_learned(_ptr(d_ref), ref_len, ctypes.byref(p),
                                             _ptr(d_ref_delta), _ptr(d_buf), buf_bytes,
                                             ctypes.byref(out), _stream(stream)),
           "rm_encode_reference_learned")
    return out


def rm_encode_reads_learned(idx: rm_index, d_seq, d_off, n_reads: int, d_read_delta, d_read_emb,
                            d_read_scale=None, stream=None) -> None:
    _check(lib().rm_encode_reads_learned(ctypes.byref(idx), _ptr(d_seq), _ptr(d_off), n_reads,
                                         _ptr(d_read_delta), _ptr(d_read_emb), _ptr(d_read_scale),
                                         _stream(stream)), "rm_encode_reads_learned")


def rm_rescore_learned(idx: rm_index, d_ref, d_ref_delta, d_seq, d_off, d_read_delta, n_reads: int,
                       k_fetch: int, d_cand_idx, k: int, d_top_idx, d_top_score,
                       stream=None) -> None:
    _check(lib().rm_rescore_learned(ctypes.byref(idx), _ptr(d_ref), _ptr(d_ref_delta), _ptr(d_seq),
                                    _ptr(d_off), _ptr(d_read_delta), n_reads, k_fetch,
                                    _ptr(d_cand_idx), k, _ptr(d_top_idx), _ptr(d_top_score),
                                    _stream(stream)), "rm_rescore_learned")


def rm_correlation_score(d_F, d_err, n_rates: int, per_rate: int, d_E, d_rmse,
                         stream=None) -> None:
    _check(lib().rm_correlation_score(_ptr(d_F), _ptr(d_err), n_rates, per_rate, _ptr(d_E),
                                      _ptr(d_rmse), _stream(stream)), "rm_correlation_score")


def rm_window_thresholds(idx: rm_index, d_ref, err: float, copies: int, rank: int, seed: int,
                         d_thr, stream=None) -> None:
    tp = rm_threshold_params(err, copies, rank, seed)
    _check(lib().rm_window_thresholds(ctypes.byref(idx), _ptr(d_ref), ctypes.byref(tp),
                                      _ptr(d_thr), _stream(stream)), "rm_window_thresholds")


def rm_threshold_workspace_bytes(n_reads: int, capacity: int) -> int:
    return int(lib().rm_threshold_workspace_bytes(n_reads, capacity))


def rm_score_threshold(idx: rm_index, d_ref, d_read_emb, d_read_scale, d_seq, d_off, n_reads: int,
                       d_thr, floor_fidelity: float, capacity: int, d_hit_off, d_n_found,
                       d_hit_idx, d_hit_score, d_total, d_ws, ws_bytes: int, stream=None) -> None:
    _check(lib().rm_score_threshold(ctypes.byref(idx), _ptr(d_ref), _ptr(d_read_emb),
                                    _ptr(d_read_scale), _ptr(d_seq), _ptr(d_off), n_reads,
                                    _ptr(d_thr), floor_fidelity, capacity, _ptr(d_hit_off),
                                    _ptr(d_n_found), _ptr(d_hit_idx), _ptr(d_hit_score),
                                    _ptr(d_total), _ptr(d_ws), ws_bytes, _stream(stream)),
           "rm_score_threshold")
