// Host side of the C ABI: argument validation (always before anything is
// enqueued), the layout of the caller's index buffer, and kernel launches.
#include <hip/hip_runtime.h>

#include <new>

#include <mutex>

#include "rm_internal.h"
#include "rm_tokens.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// The letter encoding: single letters, no map, 4 classes (the zero-initialised
// token fields).  Anything else is a token encoding.
bool letter_encoding(const rm_params* p) {
  return p->mer_len <= 1 && p->d_token_map == nullptr && (p->n_class == 0 || p->n_class == 4);
}

int mer_of(const rm_params* p) { return p->mer_len > 1 ? p->mer_len : 1; }

// Components per factor: n_class, or 4^s (0 when 4^s exceeds 256).
int classes_of(const rm_params* p) {
  const int s = mer_of(p);
  return p->n_class != 0 ? p->n_class : (s <= 4 ? 1 << (2 * s) : 0);
}

// A token encoding of 1,024 complex components (FP16 or FP8, own kernels).
bool wide_encoding(const rm_params* p) {
  return !letter_encoding(p) && (int64_t)p->n_freq * classes_of(p) == rm::kWideComplex;
}

// Reals per stored row (and per read-embedding row).
size_t real_dim(const rm_params* p) {
  return wide_encoding(p) ? 2 * rm::kWideComplex : p->reduced ? rm::kRealReduced : rm::kReal;
}

bool params_ok(const rm_params* p, int* why) {
  if (p == nullptr) return (*why = RM_EINVAL), false;
  if (p->mer_len < 0 || p->mer_len > RM_MAX_MER) return (*why = RM_ESIZE), false;
  if (letter_encoding(p)) {
    if (p->n_freq != RM_DIM) return (*why = RM_EUNSUPPORTED), false;
  } else {
    const int s = mer_of(p);
    const int C = classes_of(p);
    if (C < 2 || C % 2 != 0 || C > 256 || p->n_freq < 1) return (*why = RM_EUNSUPPORTED), false;
    if (C * p->n_freq == rm::kWideComplex) {
      if (C % 16 != 0 || p->precision == RM_FP32) return (*why = RM_EUNSUPPORTED), false;
    } else if (C * p->n_freq != rm::kComplex) {
      return (*why = RM_EUNSUPPORTED), false;
    }
    if (p->d_token_map == nullptr && C != (1 << (2 * s))) return (*why = RM_EUNSUPPORTED), false;
    if (p->window_len < s) return (*why = RM_ESIZE), false;
  }
  if (p->schedule != RM_SCHED_DEFAULT && p->schedule != RM_SCHED_FINETUNED)
    return (*why = RM_EINVAL), false;
  if (p->precision != RM_FP32 && p->precision != RM_FP16 && p->precision != RM_FP8_E4M3)
    return (*why = RM_EINVAL), false;
  if (p->window_len < 1 || p->window_len > RM_MAX_WINDOW) return (*why = RM_ESIZE), false;
  if (p->stride < 1) return (*why = RM_ESIZE), false;
  if (p->reanchor < 0) return (*why = RM_ESIZE), false;
  if (p->reduced != 0 && p->reduced != 1) return (*why = RM_EINVAL), false;
  // the letter-sum form: integer factors (f_k = k < N for every window of at
  // least RM_DIM + 1 letters), letters
  if (p->reduced && (!letter_encoding(p) || p->schedule != RM_SCHED_DEFAULT ||
                     p->window_len <= RM_DIM))
    return (*why = RM_EUNSUPPORTED), false;
  return true;
}

int64_t windows_of(int64_t ref_len, const rm_params* p) {
  if (ref_len < p->window_len) return -1;
  return (ref_len - p->window_len) / p->stride + 1;
}

struct Layout {
  size_t emb, scale, norm2, phase64, phase32, step32, token_class, total;
};

Layout layout(int64_t W, const rm_params* p) {
  Layout L{};
  size_t off = 0;
  L.emb = off;
  off = align_up(off + (size_t)W * real_dim(p) * rm::elem_bytes(p->precision));
  L.scale = off;  // [W] scales and, at [W], the FP8 windows' scale bound
  off = align_up(off + (size_t)(W + 1) * sizeof(float));
  L.norm2 = off;
  off = align_up(off + (size_t)W * sizeof(float));
  L.phase64 = off;
  off = align_up(off + (size_t)p->window_len * p->n_freq * 2 * sizeof(double));
  L.phase32 = off;
  off = align_up(off + (size_t)p->window_len * p->n_freq * 2 * sizeof(float));
  L.step32 = off;
  off = align_up(off + (size_t)p->n_freq * 4 * sizeof(float));
  L.token_class = off;
  if (!letter_encoding(p)) off = align_up(off + ((size_t)1 << (2 * mer_of(p))));
  L.total = off;
  return L;
}

int index_ok(const rm_index* idx) {
  if (idx == nullptr) return RM_EINVAL;
  int why = RM_OK;
  if (!params_ok(&idx->p, &why)) return why;
  int64_t W = windows_of(idx->ref_len, &idx->p);
  if (W < 1 || W != idx->n_windows) return RM_EINVAL;
  if (!idx->d_emb || !idx->d_scale || !idx->d_norm2 || !idx->d_phase64 || !idx->d_phase32 ||
      !idx->d_step32)
    return RM_EINVAL;
  if (!letter_encoding(&idx->p) && !idx->d_token_class) return RM_EINVAL;
  return RM_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? RM_OK : RM_EHIP; }

// Workspace of rm_score_topk_noalloc: a device array of the library, one copy
// per GPU, held until the process ends.  In host code `scratch` names a host
// stand-in, not device memory; its device address is looked up once per
// device (with that device current) and only that address is used.
constexpr size_t kNoallocAlign = 256;
__device__ __align__(256) static uint8_t scratch[RM_NOALLOC_SCRATCH_BYTES];
constexpr int kNoallocDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoallocDevices] = {};

// The current device's copy of `scratch`.
int noalloc_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RM_EHIP;
  if (dev < 0 || dev >= kNoallocDevices) return RM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return RM_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RM_OK;
}

}  // namespace

extern "C" {

const char* rm_status_str(int status) {
  switch (status) {
    case RM_OK: return "ok";
    case RM_EINVAL: return "invalid argument";
    case RM_ESIZE: return "size out of range or buffer too small";
    case RM_EUNSUPPORTED: return "unsupported parameters";
    case RM_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* rm_version(void) { return "rotormap-gfx950 0.1"; }

int64_t rm_num_windows(int64_t ref_len, const rm_params* p) {
  int why = RM_OK;
  if (!params_ok(p, &why)) return -1;
  return windows_of(ref_len, p);
}

size_t rm_index_bytes(int64_t ref_len, const rm_params* p) {
  int why = RM_OK;
  if (!params_ok(p, &why)) return 0;
  int64_t W = windows_of(ref_len, p);
  if (W < 1 || W > INT32_MAX) return 0;
  return layout(W, p).total;
}

static int encode_reference_impl(const uint8_t* d_ref, int64_t ref_len, const rm_params* p,
                                 const float* d_delta, void* d_buf, size_t buf_bytes,
                                 rm_index* out, void* stream);

int rm_encode_reference(const uint8_t* d_ref, int64_t ref_len, const rm_params* p, void* d_buf,
                        size_t buf_bytes, rm_index* out, void* stream) {
  return encode_reference_impl(d_ref, ref_len, p, nullptr, d_buf, buf_bytes, out, stream);
}

int rm_encode_reference_learned(const uint8_t* d_ref, int64_t ref_len, const rm_params* p,
                                const float* d_ref_delta, void* d_buf, size_t buf_bytes,
                                rm_index* out, void* stream) {
  if (d_ref_delta == nullptr) return RM_EINVAL;
  if (p != nullptr && p->window_len < 9) return RM_ESIZE;
  if (p != nullptr && (!letter_encoding(p) || p->reduced)) return RM_EUNSUPPORTED;
  return encode_reference_impl(d_ref, ref_len, p, d_ref_delta, d_buf, buf_bytes, out, stream);
}

static int encode_reference_impl(const uint8_t* d_ref, int64_t ref_len, const rm_params* p,
                                 const float* d_delta, void* d_buf, size_t buf_bytes,
                                 rm_index* out, void* stream) {
  int why = RM_OK;
  if (!params_ok(p, &why)) return why;
  if (d_ref == nullptr || d_buf == nullptr || out == nullptr) return RM_EINVAL;
  if (reinterpret_cast<uintptr_t>(d_buf) % kAlign != 0) return RM_EINVAL;
  int64_t W = windows_of(ref_len, p);
  if (W < 1 || W > INT32_MAX) return RM_ESIZE;
  Layout L = layout(W, p);
  if (buf_bytes < L.total) return RM_ESIZE;

  uint8_t* base = static_cast<uint8_t*>(d_buf);
  rm_index idx{};
  idx.p = *p;
  idx.ref_len = ref_len;
  idx.n_windows = W;
  idx.d_emb = base + L.emb;
  idx.d_scale = reinterpret_cast<float*>(base + L.scale);
  idx.d_norm2 = reinterpret_cast<float*>(base + L.norm2);
  idx.d_phase64 = reinterpret_cast<double*>(base + L.phase64);
  idx.d_phase32 = reinterpret_cast<float*>(base + L.phase32);
  idx.d_step32 = reinterpret_cast<float*>(base + L.step32);
  idx.d_token_class = letter_encoding(p) ? nullptr : base + L.token_class;

  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = hip_status(rm::launch_tables(*p, idx.d_phase64, idx.d_phase32, idx.d_step32, s));
  if (st == RM_OK)  // the encoders raise d_scale[W] to their windows' largest FP8 scale bound
    st = hip_status(rm::launch_zero_word(reinterpret_cast<uint32_t*>(idx.d_scale + W), s));
  if (st != RM_OK) return st;
  if (idx.d_token_class != nullptr) {
    const bool wide = wide_encoding(p);
    const int C = (wide ? rm::kWideComplex : rm::kComplex) / p->n_freq;
    st = hip_status(rm::launch_token_table(p->d_token_map, mer_of(p), C, idx.d_token_class, s));
    if (st == RM_OK && wide)
      st = hip_status(rm::launch_encode_reference_wide(d_ref, W, *p, idx.d_phase64, idx.d_step32,
                                                       idx.d_token_class, idx.d_emb, idx.d_scale,
                                                       idx.d_norm2, s));
    else if (st == RM_OK)
      st = hip_status(rm::launch_encode_reference_tokens(d_ref, W, *p, idx.d_phase64,
                                                         idx.d_step32, idx.d_token_class,
                                                         idx.d_emb, idx.d_scale, idx.d_norm2, s));
  } else if (d_delta == nullptr)
    st = hip_status(rm::launch_encode_reference(d_ref, W, *p, idx.d_phase64, idx.d_step32,
                                                idx.d_emb, idx.d_scale, idx.d_norm2, s));
  else
    st = hip_status(rm::launch_encode_reference_learned(d_ref, W, *p, idx.d_phase64,
                                                        idx.d_phase32, idx.d_step32, d_delta,
                                                        idx.d_emb, idx.d_scale, idx.d_norm2, s));
  if (st != RM_OK) return st;
  *out = idx;
  return RM_OK;
}

size_t rm_read_emb_bytes(int32_t n_reads, const rm_params* p) {
  int why = RM_OK;
  if (!params_ok(p, &why) || n_reads < 1) return 0;
  return (size_t)n_reads * 2 * real_dim(p) * rm::elem_bytes(p->precision);
}

int rm_encode_reads(const rm_index* idx, const uint8_t* d_seq, const int64_t* d_off,
                    int32_t n_reads, void* d_read_emb, float* d_read_scale, void* stream) {
  int st = index_ok(idx);
  if (st != RM_OK) return st;
  if (d_seq == nullptr || d_off == nullptr || d_read_emb == nullptr) return RM_EINVAL;
  if (idx->p.precision == RM_FP8_E4M3 && d_read_scale == nullptr) return RM_EINVAL;
  if (n_reads < 1) return RM_ESIZE;
  if (wide_encoding(&idx->p))
    return hip_status(rm::launch_encode_reads_wide(idx->p, idx->d_phase32, idx->d_token_class,
                                                   d_seq, d_off, n_reads, d_read_emb, d_read_scale,
                                                   static_cast<hipStream_t>(stream)));
  if (!letter_encoding(&idx->p))
    return hip_status(rm::launch_encode_reads_tokens(idx->p, idx->d_phase32, idx->d_token_class,
                                                     d_seq, d_off, n_reads, d_read_emb,
                                                     d_read_scale,
                                                     static_cast<hipStream_t>(stream)));
  return hip_status(rm::launch_encode_reads(idx->p, idx->d_phase32, d_seq, d_off, n_reads,
                                            d_read_emb, d_read_scale,
                                            static_cast<hipStream_t>(stream)));
}

int rm_encode_reads_learned(const rm_index* idx, const uint8_t* d_seq, const int64_t* d_off,
                            int32_t n_reads, const float* d_read_delta, void* d_read_emb,
                            float* d_read_scale, void* stream) {
  int st = index_ok(idx);
  if (st != RM_OK) return st;
  if (d_seq == nullptr || d_off == nullptr || d_read_emb == nullptr || d_read_delta == nullptr)
    return RM_EINVAL;
  if (idx->p.precision == RM_FP8_E4M3 && d_read_scale == nullptr) return RM_EINVAL;
  if (n_reads < 1 || idx->p.window_len < 9) return RM_ESIZE;
  if (!letter_encoding(&idx->p) || idx->p.reduced) return RM_EUNSUPPORTED;
  return hip_status(rm::launch_encode_reads_learned(idx->p, idx->d_phase32, d_seq, d_off, n_reads,
                                                    d_read_delta, d_read_emb, d_read_scale,
                                                    static_cast<hipStream_t>(stream)));
}

size_t rm_score_workspace_bytes(const rm_index* idx, int32_t n_reads, int32_t k_fetch) {
  if (idx != nullptr && wide_encoding(&idx->p)) {
    if (index_ok(idx) != RM_OK || n_reads < 1 || k_fetch < 1 || k_fetch > RM_WIDE_MAX_KFETCH)
      return 0;
    return rm::wide_workspace_bytes(n_reads, idx->n_windows, k_fetch);
  }
  return rm_score_groups_workspace_bytes(idx, 1, &n_reads, k_fetch, nullptr);
}

int rm_score_topk(const rm_index* idx, const void* d_read_emb, const float* d_read_scale,
                  int32_t n_reads, int32_t k_fetch, int32_t* d_cand_idx, float* d_cand_score,
                  void* d_ws, size_t ws_bytes, void* stream) {
  if (idx != nullptr && wide_encoding(&idx->p)) {
    int st = index_ok(idx);
    if (st != RM_OK) return st;
    if (!d_read_emb || !d_cand_idx || !d_cand_score || !d_ws) return RM_EINVAL;
    if (idx->p.precision == RM_FP8_E4M3 && !d_read_scale) return RM_EINVAL;
    if (n_reads < 1 || k_fetch < 1 || k_fetch > RM_WIDE_MAX_KFETCH) return RM_ESIZE;
    if (ws_bytes < rm::wide_workspace_bytes(n_reads, idx->n_windows, k_fetch)) return RM_ESIZE;
    return hip_status(rm::launch_score_wide(*idx, d_read_emb, d_read_scale, n_reads, k_fetch,
                                            d_cand_idx, d_cand_score, d_ws,
                                            static_cast<hipStream_t>(stream)));
  }
  return rm_score_topk_groups(idx, 1, &d_read_emb, &d_read_scale, &n_reads, k_fetch, &d_cand_idx,
                              &d_cand_score, d_ws, ws_bytes, nullptr, stream);
}

int rm_score_topk_noalloc(const rm_index* idx, const void* d_read_emb, const float* d_read_scale,
                          int32_t n_reads, int32_t k_fetch, int32_t* d_cand_idx,
                          float* d_cand_score, void* stream) {
  if (idx == nullptr || d_read_emb == nullptr || d_cand_idx == nullptr || d_cand_score == nullptr)
    return RM_EINVAL;
  if (idx->p.precision == RM_FP8_E4M3 && d_read_scale == nullptr) return RM_EINVAL;
  const size_t need = rm_score_workspace_bytes(idx, n_reads, k_fetch);
  if (need == 0)  // invalid arguments: rm_score_topk names the error and enqueues nothing
    return rm_score_topk(idx, d_read_emb, d_read_scale, n_reads, k_fetch, d_cand_idx,
                         d_cand_score, reinterpret_cast<void*>(kNoallocAlign), 0, stream);
  if (need > (size_t)RM_NOALLOC_SCRATCH_BYTES) return RM_ESIZE;
  void* ws = nullptr;
  const int st = noalloc_scratch(&ws);
  if (st != RM_OK) return st;
  return rm_score_topk(idx, d_read_emb, d_read_scale, n_reads, k_fetch, d_cand_idx, d_cand_score,
                       ws, (size_t)RM_NOALLOC_SCRATCH_BYTES, stream);
}

int rm_rescore(const rm_index* idx, const uint8_t* d_ref, const uint8_t* d_seq,
               const int64_t* d_off, int32_t n_reads, int32_t k_fetch, const int32_t* d_cand_idx,
               int32_t k, int32_t* d_top_idx, float* d_top_score, void* stream) {
  int st = index_ok(idx);
  if (st != RM_OK) return st;
  if (d_ref == nullptr || d_seq == nullptr || d_off == nullptr || d_cand_idx == nullptr ||
      d_top_idx == nullptr || d_top_score == nullptr)
    return RM_EINVAL;
  if (n_reads < 1 || k_fetch < 1 || k_fetch > RM_MAX_KFETCH || k < 1 || k > k_fetch)
    return RM_ESIZE;
  if (wide_encoding(&idx->p))
    return hip_status(rm::launch_rescore_wide(*idx, d_ref, d_seq, d_off, n_reads, k_fetch,
                                              d_cand_idx, k, d_top_idx, d_top_score,
                                              static_cast<hipStream_t>(stream)));
  if (!letter_encoding(&idx->p))
    return hip_status(rm::launch_rescore_tokens(*idx, d_ref, d_seq, d_off, n_reads, k_fetch,
                                                d_cand_idx, k, d_top_idx, d_top_score,
                                                static_cast<hipStream_t>(stream)));
  return hip_status(rm::launch_rescore(*idx, d_ref, d_seq, d_off, n_reads, k_fetch, d_cand_idx, k,
                                       d_top_idx, d_top_score, static_cast<hipStream_t>(stream)));
}

size_t rm_token_counts_bytes(int32_t mer_len) {
  if (mer_len < 1 || mer_len > RM_MAX_MER) return 0;
  return ((size_t)1 << (2 * mer_len)) * sizeof(uint32_t);
}

int rm_token_counts(const uint8_t* d_ref, int64_t ref_len, int32_t mer_len, uint32_t* d_counts,
                    void* stream) {
  if (d_ref == nullptr || d_counts == nullptr) return RM_EINVAL;
  if (mer_len < 1 || mer_len > RM_MAX_MER || ref_len < mer_len) return RM_ESIZE;
  return hip_status(rm::launch_token_counts(d_ref, ref_len, mer_len, d_counts,
                                            static_cast<hipStream_t>(stream)));
}

int rm_token_map_frequent(const uint32_t* d_counts, int32_t mer_len, int32_t n_class,
                          uint8_t* d_map, void* stream) {
  if (d_counts == nullptr || d_map == nullptr) return RM_EINVAL;
  if (mer_len < 1 || mer_len > RM_MAX_MER || n_class < 1 || n_class > RM_MAX_FREQUENT ||
      (int64_t)n_class > ((int64_t)1 << (2 * mer_len)))
    return RM_ESIZE;
  return hip_status(rm::launch_token_select(d_counts, mer_len, n_class, d_map,
                                            static_cast<hipStream_t>(stream)));
}

int rm_reverse_complement(const uint8_t* d_seq, const int64_t* d_off, int32_t n_reads,
                          int64_t n_letters, uint8_t* d_out, void* stream) {
  if (d_seq == nullptr || d_off == nullptr || d_out == nullptr || d_out == d_seq) return RM_EINVAL;
  if (n_reads < 1 || n_letters < 1) return RM_ESIZE;
  return hip_status(rm::launch_reverse_complement(d_seq, d_off, n_reads, n_letters, d_out,
                                                  static_cast<hipStream_t>(stream)));
}

int rm_merge_strands(const int32_t* d_fwd_idx, const float* d_fwd_score, const int32_t* d_rev_idx,
                     const float* d_rev_score, int32_t n_reads, int32_t k, float min_fidelity,
                     int32_t* d_top_idx, float* d_top_score, int8_t* d_top_strand,
                     int32_t* d_n_found, void* stream) {
  if (d_fwd_idx == nullptr || d_fwd_score == nullptr || d_rev_idx == nullptr ||
      d_rev_score == nullptr || d_top_idx == nullptr || d_top_score == nullptr ||
      d_top_strand == nullptr || d_n_found == nullptr)
    return RM_EINVAL;
  if (n_reads < 1 || k < 1 || k > RM_MAX_KFETCH) return RM_ESIZE;
  return hip_status(rm::launch_merge_strands(d_fwd_idx, d_fwd_score, d_rev_idx, d_rev_score,
                                             n_reads, k, min_fidelity, d_top_idx, d_top_score,
                                             d_top_strand, d_n_found,
                                             static_cast<hipStream_t>(stream)));
}

int rm_window_thresholds(const rm_index* idx, const uint8_t* d_ref,
                         const rm_threshold_params* tp, float* d_thr, void* stream) {
  int st = index_ok(idx);
  if (st != RM_OK) return st;
  if (d_ref == nullptr || tp == nullptr || d_thr == nullptr) return RM_EINVAL;
  if (!letter_encoding(&idx->p)) return RM_EUNSUPPORTED;
  if (!(tp->err >= 0.f && tp->err < 1.f)) return RM_EINVAL;
  if (tp->copies < 1 || tp->copies > RM_THRESH_MAX_COPIES || tp->rank < 0 ||
      tp->rank >= tp->copies)
    return RM_ESIZE;
  return hip_status(rm::launch_window_thresholds(*idx, d_ref, tp->err, tp->copies, tp->rank,
                                                 tp->seed, d_thr,
                                                 static_cast<hipStream_t>(stream)));
}

size_t rm_threshold_workspace_bytes(int32_t n_reads, int64_t capacity) {
  if (n_reads < 1 || capacity < 1 || capacity > ((int64_t)1 << 40)) return 0;
  return rm::threshold_ws_layout(n_reads, capacity).total;
}

int rm_score_threshold(const rm_index* idx, const uint8_t* d_ref, const void* d_read_emb,
                       const float* d_read_scale, const uint8_t* d_seq, const int64_t* d_off,
                       int32_t n_reads, const float* d_thr, float floor_fidelity,
                       int64_t capacity, int64_t* d_hit_off, int32_t* d_n_found,
                       int32_t* d_hit_idx, float* d_hit_score, int64_t* d_total, void* d_ws,
                       size_t ws_bytes, void* stream) {
  int st = index_ok(idx);
  if (st != RM_OK) return st;
  if (d_ref == nullptr || d_read_emb == nullptr || d_seq == nullptr || d_off == nullptr ||
      d_thr == nullptr || d_hit_off == nullptr || d_n_found == nullptr || d_hit_idx == nullptr ||
      d_hit_score == nullptr || d_total == nullptr || d_ws == nullptr)
    return RM_EINVAL;
  if (idx->p.precision == RM_FP8_E4M3 && d_read_scale == nullptr) return RM_EINVAL;
  if (!letter_encoding(&idx->p)) return RM_EUNSUPPORTED;
  if (!(floor_fidelity >= 0.f && floor_fidelity <= 1.f)) return RM_EINVAL;
  if (n_reads < 1 || capacity < 1 || idx->n_windows > INT32_MAX) return RM_ESIZE;
  const size_t need = rm_threshold_workspace_bytes(n_reads, capacity);
  if (need == 0 || ws_bytes < need) return RM_ESIZE;
  return hip_status(rm::launch_score_threshold(*idx, d_ref, d_read_emb, d_read_scale, d_seq,
                                               d_off, n_reads, d_thr, floor_fidelity,
                                               d_hit_off, d_n_found, d_hit_idx, d_hit_score,
                                               d_total, capacity, d_ws,
                                               static_cast<hipStream_t>(stream)));
}

size_t rm_refine_workspace_bytes(int32_t n_reads, int32_t k_fetch, int32_t radius) {
  if (n_reads < 1 || k_fetch < 1 || k_fetch > RM_MAX_KFETCH || radius < 0 ||
      radius > RM_REFINE_MAX_RADIUS)
    return 0;
  return rm::refine_workspace_bytes(n_reads, k_fetch, radius);
}

int rm_refine(const rm_index* coarse, const uint8_t* d_ref, const uint8_t* d_seq,
              const int64_t* d_off, int32_t n_reads, int32_t k_fetch, const int32_t* d_cand_idx,
              int32_t radius, int32_t k, int32_t* d_top_idx, float* d_top_score, void* d_ws,
              size_t ws_bytes, void* stream) {
  int st = index_ok(coarse);
  if (st != RM_OK) return st;
  if (d_ref == nullptr || d_seq == nullptr || d_off == nullptr || d_cand_idx == nullptr ||
      d_top_idx == nullptr || d_top_score == nullptr || d_ws == nullptr)
    return RM_EINVAL;
  if (n_reads < 1 || k_fetch < 1 || k_fetch > RM_MAX_KFETCH || radius < 0 ||
      radius > RM_REFINE_MAX_RADIUS || k < 1 || k > RM_MAX_KFETCH ||
      (int64_t)k > (int64_t)k_fetch * (2 * radius + 1))
    return RM_ESIZE;
  if (ws_bytes < rm::refine_workspace_bytes(n_reads, k_fetch, radius)) return RM_ESIZE;
  if (coarse->ref_len - coarse->p.window_len + 1 > (int64_t)INT32_MAX) return RM_ESIZE;
  auto launch = letter_encoding(&coarse->p) ? rm::launch_refine
                : wide_encoding(&coarse->p) ? rm::launch_refine_wide
                                            : rm::launch_refine_tokens;
  return hip_status(launch(*coarse, d_ref, d_seq, d_off, n_reads, k_fetch, d_cand_idx, radius, k,
                           d_top_idx, d_top_score, d_ws, static_cast<hipStream_t>(stream)));
}

int rm_rescore_learned(const rm_index* idx, const uint8_t* d_ref, const float* d_ref_delta,
                       const uint8_t* d_seq, const int64_t* d_off, const float* d_read_delta,
                       int32_t n_reads, int32_t k_fetch, const int32_t* d_cand_idx, int32_t k,
                       int32_t* d_top_idx, float* d_top_score, void* stream) {
  int st = index_ok(idx);
  if (st != RM_OK) return st;
  if (d_ref == nullptr || d_ref_delta == nullptr || d_seq == nullptr || d_off == nullptr ||
      d_read_delta == nullptr || d_cand_idx == nullptr || d_top_idx == nullptr ||
      d_top_score == nullptr)
    return RM_EINVAL;
  if (n_reads < 1 || k_fetch < 1 || k_fetch > RM_MAX_KFETCH || k < 1 || k > k_fetch ||
      idx->p.window_len < 9)
    return RM_ESIZE;
  if (!letter_encoding(&idx->p)) return RM_EUNSUPPORTED;
  return hip_status(rm::launch_rescore(*idx, d_ref, d_seq, d_off, n_reads, k_fetch, d_cand_idx, k,
                                       d_top_idx, d_top_score, static_cast<hipStream_t>(stream),
                                       d_ref_delta, d_read_delta));
}

size_t rm_delta_bytes(int64_t n_letters) {
  if (n_letters < 9) return 0;
  return (size_t)(n_letters - 8) * 32 * sizeof(float);
}

int rm_mlp_infer(const float* d_params, const uint8_t* d_seq, int64_t n_letters, float* d_delta,
                 void* stream) {
  if (d_params == nullptr || d_seq == nullptr || d_delta == nullptr) return RM_EINVAL;
  if (n_letters < 9) return RM_ESIZE;
  if (reinterpret_cast<uintptr_t>(d_delta) % 16 != 0) return RM_EINVAL;
  return hip_status(rm::launch_mlp_infer(d_params, d_seq, n_letters, d_delta,
                                         static_cast<hipStream_t>(stream)));
}

// ------------------------------------------------------------------ batching

int rm_bucket_reads(const int64_t* h_off, int32_t n_reads, const int32_t* bucket_len,
                    int32_t n_buckets, int32_t* h_bucket, int32_t* h_count) {
  if (!h_off || !bucket_len || !h_bucket || !h_count) return RM_EINVAL;
  if (n_reads < 0 || n_buckets < 1) return RM_ESIZE;
  for (int b = 0; b < n_buckets; ++b) {
    if (bucket_len[b] < 1 || (b > 0 && bucket_len[b] <= bucket_len[b - 1])) return RM_EINVAL;
    h_count[b] = 0;
  }
  for (int32_t r = 0; r < n_reads; ++r) {
    int64_t len = h_off[r + 1] - h_off[r];
    int b = -1;
    while (b + 1 < n_buckets && bucket_len[b + 1] <= len) ++b;
    h_bucket[r] = b;
    if (b >= 0) ++h_count[b];
  }
  return RM_OK;
}

static int groups_ok(const rm_index* idx, int32_t n_groups, const int32_t* n_reads,
                     int32_t k_fetch) {
  if (idx == nullptr || n_reads == nullptr) return RM_EINVAL;
  if (n_groups < 1 || n_groups > RM_MAX_GROUPS) return RM_ESIZE;
  if (k_fetch < 1 || k_fetch > RM_MAX_KFETCH) return RM_ESIZE;
  for (int i = 0; i < n_groups; ++i) {
    int st = index_ok(&idx[i]);
    if (st != RM_OK) return st;
    if (idx[i].p.precision != idx[0].p.precision) return RM_EINVAL;
    if (wide_encoding(&idx[i].p)) return RM_EUNSUPPORTED;  // scored by rm_score_topk only
    if (n_reads[i] < 1) return RM_ESIZE;
  }
  return RM_OK;
}

static rm::ScorePlan groups_plan(const rm_index* idx, int32_t n_groups, const int32_t* n_reads,
                                 int32_t k_fetch, const rm_tuning* tune) {
  int64_t W[RM_MAX_GROUPS];
  for (int i = 0; i < n_groups; ++i) W[i] = idx[i].n_windows;
  rm::Tuning t{tune ? tune->read_tile : 0, tune ? tune->chunk_tiles : 0};
  return rm::plan_score(idx[0].p.precision, n_groups, W, n_reads, k_fetch, t);
}

size_t rm_score_groups_workspace_bytes(const rm_index* idx, int32_t n_groups,
                                       const int32_t* n_reads, int32_t k_fetch,
                                       const rm_tuning* tune) {
  if (groups_ok(idx, n_groups, n_reads, k_fetch) != RM_OK) return 0;
  rm::ScorePlan plan = groups_plan(idx, n_groups, n_reads, k_fetch, tune);
  return plan.ok ? plan.ws_bytes : 0;
}

int rm_score_topk_groups(const rm_index* idx, int32_t n_groups, const void* const* d_read_emb,
                         const float* const* d_read_scale, const int32_t* n_reads,
                         int32_t k_fetch, int32_t* const* d_cand_idx,
                         float* const* d_cand_score, void* d_ws, size_t ws_bytes,
                         const rm_tuning* tune, void* stream) {
  int st = groups_ok(idx, n_groups, n_reads, k_fetch);
  if (st != RM_OK) return st;
  if (!d_read_emb || !d_cand_idx || !d_cand_score || !d_ws) return RM_EINVAL;
  const bool fp8 = idx[0].p.precision == RM_FP8_E4M3;
  if (fp8 && !d_read_scale) return RM_EINVAL;
  for (int i = 0; i < n_groups; ++i) {
    if (!d_read_emb[i] || !d_cand_idx[i] || !d_cand_score[i]) return RM_EINVAL;
    if (fp8 && !d_read_scale[i]) return RM_EINVAL;
  }
  if (tune && (tune->chunk_tiles < 0 ||
               (tune->read_tile != 0 && tune->read_tile != 128 && tune->read_tile != 256)))
    return RM_EUNSUPPORTED;
  rm::ScorePlan plan = groups_plan(idx, n_groups, n_reads, k_fetch, tune);
  if (!plan.ok) return tune && tune->read_tile ? RM_EUNSUPPORTED : RM_ESIZE;
  if (ws_bytes < plan.ws_bytes) return RM_ESIZE;
  return hip_status(rm::launch_score_topk(idx, plan, d_read_emb, d_read_scale, n_reads, k_fetch,
                                          d_cand_idx, d_cand_score, d_ws,
                                          static_cast<hipStream_t>(stream)));
}

// ------------------------------------------------------------------ learned offsets

size_t rm_learned_workspace_bytes(int32_t n_pairs) {
  if (n_pairs < 2 || n_pairs > RM_LEARNED_MAX_PAIRS) return 0;
  return rm::learned_workspace_bytes(n_pairs);
}

int rm_learned_encode(const float* d_params, const uint8_t* d_seq, const int64_t* d_off,
                      int32_t n_strings, int32_t nominal_len, float* d_c, void* stream) {
  if (!d_seq || !d_off || !d_c) return RM_EINVAL;
  if (n_strings < 1 || nominal_len < 1) return RM_ESIZE;
  return hip_status(rm::launch_learned_encode(d_params, d_seq, d_off, n_strings, nominal_len, d_c,
                                              static_cast<hipStream_t>(stream)));
}

int rm_pair_fidelity(const float* d_ca, const float* d_cb, int32_t n_pairs, float* d_F,
                     void* stream) {
  if (!d_ca || !d_cb || !d_F) return RM_EINVAL;
  if (n_pairs < 1) return RM_ESIZE;
  return hip_status(
      rm::launch_pair_fidelity(d_ca, d_cb, n_pairs, d_F, static_cast<hipStream_t>(stream)));
}

static int learned_args_ok(const void* p, const uint8_t* a, const int64_t* aoff, const uint8_t* b,
                           const int64_t* boff, const int32_t* ld, int32_t n_pairs,
                           int32_t nominal_len, void* ws, size_t ws_bytes, const float* loss) {
  if (!p || !a || !aoff || !b || !boff || !ld || !ws || !loss) return RM_EINVAL;
  if (n_pairs < 2 || n_pairs > RM_LEARNED_MAX_PAIRS || nominal_len < 1) return RM_ESIZE;
  if (ws_bytes < rm::learned_workspace_bytes(n_pairs)) return RM_ESIZE;
  return RM_OK;
}

int rm_learned_train_step(float* d_state, float lr, const uint8_t* d_a, const int64_t* d_aoff,
                          const uint8_t* d_b, const int64_t* d_boff, const int32_t* d_ld,
                          int32_t n_pairs, int32_t nominal_len, void* d_ws, size_t ws_bytes,
                          float* d_loss, void* stream) {
  int st = learned_args_ok(d_state, d_a, d_aoff, d_b, d_boff, d_ld, n_pairs, nominal_len, d_ws,
                           ws_bytes, d_loss);
  if (st != RM_OK) return st;
  return hip_status(rm::launch_learned_step(d_state, lr, d_a, d_aoff, d_b, d_boff, d_ld, n_pairs,
                                            nominal_len, d_ws, nullptr, d_loss,
                                            static_cast<hipStream_t>(stream)));
}

int rm_learned_gradient(const float* d_params, const uint8_t* d_a, const int64_t* d_aoff,
                        const uint8_t* d_b, const int64_t* d_boff, const int32_t* d_ld,
                        int32_t n_pairs, int32_t nominal_len, void* d_ws, size_t ws_bytes,
                        float* d_grad, float* d_loss, void* stream) {
  int st = learned_args_ok(d_params, d_a, d_aoff, d_b, d_boff, d_ld, n_pairs, nominal_len, d_ws,
                           ws_bytes, d_loss);
  if (st != RM_OK) return st;
  if (!d_grad) return RM_EINVAL;
  return hip_status(rm::launch_learned_step(const_cast<float*>(d_params), 0.f, d_a, d_aoff, d_b,
                                            d_boff, d_ld, n_pairs, nominal_len, d_ws, d_grad,
                                            d_loss, static_cast<hipStream_t>(stream)));
}

int rm_levenshtein(const uint8_t* d_a, const int64_t* d_aoff, const uint8_t* d_b,
                   const int64_t* d_boff, int64_t n, int32_t* d_out, void* stream) {
  if (!d_a || !d_aoff || !d_b || !d_boff || !d_out) return RM_EINVAL;
  if (n < 1 || n > (int64_t)INT32_MAX * 256) return RM_ESIZE;  // one thread per pair
  return hip_status(rm::launch_levenshtein(d_a, d_aoff, d_b, d_boff, n, d_out,
                                           static_cast<hipStream_t>(stream)));
}

// ------------------------------------------------------------------ graphs

struct rm_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

int rm_capture_begin(void* stream) {
  if (stream == nullptr) return RM_EINVAL;
  return hip_status(
      hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal));
}

int rm_capture_end(void* stream, rm_graph* out) {
  if (stream == nullptr || out == nullptr) return RM_EINVAL;
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(static_cast<hipStream_t>(stream), &g) != hipSuccess || g == nullptr)
    return RM_EHIP;
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return RM_EHIP;
  }
  rm_graph h = new (std::nothrow) rm_graph_s{g, ex};
  if (h == nullptr) {
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
    return RM_EHIP;
  }
  *out = h;
  return RM_OK;
}

int rm_graph_launch(rm_graph graph, void* stream) {
  if (graph == nullptr) return RM_EINVAL;
  return hip_status(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
}

int rm_graph_destroy(rm_graph graph) {
  if (graph == nullptr) return RM_EINVAL;
  (void)hipGraphExecDestroy(graph->exec);
  (void)hipGraphDestroy(graph->graph);
  delete graph;
  return RM_OK;
}

}  // extern "C"
