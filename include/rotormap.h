/* rotormap.h -- C ABI of the RotorMap hot path on AMD MI355X (gfx950).
 *
 * What is computed (RotorMap paper, arXiv 2603.22245):
 *  - §3 (the mapping problem): given a reference and reads, find for each read
 *    the reference positions it most likely comes from;
 *  - §3.1 (basic idea): windows of N letters slide over the reference with a
 *    step; each window's RoPE encoding is stored in an index; each read's head
 *    (its first N letters) is encoded; the fidelity of the head with every
 *    window is computed (a matrix product at its core) and the best windows are
 *    kept;
 *  - §2.1-§2.3 (the encoding, tokens of one letter, s = 1): component (k, L) of
 *    a string is the sum over the locations p of letter L of omega^(f_k p),
 *    omega = exp(2 pi i / N), k = 1..m (§2.2 eq. mult-factor: f_k = k; §3.3 eq.
 *    mult-factor-finetune: f_k = 2(k-1)/(m-1)+1), ordered (k-1)*4 + L as in the
 *    D^loc form of §2.10, then normalised;
 *  - §2.4: fidelity F = |<x|c>|^2 / (|x|^2 |c|^2);
 *  - §3.4: the window encoding is updated letter by letter as the window slides
 *    (rotate by omega^-f_k, remove the outgoing letter, add the incoming one).
 *
 * Conventions shared by every call:
 *  - Letters are uint8 codes A,C,G,T = 0,1,2,3.  Any other code contributes no
 *    token (it is skipped, as a letter of unknown identity with no weight).
 *  - Every pointer named d_* is DEVICE memory owned by the caller.  The library
 *    never allocates or frees device memory and keeps no state between calls.
 *  - Calls that take `stream` (a hipStream_t; NULL = the null stream) only
 *    enqueue work on it and return; results are ready once the stream is
 *    synchronised.  Faults inside a kernel surface at that synchronisation.
 *  - Every argument is validated on the host before anything is enqueued; a
 *    call that returns anything but RM_OK has enqueued nothing.  A HIP launch
 *    error after validation returns RM_EHIP.
 *  - A window or read whose squared norm (before normalisation) is below
 *    1e-4 * N in FP32 is degenerate (e.g. one letter repeated, or a period that
 *    divides N, §3.3): it is stored as the zero vector and its fidelity with
 *    anything is 0.
 *  - Candidate lists are ordered by fidelity descending, then by window id
 *    ascending.  Window id j is the window starting at reference position
 *    j * stride.
 *  - §3 asks for a read's position only if one exists.  An entry whose
 *    fidelity is 0 (the read head or the window is the zero vector: a
 *    degenerate string, or a read shorter than N) is no location and is
 *    written as id -1 with score 0; so is a slot left empty because there
 *    are fewer candidates than slots.  A read with no location has id -1,
 *    score 0 in every slot.
 */
#ifndef ROTORMAP_H
#define ROTORMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define RM_OK 0
#define RM_EINVAL (-1)        /* a null pointer, a bad enum or an inconsistent argument */
#define RM_ESIZE (-2)         /* a size out of range or a buffer that is too small */
#define RM_EUNSUPPORTED (-3)  /* a parameter combination the kernels do not implement */
#define RM_EHIP (-4)          /* a HIP runtime error when enqueuing */

/* ---- enums --------------------------------------------------------------- */
#define RM_FP32 0      /* embeddings stored as float32 */
#define RM_FP16 1      /* embeddings stored as IEEE binary16, round to nearest even */
#define RM_FP8_E4M3 2  /* embeddings stored as OCP FP8 e4m3 codes of v / 2^e (RNE)
                          plus one FP32 scale per window / per read chosen so
                          that code * scale has unit norm; 2^e = 2^-8 for every
                          window row of 128 complex components (a unit vector's
                          reals are at most 1, and e4m3's relative precision is
                          the same across its normal range), else the smallest
                          power of two with max|v| / 2^e <= 448 */

#define RM_SCHED_DEFAULT 0    /* f_k = k            (§2.2 eq. mult-factor) */
#define RM_SCHED_FINETUNED 1  /* f_k = 2(k-1)/(m-1)+1 (§3.3 eq. mult-factor-finetune) */

#define RM_DIM 32          /* number of factors m of the letter encoding: 4*m = 128 complex
                              components; token encodings use m * n_class = 128 */
#define RM_MAX_MER 8       /* longest token (s-mer) of a token encoding */
#define RM_TOKEN_SKIP 255  /* token-map value of an s-mer that adds nothing */
#define RM_MAX_WINDOW 16384 /* largest supported N */
#define RM_MAX_KFETCH 64   /* largest candidate list per read */
#define RM_WIDE_MAX_KFETCH 32  /* ... with a 1,024-component token encoding */

/* Parameters of an index.  Plain data; zero-initialise and fill. */
typedef struct rm_params {
  int32_t window_len; /* N: letters per window and per read head, 1..RM_MAX_WINDOW */
  int32_t stride;     /* window step (>= 1); window j starts at j * stride */
  int32_t n_freq;     /* m; must be RM_DIM */
  int32_t schedule;   /* RM_SCHED_* */
  int32_t precision;  /* RM_FP32, RM_FP16 or RM_FP8_E4M3 */
  int32_t reanchor;   /* window starts between two FP64 re-computations of the
                         rolling state (>= 1), or 0: chosen by the library,
                         at most 4096 */
  /* Tokens (§2.1: s-mers; §2.6: compact versions).  Zero-initialised fields
   * give the letter encoding (s = 1, n_class 4, n_freq RM_DIM).  Otherwise the
   * encoding is a token encoding: the token at location loc = 0..N-s is the
   * s-mer w[loc .. loc+s), with code sum_i w[loc+i] 4^(s-1-i) (first letter
   * most significant; an s-mer holding a letter outside 0..3 is no token); its
   * class is the code itself (no map: n_class must be 4^s) or d_token_map[code]
   * (values >= n_class, e.g. RM_TOKEN_SKIP, add nothing: the variant keeping
   * only selected s-mers, e.g. rm_token_map_frequent's).  Component index
   * (k-1)*n_class + class, with n_class even and at most 256, and
   * n_class * n_freq either 128 ((s, m) = (2, 8) or (3, 2) without a map, any
   * s <= RM_MAX_MER with one, e.g. s = 8 mapped to 16 classes, m = 8; every
   * precision) or 1,024 (n_class a multiple of 16, e.g. s = 8 mapped to 256
   * classes with m = 4 -- the paper's s = 8, m = 4, t = 4 shape -- or s = 4,
   * m = 4; FP16 or FP8 index, 2,048 reals per row). */
  int32_t mer_len;    /* s, 1..RM_MAX_MER; 0 means 1 */
  int32_t n_class;    /* components per factor; 0 means 4^s */
  const uint8_t* d_token_map; /* NULL, or DEVICE [4^s] class per s-mer code; read
                                 by rm_encode_reference only (copied into the
                                 index buffer) */
  /* Letter-sum form (letter encoding, default schedule, N > RM_DIM; 0
   * otherwise).  With integer factors f_k = k < N (§2.2) the components of
   * factor k of a window sum over the four letters to sum_p omega^(k p) = 0,
   * since each location holds one letter: 1 stores every window and read head
   * by its coordinates on an orthonormal basis of that 3m-dimensional
   * subspace (per factor, the letter weights (1,1,-1,-1)/2, (1,-1,1,-1)/2,
   * (1,-1,-1,1)/2 for A,C,G,T), 96 complex components = 192 reals per row
   * (re, im interleaved per component, factor-major) instead of 256.  Norms
   * are taken over all 128 components first, and every fidelity is the same
   * as with the full rows, provided every reference window holds letters only
   * (codes 0..3); a window holding another code loses the part of its vector
   * along the all-letters direction, which matters only against read heads
   * that hold such codes too. */
  int32_t reduced;
} rm_params;

/* Descriptor of an index living in a caller-owned device buffer.  Filled by
 * rm_encode_reference; the pointers point into that buffer.  Plain data: it may
 * be copied, and stays valid while the buffer lives. */
typedef struct rm_index {
  rm_params p;
  int64_t ref_len;     /* G, letters in the reference */
  int64_t n_windows;   /* W = floor((G - N) / stride) + 1 */
  void* d_emb;         /* [W][256] embeddings (re, im interleaved per component);
                          [W][192] in the letter-sum form; [W][2048] for
                          1,024-component token encodings */
  float* d_scale;      /* [W] FP8 dequantisation scale per window (1.0 for FP32/FP16);
                          d_scale[W] = the largest (256 d_scale[j])^2 over the FP8
                          windows of 128 components (a bound the product's
                          threshold test uses), else 0 */
  float* d_norm2;      /* [W] squared norm of each window's vector before normalising */
  double* d_phase64;   /* [N][m] complex omega^(f_k p), FP64 (re, im) */
  float* d_phase32;    /* [N][m] the same rounded to FP32 */
  float* d_step32;     /* [m][4] FP32 omega^-f_k (re, im) and omega^(f_k (N-s)) (re, im) */
  uint8_t* d_token_class; /* token encodings: [4^s] class per s-mer code (the map with
                             values >= n_class replaced by RM_TOKEN_SKIP, or the
                             identity); NULL for the letter encoding */
} rm_index;

/* Human-readable text of a status code (static storage). */
const char* rm_status_str(int status);

/* Library version string (static storage). */
const char* rm_version(void);

/* Number of windows for (ref_len, p), or -1 if the parameters are invalid. */
int64_t rm_num_windows(int64_t ref_len, const rm_params* p);

/* Bytes of the device buffer rm_encode_reference needs, or 0 if the
 * parameters are invalid.  The buffer must be 256-byte aligned. */
size_t rm_index_bytes(int64_t ref_len, const rm_params* p);

/* Build the index (§3.1) of the reference d_ref[0..ref_len) into d_buf:
 * FP64 angle tables, then every window's encoding by the rolling update of
 * §3.4 in FP32 with an FP64 re-computation every p->reanchor starts,
 * normalised and stored in p->precision.  Fills *out.
 * Errors: RM_EINVAL (null pointer, bad enum), RM_ESIZE (ref_len < N, N out of
 * range, stride < 1, buf_bytes < rm_index_bytes, more than 2^31-1 windows,
 * mer_len out of range, N < s), RM_EUNSUPPORTED (letter encoding with n_freq
 * != RM_DIM; token encoding with n_class odd or above 256, n_class * n_freq
 * neither 128 nor 1,024, 1,024 components with n_class not a multiple of 16
 * or an FP32 index, or no map and n_class != 4^s; the letter-sum form with
 * a token encoding, the fine-tuned schedule or N <= RM_DIM). */
int rm_encode_reference(const uint8_t* d_ref, int64_t ref_len, const rm_params* p,
                        void* d_buf, size_t buf_bytes, rm_index* out, void* stream);

/* Bytes of the read-embedding buffer for n_reads reads: [n_reads][2][256]
 * ([n_reads][2][192] in the letter-sum form, [n_reads][2][2048] for
 * 1,024-component token encodings) elements of the
 * index precision (row 2r holds (Re x, Im x) per component and
 * row 2r+1 holds (-Im x, Re x), so that one real product of the two rows with a
 * window row gives Re and Im of <x|c>).  0 if invalid. */
size_t rm_read_emb_bytes(int32_t n_reads, const rm_params* p);

/* Encode the head (first N letters) of every read (§3.1): FP32 direct sum of the
 * FP32 angle table (rounded from the FP64 one) over the head's letters,
 * normalised, stored in the index precision.  Read r is
 * d_seq[d_off[r] .. d_off[r+1]) (d_off: n_reads+1 int64, device).  A read
 * shorter than N is encoded as the zero vector.  A token index sums the
 * head's tokens (locations 0..N-s) by class.  d_read_scale [n_reads]
 * receives the FP8 scale per read (1.0 otherwise); it may be NULL unless the
 * precision is FP8.  Errors: RM_EINVAL, RM_ESIZE (n_reads < 1). */
int rm_encode_reads(const rm_index* idx, const uint8_t* d_seq, const int64_t* d_off,
                    int32_t n_reads, void* d_read_emb, float* d_read_scale, void* stream);

/* Bytes of the workspace rm_score_topk needs. 0 if invalid. */
size_t rm_score_workspace_bytes(const rm_index* idx, int32_t n_reads, int32_t k_fetch);

/* Score every read against every window and keep, per read, the k_fetch best
 * windows (§3.1: fidelities of the read's encoding with all index vectors as a
 * matrix product, then the best locations).  The product runs on MFMA in the
 * index precision with FP32 accumulation; the full score matrix is never
 * stored.  Outputs [n_reads][k_fetch]: window ids (int32) and fidelities
 * (float, computed from the stored embeddings).  Ties are broken by lower
 * window id, exactly.  If W < k_fetch the tail is filled with id -1, score 0;
 * a read with no location (see the conventions) has id -1, score 0 throughout.
 * d_read_scale may be NULL unless the precision is FP8.
 * Errors: RM_EINVAL, RM_ESIZE (k_fetch outside 1..RM_MAX_KFETCH -- 1..RM_WIDE_MAX_KFETCH
 * for 1,024-component token encodings -- ws too small). */
int rm_score_topk(const rm_index* idx, const void* d_read_emb, const float* d_read_scale,
                  int32_t n_reads, int32_t k_fetch, int32_t* d_cand_idx, float* d_cand_score,
                  void* d_ws, size_t ws_bytes, void* stream);

/* ---- rm_score_topk without a caller workspace ---------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  The same
 * call as rm_score_topk, with its workspace in a device array the library
 * owns: RM_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on that GPU
 * until the process ends (enough for rm_score_workspace_bytes of 100,000
 * reads against 10^7 windows with 16 candidates).  The array of the CURRENT
 * device is used, so call it with the stream's device current.  Its device
 * address is looked up on the first call on each device; no call allocates or
 * frees memory.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other streams, other host threads) race and
 * must be serialised by the caller; each call clears what must start at zero.
 * Errors: as rm_score_topk; RM_ESIZE also when rm_score_workspace_bytes
 * exceeds RM_NOALLOC_SCRATCH_BYTES; RM_EHIP if the array's address cannot be
 * found; RM_EUNSUPPORTED for a device index of 64 or more. */
#define RM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int rm_score_topk_noalloc(const rm_index* idx, const void* d_read_emb, const float* d_read_scale,
                          int32_t n_reads, int32_t k_fetch, int32_t* d_cand_idx,
                          float* d_cand_score, void* stream);

/* Rescore the candidates in FP32 and keep the k best (the refinement idea of
 * §3.4 applied to the candidates): each candidate window's encoding and the
 * read head's encoding are recomputed directly from the letters with the
 * FP32 angle table (never from the stored low-precision index), F =
 * |<x|c>|^2 / (X C) in FP32, sorted by (F desc, window id asc).  Candidates
 * with id < 0 are skipped; missing entries and entries with F = 0 are id -1,
 * score 0 (a read shorter than N, or with a degenerate head, has no location).
 * A token index recomputes the encodings over its tokens and classes the same
 * way.  Errors: RM_EINVAL, RM_ESIZE (k < 1 or k > k_fetch). */
int rm_rescore(const rm_index* idx, const uint8_t* d_ref, const uint8_t* d_seq,
               const int64_t* d_off, int32_t n_reads, int32_t k_fetch,
               const int32_t* d_cand_idx, int32_t k, int32_t* d_top_idx, float* d_top_score,
               void* stream);

/* ---- the compact context-aware token map (§2.6) ------------------------------
 * Only the reference's most frequent s-mers are tokens: count every s-mer of
 * the reference, then keep the n_class first by (count descending, code
 * ascending) as classes 0..n_class-1 in code order; every other s-mer maps to
 * RM_TOKEN_SKIP.  The map is then passed as rm_params.d_token_map. */
#define RM_MAX_FREQUENT 128  /* largest n_class for the selection (RM_TOKEN_SKIP stays free) */

/* Bytes of the count buffer for s-mers of mer_len letters (4^s uint32); 0 if invalid. */
size_t rm_token_counts_bytes(int32_t mer_len);

/* d_counts[code] = occurrences of the s-mer `code` (code as in rm_params) at
 * the locations 0..ref_len-s of d_ref; s-mers holding a letter outside 0..3
 * are not counted.  d_counts: caller-owned device buffer of
 * rm_token_counts_bytes(mer_len), overwritten.  Errors: RM_EINVAL (null
 * pointer), RM_ESIZE (mer_len outside 1..RM_MAX_MER, ref_len < mer_len). */
int rm_token_counts(const uint8_t* d_ref, int64_t ref_len, int32_t mer_len, uint32_t* d_counts,
                    void* stream);

/* d_map[code] (4^s uint8, device, caller-owned) = the class of the n_class
 * most frequent s-mers of d_counts, ranked by (count desc, code asc) and
 * numbered in code order; RM_TOKEN_SKIP for the others.  Errors: RM_EINVAL,
 * RM_ESIZE (mer_len out of range, n_class outside 1..min(RM_MAX_FREQUENT, 4^s))). */
int rm_token_map_frequent(const uint32_t* d_counts, int32_t mer_len, int32_t n_class,
                          uint8_t* d_map, void* stream);

/* ---- both strands and the threshold regime ---------------------------------
 * The paper maps reads in both directions: a read from the other strand
 * matches the reference after reverse complementing it.  Map the reads and
 * their reverse complements as one batch (2 n_reads heads), then combine each
 * read's two lists.  §3.1 takes the fidelities above a threshold as the
 * matching locations, and §3.5 describes the regime that reports every
 * location passing it: rm_merge_strands drops entries below min_fidelity, and
 * a read with none left is unmapped. */

/* Reverse complement of every read: d_out[d_off[r] .. d_off[r+1]) receives
 * the letters of read r reversed, codes 0..3 (A, C, G, T) mapped to 3 - L
 * (other codes copied).  d_out has the layout of d_seq (n_letters =
 * d_off[n_reads] - d_off[0] letters from offset d_off[0]) and must not
 * overlap it.  Errors: RM_EINVAL (null pointer, d_out == d_seq), RM_ESIZE
 * (n_reads < 1, n_letters < 1). */
int rm_reverse_complement(const uint8_t* d_seq, const int64_t* d_off, int32_t n_reads,
                          int64_t n_letters, uint8_t* d_out, void* stream);

/* Combine, per read, the forward list (d_fwd_idx / d_fwd_score [n_reads][k])
 * and the reverse-complement list (d_rev_*, same shape), each ranked by
 * (F desc, window id asc) as rm_rescore returns them, into the k best ranked
 * the same way, the forward entry first on a full tie; entries with id < 0 or
 * F < min_fidelity are dropped.  Outputs [n_reads][k]: window ids, F, strand
 * (int8: 0 forward, 1 reverse complement; -1 with id -1 and F 0 past the
 * kept entries) and d_n_found [n_reads], the number kept (0 = unmapped).
 * Errors: RM_EINVAL (null pointer), RM_ESIZE (n_reads < 1, k outside
 * 1..RM_MAX_KFETCH). */
int rm_merge_strands(const int32_t* d_fwd_idx, const float* d_fwd_score, const int32_t* d_rev_idx,
                     const float* d_rev_score, int32_t n_reads, int32_t k, float min_fidelity,
                     int32_t* d_top_idx, float* d_top_score, int8_t* d_top_strand,
                     int32_t* d_n_found, void* stream);

/* ---- per-fragment thresholds and the threshold regime (§3.3, §3.5) ----------
 * §3.3 closes by noting that, for a target mutation rate, the fidelity
 * expected of each reference fragment can be estimated and used as that
 * fragment's cutting threshold; §3.5 describes the regime that reports every
 * location whose fidelity passes its fragment's precomputed threshold (many
 * for some reads, none for others).  Estimate used here: window j is mutated
 * `copies` times at rate err by a streaming mutator (walking the reference
 * from the window's start, each step an insertion, a deletion or a
 * substitution with probability err/3 each, else a match, until N letters are
 * out; a step that needs a letter past the reference's end inserts; at most
 * 8 N + 64 steps), and its threshold is the `rank`-th smallest fidelity
 * (0 = the smallest) of the window with its copies, in FP32.  The draws come
 * from the counter-based generator Philox4x32-10 (Salmon et al., SC 2011):
 * step t of copy c of window j uses the four words of counter (j mod 2^32,
 * j >> 32, c, t) under key (seed, 0); word 0 below 1x / 2x / 3x
 * floor(err / 3 * 2^32) is an insertion / deletion / substitution (err as the
 * FP32 value converted to double), word 1 & 3 an inserted letter and
 * 1 + word 2 mod 3 a substitution's shift ((old + shift) mod 4).  Letter
 * encoding only. */
#define RM_THRESH_MAX_COPIES 64

typedef struct rm_threshold_params {
  float err;       /* target mutation rate, 0 <= err < 1 */
  int32_t copies;  /* mutated copies per window, 1..RM_THRESH_MAX_COPIES */
  int32_t rank;    /* order statistic of the copies' fidelities, 0..copies-1 */
  uint32_t seed;   /* the generator's key word 0 */
} rm_threshold_params;

/* d_thr [W] (device, caller-owned, FP32) = the threshold of every window of
 * idx (d_ref its reference).  Errors: RM_EINVAL (null pointer, invalid index,
 * err outside [0, 1)), RM_ESIZE (copies or rank out of range),
 * RM_EUNSUPPORTED (a token index). */
int rm_window_thresholds(const rm_index* idx, const uint8_t* d_ref,
                         const rm_threshold_params* tp, float* d_thr, void* stream);

/* Bytes of the workspace rm_score_threshold needs for n_reads reads and a
 * candidate capacity; 0 if invalid. */
size_t rm_threshold_workspace_bytes(int32_t n_reads, int64_t capacity);

/* The threshold regime: for every read r, every window j with
 * F(r, j) >= max(d_thr[j], floor_fidelity) and F(r, j) > 0, F recomputed in
 * FP32 from the letters (as rm_rescore does), ranked by (F desc, window id
 * asc).  The product in the index precision (reads from rm_encode_reads of the
 * same index; d_read_scale as for rm_score_topk) proposes every pair within
 * the product's error of the cut (2e-2 FP8, 2e-3 FP16, 1e-4 FP32), at most
 * `capacity` pairs in all.  Output (device, caller-owned): d_hit_off
 * [n_reads + 1] int64 offsets of each read's span in d_hit_idx / d_hit_score
 * [capacity] (the spans hold the read's proposals); d_n_found [n_reads] the
 * hits of each read, at d_hit_idx[d_hit_off[r] ..] ranked, the rest of the
 * span id -1, score 0; *d_total the number of proposals found.  If *d_total
 * exceeds capacity, proposals were dropped and the result is incomplete: call
 * again with a capacity of at least *d_total.  Errors: RM_EINVAL (null
 * pointer, invalid index, FP8 without read scales, floor_fidelity outside
 * [0, 1]), RM_ESIZE (n_reads < 1, capacity < 1, workspace too small, 2^31 or
 * more windows), RM_EUNSUPPORTED (a token index). */
int rm_score_threshold(const rm_index* idx, const uint8_t* d_ref, const void* d_read_emb,
                       const float* d_read_scale, const uint8_t* d_seq, const int64_t* d_off,
                       int32_t n_reads, const float* d_thr, float floor_fidelity,
                       int64_t capacity, int64_t* d_hit_off, int32_t* d_n_found,
                       int32_t* d_hit_idx, float* d_hit_score, int64_t* d_total, void* d_ws,
                       size_t ws_bytes, void* stream);

/* ---- the correlation score (§2.4) -------------------------------------------
 * How well fidelity predicts the mutation rate: pairs (dna, mut) are sampled at
 * mutation rates err; per rate, E_fid is the mean fidelity of its pairs; the
 * points (E_fid(err), err), joined in order of E_fid, form the fitting curve
 * (extended flat past its ends); per rate, the RMSE is the root mean square of
 * the vertical distances curve(fid) - err of its pairs' points.  Fidelities
 * come from rm_pair_fidelity (plain or learned encoding). */
#define RM_CORR_MAX_RATES 256

/* From d_F [n_rates][per_rate] (FP32 fidelities, rate-major) and d_err
 * [n_rates] (the rates), write d_E [n_rates] (E_fid) and d_rmse [n_rates].
 * All device memory, caller-owned; FP32 sums.  Errors: RM_EINVAL (null
 * pointer), RM_ESIZE (n_rates outside 1..RM_CORR_MAX_RATES, per_rate < 1). */
int rm_correlation_score(const float* d_F, const float* d_err, int32_t n_rates, int32_t per_rate,
                         float* d_E, float* d_rmse, void* stream);

/* ---- refinement around found locations (§3.4) ------------------------------
 * With a coarse index (stride sigma > 1) the product finds the coarse window
 * nearest each good location; rm_refine then scores the step-1 windows whose
 * starts lie within `radius` of each candidate's start (j * sigma - radius ..
 * j * sigma + radius, clamped to the reference) exactly in FP32 -- the first
 * by a direct sum of its letters, the rest by the one-letter slide relations
 * of §3.4 -- and keeps the k best distinct starts over all of a read's
 * neighbourhoods, ordered by (F desc, start asc).  F = |<x|c>|^2 / (X C)
 * (§2.4) with each window's norm recomputed.  Every encoding rm_build_index
 * takes: with tokens (§2.1, §2.6) the first window is a direct sum over its
 * tokens and a slide turns every component by omega^-f, takes omega^-f off
 * the class of the token leaving and adds omega^{f (N-s)} to the class of the
 * token entering. */
#define RM_REFINE_MAX_RADIUS 31  /* 2 radius + 1 <= 63 starts per candidate */

/* Bytes of the workspace rm_refine needs (256-byte multiple); 0 if invalid. */
size_t rm_refine_workspace_bytes(int32_t n_reads, int32_t k_fetch, int32_t radius);

/* Refine the coarse candidates d_cand_idx [n_reads][k_fetch] (window ids of
 * the coarse index `coarse`, e.g. rm_score_topk's output; ids < 0 or >= W are
 * skipped) into d_top_idx / d_top_score [n_reads][k]: step-1 window starts
 * (the window ids of a stride-1 index of the same reference) and their FP32
 * fidelities; missing entries and entries with F = 0 are id -1, score 0.
 * d_ref is the coarse index's reference, d_seq / d_off the reads as in
 * rm_encode_reads (a read shorter than N scores 0 everywhere, so it has no
 * location).  d_ws: caller-owned device workspace of
 * rm_refine_workspace_bytes.  Asynchronous on `stream`.
 * Errors: RM_EINVAL (null pointer, invalid index), RM_ESIZE (n_reads < 1,
 * k_fetch outside 1..RM_MAX_KFETCH, radius outside 0..RM_REFINE_MAX_RADIUS,
 * k outside 1..min(RM_MAX_KFETCH, k_fetch (2 radius + 1)), ws too small,
 * 2^31 or more step-1 windows). */
int rm_refine(const rm_index* coarse, const uint8_t* d_ref, const uint8_t* d_seq,
              const int64_t* d_off, int32_t n_reads, int32_t k_fetch, const int32_t* d_cand_idx,
              int32_t radius, int32_t k, int32_t* d_top_idx, float* d_top_score, void* d_ws,
              size_t ws_bytes, void* stream);

/* ---- batching: several (index, read batch) groups in one launch -------------
 * Reads of uneven length are mapped by bucketing them by head length (§2.9:
 * strings of different lengths are only compared at one window length), one
 * index per bucket length, and scoring every bucket's reads against its index
 * in ONE persistent launch (grouped work queue), followed by one merge per
 * group.  The sequence encode -> score -> rescore may be captured in a HIP
 * graph with rm_capture_begin / rm_capture_end and replayed with
 * rm_graph_launch. */

#define RM_MAX_GROUPS 8

/* Tile shape of the scoring kernel; zero fields select the library default. */
typedef struct rm_tuning {
  int32_t read_tile;   /* reads per block: 0, 128 or 256 (256 is not available for
                          FP32) */
  int32_t chunk_tiles; /* 64-window units per work item: 0 or >= 1 */
} rm_tuning;

/* Assign each read to the longest bucket length not above its length (host
 * memory; a pure CPU helper).  h_off: n_reads+1 offsets; bucket_len: n_buckets
 * strictly increasing lengths.  Writes h_bucket[n_reads] (the bucket index, or
 * -1 for a read shorter than bucket_len[0]) and h_count[n_buckets].
 * Errors: RM_EINVAL (null pointer, lengths not increasing), RM_ESIZE. */
int rm_bucket_reads(const int64_t* h_off, int32_t n_reads, const int32_t* bucket_len,
                    int32_t n_buckets, int32_t* h_bucket, int32_t* h_count);

/* Workspace bytes of rm_score_topk_groups; 0 if invalid.  idx and n_reads are
 * host arrays of n_groups entries; tune may be NULL. */
size_t rm_score_groups_workspace_bytes(const rm_index* idx, int32_t n_groups,
                                       const int32_t* n_reads, int32_t k_fetch,
                                       const rm_tuning* tune);

/* rm_score_topk for n_groups (index, read batch) pairs in one persistent launch
 * (§3.1 per group).  idx, d_read_emb, d_read_scale, n_reads, d_cand_idx and
 * d_cand_score are HOST arrays of n_groups entries (the entries are device
 * pointers); d_read_scale may be NULL unless the precision is FP8.  All groups
 * share one precision and k_fetch.  Output per group as rm_score_topk.
 * Errors: RM_EINVAL (null pointer, mixed precisions), RM_ESIZE (n_groups outside
 * 1..RM_MAX_GROUPS, a group without reads, k_fetch out of range, ws too small),
 * RM_EUNSUPPORTED (a tuning the kernels do not implement, or an index of
 * 1,024 components: those are scored by rm_score_topk only). */
int rm_score_topk_groups(const rm_index* idx, int32_t n_groups, const void* const* d_read_emb,
                         const float* const* d_read_scale, const int32_t* n_reads,
                         int32_t k_fetch, int32_t* const* d_cand_idx,
                         float* const* d_cand_score, void* d_ws, size_t ws_bytes,
                         const rm_tuning* tune, void* stream);

/* Autotuner: times candidate tile shapes of rm_score_topk_groups on these very
 * inputs (each candidate once after a warm-up run, with HIP events; the stream
 * is synchronised, so do not call it while capturing) and returns the fastest
 * in *best (and its time in *best_ms if not NULL).  Candidates whose workspace
 * exceeds ws_bytes are skipped.  If cache_path is not NULL, a previous result
 * for the same device architecture, precision, k_fetch and group shapes is
 * returned from that file without timing, and a new result is appended to it
 * (one JSON object per line).  The outputs hold the last candidate's results.
 * Errors: as rm_score_topk_groups; RM_EHIP if timing fails. */
int rm_autotune_score(const rm_index* idx, int32_t n_groups, const void* const* d_read_emb,
                      const float* const* d_read_scale, const int32_t* n_reads, int32_t k_fetch,
                      int32_t* const* d_cand_idx, float* const* d_cand_score, void* d_ws,
                      size_t ws_bytes, const char* cache_path, rm_tuning* best, float* best_ms,
                      void* stream);

/* HIP graph capture of a sequence of rm_* calls on one stream (which must not
 * be the null stream).  Between begin and end the calls are recorded, not run;
 * they enqueue kernels only (no allocation, copy or memset).  rm_capture_end
 * instantiates the graph; rm_graph_launch replays it on a stream;
 * rm_graph_destroy frees it (host objects only).  Errors: RM_EINVAL, RM_EHIP. */
typedef struct rm_graph_s* rm_graph;
int rm_capture_begin(void* stream);
int rm_capture_end(void* stream, rm_graph* out);
int rm_graph_launch(rm_graph graph, void* stream);
int rm_graph_destroy(rm_graph graph);

/* ---- learned angle offsets ------------------------------------------------
 * Not in the paper, which notes that token definitions, initial encodings or
 * rotations could be altered (§2.10).  Tokens are 9-mers at locations
 * p = 0..n-9 (s-mer locations, §2.1); the middle letter L selects the
 * component; the 8 flanking letters, one-hot (32 inputs), feed
 * o = W2 relu(W1 x + b1) + b2 (128 outputs = 4 letters x 32 factors); the token
 * adds exp(i (theta_k p + o[L*32 + k])) to component (k, L), theta_k =
 * 2 pi (k+1) / N with N the nominal length (§2.2).  With W2 = b2 = 0 this is
 * the plain encoding of w[4 .. n-4).  Parameters: W1 [64][32], b1 [64],
 * W2 [128][64], b2 [128], row-major FP32 (RM_LEARNED_PARAMS values).
 * Training: fidelity (§2.4) of string pairs, pairwise logistic ranking loss
 * softplus(-(F_i - F_j)/0.05) averaged over pairs with Levenshtein label
 * d_i < d_j (§1), Adam (beta 0.9 / 0.999, eps 1e-8). */

#define RM_LEARNED_PARAMS 10432
#define RM_LEARNED_MAX_LEN 256    /* letters of a string the learned kernels use */
#define RM_LEARNED_MAX_PAIRS 1024 /* pairs per training step */

/* Workspace bytes of rm_learned_train_step / rm_learned_gradient for n_pairs
 * pairs; 0 if n_pairs is outside 2..RM_LEARNED_MAX_PAIRS. */
size_t rm_learned_workspace_bytes(int32_t n_pairs);

/* Encodings of n_strings strings (string s = d_seq[d_off[s] .. d_off[s+1]),
 * device memory) into d_c [n_strings][256] floats (component k*4 + letter,
 * re/im interleaved), FP32, unnormalised.  d_params non-null: the learned
 * encoding above, of the first RM_LEARNED_MAX_LEN letters.  d_params null: the
 * plain encoding (§2.2, s = 1, f_k = k) of the whole string, the baseline the
 * learned one is compared with.  nominal_len is N of the phases.
 * Errors: RM_EINVAL (null pointer), RM_ESIZE (n_strings < 1, nominal_len < 1). */
int rm_learned_encode(const float* d_params, const uint8_t* d_seq, const int64_t* d_off,
                      int32_t n_strings, int32_t nominal_len, float* d_c, void* stream);

/* Fidelity (§2.4) of pairs of encodings: d_F[i] = F(d_ca[i], d_cb[i]), rows of
 * 256 floats as written by rm_learned_encode; 0 if either vector is zero.
 * Errors: RM_EINVAL, RM_ESIZE (n_pairs < 1). */
int rm_pair_fidelity(const float* d_ca, const float* d_cb, int32_t n_pairs, float* d_F,
                     void* stream);

/* One Adam step of the network on n_pairs pairs (a_i, b_i) = (d_a[d_aoff[i] ..
 * d_aoff[i+1]), d_b[d_boff[i] .. d_boff[i+1])) with labels d_ld[i] (edit
 * distances; only their order matters).  d_state = [params | m | v | step],
 * 3 * RM_LEARNED_PARAMS + 1 floats of device memory owned by the caller (start
 * with m = v = step = 0); the step count lives there, so a captured sequence
 * of calls can be replayed.  *d_loss (device) receives the batch loss before
 * the update.  d_ws: ws_bytes >= rm_learned_workspace_bytes(n_pairs).
 * Errors: RM_EINVAL (null pointer), RM_ESIZE (n_pairs outside
 * 2..RM_LEARNED_MAX_PAIRS, nominal_len < 1, workspace too small). */
int rm_learned_train_step(float* d_state, float lr, const uint8_t* d_a, const int64_t* d_aoff,
                          const uint8_t* d_b, const int64_t* d_boff, const int32_t* d_ld,
                          int32_t n_pairs, int32_t nominal_len, void* d_ws, size_t ws_bytes,
                          float* d_loss, void* stream);

/* The loss and its gradient with respect to the parameters (no update):
 * d_grad [RM_LEARNED_PARAMS], *d_loss.  Arguments and errors as above. */
int rm_learned_gradient(const float* d_params, const uint8_t* d_a, const int64_t* d_aoff,
                        const uint8_t* d_b, const int64_t* d_boff, const int32_t* d_ld,
                        int32_t n_pairs, int32_t nominal_len, void* d_ws, size_t ws_bytes,
                        float* d_grad, float* d_loss, void* stream);

/* ---- mapping with the learned encoding --------------------------------------
 * Inference in BF16 (weights and hidden values rounded to bfloat16, nearest
 * even; FP32 accumulation and biases).  The token offsets of a letter string
 * are computed once (a token's offsets depend on its 9 letters only); the
 * encoders and the FP32 rescore then use them in place of the network.
 * Window and read-head encodings hold the tokens at locations 0..N-9 of the N
 * letters (N >= 9); a slide of the rolling encoder (§3.4) removes the token at
 * the old start and adds the one at location N-9.  The scoring calls
 * (rm_score_topk, rm_score_topk_groups) are unchanged. */

/* Bytes of the token offsets of a string of n_letters letters:
 * (n_letters - 8) * 32 floats; 0 if n_letters < 9. */
size_t rm_delta_bytes(int64_t n_letters);

/* Token offsets d_delta[t][k] (row-major, FP32, 16-byte aligned) for the
 * tokens t = 0..n_letters-9 of d_seq: the middle letter's 32 network outputs
 * (0 if it is not a code 0..3).  For a concatenation of reads, rows whose
 * token crosses a read boundary are computed but never used.
 * Errors: RM_EINVAL (null or misaligned pointer), RM_ESIZE (n_letters < 9). */
int rm_mlp_infer(const float* d_params, const uint8_t* d_seq, int64_t n_letters, float* d_delta,
                 void* stream);

/* As rm_encode_reference, with the learned encoding; d_ref_delta = the token
 * offsets of d_ref (rm_mlp_infer over the reference), caller-owned, read
 * during this call only.  Errors as rm_encode_reference, plus RM_EINVAL
 * (null d_ref_delta), RM_ESIZE (window_len < 9) and RM_EUNSUPPORTED (token
 * parameters: the learned encoding has its own 9-letter tokens). */
int rm_encode_reference_learned(const uint8_t* d_ref, int64_t ref_len, const rm_params* p,
                                const float* d_ref_delta, void* d_buf, size_t buf_bytes,
                                rm_index* out, void* stream);

/* As rm_encode_reads, with the learned encoding of each read head;
 * d_read_delta = the token offsets of d_seq (rows indexed by positions in
 * d_seq).  Errors as rm_encode_reads, plus RM_EINVAL (null d_read_delta) and
 * RM_EUNSUPPORTED (a token index). */
int rm_encode_reads_learned(const rm_index* idx, const uint8_t* d_seq, const int64_t* d_off,
                            int32_t n_reads, const float* d_read_delta, void* d_read_emb,
                            float* d_read_scale, void* stream);

/* As rm_rescore, recomputing the fidelities in FP32 from the letters and the
 * token offsets of the reference and of the reads.  Errors as rm_rescore,
 * plus RM_EUNSUPPORTED (a token index). */
int rm_rescore_learned(const rm_index* idx, const uint8_t* d_ref, const float* d_ref_delta,
                       const uint8_t* d_seq, const int64_t* d_off, const float* d_read_delta,
                       int32_t n_reads, int32_t k_fetch, const int32_t* d_cand_idx, int32_t k,
                       int32_t* d_top_idx, float* d_top_score, void* stream);

/* Exact Levenshtein distance (unit costs) of n pairs (a_i, b_i), device
 * memory, into d_out[i] (int32): the labels of the ranking loss and the
 * reference for rank correlations.  Letters must be codes 0..3 (any other code
 * matches nothing, itself included).  The shorter string of a pair may have at
 * most 256 letters; a longer one gives -1.  Errors: RM_EINVAL, RM_ESIZE (n < 1 or
 * n > 2^31 * 256 - 256). */
int rm_levenshtein(const uint8_t* d_a, const int64_t* d_aoff, const uint8_t* d_b,
                   const int64_t* d_boff, int64_t n, int32_t* d_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ROTORMAP_H */
