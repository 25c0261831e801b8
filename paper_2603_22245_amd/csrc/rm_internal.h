// Internal declarations shared by the HIP translation units of librotormap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rotormap.h"

namespace rm {

constexpr int kLetters = 4;
constexpr int kM = RM_DIM;                 // factors per encoding (m)
constexpr int kComplex = kLetters * kM;    // 128 complex components
constexpr int kReal = 2 * kComplex;        // 256 reals per embedding row
constexpr int kRealReduced = 2 * 3 * kM;   // 192 reals per row of the letter-sum form
constexpr float kDegenerateRel = 1e-4f;    // squared norm < this * N -> zero vector
constexpr float kFp8Max = 448.0f;          // largest finite OCP e4m3 value
// FP8 window rows of 128 complex components are codes of 256 v (a common
// power of two).  Their scale s_j = 1 / |codes| then satisfies
// (256 s_j)^2 <= kFp8WindowBound: e4m3 rounds a normal value to within 2^-4
// relative and a subnormal one to within 2^-10, so over 256 reals of a unit
// vector |codes - 256 v| <= 2^-4 256 + 16 2^-10 = 16.015625 and
// |codes| >= 239.984375; (256 / 239.984375)^2 = 1.13792...
constexpr float kFp8WindowScale = 1.0f / 256.0f;
constexpr float kFp8WindowBound = 1.138f;

inline int elem_bytes(int precision) {
  return precision == RM_FP32 ? 4 : precision == RM_FP16 ? 2 : 1;
}

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Cross-lane move within rows of 16 lanes (DPP); every lane of the wavefront
// must be active.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

// Sum over the 64 lanes, returned in every lane: within each row of 16 lanes by
// DPP (xor 1, xor 2, half-row mirror, row mirror), then the four row sums in a
// fixed order.  Every lane must be active.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  const float a = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
  const float b = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
  const float c = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
  const float d = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
  return (a + b) + (c + d);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x141>(v));
  v = fmaxf(v, dpp<0x140>(v));
  const float a = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
  const float b = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
  const float c = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
  const float d = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
  return fmaxf(fmaxf(a, b), fmaxf(c, d));
}

// Maximum of non-negative floats over the 64 lanes, in every lane.  For
// non-negative floats the order of the bit patterns as unsigned integers is
// the numeric order, so the integer maximum needs none of the NaN handling of
// fmaxf.  Every lane must be active.
__device__ __forceinline__ float wave_max_nonneg(float v) {
  uint32_t u = __float_as_uint(v);
  u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, 0xB1, 0xf, 0xf, false));
  u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, 0x4E, 0xf, 0xf, false));
  u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, 0x141, 0xf, 0xf, false));
  u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, 0x140, 0xf, 0xf, false));
  const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)u, 0);
  const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)u, 16);
  const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)u, 32);
  const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)u, 48);
  return __uint_as_float(max(max(a, b), max(c, d)));
}

// Power-of-two scale s with maxabs / s <= 448 (the smallest such power), so that
// dividing by s is exact and nothing saturates.  maxabs == 0 gives 1.  With
// maxabs = m 2^E (m in [1, 2)) and 448 = 1.75 2^8, the exponent is E - 8 when
// m <= 1.75 and E - 7 otherwise: read off the float's bits, no rounding.
__device__ __forceinline__ float fp8_pow2_scale(float maxabs) {
  if (!(maxabs > 0.f)) return 1.f;
  const uint32_t b = __float_as_uint(maxabs);
  const int E = (int)(b >> 23) - 127;
  const int e = E - 8 + ((b & 0x7fffffu) > 0x600000u ? 1 : 0);
  if (E == -127 || e < -126 || e > 127) {  // subnormal or huge: the general route
    int x;
    float f = frexpf(maxabs / kFp8Max, &x);
    if (f == 0.5f) x -= 1;
    return ldexpf(1.f, x);
  }
  return __uint_as_float((uint32_t)(e + 127) << 23);
}

// 1 / s for a power of two s: exact.  Normal s with a normal reciprocal (the
// scales of unit rows, 2^-12 .. 2^-7) by exponent arithmetic, others by division.
__device__ __forceinline__ float pow2_reciprocal(float s) {
  const uint32_t ex = __float_as_uint(s) >> 23;
  return ex >= 2u && ex <= 252u ? __uint_as_float(0x7f000000u - __float_as_uint(s)) : 1.f / s;
}

// Two floats -> two OCP e4m3 bytes in the low half of the result, round to
// nearest even (gfx950 converts to the OCP format).
__device__ __forceinline__ uint32_t pack_fp8x2(float a, float b) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}

// Low two OCP e4m3 bytes of `w` -> two floats (exact).
__device__ __forceinline__ float2 unpack_fp8x2(uint32_t w) {
  auto v = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  return make_float2(v[0], v[1]);
}

// ---------------------------------------------------------------- shared device code

// One slide of the window state of this lane's components (k, 2h) and
// (k, 2h+1): rotate by `rot`, remove `uo` from the outgoing letter's component
// and add `ui` to the incoming one's.  o and n are wavefront-uniform letter
// codes; codes above 3 touch nothing.
__device__ __forceinline__ void slide(float2& c0, float2& c1, float2 rot, int o, int n, int h,
                                      float2 uo, float2 ui) {
  c0 = cmul(c0, rot);
  c1 = cmul(c1, rot);
  if ((o >> 1) != h) uo = make_float2(0.f, 0.f);
  if ((n >> 1) != h) ui = make_float2(0.f, 0.f);
  if (o & 1) {
    c1.x -= uo.x;
    c1.y -= uo.y;
  } else {
    c0.x -= uo.x;
    c0.y -= uo.y;
  }
  if (n & 1) {
    c1.x += ui.x;
    c1.y += ui.y;
  } else {
    c0.x += ui.x;
    c0.y += ui.y;
  }
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xf, 0xf, false);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t max64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Maximum over the 64 lanes, in every lane: within rows of 16 by DPP (xor 1,
// xor 2, half-row mirror, row mirror), then the four row maxima.  Every lane
// must be active.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  v = max64(v, dpp64<0xB1>(v));
  v = max64(v, dpp64<0x4E>(v));
  v = max64(v, dpp64<0x141>(v));
  v = max64(v, dpp64<0x140>(v));
  return max64(max64(readlane64(v, 0), readlane64(v, 16)), max64(readlane64(v, 32), readlane64(v, 48)));
}

// One entry of a ranked list from its 64-bit key (high word = float bits of F
// plus one, low word = ~window id).  Key 0 is an empty slot (fewer candidates
// than slots).  F = 0 means the read head or the window is the zero vector (a
// degenerate string, or a read shorter than N): that window is no location of
// the read (§3 asks for the read's position only if one exists).  Both are
// written as id -1 with score 0.
__device__ __forceinline__ void write_list_entry(uint64_t key, int32_t* __restrict__ idx,
                                                 float* __restrict__ score) {
  const uint32_t hi = (uint32_t)(key >> 32);
  const bool loc = hi > 1u;
  *idx = loc ? (int32_t)(0xffffffffu - (uint32_t)key) : -1;
  *score = loc ? __uint_as_float(hi - 1u) : 0.f;
}

// FP32 direct sum over letters [0, n) for this lane's two components (positions
// past n in the last group of 8 read letter code 255 and add nothing).
__device__ __forceinline__ void direct_sum32(const uint8_t* __restrict__ str, int n,
                                             const float2* __restrict__ phase32, int lane,
                                             float2& a0, float2& a1) {
  const int k = lane >> 1, h = lane & 1;
  const int L0 = 2 * h, L1 = 2 * h + 1;
  a0 = make_float2(0.f, 0.f);
  a1 = make_float2(0.f, 0.f);
  for (int pb = 0; pb < n; pb += 64) {
    int mine = (pb + lane < n) ? (int)str[pb + lane] : 255;
    int cnt = min(64, n - pb);
    // groups of 8 positions with their table loads in flight together
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      float2 e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) e[u] = phase32[(int64_t)min(pb + i0 + u, n - 1) * kM + k];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int L = __builtin_amdgcn_readlane(mine, i0 + u);
        a0.x += (L == L0) ? e[u].x : 0.f;
        a0.y += (L == L0) ? e[u].y : 0.f;
        a1.x += (L == L1) ? e[u].x : 0.f;
        a1.y += (L == L1) ? e[u].y : 0.f;
      }
    }
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_tables(const rm_params& p, double* phase64, float* phase32, float* step32,
                         hipStream_t s);
hipError_t launch_zero_word(uint32_t* p, hipStream_t s);

hipError_t launch_encode_reference(const uint8_t* ref, int64_t W, const rm_params& p,
                                   const double* phase64, const float* step32, void* emb,
                                   float* scale, float* norm2, hipStream_t s);

hipError_t launch_encode_reads(const rm_params& p, const float* phase32, const uint8_t* seq,
                               const int64_t* off, int32_t n_reads, void* emb, float* scale,
                               hipStream_t s);

constexpr int kMaxGroups = 8;

// One (index, read batch) pair of a scoring launch; passed by value in the
// kernel arguments.
// Per read, the scoring launch keeps kScoreSlots keys of windows from
// finished window chunks, slot = window id mod kScoreSlots: the slots always
// hold distinct windows, so the kp-th largest of them bounds the read's final
// kp-th best from below.
constexpr int kScoreSlots = 32;

// Rows of the letter-sum form (rm_params.reduced).
inline bool reduced_rows(const rm_params& p) { return p.reduced != 0; }

struct ScoreGroup {
  const uint8_t* index;      // [W][256] window embeddings
  const float* win_scale;    // [W]
  int64_t W;
  const uint8_t* reads;      // [R][2][256] read rows
  const float* read_scale;   // [R]
  int32_t R;
  int32_t read_tiles;
  int64_t chunk_windows;
  int32_t P;                 // window chunks
  int32_t item_begin;        // first work item of this group
  int32_t thin;              // 1: read tiles of half the block's reads (a group whose
                             // reads would leave most of a full tile empty)
  uint64_t* lists;           // [R][P][kp] keys
  uint32_t* gthr;            // [R] shared k-th-best per read
  uint64_t* gslot;           // [R][kScoreSlots] keys of finished chunks (slot = id mod kScoreSlots)
};

struct ScoreLaunch {
  ScoreGroup g[kMaxGroups];
  int32_t n_groups;
  int32_t total_items;
  int* counter;
};

struct Tuning {
  int read_tile;    // reads per block (128 or 256); 0 = default
  int chunk_tiles;  // 64-window units per work item; 0 = default
};

struct GroupPlan {
  int read_tiles;
  int thin;  // read tiles of half the launch's read tile
  int chunks;
  int64_t chunk_windows;
  size_t lists_offset;
  size_t thr_offset;
  size_t slot_offset;
};

struct ScorePlan {
  int kp;           // list length per (read, chunk): 8, 16 or 32
  int read_tile;    // reads per block
  int n_groups;
  GroupPlan g[kMaxGroups];
  int64_t total_items;
  size_t counter_offset;
  size_t ws_bytes;
  bool ok;
};

// Read-tile sizes the kernels implement for a precision and list length.
bool read_tile_ok(int precision, int kp, int read_tile);

ScorePlan plan_score(int precision, int n_groups, const int64_t* W, const int32_t* R, int k_fetch,
                     Tuning t);

hipError_t launch_score_topk(const rm_index* idx, const ScorePlan& plan,
                             const void* const* read_emb, const float* const* read_scale,
                             const int32_t* R, int k_fetch, int32_t* const* cand_idx,
                             float* const* cand_score, void* ws, hipStream_t s);

hipError_t launch_mlp_infer(const float* params, const uint8_t* seq, int64_t n_letters,
                            float* delta, hipStream_t s);
hipError_t launch_encode_reference_learned(const uint8_t* ref, int64_t W, const rm_params& p,
                                           const double* phase64, const float* phase32,
                                           const float* step32, const float* delta, void* emb,
                                           float* scale, float* norm2, hipStream_t s);
hipError_t launch_encode_reads_learned(const rm_params& p, const float* phase32,
                                       const uint8_t* seq, const int64_t* off, int32_t n_reads,
                                       const float* delta, void* emb, float* scale,
                                       hipStream_t s);

size_t learned_workspace_bytes(int32_t n_pairs);
hipError_t launch_learned_encode(const float* params, const uint8_t* seq, const int64_t* off,
                                 int32_t n_strings, int N, float* out, hipStream_t s);
hipError_t launch_pair_fidelity(const float* ca, const float* cb, int32_t n_pairs, float* F,
                                hipStream_t s);
hipError_t launch_learned_step(float* state, float lr, const uint8_t* a, const int64_t* aoff,
                               const uint8_t* b, const int64_t* boff, const int32_t* ld,
                               int32_t n_pairs, int N, void* ws, float* grad_out,
                               float* loss_out, hipStream_t s);
hipError_t launch_levenshtein(const uint8_t* a, const int64_t* aoff, const uint8_t* b,
                              const int64_t* boff, int64_t n, int32_t* out, hipStream_t s);

// per-fragment thresholds and the threshold regime (rm_thresh.hip)
struct ThresholdWs {
  size_t pool, keys, cand, cnt, fill, pool_n, total;  // byte offsets; total = size
};
ThresholdWs threshold_ws_layout(int32_t n_reads, int64_t capacity);
hipError_t launch_window_thresholds(const rm_index& idx, const uint8_t* ref, float err,
                                    int copies, int rank, uint32_t seed, float* thr,
                                    hipStream_t s);
hipError_t launch_score_threshold(const rm_index& idx, const uint8_t* ref,
                                  const void* read_emb, const float* read_scale,
                                  const uint8_t* seq, const int64_t* soff, int32_t R,
                                  const float* thr, float floor_f, int64_t* hit_off,
                                  int32_t* n_found, int32_t* hit_idx, float* hit_score,
                                  int64_t* total, int64_t capacity, void* ws, hipStream_t s);

hipError_t launch_correlation_score(const float* F, const float* err, int32_t n_rates,
                                    int32_t per, float* E, float* rmse, hipStream_t s);

hipError_t launch_reverse_complement(const uint8_t* seq, const int64_t* off, int32_t n_reads,
                                     int64_t n_letters, uint8_t* out, hipStream_t s);
hipError_t launch_merge_strands(const int32_t* fi, const float* ff, const int32_t* ri,
                                const float* rf, int32_t n_reads, int32_t k, float min_fidelity,
                                int32_t* top_idx, float* top_score, int8_t* top_strand,
                                int32_t* n_found, hipStream_t s);

size_t refine_workspace_bytes(int32_t n_reads, int32_t k_fetch, int32_t radius);
hipError_t launch_refine(const rm_index& coarse, const uint8_t* ref, const uint8_t* seq,
                         const int64_t* off, int32_t n_reads, int32_t k_fetch,
                         const int32_t* cand_idx, int32_t radius, int32_t k, int32_t* top_idx,
                         float* top_score, void* ws, hipStream_t s);

hipError_t launch_rescore(const rm_index& idx, const uint8_t* ref, const uint8_t* seq,
                          const int64_t* off, int32_t n_reads, int32_t k_fetch,
                          const int32_t* cand_idx, int32_t k, int32_t* top_idx, float* top_score,
                          hipStream_t s, const float* ref_delta = nullptr,
                          const float* read_delta = nullptr);

}  // namespace rm
