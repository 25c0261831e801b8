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
constexpr float kDegenerateRel = 1e-4f;    // squared norm < this * N -> zero vector
constexpr float kFp8Max = 448.0f;          // largest finite OCP e4m3 value

inline int elem_bytes(int precision) {
  return precision == RM_FP32 ? 4 : precision == RM_FP16 ? 2 : 1;
}

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  return v;
}

// Power-of-two scale s with maxabs / s <= 448 (the smallest such power), so that
// dividing by s is exact and nothing saturates.  maxabs == 0 gives 1.
__device__ __forceinline__ float fp8_pow2_scale(float maxabs) {
  if (!(maxabs > 0.f)) return 1.f;
  int e;
  float f = frexpf(maxabs / kFp8Max, &e);  // maxabs/448 = f * 2^e, f in [0.5, 1)
  // 2^(e-1) < maxabs/448 <= 2^e unless f == 0.5 exactly (then maxabs/448 = 2^(e-1))
  if (f == 0.5f) e -= 1;
  return ldexpf(1.f, e);
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

// ---------------------------------------------------------------- launchers

hipError_t launch_tables(const rm_params& p, double* phase64, float* phase32, float* step32,
                         hipStream_t s);

hipError_t launch_encode_reference(const uint8_t* ref, int64_t W, const rm_params& p,
                                   const double* phase64, const float* step32, void* emb,
                                   float* scale, float* norm2, hipStream_t s);

hipError_t launch_encode_reads(const rm_params& p, const double* phase64, const uint8_t* seq,
                               const int64_t* off, int32_t n_reads, void* emb, float* scale,
                               hipStream_t s);

struct ScorePlan {
  int reads_per_block;
  int read_tiles;
  int chunks;          // P: window chunks per read
  int64_t chunk_windows;
  int kp;              // list length kept per (read, chunk): 8, 16 or 32
  size_t thr_offset;   // byte offset of the shared per-read thresholds in the workspace
  size_t ws_bytes;
};

ScorePlan plan_score(int precision, int64_t W, int32_t n_reads, int32_t k_fetch);

hipError_t launch_score_topk(const rm_index& idx, const ScorePlan& plan, const void* read_emb,
                             const float* read_scale, int32_t n_reads, int32_t k_fetch,
                             int32_t* cand_idx, float* cand_score, void* ws, hipStream_t s);

hipError_t launch_rescore(const rm_index& idx, const uint8_t* ref, const uint8_t* seq,
                          const int64_t* off, int32_t n_reads, int32_t k_fetch,
                          const int32_t* cand_idx, int32_t k, int32_t* top_idx, float* top_score,
                          hipStream_t s);

}  // namespace rm
