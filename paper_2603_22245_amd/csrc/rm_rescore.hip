// FP32 rescore of each read's candidate windows (plain and learned encodings).
//
// The candidates come from the low-precision product; their fidelities are
// recomputed from the letters -- never from the stored index -- in FP32: the
// read head's and each candidate window's RoPE vector are direct sums of the
// FP32-rounded angle table (§2.1-§2.2), and F = |<x|c>|^2 / (X C) (§2.4).
// The candidates are then ordered by (F desc, window id asc) and the k best
// kept.  Lane layout of the per-string results as in the encoders (lane l owns
// factor l/2 and letters 2(l&1), 2(l&1)+1).
//
// Plain encoding: one wavefront per read.  The encodings of the read head and
// of its candidate windows are one matrix product: rows (string, letter) of
// one-hot indicators [letter at position p], times the FP32 phase table
// [p][factor] (§2.1-§2.2: component (k, L) sums the phases of the positions
// holding L).  The table is split exactly into three bfloat16 parts (x = hi +
// mid + lo) and the indicators are exact in bfloat16, so three bf16 MFMAs with
// FP32 accumulation reproduce the FP32 direct sums up to the order of FP32
// additions; each table row is read once per read instead of once per string.
#include "rm_bf16.h"
#include "rm_internal.h"
#include "rm_tokens.h"

namespace rm {

namespace {

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int d) {
  uint32_t lo = __shfl_xor((uint32_t)v, d, 64);
  uint32_t hi = __shfl_xor((uint32_t)(v >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}

// FP32 direct sum over T tokens of a string whose token offsets are rows
// drow[p]: token p adds phase32[p] exp(i delta) to component (k, str[p+4]).
// A range of tokens is summed by advancing str, drow and phase32 together.
__device__ __forceinline__ void direct_sum32_learned(const uint8_t* __restrict__ str, int T,
                                                     const float* __restrict__ drow,
                                                     const float2* __restrict__ phase32, int lane,
                                                     float2& a0, float2& a1) {
  const int k = lane >> 1, h = lane & 1;
  const int L0 = 2 * h, L1 = 2 * h + 1;
  a0 = make_float2(0.f, 0.f);
  a1 = make_float2(0.f, 0.f);
  for (int pb = 0; pb < T; pb += 64) {
    int mine = (pb + lane < T) ? (int)str[pb + lane + 4] : 255;
    int cnt = min(64, T - pb);
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      float2 ph[8];
      float d[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int p = min(pb + i0 + u, T - 1);
        ph[u] = phase32[(int64_t)p * kM + k];
        d[u] = drow[(int64_t)p * 32 + k];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int L = __builtin_amdgcn_readlane(mine, i0 + u);
        float sn, cs;
        __sincosf(d[u], &sn, &cs);  // hardware sin/cos: ~1e-6 for offsets of a few radians
        const float2 e = cmul(ph[u], make_float2(cs, sn));
        a0.x += (L == L0) ? e.x : 0.f;
        a0.y += (L == L0) ? e.y : 0.f;
        a1.x += (L == L1) ? e.x : 0.f;
        a1.y += (L == L1) ? e.y : 0.f;
      }
    }
  }
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Bitonic sort of one key per lane, descending over the 64 lanes, then the
// first k keys as (window id, F) -- empty keys and F = 0 give (-1, 0).
__device__ __forceinline__ void sort_and_write(uint64_t key, int lane, int64_t r, int k,
                                               int32_t* __restrict__ top_idx,
                                               float* __restrict__ top_score) {
#pragma unroll
  for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
    for (int d = kk >> 1; d > 0; d >>= 1) {
      uint64_t other = shfl_xor64(key, d);
      bool desc_block = (lane & kk) == 0;
      bool lower = (lane & d) == 0;
      uint64_t mx = key > other ? key : other;
      uint64_t mn = key > other ? other : key;
      key = (lower == desc_block) ? mx : mn;
    }
  }
  if (lane < k) write_list_entry(key, &top_idx[r * k + lane], &top_score[r * k + lane]);
}

// Plain rescore, one wavefront per read (four per block).  Strings: s = 0 is
// the read head, s = 1 .. k_fetch the candidates, taken in passes of 8 RB:
// RB blocks of 32 rows hold the rows (s, L), row = 4 (s - s0) + L, of the
// pass's strings s0 .. s0 + 8 RB - 1 (the head, in the first pass, stays in
// registers for the later ones).  Positions go 64 at a time: the block splits
// that chunk of the table into its three bfloat16 parts in LDS, each wavefront
// stages its strings' letters, then four steps of 16 positions take
// 32x32x16 bf16 MFMAs: A[row = lane % 32][p] = 2 [letter == L] for the eight
// positions p = 16 st + 8 (lane / 32) + 0..7 (2 keeps one byte of the bf16
// pattern; the sums are halved at the end, exactly), B the table part's
// [p][col = lane % 32] for the two 32-column blocks of the 64 table reals.
template <int RB>
__global__ __launch_bounds__(256) void rescore_mfma_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride,
    const float* __restrict__ tab, const uint8_t* __restrict__ seq,
    const int64_t* __restrict__ off, int32_t R, int k_fetch, const int32_t* __restrict__ cand,
    int k, int32_t* __restrict__ top_idx, float* __restrict__ top_score) {
  constexpr int SMAX = 8 * RB;
  // letters 0..3, 4 for none (past N, a short head, an invalid candidate, a code above 3)
  __shared__ __attribute__((aligned(16))) uint8_t letters_all[4][SMAX][64];
  // the table chunk's parts: [part][column block][8 positions][column] of 8 bf16
  __shared__ u32x4 tparts[3][2][8][32];
  __shared__ float mat_all[4][32][2 * kM + 1];  // one row block of the product
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r = (int64_t)blockIdx.x * 4 + wave;
  const bool active = r < R;  // inactive wavefronts still stage the table
  uint8_t(*letters)[64] = letters_all[wave];
  float(*mat)[2 * kM + 1] = mat_all[wave];
  const int S = 1 + k_fetch;
  const int64_t start = active ? off[r] : 0;
  const bool head_ok = active && off[r + 1] - start >= N;
  const int half = lane >> 5, col = lane & 31;
  const int kf = lane >> 1, h = lane & 1;
  // byte lookup: letter b -> 0x40 (the high byte of bf16 2.0) when b is this
  // lane's row letter (row & 3 = col & 3), else 0
  const uint32_t onehot_tab = 0x40u << (8 * (col & 3));
  float2 x0 = make_float2(0.f, 0.f), x1 = make_float2(0.f, 0.f);
  float X = 0.f;
  bool xdeg = true;
  uint64_t mykey = 0;

  for (int s0 = 0; s0 < S; s0 += SMAX) {
    const int SP = min(SMAX, S - s0);  // strings of this pass
    f32x16 acc[RB][2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb][0] = acc[rb][1] = f32x16{};

    for (int pb = 0; pb < N; pb += 64) {
      __syncthreads();  // the previous chunk's table parts and letters are read
      stage_table_parts(tab, pb, N, tparts, threadIdx.x, 256);
      // this wavefront's strings: the 64 letters at positions pb .. pb+63
      if (active) {
        for (int sl = 0; sl < SMAX; ++sl) {
          const int sx = s0 + sl;
          const uint8_t* base = nullptr;
          if (sl < SP) {
            if (sx == 0) {
              if (head_ok) base = seq + start;
            } else {
              const int32_t j = cand[r * k_fetch + sx - 1];
              if (j >= 0 && j < W) base = ref + (int64_t)j * stride;
            }
          }
          const int L = (base != nullptr && pb + lane < N) ? (int)base[pb + lane] : 4;
          letters[sl][lane] = (uint8_t)min(L, 4);
        }
      }
      __syncthreads();
      if (active) {
        const int steps = min(4, (N - pb + 15) >> 4);
        for (int st = 0; st < steps; ++st) {
          bf16x8 b[3][2];
#pragma unroll
          for (int pt = 0; pt < 3; ++pt)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
              b[pt][cb] = __builtin_bit_cast(bf16x8, tparts[pt][cb][2 * st + half][col]);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            // row rb*32 + col: string rb*8 + col/4, letter col & 3
            const uint2 w = *reinterpret_cast<const uint2*>(&letters[rb * 8 + (col >> 2)][16 * st + 8 * half]);
            const bf16x8 a = onehot_fragment(w, onehot_tab);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
              for (int pt = 2; pt >= 0; --pt)  // small parts first
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[pt][cb], acc[rb][cb], 0, 0, 0);
          }
        }
      }
    }

    if (!active) continue;  // (no barrier below)
    // ---- per string: components of this lane (factor kf, letters 2h, 2h+1)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      // result block: lane holds column cb*32 + col of rows 8 (v/4) + 4 half + v%4;
      // the indicators were 2, so the sums are halved (exactly)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          mat[8 * (v >> 2) + 4 * half + (v & 3)][cb * 32 + col] = 0.5f * acc[rb][cb][v];
      __builtin_amdgcn_wave_barrier();
      for (int sl = 0; sl < 8; ++sl) {
        const int sx = s0 + rb * 8 + sl;
        if (rb * 8 + sl >= SP) break;
        const float2 c0 = make_float2(mat[4 * sl + 2 * h][2 * kf], mat[4 * sl + 2 * h][2 * kf + 1]);
        const float2 c1 = make_float2(mat[4 * sl + 2 * h + 1][2 * kf], mat[4 * sl + 2 * h + 1][2 * kf + 1]);
        if (sx == 0) {
          x0 = c0;
          x1 = c1;
          X = wave_sum(x0.x * x0.x + x0.y * x0.y + x1.x * x1.x + x1.y * x1.y);
          xdeg = X < kDegenerateRel * (float)N;
          continue;
        }
        const int e = sx - 1;
        const int32_t j = cand[r * k_fetch + e];
        if (j < 0 || j >= W) continue;  // uniform: stays an empty key
        const float C = wave_sum(c0.x * c0.x + c0.y * c0.y + c1.x * c1.x + c1.y * c1.y);
        // <x|c> = sum conj(x) c
        const float ipr = wave_sum(x0.x * c0.x + x0.y * c0.y + x1.x * c1.x + x1.y * c1.y);
        const float ipi = wave_sum(x0.x * c0.y - x0.y * c0.x + x1.x * c1.y - x1.y * c1.x);
        const bool deg = xdeg || C < kDegenerateRel * (float)N;
        const float F = deg ? 0.f : (ipr * ipr + ipi * ipi) / (X * C);
        const uint32_t hi = __float_as_uint(F) + 1u;
        if (lane == e) mykey = ((uint64_t)hi << 32) | (0xffffffffu - (uint32_t)j);
      }
      __builtin_amdgcn_wave_barrier();  // before the next block overwrites mat
    }
  }  // passes
  if (active) sort_and_write(mykey, lane, r, k, top_idx, top_score);
}

// Learned encoding, with the token offsets of the reference (rows = reference
// positions) and of the reads (rows = positions in seq).  Its phases depend
// on each string's tokens, so there is no table shared by the strings to
// contract with: every string is its own direct sum.
//
// One block of four wavefronts per read: each wavefront sums a quarter of the
// read head (the quarters are added in a fixed order), then scores every
// fourth candidate; wavefront 0 sorts the keys.
constexpr int kRescoreWaves = 4;

__global__ __launch_bounds__(64 * kRescoreWaves) void rescore_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride,
    const float2* __restrict__ phase32, const uint8_t* __restrict__ seq,
    const int64_t* __restrict__ off, int32_t R, int k_fetch, const int32_t* __restrict__ cand,
    int k, int32_t* __restrict__ top_idx, float* __restrict__ top_score,
    const float* __restrict__ ref_delta, const float* __restrict__ read_delta) {
  __shared__ float4 part[kRescoreWaves][64];
  __shared__ uint64_t keys[RM_MAX_KFETCH];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r = blockIdx.x;
  const int64_t start = off[r];
  const int64_t len = off[r + 1] - start;
  const int T = N - 8;  // tokens of an encoding

  // ---- read head, a quarter per wavefront
  float2 x0 = make_float2(0.f, 0.f), x1 = make_float2(0.f, 0.f);
  if (len >= N) {
    const int q0 = wave * T / kRescoreWaves, q1 = (wave + 1) * T / kRescoreWaves;
    direct_sum32_learned(seq + start + q0, q1 - q0, read_delta + (start + q0) * 32,
                         phase32 + (int64_t)q0 * kM, lane, x0, x1);
  }
  part[wave][lane] = make_float4(x0.x, x0.y, x1.x, x1.y);
  __syncthreads();
  {
    float4 v = part[0][lane];
#pragma unroll
    for (int w = 1; w < kRescoreWaves; ++w) {
      const float4 u = part[w][lane];
      v.x += u.x; v.y += u.y; v.z += u.z; v.w += u.w;
    }
    x0 = make_float2(v.x, v.y);
    x1 = make_float2(v.z, v.w);
  }
  const float X = wave_sum(x0.x * x0.x + x0.y * x0.y + x1.x * x1.x + x1.y * x1.y);
  const bool xdeg = X < kDegenerateRel * (float)N;

  // ---- candidates e = wave, wave + 4, ...
  for (int e = wave; e < k_fetch; e += kRescoreWaves) {
    const int32_t j = cand[r * k_fetch + e];
    uint64_t key = 0;
    if (j >= 0 && j < W) {  // uniform per wavefront
      float2 c0, c1;
      direct_sum32_learned(ref + (int64_t)j * stride, T, ref_delta + (int64_t)j * stride * 32,
                           phase32, lane, c0, c1);
      float C = wave_sum(c0.x * c0.x + c0.y * c0.y + c1.x * c1.x + c1.y * c1.y);
      // <x|c> = sum conj(x) c
      float ipr = wave_sum(x0.x * c0.x + x0.y * c0.y + x1.x * c1.x + x1.y * c1.y);
      float ipi = wave_sum(x0.x * c0.y - x0.y * c0.x + x1.x * c1.y - x1.y * c1.x);
      bool deg = xdeg || C < kDegenerateRel * (float)N;
      float F = deg ? 0.f : (ipr * ipr + ipi * ipi) / (X * C);
      uint32_t hi = __float_as_uint(F) + 1u;
      key = ((uint64_t)hi << 32) | (0xffffffffu - (uint32_t)j);
    }
    if (lane == 0) keys[e] = key;
  }
  __syncthreads();
  if (wave != 0) return;

  sort_and_write(lane < k_fetch ? keys[lane] : 0, lane, r, k, top_idx, top_score);
}

// Token encodings (§2.1 s-mers, §2.6 compact versions; lane layout of
// rm_tokens.h): the block layout of rescore_kernel, with FP32 direct sums over
// the tokens at locations 0..N-s by class.
__global__ __launch_bounds__(64 * kRescoreWaves) void rescore_tokens_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride, int s, int m, int n_class,
    const float2* __restrict__ phase32, const uint8_t* __restrict__ table,
    const uint8_t* __restrict__ seq, const int64_t* __restrict__ off, int32_t R, int k_fetch,
    const int32_t* __restrict__ cand, int k, int32_t* __restrict__ top_idx,
    float* __restrict__ top_score) {
  __shared__ float4 part[kRescoreWaves][64];
  __shared__ uint64_t keys[RM_MAX_KFETCH];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r = blockIdx.x;
  const int64_t start = off[r];
  const int64_t len = off[r + 1] - start;
  const int T = N - s + 1;  // tokens of an encoding
  const int kf = 2 * lane / n_class, c0 = 2 * lane - kf * n_class;

  // ---- read head, a quarter of its token locations per wavefront
  float2 x0 = make_float2(0.f, 0.f), x1 = make_float2(0.f, 0.f);
  if (len >= N) {
    const int q0 = wave * T / kRescoreWaves, q1 = (wave + 1) * T / kRescoreWaves;
    direct_sum_tokens(seq + start + q0, q1 - q0, s, table, phase32 + (int64_t)q0 * m, m, kf, c0,
                      lane, x0, x1);
  }
  part[wave][lane] = make_float4(x0.x, x0.y, x1.x, x1.y);
  __syncthreads();
  {
    float4 v = part[0][lane];
#pragma unroll
    for (int w = 1; w < kRescoreWaves; ++w) {
      const float4 u = part[w][lane];
      v.x += u.x; v.y += u.y; v.z += u.z; v.w += u.w;
    }
    x0 = make_float2(v.x, v.y);
    x1 = make_float2(v.z, v.w);
  }
  const float X = wave_sum(x0.x * x0.x + x0.y * x0.y + x1.x * x1.x + x1.y * x1.y);
  const bool xdeg = X < kDegenerateRel * (float)N;

  // ---- candidates e = wave, wave + 4, ...
  for (int e = wave; e < k_fetch; e += kRescoreWaves) {
    const int32_t j = cand[r * k_fetch + e];
    uint64_t key = 0;
    if (j >= 0 && j < W) {  // uniform per wavefront
      float2 c0v, c1v;
      direct_sum_tokens(ref + (int64_t)j * stride, T, s, table, phase32, m, kf, c0, lane, c0v,
                        c1v);
      const float C = wave_sum(c0v.x * c0v.x + c0v.y * c0v.y + c1v.x * c1v.x + c1v.y * c1v.y);
      // <x|c> = sum conj(x) c
      const float ipr = wave_sum(x0.x * c0v.x + x0.y * c0v.y + x1.x * c1v.x + x1.y * c1v.y);
      const float ipi = wave_sum(x0.x * c0v.y - x0.y * c0v.x + x1.x * c1v.y - x1.y * c1v.x);
      const bool deg = xdeg || C < kDegenerateRel * (float)N;
      const float F = deg ? 0.f : (ipr * ipr + ipi * ipi) / (X * C);
      key = ((uint64_t)(__float_as_uint(F) + 1u) << 32) | (0xffffffffu - (uint32_t)j);
    }
    if (lane == 0) keys[e] = key;
  }
  __syncthreads();
  if (wave != 0) return;

  sort_and_write(lane < k_fetch ? keys[lane] : 0, lane, r, k, top_idx, top_score);
}

}  // namespace

hipError_t launch_rescore(const rm_index& idx, const uint8_t* ref, const uint8_t* seq,
                          const int64_t* off, int32_t n_reads, int32_t k_fetch,
                          const int32_t* cand_idx, int32_t k, int32_t* top_idx, float* top_score,
                          hipStream_t s, const float* ref_delta, const float* read_delta) {
  if (ref_delta == nullptr) {
    // rows 4 (1 + k_fetch) in blocks of 32, at most 5 blocks (40 strings) a pass
    const int rb = min(5, (1 + k_fetch + 7) / 8);
    auto kern = rb <= 1 ? rescore_mfma_kernel<1> : rb == 2 ? rescore_mfma_kernel<2>
              : rb == 3 ? rescore_mfma_kernel<3> : rb == 4 ? rescore_mfma_kernel<4>
                                                  : rescore_mfma_kernel<5>;
    hipLaunchKernelGGL(kern, dim3((unsigned)(((int64_t)n_reads + 3) / 4)), dim3(256), 0, s, ref,
                       idx.n_windows, idx.p.window_len, idx.p.stride,
                       reinterpret_cast<const float*>(idx.d_phase32), seq, off, n_reads, k_fetch,
                       cand_idx, k, top_idx, top_score);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(rescore_kernel, dim3((unsigned)n_reads), dim3(64 * kRescoreWaves), 0, s, ref,
                     idx.n_windows,
                     idx.p.window_len, idx.p.stride, reinterpret_cast<const float2*>(idx.d_phase32),
                     seq, off, n_reads, k_fetch, cand_idx, k, top_idx, top_score, ref_delta,
                     read_delta);
  return hipGetLastError();
}

hipError_t launch_rescore_tokens(const rm_index& idx, const uint8_t* ref, const uint8_t* seq,
                                 const int64_t* off, int32_t n_reads, int32_t k_fetch,
                                 const int32_t* cand_idx, int32_t k, int32_t* top_idx,
                                 float* top_score, hipStream_t st) {
  const int s = idx.p.mer_len > 1 ? idx.p.mer_len : 1;
  hipLaunchKernelGGL(rescore_tokens_kernel, dim3((unsigned)n_reads), dim3(64 * kRescoreWaves), 0,
                     st, ref, idx.n_windows, idx.p.window_len, idx.p.stride, s, idx.p.n_freq,
                     128 / idx.p.n_freq, reinterpret_cast<const float2*>(idx.d_phase32),
                     idx.d_token_class, seq, off, n_reads, k_fetch, cand_idx, k, top_idx,
                     top_score);
  return hipGetLastError();
}

}  // namespace rm
