// Refinement around found locations (§3.4, "Increasing the accuracy").
//
// The product scores the windows of a coarse index (starts j*sigma).  Around
// each candidate window the step-1 windows with starts j*sigma - h .. j*sigma
// + h are scored exactly in FP32: the first one as a direct sum over its
// letters with the FP32 phase table (§2.1-§2.2), the next ones by sliding one
// letter at a time with the relations of §3.4 (every component turns by
// omega^-f, the outgoing letter's component loses omega^-f, the incoming
// letter's gains omega^{f (N-1)}).  The squared norm of each window is
// recomputed from its components rather than skipped, so every fidelity is
// the full F = |<x|c>|^2 / (X C) of §2.4.  The k best distinct starts over all
// of a read's neighbourhoods are kept, ordered by (F desc, start asc).
//
// Letter encoding: lane l owns factor l/2 and letters 2(l&1), 2(l&1)+1, as in
// the encoders.  Token encodings of 128 components (refine_tokens_kernel):
// lane l owns components 2l and 2l+1; a slide turns every component by
// omega^-f, takes omega^-f off the outgoing token's class (the token that
// started at location 0) and adds omega^{f (N-s)} to the incoming token's
// class (the token now at location N-s), the s-mer form of the same relations.
// The 1,024-component refinement sits with the other wide kernels.  The head's
// encoding is summed once per read in the same order as the rescore's
// (quarters added in a fixed order).
#include "rm_internal.h"
#include "rm_tokens.h"

namespace rm {

namespace {

// One block of four wavefronts per read: the read head is summed once, a
// quarter per wavefront (the quarters added in a fixed order), then wavefront
// w refines candidates w, w + 4, ...  Slot i of a candidate's span in `pool`
// receives the key of start lo + i; slots past the clamped neighbourhood (or
// of an invalid candidate) receive 0.
__global__ __launch_bounds__(256) void refine_kernel(
    const uint8_t* __restrict__ ref, int64_t W1, int N, int cstride, int64_t Wc,
    const float2* __restrict__ phase32, const float4* __restrict__ step32,
    const uint8_t* __restrict__ seq, const int64_t* __restrict__ off, int32_t R, int k_fetch,
    const int32_t* __restrict__ cand, int radius, uint64_t* __restrict__ pool) {
  __shared__ float4 part[4][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r = blockIdx.x;
  const int span = 2 * radius + 1;

  // ---- read head, a quarter of its letters per wavefront
  const int64_t start = off[r];
  float2 x0 = make_float2(0.f, 0.f), x1 = make_float2(0.f, 0.f);
  if (off[r + 1] - start >= N) {
    const int q0 = wave * N / 4, q1 = (wave + 1) * N / 4;
    direct_sum32(seq + start + q0, q1 - q0, phase32 + (int64_t)q0 * kM, lane, x0, x1);
  }
  part[wave][lane] = make_float4(x0.x, x0.y, x1.x, x1.y);
  __syncthreads();
  {
    float4 v = part[0][lane];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      const float4 u = part[w][lane];
      v.x += u.x; v.y += u.y; v.z += u.z; v.w += u.w;
    }
    x0 = make_float2(v.x, v.y);
    x1 = make_float2(v.z, v.w);
  }
  const float X = wave_sum(x0.x * x0.x + x0.y * x0.y + x1.x * x1.x + x1.y * x1.y);
  const bool xdeg = X < kDegenerateRel * (float)N;
  const int h = lane & 1;
  const float4 st = step32[lane >> 1];
  const float2 rot = make_float2(st.x, st.y);  // omega^-f
  const float2 inc = make_float2(st.z, st.w);  // omega^(f (N-1))

  for (int e = wave; e < k_fetch; e += 4) {
    uint64_t* out = pool + (r * k_fetch + e) * span;
    const int32_t j = cand[r * k_fetch + e];
    int64_t lo = 0, hi = -1;
    if (j >= 0 && j < Wc) {
      const int64_t c = (int64_t)j * cstride;
      lo = c - radius < 0 ? 0 : c - radius;
      hi = c + radius > W1 - 1 ? W1 - 1 : c + radius;
    }
    if (lane < span && lo + lane > hi) out[lane] = 0;
    if (hi < lo) continue;  // uniform
    float2 c0, c1;
    direct_sum32(ref + lo, N, phase32, lane, c0, c1);
    uint64_t mine = 0;
    for (int64_t s = lo; s <= hi; ++s) {
      const float C = wave_sum(c0.x * c0.x + c0.y * c0.y + c1.x * c1.x + c1.y * c1.y);
      // <x|c> = sum conj(x) c
      const float ipr = wave_sum(x0.x * c0.x + x0.y * c0.y + x1.x * c1.x + x1.y * c1.y);
      const float ipi = wave_sum(x0.x * c0.y - x0.y * c0.x + x1.x * c1.y - x1.y * c1.x);
      const bool deg = xdeg || C < kDegenerateRel * (float)N;
      const float F = deg ? 0.f : (ipr * ipr + ipi * ipi) / (X * C);
      if (lane == (int)(s - lo))
        mine = ((uint64_t)(__float_as_uint(F) + 1u) << 32) | (0xffffffffu - (uint32_t)s);
      // s + N <= hi - 1 + N <= W1 - 2 + N = ref_len - 1
      if (s < hi) slide(c0, c1, rot, (int)ref[s], (int)ref[s + N], h, rot, inc);
    }
    if (lane <= (int)(hi - lo)) out[lane] = mine;
  }
}

// refine_kernel for a token encoding of 128 components (n_class * m = 128).
__global__ __launch_bounds__(256) void refine_tokens_kernel(
    const uint8_t* __restrict__ ref, int64_t W1, int N, int cstride, int64_t Wc, int s, int m,
    int n_class, const float2* __restrict__ phase32, const float4* __restrict__ step32,
    const uint8_t* __restrict__ table, const uint8_t* __restrict__ seq,
    const int64_t* __restrict__ off, int32_t R, int k_fetch, const int32_t* __restrict__ cand,
    int radius, uint64_t* __restrict__ pool) {
  __shared__ float4 part[4][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r = blockIdx.x;
  const int span = 2 * radius + 1;
  const int T = N - s + 1;  // tokens of an encoding
  const int kf = 2 * lane / n_class, cl = 2 * lane - kf * n_class;

  // ---- read head, a quarter of its token locations per wavefront
  const int64_t start = off[r];
  float2 x0 = make_float2(0.f, 0.f), x1 = make_float2(0.f, 0.f);
  if (off[r + 1] - start >= N) {
    const int q0 = wave * T / 4, q1 = (wave + 1) * T / 4;
    direct_sum_tokens(seq + start + q0, q1 - q0, s, table, phase32 + (int64_t)q0 * m, m, kf, cl,
                      lane, x0, x1);
  }
  part[wave][lane] = make_float4(x0.x, x0.y, x1.x, x1.y);
  __syncthreads();
  {
    float4 v = part[0][lane];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      const float4 u = part[w][lane];
      v.x += u.x; v.y += u.y; v.z += u.z; v.w += u.w;
    }
    x0 = make_float2(v.x, v.y);
    x1 = make_float2(v.z, v.w);
  }
  const float X = wave_sum(x0.x * x0.x + x0.y * x0.y + x1.x * x1.x + x1.y * x1.y);
  const bool xdeg = X < kDegenerateRel * (float)N;
  const float4 st = step32[kf];
  const float2 rot = make_float2(st.x, st.y);  // omega^-f
  const float2 inc = make_float2(st.z, st.w);  // omega^(f (N-s))

  for (int e = wave; e < k_fetch; e += 4) {
    uint64_t* out = pool + (r * k_fetch + e) * span;
    const int32_t j = cand[r * k_fetch + e];
    int64_t lo = 0, hi = -1;
    if (j >= 0 && j < Wc) {
      const int64_t c = (int64_t)j * cstride;
      lo = c - radius < 0 ? 0 : c - radius;
      hi = c + radius > W1 - 1 ? W1 - 1 : c + radius;
    }
    if (lane < span && lo + lane > hi) out[lane] = 0;
    if (hi < lo) continue;  // uniform
    float2 c0, c1;
    direct_sum_tokens(ref + lo, T, s, table, phase32, m, kf, cl, lane, c0, c1);
    // lane i holds the classes of slide lo + i: the token leaving (at lo + i)
    // and the one entering (at lo + i + T, whose last letter lo + i + N <=
    // hi - 1 + N <= W1 - 2 + N = ref_len - 1)
    const int64_t tl = lo + lane;
    const int out_c = tl < hi ? token_class(ref + tl, s, table) : kNoToken;
    const int in_c = tl < hi ? token_class(ref + tl + T, s, table) : kNoToken;
    uint64_t mine = 0;
    for (int64_t t = lo; t <= hi; ++t) {
      const float C = wave_sum(c0.x * c0.x + c0.y * c0.y + c1.x * c1.x + c1.y * c1.y);
      // <x|c> = sum conj(x) c
      const float ipr = wave_sum(x0.x * c0.x + x0.y * c0.y + x1.x * c1.x + x1.y * c1.y);
      const float ipi = wave_sum(x0.x * c0.y - x0.y * c0.x + x1.x * c1.y - x1.y * c1.x);
      const bool deg = xdeg || C < kDegenerateRel * (float)N;
      const float F = deg ? 0.f : (ipr * ipr + ipi * ipi) / (X * C);
      if (lane == (int)(t - lo))
        mine = ((uint64_t)(__float_as_uint(F) + 1u) << 32) | (0xffffffffu - (uint32_t)t);
      if (t < hi) {
        // classes relative to this lane's first one: 0 or 1 is one of its components
        const int i = (int)(t - lo);
        const int o = __builtin_amdgcn_readlane(out_c, i) - cl;
        const int n = __builtin_amdgcn_readlane(in_c, i) - cl;
        slide(c0, c1, rot, (unsigned)o < 2u ? o : 255, (unsigned)n < 2u ? n : 255, 0, rot, inc);
      }
    }
    if (lane <= (int)(hi - lo)) out[lane] = mine;
  }
}

// One wavefront per read over its k_fetch * span keys (at most EMAX per
// lane): k rounds of a wavefront maximum; every key of the winning start
// leaves the pool (neighbourhoods of nearby candidates overlap, and their FP32
// values of a shared start may differ in the last bits).
template <int EMAX>
__global__ __launch_bounds__(256) void refine_select_kernel(const uint64_t* __restrict__ pool, int n,
                                                            int32_t R, int k,
                                                            int32_t* __restrict__ top_idx,
                                                            float* __restrict__ top_score) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= R) return;  // whole wavefront
  const uint64_t* src = pool + r * n;
  uint64_t mine[EMAX];
#pragma unroll
  for (int e = 0; e < EMAX; ++e) {
    const int i = e * 64 + lane;
    mine[e] = i < n ? src[i] : 0;
  }
  uint64_t res = 0;
  for (int out = 0; out < k; ++out) {
    uint64_t best = 0;
#pragma unroll
    for (int e = 0; e < EMAX; ++e) best = mine[e] > best ? mine[e] : best;
    const uint64_t g = wave_max_u64(best);
    if (g != 0) {
#pragma unroll
      for (int e = 0; e < EMAX; ++e)
        if ((uint32_t)mine[e] == (uint32_t)g) mine[e] = 0;
    }
    if (lane == out) res = g;
  }
  if (lane < k) write_list_entry(res, &top_idx[r * k + lane], &top_score[r * k + lane]);
}

}  // namespace

size_t refine_workspace_bytes(int32_t n_reads, int32_t k_fetch, int32_t radius) {
  return ((size_t)n_reads * (size_t)k_fetch * (size_t)(2 * radius + 1) * sizeof(uint64_t) + 255) /
         256 * 256;
}

hipError_t launch_refine(const rm_index& coarse, const uint8_t* ref, const uint8_t* seq,
                         const int64_t* off, int32_t n_reads, int32_t k_fetch,
                         const int32_t* cand_idx, int32_t radius, int32_t k, int32_t* top_idx,
                         float* top_score, void* ws, hipStream_t s) {
  const int N = coarse.p.window_len;
  const int64_t W1 = coarse.ref_len - N + 1;  // step-1 windows
  uint64_t* pool = static_cast<uint64_t*>(ws);
  hipLaunchKernelGGL(refine_kernel, dim3((unsigned)n_reads), dim3(256), 0, s, ref, W1, N,
                     coarse.p.stride, coarse.n_windows,
                     reinterpret_cast<const float2*>(coarse.d_phase32),
                     reinterpret_cast<const float4*>(coarse.d_step32), seq, off, n_reads, k_fetch,
                     cand_idx, radius, pool);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_refine_select(pool, k_fetch * (2 * radius + 1), n_reads, k, top_idx, top_score, s);
}

hipError_t launch_refine_select(const uint64_t* pool, int n, int32_t n_reads, int32_t k,
                                int32_t* top_idx, float* top_score, hipStream_t s) {
  // n = k_fetch (2 radius + 1) <= 64 x 63 keys per read
  auto kern = n <= 512    ? refine_select_kernel<8>
              : n <= 1024 ? refine_select_kernel<16>
              : n <= 2048 ? refine_select_kernel<32>
                          : refine_select_kernel<64>;
  hipLaunchKernelGGL(kern, dim3((unsigned)(((int64_t)n_reads + 3) / 4)), dim3(256), 0, s, pool, n,
                     n_reads, k, top_idx, top_score);
  return hipGetLastError();
}

hipError_t launch_refine_tokens(const rm_index& coarse, const uint8_t* ref, const uint8_t* seq,
                                const int64_t* off, int32_t n_reads, int32_t k_fetch,
                                const int32_t* cand_idx, int32_t radius, int32_t k,
                                int32_t* top_idx, float* top_score, void* ws, hipStream_t s) {
  const int N = coarse.p.window_len;
  const int64_t W1 = coarse.ref_len - N + 1;  // step-1 windows
  uint64_t* pool = static_cast<uint64_t*>(ws);
  hipLaunchKernelGGL(refine_tokens_kernel, dim3((unsigned)n_reads), dim3(256), 0, s, ref, W1, N,
                     coarse.p.stride, coarse.n_windows,
                     coarse.p.mer_len > 1 ? coarse.p.mer_len : 1, coarse.p.n_freq,
                     128 / coarse.p.n_freq, reinterpret_cast<const float2*>(coarse.d_phase32),
                     reinterpret_cast<const float4*>(coarse.d_step32), coarse.d_token_class, seq,
                     off, n_reads, k_fetch, cand_idx, radius, pool);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_refine_select(pool, k_fetch * (2 * radius + 1), n_reads, k, top_idx, top_score, s);
}

}  // namespace rm
