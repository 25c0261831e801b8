// Encoders: the rolling window encoder that builds the index, and the read-head
// encoder.
//
// Lane layout (one wavefront = one string): lane l owns factor k = l >> 1 and
// the two letters 2h, 2h+1 with h = l & 1, i.e. complex components
// (k, 2h) and (k, 2h+1), stored at reals [4l, 4l+4) of the 256-real row
// (component index k*4 + letter, re/im interleaved).  One wavefront therefore
// writes a whole row with one coalesced store.
//
// Window encoder (§3.4): window j (start j*stride) follows from window j-1 by
// `stride` one-letter slides; a slide multiplies every component by omega^-f_k,
// subtracts omega^-f_k from the outgoing letter's component and adds
// omega^(f_k (N-1)) to the incoming letter's component.  Each wavefront walks a
// segment of consecutive windows; at the segment start the state is computed
// directly from the letters in FP64 (the re-anchor), then rolled in FP32.
// Each window is normalised (§2.3) and written in the index precision.
#include "rm_internal.h"

namespace rm {

namespace {

struct Row4 {
  float v[4];
};

// Write one normalised row (4 reals per lane) in the requested precision.
// Returns the FP8 scale used (1 for FP32/FP16).
template <int PREC>
__device__ __forceinline__ float store_row(void* base, int64_t row, int lane, Row4 x) {
  if constexpr (PREC == RM_FP32) {
    float4* dst = reinterpret_cast<float4*>(static_cast<float*>(base) + row * kReal) + lane;
    *dst = make_float4(x.v[0], x.v[1], x.v[2], x.v[3]);
    return 1.f;
  } else if constexpr (PREC == RM_FP16) {
    _Float16 h0 = (_Float16)x.v[0], h1 = (_Float16)x.v[1], h2 = (_Float16)x.v[2],
             h3 = (_Float16)x.v[3];
    uint32_t lo = (uint32_t)__builtin_bit_cast(uint16_t, h0) |
                  ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
    uint32_t hi = (uint32_t)__builtin_bit_cast(uint16_t, h2) |
                  ((uint32_t)__builtin_bit_cast(uint16_t, h3) << 16);
    uint2* dst = reinterpret_cast<uint2*>(static_cast<_Float16*>(base) + row * kReal) + lane;
    *dst = make_uint2(lo, hi);
    return 1.f;
  } else {
    float m = fmaxf(fmaxf(fabsf(x.v[0]), fabsf(x.v[1])), fmaxf(fabsf(x.v[2]), fabsf(x.v[3])));
    m = wave_max(m);
    float s = fp8_pow2_scale(m);
    float inv = 1.f / s;  // exact: s is a power of two
    uint32_t w = pack_fp8x2(x.v[0] * inv, x.v[1] * inv) |
                 (pack_fp8x2(x.v[2] * inv, x.v[3] * inv) << 16);
    uint32_t* dst = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(base) + row * kReal) + lane;
    *dst = w;
    // Norm correction: the returned scale makes the dequantised row (code * scale)
    // exactly unit length.  For a pair of nearly equal vectors the first-order
    // error of F = |<x|c>|^2 is the change of squared norm Re<c, e_c> caused by
    // quantisation; renormalising removes it (phase errors only enter F at
    // second order).
    float2 d01 = unpack_fp8x2(w), d23 = unpack_fp8x2(w >> 16);
    float q2 = wave_sum(d01.x * d01.x + d01.y * d01.y + d23.x * d23.x + d23.y * d23.y);
    return q2 > 0.f ? 1.f / sqrtf(q2) : s;
  }
}

// FP64 direct sum over letters [0, n) of `str` for this lane's two components.
__device__ __forceinline__ void direct_sum(const uint8_t* __restrict__ str, int n,
                                           const double2* __restrict__ phase64, int lane,
                                           double2& a0, double2& a1) {
  const int k = lane >> 1, h = lane & 1;
  const int L0 = 2 * h, L1 = 2 * h + 1;
  a0 = make_double2(0.0, 0.0);
  a1 = make_double2(0.0, 0.0);
  for (int pb = 0; pb < n; pb += 64) {
    int mine = (pb + lane < n) ? (int)str[pb + lane] : 255;
    int cnt = min(64, n - pb);

    for (int i = 0; i < cnt; ++i) {
      int L = __builtin_amdgcn_readlane(mine, i);
      double2 e = phase64[(int64_t)(pb + i) * kM + k];
      a0.x += (L == L0) ? e.x : 0.0;
      a0.y += (L == L0) ? e.y : 0.0;
      a1.x += (L == L1) ? e.x : 0.0;
      a1.y += (L == L1) ? e.y : 0.0;
    }
  }
}

template <int PREC>
__device__ __forceinline__ void emit_window(int64_t j, int lane, int N, float2 c0, float2 c1,
                                            void* emb, float* scale, float* norm2) {
  float n2 = wave_sum(c0.x * c0.x + c0.y * c0.y + c1.x * c1.x + c1.y * c1.y);
  bool deg = n2 < kDegenerateRel * (float)N;
  float inv = deg ? 0.f : 1.f / sqrtf(n2);
  Row4 x{{c0.x * inv, c0.y * inv, c1.x * inv, c1.y * inv}};
  float s = store_row<PREC>(emb, j, lane, x);
  if (lane == 0) {
    norm2[j] = n2;
    scale[j] = s;
  }
}

template <int PREC>
__global__ __launch_bounds__(256) void encode_reference_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride, int64_t seg_len, int64_t n_seg,
    const double2* __restrict__ phase64, const float4* __restrict__ step32, void* __restrict__ emb,
    float* __restrict__ scale, float* __restrict__ norm2) {
  const int lane = threadIdx.x & 63;
  const int64_t seg = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (seg >= n_seg) return;
  const int k = lane >> 1, h = lane & 1;
  const int L0 = 2 * h, L1 = 2 * h + 1;
  const int64_t j0 = seg * seg_len;
  const int64_t j1 = min(W, j0 + seg_len);

  // Re-anchor: the first window of the segment, directly, in FP64.
  double2 a0, a1;
  direct_sum(ref + j0 * stride, N, phase64, lane, a0, a1);
  float2 c0 = make_float2((float)a0.x, (float)a0.y);
  float2 c1 = make_float2((float)a1.x, (float)a1.y);
  emit_window<PREC>(j0, lane, N, c0, c1, emb, scale, norm2);

  const float4 st = step32[k];
  const float2 rot = make_float2(st.x, st.y);   // omega^-f
  const float2 inc = make_float2(st.z, st.w);   // omega^(f (N-1))

  // Slides t = 0 .. n_slides-1 move the window start from j0*stride+t to +1.
  const int64_t s0 = j0 * stride;
  const int64_t n_slides = (j1 - 1 - j0) * stride;
  int64_t j = j0;
  int until_emit = stride;
  for (int64_t tb = 0; tb < n_slides; tb += 64) {
    // outgoing letter of slide t is ref[s0+t], incoming is ref[s0+t+N]
    int64_t t = tb + lane;
    int out_l = (t < n_slides) ? (int)ref[s0 + t] : 255;
    int in_l = (t < n_slides) ? (int)ref[s0 + t + N] : 255;
    int cnt = (int)min<int64_t>(64, n_slides - tb);
    for (int i = 0; i < cnt; ++i) {
      int o = __builtin_amdgcn_readlane(out_l, i);
      int n = __builtin_amdgcn_readlane(in_l, i);
      c0 = cmul(c0, rot);
      c1 = cmul(c1, rot);
      if (o == L0) { c0.x -= rot.x; c0.y -= rot.y; }
      if (o == L1) { c1.x -= rot.x; c1.y -= rot.y; }
      if (n == L0) { c0.x += inc.x; c0.y += inc.y; }
      if (n == L1) { c1.x += inc.x; c1.y += inc.y; }
      if (--until_emit == 0) {
        until_emit = stride;
        ++j;
        emit_window<PREC>(j, lane, N, c0, c1, emb, scale, norm2);
      }
    }
  }
}

template <int PREC>
__global__ __launch_bounds__(256) void encode_reads_kernel(
    const uint8_t* __restrict__ seq, const int64_t* __restrict__ off, int32_t n_reads, int N,
    const double2* __restrict__ phase64, void* __restrict__ emb, float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= n_reads) return;
  const int64_t start = off[r];
  const int64_t len = off[r + 1] - start;
  double2 a0 = make_double2(0.0, 0.0), a1 = make_double2(0.0, 0.0);
  if (len >= N) direct_sum(seq + start, N, phase64, lane, a0, a1);
  double X = wave_sum(a0.x * a0.x + a0.y * a0.y + a1.x * a1.x + a1.y * a1.y);
  bool deg = X < (double)kDegenerateRel * N;
  double inv = deg ? 0.0 : 1.0 / sqrt(X);
  float xr0 = (float)(a0.x * inv), xi0 = (float)(a0.y * inv);
  float xr1 = (float)(a1.x * inv), xi1 = (float)(a1.y * inv);
  // row 2r: (Re x, Im x) per component; row 2r+1: (-Im x, Re x).  A window row
  // (Re c, Im c) dotted with them gives Re and Im of sum conj(x) c.
  Row4 re{{xr0, xi0, xr1, xi1}};
  Row4 im{{-xi0, xr0, -xi1, xr1}};
  float s = store_row<PREC>(emb, 2 * r, lane, re);
  store_row<PREC>(emb, 2 * r + 1, lane, im);
  if (scale != nullptr && lane == 0) scale[r] = s;
}

}  // namespace

hipError_t launch_encode_reference(const uint8_t* ref, int64_t W, const rm_params& p,
                                   const double* phase64, const float* step32, void* emb,
                                   float* scale, float* norm2, hipStream_t s) {
  // Segment = window starts between two FP64 re-anchors: the caller's value,
  // or enough segments for the chip (about 8192) with at most 4096 starts each.
  int64_t seg = p.reanchor;
  if (seg <= 0) {
    seg = (W + 8191) / 8192;
    if (seg < 256) seg = 256;
    if (seg > 4096) seg = 4096;
  }
  int64_t n_seg = (W + seg - 1) / seg;
  const int waves = 4;
  int64_t blocks = (n_seg + waves - 1) / waves;
  auto* ph = reinterpret_cast<const double2*>(phase64);
  auto* st = reinterpret_cast<const float4*>(step32);
  switch (p.precision) {
    case RM_FP32:
      hipLaunchKernelGGL(encode_reference_kernel<RM_FP32>, dim3((unsigned)blocks), dim3(64 * waves),
                         0, s, ref, W, p.window_len, p.stride, seg, n_seg, ph, st, emb, scale, norm2);
      break;
    case RM_FP16:
      hipLaunchKernelGGL(encode_reference_kernel<RM_FP16>, dim3((unsigned)blocks), dim3(64 * waves),
                         0, s, ref, W, p.window_len, p.stride, seg, n_seg, ph, st, emb, scale, norm2);
      break;
    default:
      hipLaunchKernelGGL(encode_reference_kernel<RM_FP8_E4M3>, dim3((unsigned)blocks),
                         dim3(64 * waves), 0, s, ref, W, p.window_len, p.stride, seg, n_seg, ph, st,
                         emb, scale, norm2);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_encode_reads(const rm_params& p, const double* phase64, const uint8_t* seq,
                               const int64_t* off, int32_t n_reads, void* emb, float* scale,
                               hipStream_t s) {
  const int waves = 4;
  int64_t blocks = ((int64_t)n_reads + waves - 1) / waves;
  auto* ph = reinterpret_cast<const double2*>(phase64);
  switch (p.precision) {
    case RM_FP32:
      hipLaunchKernelGGL(encode_reads_kernel<RM_FP32>, dim3((unsigned)blocks), dim3(64 * waves), 0, s,
                         seq, off, n_reads, p.window_len, ph, emb, scale);
      break;
    case RM_FP16:
      hipLaunchKernelGGL(encode_reads_kernel<RM_FP16>, dim3((unsigned)blocks), dim3(64 * waves), 0, s,
                         seq, off, n_reads, p.window_len, ph, emb, scale);
      break;
    default:
      hipLaunchKernelGGL(encode_reads_kernel<RM_FP8_E4M3>, dim3((unsigned)blocks), dim3(64 * waves),
                         0, s, seq, off, n_reads, p.window_len, ph, emb, scale);
      break;
  }
  return hipGetLastError();
}

}  // namespace rm
