// BF16 inference of the learned token offsets on the matrix cores.
//
// For every 9-mer token location t of a letter string (t = 0..n-9) the network
// maps the one-hot of the 8 flanking letters (w[t..t+3], w[t+5..t+8]) to 128
// outputs, o = W2 relu(W1 x + b1) + b2, and keeps the 32 of the middle letter
// w[t+4]: delta[t][k] = o[w[t+4]*32 + k] (0 if the middle letter is not A, C,
// G or T).  Weights and hidden values are rounded to bfloat16 (nearest, ties
// to even); products accumulate in FP32; biases are added in FP32.
//
// Layout on the 32x32x16 bf16 MFMA, one wavefront per tile of 32 tokens, both
// layers transposed so that no data crosses lanes:
//   layer 1: P^T [64 hidden x 32 tokens] = W1 [64 x 32] * X^T [32 x 32]
//            (2 hidden tiles x 2 K steps; X^T is built from the letters in the
//            lane that owns the token column);
//   layer 2: O^T [128 x 32 tokens] = W2 [128 x 64] * H^T [64 x 32]
//            (4 output tiles = the 4 middle letters, 4 K steps).  The B
//            operand of layer 2 is the layer-1 accumulator itself, relu'd and
//            rounded: lane l holds hidden rows 8(v/4) + 4(l/32) + v%4 of its
//            token column, so K step (mt, half) pairs slot j of lane l with
//            hidden 32mt + 16half + 8(j/4) + 4(l/32) + j%4, and W2's fragments
//            are gathered in that order.
// Lane l (column token l%32) then holds 16 of its token's 32 outputs per
// letter tile and keeps the tile of its own middle letter.
#include "rm_internal.h"

namespace rm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kIn = 32, kHid = 64, kOut = 128;
constexpr int kW1 = 0, kB1 = kHid * kIn, kW2 = kB1 + kHid, kB2 = kW2 + kOut * kHid;
constexpr int kWavesPerBlock = 4;

__device__ __forceinline__ unsigned short bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ bf16x8 as_bf16(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

__global__ __launch_bounds__(64 * kWavesPerBlock) void mlp_infer_kernel(
    const float* __restrict__ params, const uint8_t* __restrict__ seq, int64_t n_tok,
    float* __restrict__ delta) {
  __shared__ float sb1[kHid], sb2[kOut];
  for (int i = threadIdx.x; i < kHid; i += blockDim.x) sb1[i] = params[kB1 + i];
  for (int i = threadIdx.x; i < kOut; i += blockDim.x) sb2[i] = params[kB2 + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 5, col = lane & 31;

  // weight fragments (A operands), rounded once per wavefront
  bf16x8 w1f[2][2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      u16x8 v;
      const float* src = params + kW1 + (32 * mt + col) * kIn + 16 * ks + 8 * g;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = bf16_bits(src[j]);
      w1f[mt][ks] = as_bf16(v);
    }
  bf16x8 w2f[4][4];
#pragma unroll
  for (int mo = 0; mo < 4; ++mo)
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int mt = ks >> 1, half = ks & 1;
      u16x8 v;
      const float* src = params + kW2 + (32 * mo + col) * kHid + 32 * mt + 16 * half + 4 * g;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = bf16_bits(src[8 * (j >> 2) + (j & 3)]);
      w2f[mo][ks] = as_bf16(v);
    }

  const int64_t n_tiles = (n_tok + 31) / 32;
  for (int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + wave; tile < n_tiles;
       tile += (int64_t)gridDim.x * kWavesPerBlock) {
    const int64_t t = tile * 32 + col;  // this lane's token
    const bool valid = t < n_tok;
    int let[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) let[q] = valid ? (int)seq[t + q] : 4;

    // layer 1, accumulators start at b1 of the lane's hidden rows
    floatx16 acc1[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 b = *reinterpret_cast<const float4*>(&sb1[32 * mt + 8 * q + 4 * g]);
        acc1[mt][4 * q] = b.x;
        acc1[mt][4 * q + 1] = b.y;
        acc1[mt][4 * q + 2] = b.z;
        acc1[mt][4 * q + 3] = b.w;
      }
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      // inputs 16ks + 8g + j: flank 4ks + 2g + j/4, letter j%4
      u16x8 x;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int fi = 4 * ks + 2 * g + (j >> 2);
        const int pos = fi < 4 ? fi : fi + 1;
        x[j] = let[pos] == (j & 3) ? (unsigned short)0x3F80 : (unsigned short)0;
      }
      const bf16x8 xb = as_bf16(x);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        acc1[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1f[mt][ks], xb, acc1[mt], 0, 0, 0);
    }
    // hidden values, relu'd and rounded: the B operands of layer 2
    bf16x8 hf[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int mt = ks >> 1, half = ks & 1;
      u16x8 v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = bf16_bits(fmaxf(acc1[mt][8 * half + j], 0.f));
      hf[ks] = as_bf16(v);
    }
    // layer 2, one letter tile at a time; keep the middle letter's
    const int mid = let[4];
    floatx16 res;
#pragma unroll
    for (int v = 0; v < 16; ++v) res[v] = 0.f;
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      floatx16 acc2;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc2[v] = 0.f;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2f[mo][ks], hf[ks], acc2, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; ++v) res[v] = mid == mo ? acc2[v] : res[v];
    }
    if (valid) {
      float* dst = delta + t * 32 + 4 * g;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
        if (mid < 4) {
          const float4 b = *reinterpret_cast<const float4*>(&sb2[32 * mid + 8 * q + 4 * g]);
          o = make_float4(res[4 * q] + b.x, res[4 * q + 1] + b.y, res[4 * q + 2] + b.z,
                          res[4 * q + 3] + b.w);
        }
        *reinterpret_cast<float4*>(dst + 8 * q) = o;
      }
    }
  }
}

}  // namespace

hipError_t launch_mlp_infer(const float* params, const uint8_t* seq, int64_t n_letters,
                            float* delta, hipStream_t s) {
  const int64_t n_tok = n_letters - 8;
  const int64_t tiles = (n_tok + 31) / 32;
  int64_t blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 1024) blocks = 1024;  // grid-stride beyond: weights are loaded once per wavefront
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, s,
                     params, seq, n_tok, delta);
  return hipGetLastError();
}

}  // namespace rm
