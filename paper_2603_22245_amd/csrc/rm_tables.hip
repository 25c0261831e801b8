// Angle tables of the RoPE-DNA encoding, computed in FP64 on the device.
//
// For factor index k (0-based, f = f_{k+1}) and location p < N:
//   phase64[p][k] = omega^(f p),  omega = exp(2 pi i / N)      (§2.1, §2.2)
//   step32[k]     = (omega^-f, omega^(f (N-s)))  rounded to FP32 -- the two
//                   constants of the one-letter slide of §3.4 (tokens of s
//                   letters; s = 1 for the letter encoding).
// Factors: f = k+1 (§2.2 eq. mult-factor) or 2k/(m-1)+1 (§3.3 eq.
// mult-factor-finetune).  For integer factors the exponent f*p is reduced
// modulo N in integer arithmetic, so the argument of sincospi is 2r/N exactly
// representable up to one rounding, whatever p is.
#include "rm_internal.h"
#include "rm_tokens.h"

namespace rm {

__device__ __forceinline__ double factor(int k, int m, int schedule) {
  if (schedule == RM_SCHED_FINETUNED && m > 1) return 2.0 * (double)k / (double)(m - 1) + 1.0;
  return (double)(k + 1);
}

// exp(2 pi i f q / N) for integer location q (may be negative).
__device__ __forceinline__ double2 unit(int k, int m, int schedule, int64_t q, int N) {
  double s, c;
  if (schedule == RM_SCHED_DEFAULT) {
    int64_t r = ((int64_t)(k + 1) * q) % N;
    if (r < 0) r += N;
    sincospi(2.0 * (double)r / (double)N, &s, &c);
  } else {
    sincospi(2.0 * factor(k, m, schedule) * (double)q / (double)N, &s, &c);
  }
  return make_double2(c, s);
}

__global__ void tables_kernel(int N, int m, int schedule, int s, double2* __restrict__ phase64,
                              float2* __restrict__ phase32, float4* __restrict__ step32) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)N * m;
  if (t < total) {
    int p = (int)(t / m), k = (int)(t % m);
    double2 e = unit(k, m, schedule, p, N);
    phase64[t] = e;
    phase32[t] = make_float2((float)e.x, (float)e.y);
  }
  if (t < m) {
    int k = (int)t;
    double2 back = unit(k, m, schedule, -1, N);
    double2 front = unit(k, m, schedule, N - s, N);
    step32[k] = make_float4((float)back.x, (float)back.y, (float)front.x, (float)front.y);
  }
}

__global__ void zero_word_kernel(uint32_t* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}

hipError_t launch_zero_word(uint32_t* p, hipStream_t s) {
  hipLaunchKernelGGL(zero_word_kernel, dim3(1), dim3(64), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_tables(const rm_params& p, double* phase64, float* phase32, float* step32,
                         hipStream_t s) {
  int64_t total = (int64_t)p.window_len * p.n_freq;
  int threads = 256;
  int blocks = (int)((total + threads - 1) / threads);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(tables_kernel, dim3(blocks), dim3(threads), 0, s, p.window_len, p.n_freq,
                     p.schedule, p.mer_len > 1 ? p.mer_len : 1, reinterpret_cast<double2*>(phase64),
                     reinterpret_cast<float2*>(phase32), reinterpret_cast<float4*>(step32));
  return hipGetLastError();
}

// Class table of a token index: the caller's map with out-of-range values
// replaced by RM_TOKEN_SKIP, or the identity (class = s-mer code).
__global__ void token_table_kernel(const uint8_t* __restrict__ map, int n, int n_class,
                                   uint8_t* __restrict__ table) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v = map != nullptr ? (int)map[i] : i;
  table[i] = v < n_class ? (uint8_t)v : (uint8_t)RM_TOKEN_SKIP;
}

hipError_t launch_token_table(const uint8_t* map, int s, int n_class, uint8_t* table,
                              hipStream_t st) {
  const int n = 1 << (2 * s);
  hipLaunchKernelGGL(token_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, map,
                     n, n_class, table);
  return hipGetLastError();
}

}  // namespace rm
