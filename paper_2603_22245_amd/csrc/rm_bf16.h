// Products of one-hot (string, letter) rows with the FP32 phase table on
// 32x32x16 bfloat16 MFMAs, shared by the rescore and threshold kernels.
//
// Component (k, L) of a string's RoPE vector sums the table entries
// omega^(f_k p) over the positions p holding letter L (§2.1-§2.2), so the
// vectors of a set of strings are the product of their one-hot rows with the
// table [p][factor].  The table splits exactly into three bfloat16 parts and
// the indicators are exact in bfloat16, so three bf16 MFMAs with FP32
// accumulation give the FP32 direct sums up to the order of the additions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Exact split of an FP32 value into three bfloat16 bit patterns, x = hi + mid +
// lo: hi keeps the sign, exponent and top 7 stored mantissa bits of x
// (truncated), so x - hi is exact and has at most 16 significant bits; mid
// keeps the top 8 of those, and the exact remainder has at most 8 (bfloat16
// has the exponent range of FP32, so no part underflows).
__device__ __forceinline__ void split_bf16x3(float x, uint32_t& hi, uint32_t& mid, uint32_t& lo) {
  const uint32_t h = __float_as_uint(x) & 0xffff0000u;
  const float r1 = x - __uint_as_float(h);
  const uint32_t m = __float_as_uint(r1) & 0xffff0000u;
  const float r2 = r1 - __uint_as_float(m);
  hi = h >> 16;
  mid = m >> 16;
  lo = __float_as_uint(r2) >> 16;
}

// One 64-position chunk (positions pb .. pb+63, zero past N) of the table
// [N][64 reals] as its three parts in LDS: tparts[part][column block][8
// positions][column] holds the 8 bf16 of positions 8 pg .. 8 pg + 7 (the B
// fragment layout of the 32x32x16 bf16 MFMA).  Block-cooperative: 512
// fragments over `nthreads` threads.
__device__ __forceinline__ void stage_table_parts(const float* __restrict__ tab, int pb, int N,
                                                  u32x4 (*tparts)[2][8][32], int tid,
                                                  int nthreads) {
  for (int f = tid; f < 512; f += nthreads) {
    const int c = f & 31, pg = (f >> 5) & 7, cb = f >> 8;
    uint32_t hi[8], mid[8], lo[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int pos = pb + 8 * pg + jj;
      const float x = pos < N ? tab[(int64_t)pos * 64 + cb * 32 + c] : 0.f;
      split_bf16x3(x, hi[jj], mid[jj], lo[jj]);
    }
    tparts[0][cb][pg][c] = u32x4{hi[0] | hi[1] << 16, hi[2] | hi[3] << 16, hi[4] | hi[5] << 16,
                                 hi[6] | hi[7] << 16};
    tparts[1][cb][pg][c] = u32x4{mid[0] | mid[1] << 16, mid[2] | mid[3] << 16,
                                 mid[4] | mid[5] << 16, mid[6] | mid[7] << 16};
    tparts[2][cb][pg][c] = u32x4{lo[0] | lo[1] << 16, lo[2] | lo[3] << 16, lo[4] | lo[5] << 16,
                                 lo[6] | lo[7] << 16};
  }
}

// A fragment of eight positions of one (string, letter) row: `w` holds the
// string's letters there (bytes 0..3, 4 for none), `onehot_tab` has byte L =
// 0x40 for the row's letter L and 0 elsewhere; the result is bf16 2.0 where the
// letter matches, else 0 (2 keeps one byte of the pattern: sums come out
// doubled, which halving undoes exactly).
__device__ __forceinline__ bf16x8 onehot_fragment(uint2 w, uint32_t onehot_tab) {
  const uint32_t h0 = __builtin_amdgcn_perm(0u, onehot_tab, w.x);  // bytes 0x40 / 0
  const uint32_t h1 = __builtin_amdgcn_perm(0u, onehot_tab, w.y);
  const u32x4 av{__builtin_amdgcn_perm(0u, h0, 0x010c000cu), __builtin_amdgcn_perm(0u, h0, 0x030c020cu),
                 __builtin_amdgcn_perm(0u, h1, 0x010c000cu), __builtin_amdgcn_perm(0u, h1, 0x030c020cu)};
  return __builtin_bit_cast(bf16x8, av);
}

}  // namespace rm
