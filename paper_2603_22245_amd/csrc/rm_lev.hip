// Exact Levenshtein distance of string pairs (the labels of the learned
// ranking loss, and the reference the Spearman correlation is taken against).
//
// One thread per pair.  Bit-parallel dynamic programme over the columns of the
// text: Myers (J. ACM 46(3), 1999) with the block decomposition of the same
// paper, in its global-distance form (the horizontal delta entering row 0 is
// +1 at every column, the vertical deltas of column 0 are all +1).  The shorter
// string is the pattern, at most 256 letters = 4 words of 64 bits; the score
// at the last pattern row starts at m and follows the horizontal delta leaving
// the last block.
#include "rm_internal.h"

namespace rm {

namespace {

constexpr int kWords = 4;

__global__ __launch_bounds__(256) void levenshtein_kernel(
    const uint8_t* __restrict__ a, const int64_t* __restrict__ aoff,
    const uint8_t* __restrict__ b, const int64_t* __restrict__ boff, int64_t n,
    int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t a0 = aoff[i], la = aoff[i + 1] - a0;
  const int64_t b0 = boff[i], lb = boff[i + 1] - b0;
  const uint8_t* P = a + a0;
  const uint8_t* T = b + b0;
  int64_t m = la, tn = lb;
  if (la > lb) {
    P = b + b0;
    T = a + a0;
    m = lb;
    tn = la;
  }
  if (m <= 0) {
    out[i] = (int32_t)max<int64_t>(tn, 0);
    return;
  }
  if (m > 64 * kWords) {
    out[i] = -1;
    return;
  }
  // match masks per letter and word
  uint64_t eqA[kWords] = {}, eqC[kWords] = {}, eqG[kWords] = {}, eqT[kWords] = {};
  for (int q = 0; q < (int)m; ++q) {
    const uint8_t c = P[q];
    const uint64_t bit = 1ull << (q & 63);
#pragma unroll
    for (int w = 0; w < kWords; ++w) {
      if ((q >> 6) != w) continue;
      eqA[w] |= c == 0 ? bit : 0;
      eqC[w] |= c == 1 ? bit : 0;
      eqG[w] |= c == 2 ? bit : 0;
      eqT[w] |= c == 3 ? bit : 0;
    }
  }
  const int nw = (int)((m + 63) >> 6);
  const uint64_t last_high = 1ull << ((m - 1) & 63);
  uint64_t Pv[kWords], Mv[kWords];
#pragma unroll
  for (int w = 0; w < kWords; ++w) {
    Pv[w] = ~0ull;
    Mv[w] = 0;
  }
  int64_t score = m;
  for (int64_t j = 0; j < tn; ++j) {
    const uint8_t c = T[j];
    int hin = 1;  // row 0: D[0][j] = j
#pragma unroll
    for (int w = 0; w < kWords; ++w) {
      if (w >= nw) break;
      uint64_t eq = c == 0 ? eqA[w] : c == 1 ? eqC[w] : c == 2 ? eqG[w] : c == 3 ? eqT[w] : 0;
      const uint64_t pv = Pv[w], mv = Mv[w];
      const uint64_t xv = eq | mv;
      if (hin < 0) eq |= 1;
      const uint64_t xh = (((eq & pv) + pv) ^ pv) | eq;
      uint64_t ph = mv | ~(xh | pv);
      uint64_t mh = pv & xh;
      const uint64_t high = w == nw - 1 ? last_high : (1ull << 63);
      const int hout = (ph & high) ? 1 : (mh & high) ? -1 : 0;
      ph <<= 1;
      mh <<= 1;
      if (hin < 0) mh |= 1;
      else if (hin > 0) ph |= 1;
      Pv[w] = mh | ~(xv | ph);
      Mv[w] = ph & xv;
      hin = hout;
    }
    score += hin;
  }
  out[i] = (int32_t)score;
}

}  // namespace

hipError_t launch_levenshtein(const uint8_t* a, const int64_t* aoff, const uint8_t* b,
                              const int64_t* boff, int64_t n, int32_t* out, hipStream_t s) {
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(levenshtein_kernel, dim3(blocks), dim3(256), 0, s, a, aoff, b, boff, n, out);
  return hipGetLastError();
}

}  // namespace rm
