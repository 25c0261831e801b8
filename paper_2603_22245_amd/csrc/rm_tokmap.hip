// The compact context-aware token map of §2.6: only the reference's most
// frequent s-mers are tokens.
//
// count_kernel: occurrences of every s-mer code over the reference (locations
// 0..G-s; an s-mer holding a letter outside 0..3 is not counted), with a
// per-block LDS histogram for s <= 6 and global atomics for longer s-mers.
// select_kernel (one block): the n_class codes ranked first by (count
// descending, code ascending) become classes 0..n_class-1 in code order, every
// other code RM_TOKEN_SKIP.  The n_class-th largest key is found by a binary
// search on the count, then the codes tied at that count are taken in code
// order; both steps and the class numbering use block-wide prefix counts over
// contiguous code ranges, so the result is a pure function of the counts.
#include "rm_tokens.h"

namespace rm {

namespace {

constexpr int kSelThreads = 1024;

__global__ __launch_bounds__(256) void zero_kernel(uint32_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(256) void count_kernel(const uint8_t* __restrict__ ref,
                                                    int64_t n_loc, int s,
                                                    uint32_t* __restrict__ counts) {
  extern __shared__ uint32_t hist[];  // 4^s bins when s <= 6, else unused
  const int nb = 1 << (2 * s);
  const bool local = s <= 6;
  if (local)
    for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_loc;
       q += (int64_t)gridDim.x * blockDim.x) {
    uint32_t code = 0;
    bool ok = true;
    for (int i = 0; i < s; ++i) {
      const uint32_t L = ref[q + i];
      ok = ok && L < 4u;
      code = code * 4u + (L & 3u);
    }
    if (!ok) continue;
    if (local) atomicAdd(&hist[code], 1u);
    else atomicAdd(&counts[code], 1u);
  }
  if (!local) return;
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    if (hist[i] != 0) atomicAdd(&counts[i], hist[i]);
}

// Block-wide sum of one value per thread (kSelThreads threads).
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* red) {
  // wavefront sum by shuffles
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  uint32_t t = 0;
  for (int w = 0; w < kSelThreads / 64; ++w) t += red[w];
  return t;
}

// Exclusive prefix over threads of one value per thread (in thread order).
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* scan) {
  __syncthreads();
  scan[threadIdx.x] = v;
  __syncthreads();
  // Hillis-Steele inclusive scan over kSelThreads entries
  for (int d = 1; d < kSelThreads; d <<= 1) {
    const uint32_t add = threadIdx.x >= (unsigned)d ? scan[threadIdx.x - d] : 0u;
    __syncthreads();
    scan[threadIdx.x] += add;
    __syncthreads();
  }
  return scan[threadIdx.x] - v;
}

__global__ __launch_bounds__(kSelThreads) void select_kernel(const uint32_t* __restrict__ counts,
                                                             int s, int n_class,
                                                             uint8_t* __restrict__ map) {
  __shared__ uint32_t red[kSelThreads / 64];
  __shared__ uint32_t scan[kSelThreads];
  const int nb = 1 << (2 * s);
  const int per = (nb + kSelThreads - 1) / kSelThreads;  // codes per thread (contiguous)
  const int c0 = threadIdx.x * per, c1 = min(nb, c0 + per);

  // the largest count c* with at least n_class codes at or above it
  uint32_t mx = 0;
  for (int c = c0; c < c1; ++c) mx = max(mx, counts[c]);
  for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, d, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = 0;
  for (int w = 0; w < kSelThreads / 64; ++w) mx = max(mx, red[w]);
  uint32_t lo = 0, hi = mx;  // invariant: at least n_class codes have count >= lo
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo + 1) / 2;
    uint32_t n = 0;
    for (int c = c0; c < c1; ++c) n += counts[c] >= mid ? 1u : 0u;
    if (block_sum(n, red) >= (uint32_t)n_class) lo = mid; else hi = mid - 1;
  }
  const uint32_t cstar = lo;

  // codes above c*, then the first ones (in code order) at c*
  uint32_t above = 0, tied = 0;
  for (int c = c0; c < c1; ++c) {
    above += counts[c] > cstar ? 1u : 0u;
    tied += counts[c] == cstar ? 1u : 0u;
  }
  const uint32_t n_above = block_sum(above, red);
  const uint32_t need = (uint32_t)n_class - n_above;  // taken from the ties
  uint32_t tie_rank = block_exclusive(tied, scan);
  uint32_t kept = 0;
  for (int c = c0; c < c1; ++c) {
    const bool sel = counts[c] > cstar || (counts[c] == cstar && tie_rank++ < need);
    kept += sel ? 1u : 0u;
  }
  // classes in code order
  uint32_t cls = block_exclusive(kept, scan);
  tie_rank = block_exclusive(tied, scan);
  for (int c = c0; c < c1; ++c) {
    const bool sel = counts[c] > cstar || (counts[c] == cstar && tie_rank++ < need);
    map[c] = sel ? (uint8_t)cls++ : (uint8_t)RM_TOKEN_SKIP;
  }
}

}  // namespace

hipError_t launch_token_counts(const uint8_t* ref, int64_t ref_len, int s, uint32_t* counts,
                               hipStream_t st) {
  const int nb = 1 << (2 * s);
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, counts,
                     nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n_loc = ref_len - s + 1;
  int64_t blocks = (n_loc + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  const size_t lds = s <= 6 ? (size_t)nb * sizeof(uint32_t) : 0;
  hipLaunchKernelGGL(count_kernel, dim3((unsigned)blocks), dim3(256), lds, st, ref, n_loc, s,
                     counts);
  return hipGetLastError();
}

hipError_t launch_token_select(const uint32_t* counts, int s, int n_class, uint8_t* map,
                               hipStream_t st) {
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kSelThreads), 0, st, counts, s, n_class, map);
  return hipGetLastError();
}

}  // namespace rm
