// Both mapping directions and the fidelity-threshold regime.
//
// A read from the other strand matches the reference after reverse
// complementing it (reversed, A <-> T, C <-> G: code L -> 3 - L for A,C,G,T =
// 0..3); the paper maps reads in both directions.  reverse_complement_kernel
// writes the reverse complement of every read in place of its letters in a
// second buffer (same offsets), so one product over the 2R heads scores both
// strands.  merge_strands_kernel combines a read's two ranked lists into its
// k best, ranked (F desc, window id asc, forward first), and drops the
// entries below a minimum fidelity (§3.1: fidelities above a threshold give
// the matching locations; §3.5: the regime that outputs every location
// passing the threshold).
#include "rm_internal.h"

namespace rm {

namespace {

// One thread per letter of the batch; the read of letter i is found by
// binary search over the offsets (reads are contiguous).
__global__ __launch_bounds__(256) void reverse_complement_kernel(const uint8_t* __restrict__ seq,
                                                                 const int64_t* __restrict__ off,
                                                                 int32_t n_reads,
                                                                 uint8_t* __restrict__ out) {
  const int64_t total = off[n_reads] - off[0];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = off[0] + t;
    int lo = 0, hi = n_reads - 1;  // the read r with off[r] <= i < off[r+1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const int64_t mirror = off[lo] + off[lo + 1] - 1 - i;
    const uint8_t L = seq[mirror];
    out[i] = L < 4 ? (uint8_t)(3 - L) : L;
  }
}

// One thread per read: a two-way merge of the forward and reverse lists (each
// of k entries, ranked, missing entries have id < 0).
__global__ __launch_bounds__(256) void merge_strands_kernel(
    const int32_t* __restrict__ fi, const float* __restrict__ ff, const int32_t* __restrict__ ri,
    const float* __restrict__ rf, int32_t n_reads, int k, float min_fidelity,
    int32_t* __restrict__ top_idx, float* __restrict__ top_score, int8_t* __restrict__ top_strand,
    int32_t* __restrict__ n_found) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  const int32_t* a = fi + r * k;
  const float* af = ff + r * k;
  const int32_t* b = ri + r * k;
  const float* bf = rf + r * k;
  int p = 0, q = 0, n = 0;
  auto valid = [&](const int32_t* ids, const float* sc, int i) {
    return i < k && ids[i] >= 0 && sc[i] >= min_fidelity;
  };
  while (n < k) {
    const bool va = valid(a, af, p), vb = valid(b, bf, q);
    if (!va && !vb) break;
    // the forward entry goes first unless the reverse one ranks strictly higher
    bool take_b = false;
    if (va && vb) take_b = bf[q] > af[p] || (bf[q] == af[p] && b[q] < a[p]);
    else take_b = vb;
    if (take_b) {
      top_idx[r * k + n] = b[q];
      top_score[r * k + n] = bf[q];
      top_strand[r * k + n] = 1;
      ++q;
    } else {
      top_idx[r * k + n] = a[p];
      top_score[r * k + n] = af[p];
      top_strand[r * k + n] = 0;
      ++p;
    }
    ++n;
  }
  n_found[r] = n;
  for (int e = n; e < k; ++e) {
    top_idx[r * k + e] = -1;
    top_score[r * k + e] = 0.f;
    top_strand[r * k + e] = -1;
  }
}

}  // namespace

hipError_t launch_reverse_complement(const uint8_t* seq, const int64_t* off, int32_t n_reads,
                                     int64_t n_letters, uint8_t* out, hipStream_t s) {
  int64_t blocks = (n_letters + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(reverse_complement_kernel, dim3((unsigned)blocks), dim3(256), 0, s, seq, off,
                     n_reads, out);
  return hipGetLastError();
}

hipError_t launch_merge_strands(const int32_t* fi, const float* ff, const int32_t* ri,
                                const float* rf, int32_t n_reads, int32_t k, float min_fidelity,
                                int32_t* top_idx, float* top_score, int8_t* top_strand,
                                int32_t* n_found, hipStream_t s) {
  hipLaunchKernelGGL(merge_strands_kernel, dim3((unsigned)(((int64_t)n_reads + 255) / 256)),
                     dim3(256), 0, s, fi, ff, ri, rf, n_reads, k, min_fidelity, top_idx, top_score,
                     top_strand, n_found);
  return hipGetLastError();
}

}  // namespace rm
