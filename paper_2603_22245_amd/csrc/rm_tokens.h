// Token encodings (§2.1 s-mers, §2.6 compact versions): shared device helpers
// and the launchers of the token kernels.
//
// The token at location q of a string is the s-mer str[q .. q+s); its code is
// sum_i str[q+i] 4^(s-1-i) and its class is table[code] (an index's class
// table: values below n_class, or RM_TOKEN_SKIP).  Component index
// k * n_class + class (0-based factor k), n_class * m = 128.
//
// Lane layout: lane l owns the complex components 2l and 2l+1, i.e. factor
// k = 2l / n_class and classes c0 = 2l mod n_class and c0 + 1 (n_class is
// even), stored at reals [4l, 4l+4) of the 256-real row -- the same storage
// as the letter encoding, so the scoring product is shared unchanged.
#pragma once

#include "rm_internal.h"

namespace rm {

// "No token here": an s-mer holding a letter outside 0..3, or a location
// past the end.  Negative, so it matches no component whatever n_class is (a
// table value >= n_class matches none either; with n_class = 256 every table
// value is a class).
constexpr int kNoToken = -1;

// Class of the token starting at p.
__device__ __forceinline__ int token_class(const uint8_t* __restrict__ p, int s,
                                           const uint8_t* __restrict__ table) {
  uint32_t code = 0;
  bool ok = true;
  for (int i = 0; i < s; ++i) {
    const uint32_t L = p[i];
    ok = ok && L < 4u;
    code = code * 4u + (L & 3u);
  }
  return ok ? (int)table[code] : kNoToken;
}

// Direct sum over the tokens at locations 0..T-1 of `str` of this lane's two
// components: a0 += phase[q][k] where class(q) == c0, a1 where == c0 + 1.
// `phase` is the [location][m] table (a range of locations is summed by
// advancing str and phase together).
template <typename C2, typename E2>
__device__ __forceinline__ void direct_sum_tokens(const uint8_t* __restrict__ str, int T, int s,
                                                  const uint8_t* __restrict__ table,
                                                  const E2* __restrict__ phase, int m, int k,
                                                  int c0, int lane, C2& a0, C2& a1) {
  a0.x = 0; a0.y = 0;
  a1.x = 0; a1.y = 0;
  for (int pb = 0; pb < T; pb += 64) {
    const int mine = (pb + lane < T) ? token_class(str + pb + lane, s, table) : kNoToken;
    const int cnt = min(64, T - pb);
    // groups of 8 locations with their table loads in flight together; a
    // location past the end re-reads the last row and has no token
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      E2 e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) e[u] = phase[(int64_t)min(pb + i0 + u, T - 1) * m + k];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = __builtin_amdgcn_readlane(mine, i0 + u);
        a0.x += (c == c0) ? e[u].x : 0;
        a0.y += (c == c0) ? e[u].y : 0;
        a1.x += (c == c0 + 1) ? e[u].x : 0;
        a1.y += (c == c0 + 1) ? e[u].y : 0;
      }
    }
  }
}

// table[code] for code < 4^s: the caller's map with values >= n_class set to
// RM_TOKEN_SKIP (a value no lane's classes include when n_class <= 128), or the
// identity when map is NULL.
hipError_t launch_token_table(const uint8_t* map, int s, int n_class, uint8_t* table,
                              hipStream_t st);

hipError_t launch_encode_reference_tokens(const uint8_t* ref, int64_t W, const rm_params& p,
                                          const double* phase64, const float* step32,
                                          const uint8_t* table, void* emb, float* scale,
                                          float* norm2, hipStream_t st);

hipError_t launch_encode_reads_tokens(const rm_params& p, const float* phase32,
                                      const uint8_t* table, const uint8_t* seq, const int64_t* off,
                                      int32_t n_reads, void* emb, float* scale, hipStream_t st);

// Encodings of 1,024 complex components (16 per lane), FP16 or FP8.
constexpr int kWideComplex = 1024;
constexpr int kWideMaxChunks = 16;  // window chunks per read tile (merge reads <= 16 x 32 keys)

struct WidePlan {
  int n_rt;             // read tiles (128 reads each)
  int64_t n_tiles;      // window tiles of 128
  int64_t chunk_tiles;  // window tiles per chunk
  int n_chunks;
  int n_quads;          // groups of 4 chunks
  int64_t n_blocks;     // grid size
};
WidePlan plan_wide(int32_t n_reads, int64_t W);
size_t wide_workspace_bytes(int32_t n_reads, int64_t W, int32_t k_fetch);
hipError_t launch_encode_reference_wide(const uint8_t* ref, int64_t W, const rm_params& p,
                                        const double* phase64, const float* step32,
                                        const uint8_t* table, void* emb, float* scale,
                                        float* norm2, hipStream_t st);
hipError_t launch_encode_reads_wide(const rm_params& p, const float* phase32,
                                    const uint8_t* table, const uint8_t* seq, const int64_t* off,
                                    int32_t n_reads, void* emb, float* scale, hipStream_t st);
hipError_t launch_score_wide(const rm_index& idx, const void* read_emb, const float* read_scale,
                             int32_t n_reads, int32_t k_fetch, int32_t* cand_idx,
                             float* cand_score, void* ws, hipStream_t st);
hipError_t launch_rescore_wide(const rm_index& idx, const uint8_t* ref, const uint8_t* seq,
                               const int64_t* off, int32_t n_reads, int32_t k_fetch,
                               const int32_t* cand_idx, int32_t k, int32_t* top_idx,
                               float* top_score, hipStream_t st);

// The reference's s-mer counts (4^s uint32, zeroed here) and the map that
// keeps its n_class most frequent s-mers (§2.6).
hipError_t launch_token_counts(const uint8_t* ref, int64_t ref_len, int s, uint32_t* counts,
                               hipStream_t st);
hipError_t launch_token_select(const uint32_t* counts, int s, int n_class, uint8_t* map,
                               hipStream_t st);

// Refinement around coarse candidates (§3.4) for token indexes: each read's
// k_fetch * (2 radius + 1) keys go to the workspace `ws`, in the layout of the
// letter refinement, then launch_refine_select keeps the k best distinct starts.
hipError_t launch_refine_tokens(const rm_index& coarse, const uint8_t* ref, const uint8_t* seq,
                                const int64_t* off, int32_t n_reads, int32_t k_fetch,
                                const int32_t* cand_idx, int32_t radius, int32_t k,
                                int32_t* top_idx, float* top_score, void* ws, hipStream_t st);
hipError_t launch_refine_wide(const rm_index& coarse, const uint8_t* ref, const uint8_t* seq,
                              const int64_t* off, int32_t n_reads, int32_t k_fetch,
                              const int32_t* cand_idx, int32_t radius, int32_t k, int32_t* top_idx,
                              float* top_score, void* ws, hipStream_t st);
// The k best distinct starts of each read's n pool keys (key 0 = empty slot).
hipError_t launch_refine_select(const uint64_t* pool, int n, int32_t n_reads, int32_t k,
                                int32_t* top_idx, float* top_score, hipStream_t st);

hipError_t launch_rescore_tokens(const rm_index& idx, const uint8_t* ref, const uint8_t* seq,
                                 const int64_t* off, int32_t n_reads, int32_t k_fetch,
                                 const int32_t* cand_idx, int32_t k, int32_t* top_idx,
                                 float* top_score, hipStream_t st);

}  // namespace rm
