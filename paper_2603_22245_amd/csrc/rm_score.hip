// Scoring GEMM with fused per-read top-k (§3.1): FP32 and FP8 instantiations,
// the work plan, the launch sequence and the merge of per-chunk lists.  The
// kernel itself is in rm_score_kernel.h; FP16 is instantiated in
// rm_score_f16.hip.
#include "rm_score_kernel.h"

namespace rm {

namespace {

// Clears the work counter and every group's shared per-read thresholds and
// slots ("no information" = 0).
__global__ void clear_state(ScoreLaunch L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *L.counter = 0;
  for (int gi = 0; gi < L.n_groups; ++gi)
    if (i < L.g[gi].R) {
      L.g[gi].gthr[i] = 0u;
      uint4* slot = reinterpret_cast<uint4*>(L.g[gi].gslot + i * kScoreSlots);
#pragma unroll
      for (int u = 0; u < kScoreSlots / 2; ++u) slot[u] = make_uint4(0, 0, 0, 0);
    }
}

// Merge the P per-chunk lists of each read into its k_fetch best (keys are
// unique per read).  One wavefront per read (all its lanes active): each lane
// sorts the EMAX keys it holds (descending), then every round takes the
// wavefront maximum of the lanes' heads and the lane that held it drops its
// head.  Lane `out` keeps the
// round-`out` winner, so the k_fetch results are written with one coalesced
// store each.
template <int EMAX>
__global__ __launch_bounds__(256) void merge_kernel(const uint64_t* __restrict__ ws, int n_per_read,
                                                    int32_t R, int k_fetch,
                                                    int32_t* __restrict__ cand_idx,
                                                    float* __restrict__ cand_score) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= R) return;
  const uint64_t* src = ws + r * n_per_read;
  uint64_t mine[EMAX];
#pragma unroll
  for (int e = 0; e < EMAX; ++e) {
    int i = e * 64 + lane;
    mine[e] = i < n_per_read ? src[i] : 0;
  }
  // odd-even transposition sort, descending (EMAX rounds make it complete)
#pragma unroll
  for (int p = 0; p < EMAX; ++p)
#pragma unroll
    for (int e = p & 1; e + 1 < EMAX; e += 2) {
      uint64_t x = mine[e], y = mine[e + 1];
      mine[e] = x > y ? x : y;
      mine[e + 1] = x > y ? y : x;
    }
  uint64_t res = 0;
  for (int out = 0; out < k_fetch; ++out) {
    const uint64_t gbest = wave_max_u64(mine[0]);
    if (gbest != 0 && mine[0] == gbest) {
#pragma unroll
      for (int e = 0; e + 1 < EMAX; ++e) mine[e] = mine[e + 1];
      mine[EMAX - 1] = 0;
    }
    if (lane == out) res = gbest;
  }
  if (lane < k_fetch) {
    write_list_entry(res, &cand_idx[r * k_fetch + lane], &cand_score[r * k_fetch + lane]);
  }
}

// Instantiations: (precision, reads per block, list length, row format) ->
// (fragments per wavefront, list+buffer entries, ring stages, column blocks);
// LDS stays within 160 KB.
template <int KR>
hipError_t dispatch_f8(int read_tile, int kp, const ScoreLaunch& L, hipStream_t s) {
  if (read_tile == 256) {
    switch (kp) {
      case 8: return launch_persistent<RM_FP8_E4M3, 2, 8, 32, 4, 2, KR>(L, s);
      case 16: return launch_persistent<RM_FP8_E4M3, 2, 16, 32, 4, 2, KR>(L, s);
      default: return launch_persistent<RM_FP8_E4M3, 2, 32, 48, 3, 2, KR>(L, s);
    }
  }
  switch (kp) {
    case 8: return launch_persistent<RM_FP8_E4M3, 1, 8, 32, 4, 1, KR>(L, s);
    case 16: return launch_persistent<RM_FP8_E4M3, 1, 16, 32, 4, 1, KR>(L, s);
    case 32: return launch_persistent<RM_FP8_E4M3, 1, 32, 64, 4, 1, KR>(L, s);
    // 64-key lists with a 32-slot buffer: 96 KB of lists
    default: return launch_persistent<RM_FP8_E4M3, 1, 64, 96, 4, 1, KR>(L, s);
  }
}

template <int KR>
hipError_t dispatch_f32(int kp, const ScoreLaunch& L, hipStream_t s) {
  switch (kp) {
    case 8: return launch_persistent<RM_FP32, 1, 8, 32, 3, 1, KR>(L, s);
    case 16: return launch_persistent<RM_FP32, 1, 16, 32, 3, 1, KR>(L, s);
    case 32: return launch_persistent<RM_FP32, 1, 32, 64, 2, 1, KR>(L, s);
    // 64-key lists with a 16-slot buffer (80 KB) and two stages of at most 32 KB
    default: return launch_persistent<RM_FP32, 1, 64, 80, 2, 1, KR>(L, s);
  }
}

hipError_t dispatch(int precision, bool reduced, int read_tile, int kp, const ScoreLaunch& L,
                    hipStream_t s) {
  if (precision == RM_FP32)
    return reduced ? dispatch_f32<kRealReduced>(kp, L, s) : dispatch_f32<kReal>(kp, L, s);
  if (precision == RM_FP16) return dispatch_score_f16(read_tile, kp, reduced, L, s);
  return reduced ? dispatch_f8<kRealReduced>(read_tile, kp, L, s)
                 : dispatch_f8<kReal>(read_tile, kp, L, s);
}

}  // namespace

bool read_tile_ok(int precision, int kp, int read_tile) {
  if (read_tile == 128) return true;
  if (read_tile == 256) return precision != RM_FP32 && kp <= 32;  // 64-key lists: 128 reads
  return false;
}

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

ScorePlan plan_score(int precision, int n_groups, const int64_t* W, const int32_t* R, int k_fetch,
                     Tuning t) {
  ScorePlan p{};
  p.kp = k_fetch <= 8 ? 8 : k_fetch <= 16 ? 16 : k_fetch <= 32 ? 32 : 64;
  int rt = t.read_tile;
  if (rt == 0) rt = read_tile_ok(precision, p.kp, 256) ? 256 : 128;
  if (!read_tile_ok(precision, p.kp, rt) || n_groups < 1 || n_groups > kMaxGroups) return p;
  p.read_tile = rt;
  p.n_groups = n_groups;
  size_t off = 0;
  int64_t items = 0;
  for (int i = 0; i < n_groups; ++i) {
    GroupPlan& gp = p.g[i];
    gp.read_tiles = (int)(((int64_t)R[i] + rt - 1) / rt);
    // 256-read tiles run two fragments per wavefront; a group that would leave
    // a quarter or more of its padded reads empty takes 128-read tiles (one
    // fragment per wavefront, half the work per tile) in the same launch
    gp.thin = 0;
    if (rt == 256) {
      const int64_t t128 = ((int64_t)R[i] + 127) / 128;
      if (4 * 128 * t128 <= 3 * 256 * (int64_t)gp.read_tiles) {
        gp.thin = 1;
        gp.read_tiles = (int)t128;
      }
    }
    int64_t tiles = (W[i] + kPlanW - 1) / kPlanW;
    int64_t ct = t.chunk_tiles;
    if (ct <= 0) {
      // about 30 items per CU of a 256-CU chip (a short last round), at least
      // 64 tile units each, at most 1024 keys per read for the merge; fewer,
      // longer items leave an uneven last round, more items repeat each
      // read's top-k warm-up in more chunks
      int64_t P = (256 * 30 + gp.read_tiles - 1) / gp.read_tiles;
      if (P > (tiles + 63) / 64) P = (tiles + 63) / 64;
      if (P < 1) P = 1;
      ct = (tiles + P - 1) / P;
    }
    if (ct < 1) ct = 1;
    int64_t P = (tiles + ct - 1) / ct;
    if (P > 1024 / p.kp) {  // keep the merge within 1024 keys per read
      P = 1024 / p.kp;
      ct = (tiles + P - 1) / P;
      P = (tiles + ct - 1) / ct;
    }
    gp.chunk_windows = ct * kPlanW;
    gp.chunks = (int)P;
    gp.lists_offset = off;
    off = align256(off + (size_t)R[i] * (size_t)P * (size_t)p.kp * sizeof(uint64_t));
    gp.thr_offset = off;
    off = align256(off + (size_t)R[i] * sizeof(uint32_t));
    gp.slot_offset = off;
    off = align256(off + (size_t)R[i] * kScoreSlots * sizeof(uint64_t));
    items += (int64_t)gp.read_tiles * P;
  }
  p.counter_offset = off;
  p.ws_bytes = off + 256;
  p.total_items = items;
  p.ok = items > 0 && items < INT32_MAX;
  return p;
}

hipError_t launch_score_topk(const rm_index* idx, const ScorePlan& plan,
                             const void* const* read_emb, const float* const* read_scale,
                             const int32_t* R, int k_fetch, int32_t* const* cand_idx,
                             float* const* cand_score, void* ws, hipStream_t s) {
  uint8_t* base = static_cast<uint8_t*>(ws);
  ScoreLaunch L{};
  L.n_groups = plan.n_groups;
  L.total_items = (int32_t)plan.total_items;
  L.counter = reinterpret_cast<int*>(base + plan.counter_offset);
  int32_t item = 0;
  int32_t maxR = 0;
  for (int i = 0; i < plan.n_groups; ++i) {
    const GroupPlan& gp = plan.g[i];
    ScoreGroup& G = L.g[i];
    G.index = static_cast<const uint8_t*>(idx[i].d_emb);
    G.win_scale = idx[i].d_scale;
    G.W = idx[i].n_windows;
    G.reads = static_cast<const uint8_t*>(read_emb[i]);
    G.read_scale = read_scale ? read_scale[i] : nullptr;
    G.R = R[i];
    G.read_tiles = gp.read_tiles;
    G.chunk_windows = gp.chunk_windows;
    G.P = gp.chunks;
    G.item_begin = item;
    G.thin = gp.thin;
    G.lists = reinterpret_cast<uint64_t*>(base + gp.lists_offset);
    G.gthr = reinterpret_cast<uint32_t*>(base + gp.thr_offset);
    G.gslot = reinterpret_cast<uint64_t*>(base + gp.slot_offset);
    item += gp.read_tiles * gp.chunks;
    if (R[i] > maxR) maxR = R[i];
  }
  hipLaunchKernelGGL(clear_state, dim3((unsigned)(((int64_t)maxR + 255) / 256)), dim3(256), 0, s, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = dispatch(idx[0].p.precision, reduced_rows(idx[0].p), plan.read_tile, plan.kp, L, s);
  if (e != hipSuccess) return e;
  for (int i = 0; i < plan.n_groups; ++i) {
    int n_per_read = plan.g[i].chunks * plan.kp;
    unsigned blocks = (unsigned)(((int64_t)R[i] + 3) / 4);
    // n_per_read <= 1024 (plan_score keeps the merge within 1024 keys)
    auto kern = n_per_read <= 256 ? merge_kernel<4> : n_per_read <= 512 ? merge_kernel<8>
                                                                        : merge_kernel<16>;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<const uint64_t*>(base + plan.g[i].lists_offset), n_per_read,
                       R[i], k_fetch, cand_idx[i], cand_score[i]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rm
