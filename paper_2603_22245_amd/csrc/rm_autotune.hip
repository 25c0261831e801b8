// Autotuner for the scoring launch: times candidate tile shapes on the caller's
// inputs with HIP events and keeps the fastest; results are cached as one JSON
// object per line, keyed by device architecture, precision, k_fetch and the
// groups' shapes.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rm_internal.h"

namespace {

std::mutex g_cache_mutex;  // serialises reads and appends of cache files

std::string make_key(const rm_index* idx, int32_t n_groups, const int32_t* n_reads,
                     int32_t k_fetch) {
  hipDeviceProp_t prop{};
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  std::string key = arch + "|p" + std::to_string(idx[0].p.precision) + "|k" +
                    std::to_string(k_fetch);
  for (int i = 0; i < n_groups; ++i)
    key += "|W" + std::to_string(idx[i].n_windows) + "R" + std::to_string(n_reads[i]) + "N" +
           std::to_string(idx[i].p.window_len);
  return key;
}

bool cache_lookup(const char* path, const std::string& key, rm_tuning* out, float* ms) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string needle = "\"key\": \"" + key + "\"";
  char line[4096];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    if (std::strstr(line, needle.c_str()) == nullptr) continue;
    int rt = 0, ct = 0;
    float t = 0.f;
    const char* a = std::strstr(line, "\"read_tile\": ");
    const char* b = std::strstr(line, "\"chunk_tiles\": ");
    const char* c = std::strstr(line, "\"ms\": ");
    if (a && b && c && std::sscanf(a, "\"read_tile\": %d", &rt) == 1 &&
        std::sscanf(b, "\"chunk_tiles\": %d", &ct) == 1 && std::sscanf(c, "\"ms\": %f", &t) == 1) {
      out->read_tile = rt;
      out->chunk_tiles = ct;
      if (ms) *ms = t;
      found = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_append(const char* path, const std::string& key, const rm_tuning& t, float ms) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"read_tile\": %d, \"chunk_tiles\": %d, \"ms\": %.4f}\n",
               key.c_str(), t.read_tile, t.chunk_tiles, ms);
  std::fclose(f);
}

}  // namespace

extern "C" int rm_autotune_score(const rm_index* idx, int32_t n_groups,
                                 const void* const* d_read_emb, const float* const* d_read_scale,
                                 const int32_t* n_reads, int32_t k_fetch,
                                 int32_t* const* d_cand_idx, float* const* d_cand_score,
                                 void* d_ws, size_t ws_bytes, const char* cache_path,
                                 rm_tuning* best, float* best_ms, void* stream) {
  if (best == nullptr) return RM_EINVAL;
  // validate through the default configuration's workspace query
  if (rm_score_groups_workspace_bytes(idx, n_groups, n_reads, k_fetch, nullptr) == 0)
    return idx == nullptr || n_reads == nullptr ? RM_EINVAL : RM_ESIZE;
  std::string key = make_key(idx, n_groups, n_reads, k_fetch);
  if (cache_path) {
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    if (cache_lookup(cache_path, key, best, best_ms)) return RM_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int kp = k_fetch <= 8 ? 8 : k_fetch <= 16 ? 16 : 32;
  std::vector<rm_tuning> cands;
  for (int rt : {256, 128}) {
    if (!rm::read_tile_ok(idx[0].p.precision, kp, rt)) continue;
    for (int ct : {0, 128, 512, 2048, 8192}) cands.push_back(rm_tuning{rt, ct});
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return RM_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RM_EHIP;
  }
  float best_t = -1.f;
  rm_tuning best_c{0, 0};
  int status = RM_OK;
  for (const rm_tuning& c : cands) {
    size_t need = rm_score_groups_workspace_bytes(idx, n_groups, n_reads, k_fetch, &c);
    if (need == 0 || need > ws_bytes) continue;
    // warm-up run, then one timed run
    int st = rm_score_topk_groups(idx, n_groups, d_read_emb, d_read_scale, n_reads, k_fetch,
                                  d_cand_idx, d_cand_score, d_ws, ws_bytes, &c, stream);
    if (st != RM_OK) {
      status = st;
      break;
    }
    if (hipEventRecord(e0, s) != hipSuccess) { status = RM_EHIP; break; }
    st = rm_score_topk_groups(idx, n_groups, d_read_emb, d_read_scale, n_reads, k_fetch,
                              d_cand_idx, d_cand_score, d_ws, ws_bytes, &c, stream);
    if (st != RM_OK) {
      status = st;
      break;
    }
    float ms = 0.f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      status = RM_EHIP;
      break;
    }
    if (best_t < 0.f || ms < best_t) {
      best_t = ms;
      best_c = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != RM_OK) return status;
  if (best_t < 0.f) return RM_ESIZE;  // no candidate fits the workspace
  *best = best_c;
  if (best_ms) *best_ms = best_t;
  if (cache_path) {
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    cache_append(cache_path, key, best_c, best_t);
  }
  return RM_OK;
}
