// Scoring GEMM with fused per-read top-k, and the merge of per-chunk lists.
//
// §3.1 computes the fidelity of every read head with every index vector -- a
// matrix product -- and keeps the best locations.  With reads stored as two
// real rows (Re row (xr, xi), Im row (-xi, xr)) and windows as one real row
// (cr, ci), the real product S = A B^T gives Re<x|c> = S[2r, j] and
// Im<x|c> = S[2r+1, j] (the complex/real isomorphism of §4), and
// F = Re^2 + Im^2 for unit vectors (times (s_r s_j)^2 for FP8 scales).
//
// Work item = (read tile, window chunk).  A block keeps its read tile in
// registers (each wavefront owns NF fragments of 32 rows = 16 reads, the full
// K = 256) and streams the chunk's windows through LDS in tiles of 32
// (double-buffered).  Per tile every wavefront runs NF x (256/K_mfma) MFMAs
// on 32x32 output blocks; the epilogue forms F per (read, window) in
// registers, compares with the read's current k-th best and, only for hits,
// appends (F, j) to the read's LDS buffer.  Full buffers are merged into the
// read's sorted list by a bitonic sort across lanes.  The score matrix never
// leaves registers.
//
// List entries are 64-bit keys: high word = float bits of F plus one (0 means
// empty), low word = ~j; a larger key is a better candidate (F descending,
// then window id ascending), so one integer comparison orders them exactly.
#include "rm_internal.h"

namespace rm {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kTileW = 32;  // windows per B tile (the MFMA N dimension)
// The register test re^2 + im^2 - t > 0 is computed with fused multiply-adds,
// which round differently from the F stored in a key; lowering t by 2^-20
// relative sends every candidate within rounding of the k-th best to the exact
// key comparison instead of dropping it.  (t < 0 for a list that is not full.)
constexpr float kLoose = 1.0f - 1.0f / 1048576.0f;

__device__ __forceinline__ uint64_t make_key(float F, int32_t j) {
  uint32_t hi = __float_as_uint(F) + 1u;  // F >= 0
  uint32_t lo = 0xffffffffu - (uint32_t)j;
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ float key_score(uint64_t key) {
  uint32_t hi = (uint32_t)(key >> 32);
  return hi ? __uint_as_float(hi - 1u) : -1.f;
}
__device__ __forceinline__ int32_t key_index(uint64_t key) {
  uint32_t hi = (uint32_t)(key >> 32);
  return hi ? (int32_t)(0xffffffffu - (uint32_t)key) : -1;
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int d) {
  uint32_t lo = __shfl_xor((uint32_t)v, d, 64);
  uint32_t hi = __shfl_xor((uint32_t)(v >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Sort keys descending within each group of ENT consecutive lanes (bitonic).
template <int ENT>
__device__ __forceinline__ uint64_t sort_desc(uint64_t key, int lane) {
  const int id = lane & (ENT - 1);
#pragma unroll
  for (int kk = 2; kk <= ENT; kk <<= 1) {
#pragma unroll
    for (int d = kk >> 1; d > 0; d >>= 1) {
      uint64_t other = shfl_xor64(key, d);
      bool desc_block = (id & kk) == 0;
      bool lower = (id & d) == 0;
      bool keep_max = (lower == desc_block);
      uint64_t mx = key > other ? key : other;
      uint64_t mn = key > other ? other : key;
      key = keep_max ? mx : mn;
    }
  }
  return key;
}

template <int PREC>
struct Prec;
template <>
struct Prec<RM_FP32> {
  static constexpr int esize = 4;
};
template <>
struct Prec<RM_FP16> {
  static constexpr int esize = 2;
};
template <>
struct Prec<RM_FP8_E4M3> {
  static constexpr int esize = 1;
};

// LDS byte offset of a pointer into a __shared__ array.
__device__ __forceinline__ uint32_t lds_offset(const void* p) {
  return (uint32_t)(uintptr_t)((__attribute__((address_space(3))) const void*)p);
}

// Asynchronous copy from global memory straight into LDS (gfx950
// global_load_lds_*): lane l writes 16 (dma16) or 4 (dma4) bytes at LDS
// offset lds + l * size.  Written as inline assembly, with no output register,
// so that the compiler does not drain every outstanding copy (vmcnt(0)) before
// each LDS read; completion is awaited explicitly with wait_vmcnt<N>(), which
// counts this wavefront's vector-memory operations in issue order.
__device__ __forceinline__ void dma16(const void* src, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(lds)
               : "memory");
}
__device__ __forceinline__ void dma4(const void* src, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dword %0, off" ::"v"(src), "s"(lds)
               : "memory");
}
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// B tiles in LDS: row r (one window, RB bytes) stores its logical 16-byte chunk
// c at position c ^ (r & 15).  A lane reading chunk c of row `col` therefore
// reads byte offset col*RB + 16 (c ^ (col & 15)); the 16 lanes of one LDS
// access cycle (consecutive col, same c) hit 16 different bank groups.
//
// One 32x32 output block per fragment over the full K = 256.  `a[f]` holds
// this lane's 128 K-elements of fragment f (K range [128 g, 128 g + 128),
// g = lane / 32, in natural order); `row` points at this lane's window row in
// the current LDS stage and kx = (byte offset of the lane's K half) ^
// 16 (col & 15), so logical byte offset o is found at row + (kx ^ o).  Any
// assignment of K indices to (lane group, register slot) works as long as A
// and B use the same one, which they do here.
template <int PREC, int NF, int AU4>
__device__ __forceinline__ void mfma_tile(const uint4 (&a)[NF][AU4], const uint8_t* row,
                                          uint32_t kx, f32x16 (&acc)[NF]) {
  if constexpr (PREC == RM_FP16) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      uint4 bv = *reinterpret_cast<const uint4*>(row + (kx ^ (16u * s)));
      half8 bh = __builtin_bit_cast(half8, bv);
#pragma unroll
      for (int f = 0; f < NF; ++f)
        acc[f] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a[f][s]), bh,
                                                        acc[f], 0, 0, 0);
    }
  } else if constexpr (PREC == RM_FP8_E4M3) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      uint4 b0 = *reinterpret_cast<const uint4*>(row + (kx ^ (32u * s)));
      uint4 b1 = *reinterpret_cast<const uint4*>(row + (kx ^ (32u * s + 16u)));
      i32x8 bb = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w,
                  (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const uint4 a0 = a[f][2 * s], a1 = a[f][2 * s + 1];
        i32x8 aa = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w,
                    (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
        // formats 0/0 = FP8 e4m3 for both operands; E8M0 scales 127 = 1.0
        acc[f] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(aa, bb, acc[f], 0, 0, 0, 127, 0,
                                                                  127);
      }
    }
  } else {
#pragma unroll
    for (int s4 = 0; s4 < 32; ++s4) {
      uint4 bv = *reinterpret_cast<const uint4*>(row + (kx ^ (16u * s4)));
      float bf[4] = {__uint_as_float(bv.x), __uint_as_float(bv.y), __uint_as_float(bv.z),
                     __uint_as_float(bv.w)};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const uint4 av = a[f][s4];
          uint32_t ab = q == 0 ? av.x : q == 1 ? av.y : q == 2 ? av.z : av.w;
          acc[f] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(ab), bf[q], acc[f], 0, 0, 0);
        }
      }
    }
  }
}

template <int PREC, int NF, int WAVES, int KP, int ENT, int STAGES>
struct ScoreKernel {
  static constexpr int esize = Prec<PREC>::esize;
  static constexpr int RB = kReal * esize;              // bytes per embedding row
  static constexpr int CPR = RB / 16;                   // 16-byte chunks per row
  static constexpr int AU4 = (kReal / 2) * esize / 16;  // uint4 per lane per fragment
  static constexpr int READS = WAVES * NF * 16;         // reads per block
  static constexpr int THREADS = WAVES * 64;
  static constexpr int TILE = kTileW * RB;              // bytes per B tile
  static constexpr int L = TILE / 1024 / WAVES;         // 1 KB copies per wave per tile
  static constexpr int LT = L + (PREC == RM_FP8_E4M3 ? 1 : 0);  // + the window scales
  static constexpr int CB = ENT - KP;                   // buffer slots per read
  static_assert(L >= 1 && TILE % (1024 * WAVES) == 0, "tile/waves");
  static_assert(CB >= 1, "buffer");
  static_assert(STAGES >= 2, "stages");
};

template <int PREC, int NF, int WAVES, int KP, int ENT, int STAGES>
__global__ __launch_bounds__(WAVES * 64) void score_topk_kernel(
    const uint8_t* __restrict__ index, const float* __restrict__ win_scale, int64_t W,
    const uint8_t* __restrict__ reads, const float* __restrict__ read_scale, int32_t R,
    int read_tiles, int64_t chunk_windows, int P, uint64_t* __restrict__ ws,
    uint32_t* __restrict__ gthr) {
  using K = ScoreKernel<PREC, NF, WAVES, KP, ENT, STAGES>;
  constexpr bool kFp8 = PREC == RM_FP8_E4M3;
  __shared__ __align__(1024) uint8_t ring[STAGES * K::TILE];
  __shared__ __align__(16) float ring_scale[kFp8 ? STAGES * WAVES * 32 : 4];
  __shared__ uint64_t lst[K::READS][ENT];
  __shared__ int cnt[K::READS];
  __shared__ float thr[K::READS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 5;
  const int col = lane & 31;
  const int chunk = blockIdx.x / read_tiles;
  const int tile = blockIdx.x % read_tiles;
  const int64_t read0 = (int64_t)tile * K::READS;
  const int64_t wbeg = (int64_t)chunk * chunk_windows;
  const int64_t wend = min(W, wbeg + chunk_windows);
  const int ntiles = (int)((wend - wbeg + kTileW - 1) / kTileW);

  // ---- per-read state (each wavefront owns its reads)
  const int rb0 = wave * NF * 16;
  for (int i = lane; i < NF * 16 * ENT; i += 64) lst[rb0 + i / ENT][i % ENT] = 0;
  if (lane < NF * 16) {
    cnt[rb0 + lane] = 0;
    thr[rb0 + lane] = -1.f;
  }

  // ---- A fragments: this lane's K half of row (read tile row) for each fragment
  uint4 a[NF][K::AU4];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    int64_t row = 2 * read0 + (int64_t)(wave * NF + f) * 32 + col;
    if (row < 2 * (int64_t)R) {
      const uint4* src = reinterpret_cast<const uint4*>(reads + row * K::RB + g * (K::RB / 2));
#pragma unroll
      for (int u = 0; u < K::AU4; ++u) a[f][u] = src[u];
    } else {
#pragma unroll
      for (int u = 0; u < K::AU4; ++u) a[f][u] = make_uint4(0, 0, 0, 0);
    }
  }
  // per (fragment, slot): s_r^2 and its inverse (FP8; 1 otherwise)
  float rs2[NF][8], irs2[NF][8];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      rs2[f][q] = 1.f;
      irs2[f][q] = 1.f;
      if constexpr (kFp8) {
        int64_t r = read0 + (wave * NF + f) * 16 + 4 * (q >> 1) + 2 * g + (q & 1);
        float s = r < R ? read_scale[r] : 0.f;
        rs2[f][q] = s * s;
        irs2[f][q] = rs2[f][q] > 0.f ? 1.f / rs2[f][q] : 0.f;
      }
    }
  // Wait for these loads here, before the tile loop: otherwise the compiler's
  // wait-count state from them reaches into the loop.
  {
    uint32_t any = 0;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int u = 0; u < K::AU4; ++u) any |= a[f][u].x | a[f][u].w;
    __builtin_amdgcn_s_waitcnt(0);
    if (any == 0xdeadbeefu && R < 0) ws[0] = any;  // never true; keeps the use
  }

  // thresholds in the product's units: F-threshold / s_r^2 (further divided by
  // s_j^2 per window in the epilogue), lowered by kLoose
  float th[NF][8];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int q = 0; q < 8; ++q) th[f][q] = -1.f;

  // ---- B tiles: asynchronous copies into an LDS ring of STAGES tiles
  const uint32_t ring_lds = lds_offset(ring);
  const uint32_t scale_lds = lds_offset(ring_scale);
  int drow[K::L];
  uint32_t doff[K::L];
#pragma unroll
  for (int i = 0; i < K::L; ++i) {
    int pos = (i * WAVES + wave) * 64 + lane;  // physical 16-byte chunk in the tile
    int r = pos / K::CPR;
    int c = (pos % K::CPR) ^ (r & 15);          // logical chunk stored there
    drow[i] = r;
    doff[i] = (uint32_t)c * 16u;
  }
  // copy window tile `tsrc` into ring stage `stage`
  auto issue_into = [&](int tsrc, int stage) {
    const int64_t tb = wbeg + (int64_t)tsrc * kTileW;
#pragma unroll
    for (int i = 0; i < K::L; ++i) {
      int64_t grow = min(tb + drow[i], wend - 1);  // rows past the chunk: any valid row
      dma16(index + grow * K::RB + doff[i],
            __builtin_amdgcn_readfirstlane(ring_lds + stage * K::TILE + (i * WAVES + wave) * 1024));
    }
    if constexpr (kFp8) {
      if (lane < 32)
        dma4(win_scale + min(tb + lane, wend - 1),
             __builtin_amdgcn_readfirstlane(scale_lds + (stage * WAVES + wave) * 128));
    }
  };

  // ---- thresholds: the larger of this chunk's k-th best and the best k-th
  // best any chunk has published for the read (0 = none yet)
  auto refresh_thresholds = [&]() {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        int rb = rb0 + f * 16 + 4 * (q >> 1) + 2 * g + (q & 1);
        int64_t r = read0 + rb;
        uint32_t gk = r < R ? __hip_atomic_load(&gthr[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        float gt = gk ? __uint_as_float(gk - 1u) : -1.f;
        th[f][q] = fmaxf(thr[rb], gt) * irs2[f][q] * kLoose;
      }
  };

  // ---- merge a read's buffer into its list (whole wavefront, uniform call)
  auto merge_reads = [&](uint32_t mask) {
    // ENT == 32: two reads at a time (one per half-wave); ENT == 64: one read.
    while (mask) {
      int r0 = __builtin_ctz(mask);
      mask &= mask - 1;
      int r1 = -1;
      if (ENT == 32 && mask) {
        r1 = __builtin_ctz(mask);
        mask &= mask - 1;
      }
      int my = (ENT == 32 && lane >= 32) ? r1 : r0;
      int id = lane & (ENT - 1);
      if (my >= 0) {
        int rb = rb0 + my;
        int n = min(cnt[rb], K::CB);
        uint64_t key = (id < KP + n) ? lst[rb][id] : 0;
        key = sort_desc<ENT>(key, lane);
        if (id < KP) lst[rb][id] = key;
        if (id == KP - 1) {
          float kth = key_score(key);
          thr[rb] = kth;
          // publish this chunk's k-th best: no window scoring below it can be
          // in the read's final list, whichever chunk holds it
          if (kth >= 0.f && read0 + rb < R) atomicMax(&gthr[read0 + rb], __float_as_uint(kth) + 1u);
        }
        if (id == 0) cnt[rb] = 0;
      }
    }
    __builtin_amdgcn_wave_barrier();
    refresh_thresholds();
  };

  // lane's B row offset and K-half key (see mfma_tile)
  const uint32_t kx = ((uint32_t)g * (K::RB / 2)) ^ (16u * (uint32_t)(col & 15));

  // Pipeline: the ring always has copies of the next STAGES-2 tiles in flight
  // (past the last tile the copies repeat the last tile, so every tile step
  // issues the same number of copies and waits for the same count).  A tile
  // step waits for its own tile, synchronises the block (every copy landed;
  // the stage of the previous tile is free), refills that stage and issues
  // the tile's MFMAs.  The epilogue of tile t runs after the MFMAs of tile t+1
  // have been issued, in the same basic block, so its VALU work fills the
  // MFMA pipeline's latency.
  auto start_tile = [&](int t, f32x16 (&acc)[NF], float& sj2) {
    wait_vmcnt<(STAGES - 2) * K::LT>();
    __syncthreads();
    const int stage = t % STAGES;
    if constexpr (kFp8) {
      float sc = ring_scale[(stage * WAVES + wave) * 32 + col];
      sj2 = sc * sc;
    }
    issue_into(min(t + STAGES - 1, ntiles - 1), (t + STAGES - 1) % STAGES);
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = f32x16{};
    mfma_tile<PREC, NF, K::AU4>(a, ring + stage * K::TILE + col * K::RB, kx, acc);
  };

  // re^2 + im^2 - threshold per (read slot, window col), reduced with max;
  // only a positive maximum anywhere in the wavefront leads to the (rare)
  // per-score test and appends.
  auto epilogue = [&](int t, const f32x16 (&acc)[NF], float sj2) {
    if ((t & 255) == 255) refresh_thresholds();  // pick up other chunks' progress
    const int64_t tbase = wbeg + (int64_t)t * kTileW;
    const int32_t j = (int32_t)(tbase + col);
    const bool colok = tbase + col < wend;
    float isj2 = 1.f;
    if constexpr (kFp8) isj2 = sj2 > 0.f ? 1.f / sj2 : 0.f;
    float ex = -1.f;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float re = acc[f][2 * q], im = acc[f][2 * q + 1];
        float tq = th[f][q];
        if constexpr (kFp8) tq = tq * isj2;
        ex = fmaxf(ex, __builtin_fmaf(re, re, __builtin_fmaf(im, im, -tq)));
      }
    if (!colok) ex = -1.f;

    if (__ballot(ex > 0.f)) {
      uint32_t pend = 0;
      float Fv[NF][8];
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          float re = acc[f][2 * q], im = acc[f][2 * q + 1];
          float F = re * re + im * im;
          if constexpr (kFp8) F = F * (rs2[f][q] * sj2);
          Fv[f][q] = F;
          float tq = th[f][q];
          if constexpr (kFp8) tq = tq * isj2;
          pend |= (uint32_t)(colok && __builtin_fmaf(re, re, __builtin_fmaf(im, im, -tq)) > 0.f)
                  << (f * 8 + q);
        }
      // append every hit, merging reads whose buffer is full, until nothing
      // is pending
      while (true) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const uint32_t bit = 1u << (f * 8 + q);
            if (pend & bit) {
              int rb = rb0 + f * 16 + 4 * (q >> 1) + 2 * g + (q & 1);
              int pos = atomicAdd(&cnt[rb], 1);
              if (pos < K::CB) {
                lst[rb][KP + pos] = make_key(Fv[f][q], j);
                pend &= ~bit;
              }
            }
          }
        __builtin_amdgcn_wave_barrier();
        bool full = lane < NF * 16 && cnt[rb0 + lane] >= K::CB;
        uint32_t fm = (uint32_t)__ballot(full);
        if (fm) merge_reads(fm);
        if (!__ballot(pend != 0)) break;
      }
    }
  };

#pragma unroll
  for (int t = 0; t < STAGES - 1; ++t) issue_into(min(t, ntiles - 1), t);

  // FP16 keeps one accumulator set: its A fragments take 128 VGPRs and a
  // second set would spill at two wavefronts per SIMD.
  constexpr bool kPipe = PREC != RM_FP16;
  refresh_thresholds();
  f32x16 accA[NF];
  float sjA = 1.f;
  if constexpr (kPipe) {
    f32x16 accB[NF];
    float sjB = 1.f;
    start_tile(0, accA, sjA);
    for (int t = 0;; t += 2) {
      start_tile(t + 1, accB, sjB);  // past the end: a repeat of the last tile, unused
      epilogue(t, accA, sjA);
      if (t + 1 >= ntiles) break;
      start_tile(t + 2, accA, sjA);
      epilogue(t + 1, accB, sjB);
      if (t + 2 >= ntiles) break;
    }
  } else {
    for (int t = 0; t < ntiles; ++t) {
      start_tile(t, accA, sjA);
      epilogue(t, accA, sjA);
    }
  }
  wait_vmcnt<0>();  // no copy may still be writing this block's LDS

  // ---- final merge and write-out of this chunk's lists
  {
    bool any = lane < NF * 16 && cnt[rb0 + lane] > 0;
    uint32_t m = (uint32_t)__ballot(any);
    if (m) merge_reads(m);
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < NF * 16 * KP; i += 64) {
      int rr = i / KP, e = i % KP;
      int64_t r = read0 + rb0 + rr;
      if (r < R) ws[((int64_t)r * P + chunk) * KP + e] = lst[rb0 + rr][e];
    }
  }
}

// Shared per-read thresholds start with "no information" (0).
__global__ void clear_thresholds(uint32_t* __restrict__ gthr, int32_t R) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R) gthr[i] = 0u;
}

// Merge the P per-chunk lists of each read into its k_fetch best: repeated
// wavefront-wide arg-max over the P*KP keys (keys are unique per read).
__global__ __launch_bounds__(256) void merge_kernel(const uint64_t* __restrict__ ws, int n_per_read,
                                                    int32_t R, int k_fetch,
                                                    int32_t* __restrict__ cand_idx,
                                                    float* __restrict__ cand_score) {
  constexpr int EMAX = 16;
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
  for (int out = 0; out < k_fetch; ++out) {
    uint64_t best = 0;
#pragma unroll
    for (int e = 0; e < EMAX; ++e) best = mine[e] > best ? mine[e] : best;
    uint64_t gbest = best;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      uint64_t o = shfl_xor64(gbest, d);
      gbest = o > gbest ? o : gbest;
    }
    if (gbest != 0 && best == gbest) {
#pragma unroll
      for (int e = 0; e < EMAX; ++e)
        if (mine[e] == gbest) mine[e] = 0;
    }
    if (lane == 0) {
      cand_idx[r * k_fetch + out] = key_index(gbest);
      cand_score[r * k_fetch + out] = key_score(gbest);
    }
  }
}

struct Shape {
  int nf, waves, kp, ent;
};

Shape shape_for(int precision, int k_fetch) {
  int kp = k_fetch <= 8 ? 8 : k_fetch <= 16 ? 16 : 32;
  int ent = kp <= 16 ? 32 : 64;
  int nf = precision == RM_FP32 ? 1 : 2;
  int waves = 8;
  if (precision == RM_FP16 && kp == 32) waves = 4;
  return {nf, waves, kp, ent};
}

template <int PREC, int NF, int WAVES, int KP, int ENT, int STAGES>
hipError_t launch_one(const rm_index& idx, const ScorePlan& plan, const void* read_emb,
                      const float* read_scale, int32_t R, void* ws, hipStream_t s) {
  unsigned blocks = (unsigned)plan.read_tiles * (unsigned)plan.chunks;
  hipLaunchKernelGGL((score_topk_kernel<PREC, NF, WAVES, KP, ENT, STAGES>), dim3(blocks),
                     dim3(WAVES * 64), 0, s, static_cast<const uint8_t*>(idx.d_emb), idx.d_scale,
                     idx.n_windows, static_cast<const uint8_t*>(read_emb), read_scale, R,
                     plan.read_tiles, plan.chunk_windows, plan.chunks, static_cast<uint64_t*>(ws),
                     reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(ws) + plan.thr_offset));
  return hipGetLastError();
}

// LDS per block: ring STAGES x 32 rows + lists READS x ENT x 8 B (+ FP8 scales),
// kept within 160 KB.
template <int PREC>
hipError_t dispatch_kp(const rm_index& idx, const ScorePlan& plan, const void* read_emb,
                       const float* read_scale, int32_t R, void* ws, hipStream_t s) {
  if constexpr (PREC == RM_FP32) {
    switch (plan.kp) {
      case 8: return launch_one<PREC, 1, 8, 8, 32, 3>(idx, plan, read_emb, read_scale, R, ws, s);
      case 16: return launch_one<PREC, 1, 8, 16, 32, 3>(idx, plan, read_emb, read_scale, R, ws, s);
      default: return launch_one<PREC, 1, 8, 32, 64, 2>(idx, plan, read_emb, read_scale, R, ws, s);
    }
  } else if constexpr (PREC == RM_FP16) {
    switch (plan.kp) {
      case 8: return launch_one<PREC, 2, 8, 8, 32, 4>(idx, plan, read_emb, read_scale, R, ws, s);
      case 16: return launch_one<PREC, 2, 8, 16, 32, 4>(idx, plan, read_emb, read_scale, R, ws, s);
      default: return launch_one<PREC, 2, 4, 32, 64, 4>(idx, plan, read_emb, read_scale, R, ws, s);
    }
  } else {
    switch (plan.kp) {
      case 8: return launch_one<PREC, 2, 8, 8, 32, 4>(idx, plan, read_emb, read_scale, R, ws, s);
      case 16: return launch_one<PREC, 2, 8, 16, 32, 4>(idx, plan, read_emb, read_scale, R, ws, s);
      default: return launch_one<PREC, 2, 8, 32, 64, 3>(idx, plan, read_emb, read_scale, R, ws, s);
    }
  }
}

}  // namespace

ScorePlan plan_score(int precision, int64_t W, int32_t n_reads, int32_t k_fetch) {
  Shape sh = shape_for(precision, k_fetch);
  ScorePlan p{};
  p.kp = sh.kp;
  p.reads_per_block = sh.waves * sh.nf * 16;
  p.read_tiles = (int)(((int64_t)n_reads + p.reads_per_block - 1) / p.reads_per_block);
  // Enough blocks to fill 256 CUs several times, chunks of at least 64 tiles,
  // and at most 1024 keys per read for the merge.
  int64_t target_blocks = 256 * 8;
  int64_t P = (target_blocks + p.read_tiles - 1) / p.read_tiles;
  int64_t max_by_len = (W + 64 * kTileW - 1) / (64 * kTileW);
  if (P > max_by_len) P = max_by_len;
  if (P > 1024 / sh.kp) P = 1024 / sh.kp;
  if (P < 1) P = 1;
  int64_t cw = (W + P - 1) / P;
  cw = (cw + kTileW - 1) / kTileW * kTileW;
  if (cw < kTileW) cw = kTileW;
  p.chunk_windows = cw;
  p.chunks = (int)((W + cw - 1) / cw);
  if (p.chunks < 1) p.chunks = 1;
  size_t lists = (size_t)n_reads * (size_t)p.chunks * (size_t)p.kp * sizeof(uint64_t);
  p.thr_offset = (lists + 255) / 256 * 256;
  p.ws_bytes = p.thr_offset + (size_t)n_reads * sizeof(uint32_t);
  return p;
}

hipError_t launch_score_topk(const rm_index& idx, const ScorePlan& plan, const void* read_emb,
                             const float* read_scale, int32_t n_reads, int32_t k_fetch,
                             int32_t* cand_idx, float* cand_score, void* ws, hipStream_t s) {
  hipLaunchKernelGGL(clear_thresholds, dim3((unsigned)(((int64_t)n_reads + 255) / 256)), dim3(256),
                     0, s, reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(ws) + plan.thr_offset),
                     n_reads);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (idx.p.precision) {
    case RM_FP32:
      e = dispatch_kp<RM_FP32>(idx, plan, read_emb, read_scale, n_reads, ws, s);
      break;
    case RM_FP16:
      e = dispatch_kp<RM_FP16>(idx, plan, read_emb, read_scale, n_reads, ws, s);
      break;
    default:
      e = dispatch_kp<RM_FP8_E4M3>(idx, plan, read_emb, read_scale, n_reads, ws, s);
      break;
  }
  if (e != hipSuccess) return e;
  int n_per_read = plan.chunks * plan.kp;
  unsigned blocks = (unsigned)(((int64_t)n_reads + 3) / 4);
  hipLaunchKernelGGL(merge_kernel, dim3(blocks), dim3(256), 0, s,
                     static_cast<const uint64_t*>(ws), n_per_read, n_reads, k_fetch, cand_idx,
                     cand_score);
  return hipGetLastError();
}

}  // namespace rm
