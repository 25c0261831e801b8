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
// registers (each wavefront owns NF fragments of 32 rows = 16 reads, over the
// row's full K: 256 reals, or 192 in the letter-sum form) and streams the
// chunk's windows through an LDS ring in tiles of 32 or 64.  Per tile every
// wavefront runs NF x NB x (K/K_mfma) MFMAs on 32x32 output blocks; the
// epilogue forms F per (read, window) in registers, compares with the read's
// current k-th best and, only for hits, appends (F, j) to the read's LDS
// buffer.  Full buffers are merged into the read's sorted list by a bitonic
// sort across lanes.  The score matrix never leaves registers.
//
// List entries are 64-bit keys: high word = float bits of F plus one (0 means
// empty), low word = ~j; a larger key is a better candidate (F descending,
// then window id ascending), so one integer comparison orders them exactly.
//
// This header holds the kernel templates; each translation unit that
// includes it instantiates its own precisions (internal linkage), so they can
// be compiled with different code-generation options.
#pragma once

#include "rm_internal.h"

namespace rm {

// FP16 instantiations of the scoring kernel (rm_score_f16.hip).
hipError_t dispatch_score_f16(int read_tile, int kp, bool reduced, const ScoreLaunch& L,
                              hipStream_t s);

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kBlkW = 32;   // windows per MFMA column block (the MFMA N dimension)
constexpr int kPlanW = 64;  // chunk boundaries are multiples of this many windows
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

// The slot bound of each of a wavefront's NF*16 reads (first read row0),
// written to thr[0 .. NF*16): the KP-th largest F among the keys that finished
// chunks left in the read's slots (distinct windows; -1 while fewer than KP
// slots are filled, or past the last read).  Two reads per step, one per
// half-wavefront, one slot per lane, sorted across the half.  Called once at
// the start of an item: a read's chunks are scored roughly one after another,
// since items are numbered chunk-major.  Kept out of line so that its
// registers do not add to the scoring loop's.
template <int NF, int KP>
__device__ __noinline__ void slot_bounds(const uint64_t* __restrict__ gslot, int64_t row0, int32_t R,
                                         int lane, float* thr) {
  static_assert(KP <= kScoreSlots && kScoreSlots == 32, "slots");
  const int g = lane >> 5, col = lane & 31;
#pragma unroll 1
  for (int p = 0; p < NF * 8; ++p) {
    const int i = 2 * p + g;
    const int64_t r = row0 + i;
    uint64_t key = r < R ? __hip_atomic_load(&gslot[r * kScoreSlots + col], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)
                         : 0ull;
    key = sort_desc<32>(key, lane);
    if (col == KP - 1) thr[i] = key_score(key);
  }
  __builtin_amdgcn_wave_barrier();
}

// Sort 128 keys descending, two per lane: element lane + 64 e is k[e] (the
// same bitonic network over 128 elements; its distance-64 steps compare the
// lane's own two keys).
__device__ __forceinline__ void sort_desc128(uint64_t& k0, uint64_t& k1, int lane) {
#pragma unroll
  for (int kk = 2; kk <= 128; kk <<= 1) {
#pragma unroll
    for (int d = kk >> 1; d > 0; d >>= 1) {
      if (d == 64) {  // only at kk = 128, where every block is descending
        const uint64_t mx = k0 > k1 ? k0 : k1, mn = k0 > k1 ? k1 : k0;
        k0 = mx;
        k1 = mn;
        continue;
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        uint64_t& key = e ? k1 : k0;
        const int i = lane + 64 * e;
        const uint64_t other = shfl_xor64(key, d);
        const bool keep_max = ((i & d) == 0) == ((i & kk) == 0);
        const uint64_t mx = key > other ? key : other, mn = key > other ? other : key;
        key = keep_max ? mx : mn;
      }
    }
  }
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
// counts this wavefront's vector-memory operations in issue order.  The LDS
// base goes in through an m0 operand, so the compiler itself sets m0 and
// knows that it holds the value.
__device__ __forceinline__ void dma16(const void* src, uint32_t lds) {
  asm volatile("global_load_lds_dwordx4 %0, off" ::"v"(src), "{m0}"(lds) : "memory");
}
__device__ __forceinline__ void dma4(const void* src, uint32_t lds) {
  asm volatile("global_load_lds_dword %0, off" ::"v"(src), "{m0}"(lds) : "memory");
}
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Row formats of the product.  A row holds KR reals: kReal = 256 for the
// letter encoding (128 complex components), kRealReduced = 192 for its
// letter-sum form (96 components).  B tiles in LDS: row r
// (one window, RB bytes) stores logical 16-byte chunk c at physical chunk
// swap(r, c), a permutation keyed by r's low bits that makes the 16 rows read
// together by one LDS access cycle (16 consecutive rows, the same logical
// chunk) fall in 16 different bank groups (16-byte units mod 16):
//  * 256 reals, and 192 reals in FP32 (768 B): c ^ (r & 15) (a row is a
//    multiple of 256 B, so its physical chunk index mod 16 is c ^ (r & 15));
//  * 192 reals, FP16 (24 chunks = 384 B, rows alternate between bank-group
//    offsets 0 and 8): chunks 0-15 as c ^ (r & 15), chunks 16-23 as
//    16 + ((c - 16) ^ ((r >> 1) & 7));
//  * 192 reals, FP8 (12 chunks = 192 B, rows step the bank-group offset by
//    12): c ^ ((r >> 2) & 3), which permutes each aligned group of 4 chunks.
// Each permutation is an involution, so swap() also maps physical to logical.
// A lane in half g = lane / 32 of a wavefront takes AU4 of the row's chunks,
// its share of K: register slot u holds logical chunk lane_chunk(g, u), of
// the read row (A, registers) and of the window row (B, LDS) alike -- any
// assignment of K indices to (lane half, slot) works as long as A and B use
// the same one.  keys() gives the lane's LDS byte-offset keys: slot u of the
// first region is at row + (kx ^ 16 u'), of the second at row + base2 +
// (kx2 ^ 16 u''), with u', u'' the slot's position inside its region.
template <int PREC, int KR>
struct RowFmt {
  static constexpr int esize = Prec<PREC>::esize;
  static constexpr int RB = KR * esize;  // bytes per row
  static constexpr int CPR = RB / 16;    // 16-byte chunks per row
  static constexpr int AU4 = CPR / 2;    // chunks per lane (uint4 per fragment)
  static constexpr bool kFull = KR == kReal;
  static_assert(kFull || KR == kRealReduced, "row format");
  // slots in the first region, and the byte offset of the second region
  static constexpr int U1 = kFull ? AU4 : (PREC == RM_FP32 ? 16 : PREC == RM_FP16 ? 8 : 4);
  static constexpr int BASE2 = PREC == RM_FP32 ? 512 : PREC == RM_FP16 ? 256 : 128;
  __device__ __forceinline__ static int swap(int r, int c) {
    if constexpr (kFull || PREC == RM_FP32) return c ^ (r & 15);
    else if constexpr (PREC == RM_FP16) return c < 16 ? c ^ (r & 15) : 16 + ((c - 16) ^ ((r >> 1) & 7));
    else return c ^ ((r >> 2) & 3);
  }
  __device__ __forceinline__ static int lane_chunk(int g, int u) {
    if constexpr (kFull) return g * AU4 + u;
    else if constexpr (PREC == RM_FP32) return u < 16 ? 16 * g + u : 32 + 8 * g + (u - 16);
    else if constexpr (PREC == RM_FP16) return u < 8 ? 8 * g + u : 16 + 4 * g + (u - 8);
    else return u < 4 ? 4 * g + u : 8 + 2 * g + (u - 4);
  }
  __device__ __forceinline__ static void keys(int g, int col, uint32_t& kx, uint32_t& kx2) {
    if constexpr (kFull) {
      kx = ((uint32_t)g * (RB / 2)) ^ (16u * (uint32_t)(col & 15));
      kx2 = 0;
    } else if constexpr (PREC == RM_FP32) {
      kx = (256u * g) ^ (16u * (uint32_t)(col & 15));
      kx2 = (128u * g) ^ (16u * (uint32_t)(col & 15));
    } else if constexpr (PREC == RM_FP16) {
      kx = (128u * g) ^ (16u * (uint32_t)(col & 15));
      kx2 = (64u * g) ^ (16u * (uint32_t)((col >> 1) & 7));
    } else {
      kx = (64u * g) ^ (16u * (uint32_t)((col >> 2) & 3));
      kx2 = (32u * g) ^ (16u * (uint32_t)((col >> 2) & 3));
    }
  }
  // LDS byte offset of slot u (u a compile-time constant after unrolling)
  __device__ __forceinline__ static uint32_t slot_offset(int u, uint32_t kx, uint32_t kx2) {
    return u < U1 ? (kx ^ (16u * u)) : BASE2 + (kx2 ^ (16u * (u - U1)));
  }
};

// One 32x32 output block per fragment over the row's full K.  `a[f]` holds
// this lane's AU4 chunks of fragment f's rows (slot order of RowFmt); `row`
// points at this lane's window row in the current LDS stage and kx, kx2 are
// its RowFmt keys.
template <int PREC, int NF, int NB, int KR>
__device__ __forceinline__ void mfma_tile(const uint4 (&a)[NF][RowFmt<PREC, KR>::AU4],
                                          const uint8_t* row, uint32_t kx, uint32_t kx2,
                                          f32x16 (&acc)[NF][NB]) {
  using RF = RowFmt<PREC, KR>;
  // column block nb of the tile: rows 32 nb + col (same swizzle keys: 32 nb
  // leaves the row's low five bits alone)
  constexpr int BLK = kBlkW * RF::RB;
  if constexpr (PREC == RM_FP16) {
#pragma unroll
    for (int s = 0; s < RF::AU4; ++s) {
      half8 bh[NB];
      const uint32_t o = RF::slot_offset(s, kx, kx2);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bh[nb] = __builtin_bit_cast(half8, *reinterpret_cast<const uint4*>(row + nb * BLK + o));
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int f = 0; f < NF; ++f)
          acc[f][nb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a[f][s]),
                                                              bh[nb], acc[f][nb], 0, 0, 0);
    }
  } else if constexpr (PREC == RM_FP8_E4M3) {
#pragma unroll
    for (int s = 0; s < RF::AU4 / 2; ++s) {
      i32x8 bb[NB];
      const uint32_t o0 = RF::slot_offset(2 * s, kx, kx2), o1 = RF::slot_offset(2 * s + 1, kx, kx2);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        uint4 b0 = *reinterpret_cast<const uint4*>(row + nb * BLK + o0);
        uint4 b1 = *reinterpret_cast<const uint4*>(row + nb * BLK + o1);
        bb[nb] = i32x8{(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w,
                       (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const uint4 a0 = a[f][2 * s], a1 = a[f][2 * s + 1];
        i32x8 aa = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w,
                    (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
        // formats 0/0 = FP8 e4m3 for both operands; E8M0 scales 127 = 1.0
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[f][nb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(aa, bb[nb], acc[f][nb], 0, 0,
                                                                        0, 127, 0, 127);
      }
    }
  } else {
#pragma unroll
    for (int s4 = 0; s4 < RF::AU4; ++s4) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        uint4 bv = *reinterpret_cast<const uint4*>(row + nb * BLK + RF::slot_offset(s4, kx, kx2));
        float bf[4] = {__uint_as_float(bv.x), __uint_as_float(bv.y), __uint_as_float(bv.z),
                       __uint_as_float(bv.w)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            const uint4 av = a[f][s4];
            uint32_t ab = q == 0 ? av.x : q == 1 ? av.y : q == 2 ? av.z : av.w;
            acc[f][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(ab), bf[q],
                                                              acc[f][nb], 0, 0, 0);
          }
        }
      }
    }
  }
}

template <int PREC, int NF, int WAVES, int KP, int ENT, int STAGES, int NB, int KR>
struct ScoreKernel {
  using RF = RowFmt<PREC, KR>;
  static constexpr int RB = RF::RB;                     // bytes per embedding row
  static constexpr int CPR = RF::CPR;                   // 16-byte chunks per row
  static constexpr int AU4 = RF::AU4;                   // uint4 per lane per fragment
  static constexpr int READS = WAVES * NF * 16;         // reads per block
  static constexpr int THREADS = WAVES * 64;
  static constexpr int TW = kBlkW * NB;                 // windows per B tile
  static constexpr int TILE = TW * RB;                  // bytes per B tile
  // 1 KB copies per tile: wavefronts w < NH make LH of them, the others LL
  static constexpr int C = TILE / 1024;
  static constexpr int LH = (C + WAVES - 1) / WAVES, LL = C / WAVES, NH = C % WAVES;
  // this wavefront's copies per tile, + the window scales
  static constexpr int LTH = LH + (PREC == RM_FP8_E4M3 ? 1 : 0);
  static constexpr int LTL = LL + (PREC == RM_FP8_E4M3 ? 1 : 0);
  static constexpr int CB = ENT - KP;                   // buffer slots per read
  // lanes of the bitonic merge of one read's list and buffer (ENT rounded up
  // to a power of two; lanes past ENT sort empty keys)
  static constexpr int SW = ENT <= 32 ? 32 : ENT <= 64 ? 64 : 128;
  // one block barrier per GRP tiles; copies run LEAD tiles ahead.  FP8
  // tiles carry twice the epilogue work per MFMA cycle of FP16 ones, and
  // halving their barriers pays (2%); for FP16 it costs 2.5%.
  static constexpr int GRP = PREC == RM_FP8_E4M3 && STAGES >= 4 ? 2 : 1;
  static constexpr int LEAD = STAGES - GRP;
  static_assert(C >= 1 && TILE % 1024 == 0, "tile");
  static_assert(CB >= 1 && ENT <= 128 && KP <= 64, "buffer");
  static_assert(NF * 16 <= 64, "a wavefront's reads are addressed by 64-bit lane masks");
  static_assert(NF * NB * 8 <= 64, "pending hits are 64-bit masks of (block, fragment, row pair)");
  static_assert(kPlanW % TW == 0, "chunks hold whole tiles");
  static_assert(STAGES >= 2 && LEAD >= GRP, "stages");
};

// One work item: read tile `tile` of group G against window chunk `chunk`.
template <int PREC, int NF, int WAVES, int KP, int ENT, int STAGES, int NB, int KR>
__device__ __forceinline__ void score_item(const ScoreGroup& G, int chunk, int tile,
                                           uint8_t* ring, float* ring_scale,
                                           uint64_t (*lst)[ENT], int* cnt, float* thr,
                                           float* rsq) {
  using K = ScoreKernel<PREC, NF, WAVES, KP, ENT, STAGES, NB, KR>;
  using RF = typename K::RF;
  constexpr bool kFp8 = PREC == RM_FP8_E4M3;
  const uint8_t* __restrict__ index = G.index;
  const float* __restrict__ win_scale = G.win_scale;
  const int64_t W = G.W;
  const uint8_t* __restrict__ reads = G.reads;
  const float* __restrict__ read_scale = G.read_scale;
  const int32_t R = G.R;
  const int64_t chunk_windows = G.chunk_windows;
  const int P = G.P;
  uint64_t* __restrict__ ws = G.lists;
  uint32_t* __restrict__ gthr = G.gthr;
  uint64_t* __restrict__ gslot = G.gslot;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar registers
  const int g = lane >> 5;
  const int col = lane & 31;
  const int64_t read0 = (int64_t)tile * K::READS;
  const int64_t wbeg = (int64_t)chunk * chunk_windows;
  const int64_t wend = min(W, wbeg + chunk_windows);
  const int ntiles = (int)((wend - wbeg + K::TW - 1) / K::TW);

  // ---- per-read state (each wavefront owns reads rb0 .. rb0 + NF*16 - 1 of
  // the tile: rows 32 (wave NF + f) .. +31 for fragment f)
  const int rb0 = wave * NF * 16;
  auto gread = [&](int i) -> int64_t { return read0 + rb0 + i; };
  // a wavefront whose rows all lie past the last read has nothing to score
  const bool wave_active = read0 + rb0 < (int64_t)R;
  for (int i = lane; i < NF * 16 * ENT; i += 64) lst[rb0 + i / ENT][i % ENT] = 0;
  if (lane < NF * 16) {
    cnt[rb0 + lane] = 0;
    thr[rb0 + lane] = -1.f;
  }

  // ---- the read's slot bound is the chunk's first threshold
  if constexpr (KP <= kScoreSlots) slot_bounds<NF, KP>(gslot, read0 + rb0, R, lane, thr + rb0);

  // ---- A fragments: this lane's K half of row (read tile row) for each fragment
  uint4 a[NF][K::AU4];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    int64_t row = 2 * read0 + (int64_t)(wave * NF + f) * 32 + col;
    if (row < 2 * (int64_t)R) {
      const uint4* src = reinterpret_cast<const uint4*>(reads + row * K::RB);
#pragma unroll
      for (int u = 0; u < K::AU4; ++u) a[f][u] = src[RF::lane_chunk(g, u)];
    } else {
#pragma unroll
      for (int u = 0; u < K::AU4; ++u) a[f][u] = make_uint4(0, 0, 0, 0);
    }
  }
  // FP8: the largest s_j^2 of the index's windows: the encoder's record at
  // win_scale[W] ((256 s_j)^2, typically within a few percent of 1), else the
  // proven bound kFp8WindowBound
  float wbound = 1.f;
  if constexpr (kFp8) {
    const float rec = win_scale[W];
    wbound = (rec > 0.f && rec <= kFp8WindowBound ? rec : kFp8WindowBound) *
             (kFp8WindowScale * kFp8WindowScale);
  }
  // FP8: s_r^2 per read of the block, in LDS (1 otherwise)
  if constexpr (kFp8) {
    if (lane < NF * 16) {
      int64_t r = gread(lane);
      float sc = r < R ? read_scale[r] : 0.f;
      rsq[rb0 + lane] = sc * sc;
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
    __builtin_amdgcn_wave_barrier();
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
  int drow[K::LH];
  uint32_t doff[K::LH];
#pragma unroll
  for (int i = 0; i < K::LH; ++i) {
    int pos = (i * WAVES + wave) * 64 + lane;  // physical 16-byte chunk in the tile
    int r = min(pos / K::CPR, K::TW - 1);      // (a wavefront's copy past C is never issued)
    int c = RF::swap(r, pos % K::CPR);         // logical chunk stored there
    drow[i] = r;
    doff[i] = (uint32_t)c * 16u;
  }
  // copy window tile `tsrc` into ring stage `stage`
  auto issue_into = [&](int tsrc, int stage) {
    const int64_t tb = wbeg + (int64_t)tsrc * K::TW;
#pragma unroll
    for (int i = 0; i < K::LH; ++i) {
      if (i < K::LL || wave < K::NH) {
        int64_t grow = min(tb + drow[i], wend - 1);  // rows past the chunk: any valid row
        dma16(index + grow * K::RB + doff[i],
              __builtin_amdgcn_readfirstlane(ring_lds + stage * K::TILE + (i * WAVES + wave) * 1024));
      }
    }
    if constexpr (kFp8) {
      if (lane < K::TW)
        dma4(win_scale + min(tb + lane, wend - 1),
             __builtin_amdgcn_readfirstlane(scale_lds + (stage * WAVES + wave) * K::TW * 4));
    }
  };

  // ---- thresholds: the larger of this chunk's threshold (its slot bound,
  // then its own k-th best when higher) and the best k-th best any chunk has
  // published for the read (0 = none yet); slots past the last read get an
  // unreachable threshold
  auto refresh_thresholds = [&]() {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = f * 16 + 4 * (q >> 1) + 2 * g + (q & 1);
        const int rb = rb0 + i;
        const int64_t r = gread(i);
        uint32_t gk = r < R ? __hip_atomic_load(&gthr[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        float gt = gk ? __uint_as_float(gk - 1u) : -1.f;
        float t = fmaxf(thr[rb], gt);
        if constexpr (kFp8) {
          // F = (re^2 + im^2) s_r^2 s_j^2 with s_j^2 <= wbound for every
          // window of the index: in the product's units the threshold is
          // divided by s_r^2 and that bound, so no window above it is missed
          // and the register test needs no per-window factor
          float r2 = rsq[rb] * wbound;
          t = r2 > 0.f ? t / r2 : 0.f;
        }
        th[f][q] = r < R ? t * kLoose : 3.0e38f;
      }
    // Settle the threshold loads on every path (vmcnt(0); expcnt and lgkmcnt
    // not waited): a load whose value one branch leaves unused would otherwise
    // make the compiler wait for all vector memory -- the tile copies in
    // flight included -- before the next MFMA that reuses its register.
    __builtin_amdgcn_s_waitcnt(0x0F70);
  };

  // the merged list's k-th best becomes the chunk's threshold and is published:
  // no window scoring below it can be in the read's final list, whichever
  // chunk holds it
  auto take_kth = [&](int my, uint64_t key) {
    const int rb = rb0 + my;
    float kth = key_score(key);
    thr[rb] = fmaxf(thr[rb], kth);
    const int64_t r = gread(my);
    if (kth >= 0.f && r < R) atomicMax(&gthr[r], __float_as_uint(kth) + 1u);
  };

  // ---- merge a read's buffer into its list (whole wavefront, uniform call)
  auto merge_reads = [&](uint64_t mask) {
    if constexpr (K::SW == 128) {  // one read at a time, two keys per lane
      while (mask) {
        const int my = __builtin_ctzll(mask);
        mask &= mask - 1;
        const int rb = rb0 + my;
        const int n = min(cnt[rb], K::CB);
        uint64_t k0 = lane < KP + n ? lst[rb][lane] : 0;  // KP + n <= ENT
        uint64_t k1 = lane + 64 < KP + n ? lst[rb][lane + 64] : 0;
        sort_desc128(k0, k1, lane);
        if (lane < KP) lst[rb][lane] = k0;
        if (lane + 64 < KP) lst[rb][lane + 64] = k1;
        if (lane == (KP - 1) % 64) take_kth(my, KP > 64 ? k1 : k0);
        if (lane == 0) cnt[rb] = 0;
      }
      __builtin_amdgcn_wave_barrier();
      refresh_thresholds();
      return;
    }
    // SW == 32: two reads at a time (one per half-wave); SW == 64: one read.
    while (mask) {
      int r0 = __builtin_ctzll(mask);
      mask &= mask - 1;
      int r1 = -1;
      if (K::SW == 32 && mask) {
        r1 = __builtin_ctzll(mask);
        mask &= mask - 1;
      }
      int my = (K::SW == 32 && lane >= 32) ? r1 : r0;
      int id = lane & (K::SW - 1);
      if (my >= 0) {
        int rb = rb0 + my;
        int n = min(cnt[rb], K::CB);
        uint64_t key = (id < KP + n) ? lst[rb][id] : 0;  // KP + n <= ENT
        key = sort_desc<K::SW>(key, lane);
        if (id < KP) lst[rb][id] = key;
        if (id == KP - 1) take_kth(my, key);
        if (id == 0) cnt[rb] = 0;
      }
    }
    __builtin_amdgcn_wave_barrier();
    refresh_thresholds();
  };

  // lane's LDS keys (see RowFmt)
  uint32_t kx, kx2;
  RF::keys(g, col, kx, kx2);

  // Pipeline: copies run LEAD tiles ahead of the tile being scored (past the
  // last tile they repeat the last tile, so every group issues the same
  // number of copies and waits for the same count).  Every GRP tiles the
  // block synchronises once: each wavefront first waits for its own copies of
  // the group's GRP tiles, so after the barrier they are all in LDS, and every
  // wavefront has issued its MFMAs on the previous group's tiles, whose
  // stages are then refilled with the tiles LEAD ahead.  When pipelined, the
  // epilogue of tile t runs after the MFMAs of tile t+1 have been issued, in
  // the same basic block, so its VALU work fills the MFMA pipeline's latency.
  // wait for this wavefront's copies of tile t's group and synchronise the
  // block; false (nothing done) inside a group
  auto group_barrier = [&](int t) -> bool {
    if (t % K::GRP) return false;
    if (K::NH == 0 || wave < K::NH)
      wait_vmcnt<(K::LEAD - K::GRP) * K::LTH>();
    else
      wait_vmcnt<(K::LEAD - K::GRP) * K::LTL>();
    __syncthreads();
    return true;
  };
  auto issue_group = [&](int t) {
#pragma unroll
    for (int gi = 0; gi < K::GRP; ++gi)
      issue_into(min(t + K::LEAD + gi, ntiles - 1), (t + K::LEAD + gi) % STAGES);
  };
  auto sync_tile = [&](int t) {
    if (group_barrier(t)) issue_group(t);
  };
  // FP8: squared window scales of tile t (this wavefront's copy)
  auto read_scales = [&](int t, float (&sj2)[NB]) {
    if constexpr (kFp8) {
      const int stage = t % STAGES;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        float sc = ring_scale[(stage * WAVES + wave) * K::TW + nb * kBlkW + col];
        sj2[nb] = sc * sc;
      }
    }
  };
  auto mfmas = [&](int t, f32x16 (&acc)[NF][NB]) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[f][nb] = f32x16{};
    mfma_tile<PREC, NF, NB, KR>(a, ring + (t % STAGES) * K::TILE + col * K::RB, kx, kx2, acc);
  };
  // tile t's scales and MFMAs; its data is valid from the barrier of tile t's
  // group until the barrier after it
  auto mfma_step = [&](int t, f32x16 (&acc)[NF][NB], float (&sj2)[NB]) {
    read_scales(t, sj2);
    mfmas(t, acc);
  };
  auto start_tile = [&](int t, f32x16 (&acc)[NF][NB], float (&sj2)[NB]) {
    const bool b = group_barrier(t);
    read_scales(t, sj2);
    if (b) issue_group(t);
    mfmas(t, acc);
  };

  // re^2 + im^2 - threshold per (read slot, window col), reduced with max per
  // (column block, fragment); only a positive maximum anywhere in the
  // wavefront leads to the (rare) per-score test and appends.  FP8 tiles
  // (four block-fragment groups, half the MFMA time per tile of FP16) test
  // and append only in the groups that hold a hit; for FP16 the extra live
  // registers of the group test cost more than it saves.
  constexpr bool kGroupTest = kFp8;
  auto epilogue = [&](int t, const f32x16 (&acc)[NF][NB], const float (&sj2)[NB]) {
    if ((t & 255) == 255) refresh_thresholds();  // pick up other chunks' progress
    const int64_t tbase = wbeg + (int64_t)t * K::TW;
    bool colok[NB];
    float exg[NB][NF];
    float ex = -1.f;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      colok[nb] = tbase + nb * kBlkW + col < wend;
      float exb = -1.f;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        if constexpr (kGroupTest) {
          float e = -1.f;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            float re = acc[f][nb][2 * q], im = acc[f][nb][2 * q + 1];
            e = fmaxf(e, __builtin_fmaf(re, re, __builtin_fmaf(im, im, -th[f][q])));
          }
          exg[nb][f] = e;
          exb = fmaxf(exb, e);
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            float re = acc[f][nb][2 * q], im = acc[f][nb][2 * q + 1];
            exb = fmaxf(exb, __builtin_fmaf(re, re, __builtin_fmaf(im, im, -th[f][q])));
          }
        }
      }
      ex = colok[nb] ? fmaxf(ex, exb) : ex;
    }

    if (__ballot(ex > 0.f)) {
      uint64_t pend = 0;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int f = 0; f < NF; ++f)
          if (!kGroupTest || __ballot(colok[nb] && exg[nb][f] > 0.f)) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              float re = acc[f][nb][2 * q], im = acc[f][nb][2 * q + 1];
              pend |= (uint64_t)(colok[nb] &&
                                 __builtin_fmaf(re, re, __builtin_fmaf(im, im, -th[f][q])) > 0.f)
                      << ((nb * NF + f) * 8 + q);
            }
          }
      // append every hit, merging reads whose buffer is full, until nothing
      // is pending
      while (true) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int f = 0; f < NF; ++f)
            if (!kGroupTest || __ballot(((pend >> ((nb * NF + f) * 8)) & 0xffu) != 0)) {
#pragma unroll
              for (int q = 0; q < 8; ++q) {
                const uint64_t bit = 1ull << ((nb * NF + f) * 8 + q);
                if (pend & bit) {
                  int rb = rb0 + f * 16 + 4 * (q >> 1) + 2 * g + (q & 1);
                  int pos = atomicAdd(&cnt[rb], 1);
                  if (pos < K::CB) {
                    float re = acc[f][nb][2 * q], im = acc[f][nb][2 * q + 1];
                    float F = re * re + im * im;
                    if constexpr (kFp8) F = F * (rsq[rb] * sj2[nb]);
                    lst[rb][KP + pos] = make_key(F, (int32_t)(tbase + nb * kBlkW + col));
                    pend &= ~bit;
                  }
                }
              }
            }
        __builtin_amdgcn_wave_barrier();
        bool full = lane < NF * 16 && cnt[rb0 + lane] >= K::CB;
        const uint64_t fm = __ballot(full);
        if (fm) merge_reads(fm);
        if (!__ballot(pend != 0)) break;
      }
    }
  };

#pragma unroll
  for (int t = 0; t < K::LEAD; ++t) issue_into(min(t, ntiles - 1), t);

  // FP16 keeps one accumulator set: its A fragments take 128 VGPRs and a
  // second set would spill at two wavefronts per SIMD; so do wide tiles.
  constexpr bool kPipe = PREC != RM_FP16 && NB == 1;
  if (!wave_active) {
    // No read of this wavefront is valid (the tail of the last read tile): it
    // only copies its share of every tile and joins every block barrier, for
    // as many tile steps as the scoring loop below runs (one more when
    // pipelined).
    const int steps = kPipe ? ntiles + 1 : ntiles;
    for (int t = 0; t < steps; ++t) sync_tile(t);
    wait_vmcnt<0>();
    return;  // its reads are all past R: nothing to write
  }
  refresh_thresholds();
  f32x16 accA[NF][NB];
  float sjA[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) sjA[nb] = 1.f;
  if constexpr (kPipe) {
    f32x16 accB[NF][NB];
    float sjB[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) sjB[nb] = 1.f;
    start_tile(0, accA, sjA);
    for (int t = 0;; t += 2) {
      start_tile(t + 1, accB, sjB);  // past the end: a repeat of the last tile, unused
      epilogue(t, accA, sjA);
      if (t + 1 >= ntiles) break;
      start_tile(t + 2, accA, sjA);
      epilogue(t + 1, accB, sjB);
      if (t + 2 >= ntiles) break;
    }
  } else if (wave < WAVES / 2) {
    // one accumulator set: MFMAs of tile t, then its epilogue
    for (int t = 0; t < ntiles; ++t) {
      start_tile(t, accA, sjA);
      epilogue(t, accA, sjA);
    }
  } else {
    // The other wavefront of each SIMD (wavefronts w and w + WAVES/2 share
    // one) runs half a step out of phase: after the barrier of step t it
    // first finishes the epilogue of tile t-1, then issues tile t's MFMAs, so
    // one wavefront's epilogue overlaps the other's MFMAs instead of both
    // leaving the matrix pipe idle together.  Both halves pass the same
    // barriers, and each issues its MFMAs on a tile before the barrier that
    // lets its stage be refilled.
    start_tile(0, accA, sjA);
    for (int t = 1; t < ntiles; ++t) {
      sync_tile(t);
      epilogue(t - 1, accA, sjA);
      mfma_step(t, accA, sjA);
    }
    epilogue(ntiles - 1, accA, sjA);
  }
  wait_vmcnt<0>();  // no copy may still be writing this block's LDS

  // ---- final merge and write-out of this chunk's lists
  {
    bool any = lane < NF * 16 && cnt[rb0 + lane] > 0;
    const uint64_t m = __ballot(any);
    if (m) merge_reads(m);
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < NF * 16 * KP; i += 64) {
      int rr = i / KP, e = i % KP;
      int64_t r = gread(rr);
      if (r < R) {
        const uint64_t key = lst[rb0 + rr][e];
        ws[((int64_t)r * P + chunk) * KP + e] = key;
        // this chunk's windows join the read's slots for the chunks after it
        if (KP <= kScoreSlots && (key >> 32))
          atomicMax(reinterpret_cast<unsigned long long*>(
                        &gslot[r * kScoreSlots + ((~(uint32_t)key) & (kScoreSlots - 1))]),
                    (unsigned long long)key);
      }
    }
  }
}

// Persistent grouped kernel: a grid sized to the chip pulls work items
// (group, chunk, read tile) from a device counter until all are done.  Items
// are numbered chunk-major within each group, so concurrently running blocks
// stream the same windows.  Every block leaves the loop once the counter has
// passed the last item.  With two fragments per wavefront, a thin group's
// items run with one (half the reads per tile, half the work per tile).
template <int PREC, int NF, int WAVES, int KP, int ENT, int STAGES, int NB, int KR>
__global__ __launch_bounds__(WAVES * 64) void score_topk_kernel(ScoreLaunch L) {
  using K = ScoreKernel<PREC, NF, WAVES, KP, ENT, STAGES, NB, KR>;
  constexpr bool kFp8 = PREC == RM_FP8_E4M3;
  __shared__ __align__(1024) uint8_t ring[STAGES * K::TILE];
  __shared__ __align__(16) float ring_scale[kFp8 ? STAGES * WAVES * K::TW : 4];
  __shared__ uint64_t lst[K::READS][ENT];
  __shared__ int cnt[K::READS];
  __shared__ float thr[K::READS];
  __shared__ float rsq[kFp8 ? K::READS : 1];
  __shared__ int s_item;
  while (true) {
    __syncthreads();  // the previous item is finished with s_item and all LDS
    if (threadIdx.x == 0) s_item = atomicAdd(L.counter, 1);
    __syncthreads();
    const int item = s_item;
    if (item >= L.total_items) break;
    int gi = 0;
    while (gi + 1 < L.n_groups && item >= L.g[gi + 1].item_begin) ++gi;
    const ScoreGroup& G = L.g[gi];
    const int local = item - G.item_begin;
    if constexpr (NF == 2) {
      if (G.thin) {  // half-size read tiles: one fragment per wavefront
        score_item<PREC, 1, WAVES, KP, ENT, STAGES, NB, KR>(G, local / G.read_tiles,
                                                         local % G.read_tiles, ring, ring_scale,
                                                         lst, cnt, thr, rsq);
        continue;
      }
    }
    score_item<PREC, NF, WAVES, KP, ENT, STAGES, NB, KR>(G, local / G.read_tiles,
                                                      local % G.read_tiles, ring, ring_scale, lst,
                                                      cnt, thr, rsq);
  }
}

template <int PREC, int NF, int KP, int ENT, int STAGES, int NB = 1, int KR = kReal>
hipError_t launch_persistent(const ScoreLaunch& L, hipStream_t s) {
  constexpr int WAVES = 8;
  auto kern = score_topk_kernel<PREC, NF, WAVES, KP, ENT, STAGES, NB, KR>;
  // resident blocks per CU for this instantiation (LDS and VGPR limited)
  static int per_cu = [&] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, WAVES * 64, 0) != hipSuccess || n < 1)
      n = 1;
    return n;
  }();
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  int64_t grid = (int64_t)per_cu * cus;
  if (grid > L.total_items) grid = L.total_items;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(WAVES * 64), 0, s, L);
  return hipGetLastError();
}

}  // namespace

}  // namespace rm
