// Per-fragment fidelity thresholds and the threshold regime.
//
// §3.3 (closing paragraph): for a target mutation rate, the fidelity expected
// of each reference fragment can serve as that fragment's cutting threshold.
// §3.5: in the threshold regime the mapper reports every location whose
// fidelity passes its fragment's precomputed threshold, as many as there are.
//
// Thresholds: window j is mutated `copies` times at rate err by the streaming
// mutator the reads are simulated with (per step an insertion, a deletion or
// a substitution with probability err/3 each, else a match, until N letters
// are out; a step that needs a letter past the reference's end inserts).  The
// draws come from Philox4x32-10 (Salmon et al., SC 2011) at counter (j mod
// 2^32, j >> 32, copy, step) and key (seed, 0): word 0 picks the event by
// integer comparison, word 1 & 3 is an inserted letter, 1 + word 2 mod 3 a
// substitution's shift.  The threshold is the `rank`-th smallest fidelity of
// the window with its copies (FP32 direct sums of the FP32 table).  One
// wavefront per window; the 64 lanes take 64 consecutive steps of a copy at
// once, and prefix counts over the lanes give each step's reference position
// and output position.
//
// Regime: a product pass (the index precision on MFMA, read tile in
// registers, window tiles through LDS) keeps every (read, window) whose
// product fidelity is within the product's error of max(thr_j, floor) in a
// pool; the pool is grouped by read (counts, prefix sums, scatter); then one
// wavefront per read recomputes each candidate's F in FP32 from the letters,
// keeps those with F >= max(thr_j, floor) and F > 0, and writes them ranked by
// (F desc, window id asc).

#include "rm_bf16.h"
#include "rm_score_kernel.h"

namespace rm {
namespace {

struct Words4 {
  uint32_t x, y, z, w;
};

// Philox4x32-10: ten rounds; a round multiplies words 0 and 2 by the two
// round constants (64-bit products as high and low halves) and mixes them
// with words 1 and 3 and the key; the key advances by the Weyl constants
// between rounds.
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return Words4{c0, c1, c2, c3};
}

// Number of lanes below this one whose bit is set in `mask`.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ float fidelity32(float2 a0, float2 a1, float A, float2 b0, float2 b1,
                                            float B, int N) {
  const float ipr = wave_sum(a0.x * b0.x + a0.y * b0.y + a1.x * b1.x + a1.y * b1.y);
  const float ipi = wave_sum(a0.x * b0.y - a0.y * b0.x + a1.x * b1.y - a1.y * b1.x);
  const bool deg = A < kDegenerateRel * N || B < kDegenerateRel * N;
  return deg ? 0.f : (ipr * ipr + ipi * ipi) / (A * B);
}

constexpr int kThrWaves = 4;

__global__ __launch_bounds__(64 * kThrWaves) void window_thresholds_kernel(
    const uint8_t* __restrict__ ref, int64_t G, int64_t W, int N, int stride,
    const float2* __restrict__ phase32, uint32_t T1, int copies, int rank, uint32_t seed,
    int max_steps, float* __restrict__ thr) {
  __shared__ uint8_t emitted[kThrWaves][64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * kThrWaves + wave;
  if (j >= W) return;
  const int64_t start = j * stride;
  const int k = lane >> 1, h = lane & 1;
  const int L0 = 2 * h, L1 = 2 * h + 1;

  float2 c0, c1;
  direct_sum32(ref + start, N, phase32, lane, c0, c1);
  const float C = wave_sum(c0.x * c0.x + c0.y * c0.y + c1.x * c1.x + c1.y * c1.y);
  float mine = 3.0e38f;  // lane c keeps copy c's fidelity
  for (int c = 0; c < copies; ++c) {
    float2 y0 = make_float2(0.f, 0.f), y1 = make_float2(0.f, 0.f);
    int64_t pos = start;  // next reference letter
    int n = 0;            // letters emitted
    for (int t0 = 0; t0 < max_steps && n < N; t0 += 64) {
      const int t = t0 + lane;
      const Words4 d = philox4x32_10((uint32_t)j, (uint32_t)(j >> 32), (uint32_t)c, (uint32_t)t,
                                     seed, 0u);
      const bool live = t < max_steps;
      // 0 insertion, 1 deletion, 2 substitution, 3 match
      int kind = d.x < T1 ? 0 : d.x < 2u * T1 ? 1 : d.x < 3u * T1 ? 2 : 3;
      // reference position of each step as if no step ran past the end; once
      // it reaches G every later step is an insertion, so the positions
      // before that point are exact
      const uint64_t consume = __ballot(live && kind != 0);
      const int64_t p = pos + lanes_below(consume);
      if (p >= G) kind = 0;
      const bool emit = live && kind != 1;
      const uint64_t em = __ballot(emit);
      const int q = lanes_below(em);  // this step's output index in the group
      if (emit && n + q < N) {
        int L;
        if (kind == 0) {
          L = (int)(d.y & 3u);
        } else {
          const int R0 = ref[p];
          L = (kind == 3 || R0 > 3) ? R0 : (R0 + 1 + (int)(d.z % 3u)) & 3;
        }
        emitted[wave][q] = (uint8_t)L;
      }
      __builtin_amdgcn_wave_barrier();
      const int m = min(__popcll(em), N - n);
      for (int i = 0; i < m; ++i) {
        const int L = emitted[wave][i];
        const float2 e = phase32[(int64_t)(n + i) * kM + k];
        y0.x += (L == L0) ? e.x : 0.f;
        y0.y += (L == L0) ? e.y : 0.f;
        y1.x += (L == L1) ? e.x : 0.f;
        y1.y += (L == L1) ? e.y : 0.f;
      }
      __builtin_amdgcn_wave_barrier();  // emitted[] is rewritten by the next group
      n += m;
      pos += __popcll(__ballot(live && kind != 0));
    }
    const float Y = wave_sum(y0.x * y0.x + y0.y * y0.y + y1.x * y1.x + y1.y * y1.y);
    const float F = fidelity32(c0, c1, C, y0, y1, Y, N);
    if (lane == c) mine = F;
  }
  // ascending bitonic sort of the copies' fidelities over the 64 lanes
#pragma unroll
  for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
    for (int dd = kk >> 1; dd > 0; dd >>= 1) {
      const float other = __shfl_xor(mine, dd, 64);
      const bool up = (lane & kk) == 0;
      const bool lower = (lane & dd) == 0;
      const float lo = fminf(mine, other), hi = fmaxf(mine, other);
      mine = (lower == up) ? lo : hi;
    }
  }
  if (lane == rank) thr[j] = mine;
}

// ---- the regime's product pass

// The same thresholds with the strings' vectors from one MFMA product: each
// wavefront writes the letters of its window (string 0) and of its copies
// (strings 1..copies) into LDS, drawing the copies exactly as
// window_thresholds_kernel does, then the block multiplies the one-hot
// (string, letter) rows of its four windows with the FP32 table split into
// three bfloat16 parts (rm_bf16.h), in passes of 8 RB strings and chunks of
// 64 positions, and each wavefront takes the fidelities of its copies with
// its window from the product.  `np` is N rounded up to 64, `sp` the strings
// rounded up to whole passes; letters past a string's end are 4 (none).
template <int RB>
__global__ __launch_bounds__(64 * kThrWaves) void window_thresholds_mfma_kernel(
    const uint8_t* __restrict__ ref, int64_t G, int64_t W, int N, int np, int stride,
    const float* __restrict__ tab, uint32_t T1, int copies, int sp, int rank, uint32_t seed,
    int max_steps, float* __restrict__ thr) {
  constexpr int SMAX = 8 * RB;
  typedef float f32x16 __attribute__((ext_vector_type(16)));
  extern __shared__ __attribute__((aligned(16))) uint8_t letters_dyn[];  // [waves][sp][np]
  __shared__ u32x4 tparts[3][2][8][32];
  __shared__ float mat_all[kThrWaves][32][2 * kM + 1];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t j = (int64_t)blockIdx.x * kThrWaves + wave;
  const bool active = j < W;  // inactive wavefronts still stage the table
  uint8_t* letters = letters_dyn + (size_t)wave * sp * np;
  float(*mat)[2 * kM + 1] = mat_all[wave];
  const int S = 1 + copies;
  const int half = lane >> 5, col = lane & 31;
  const int kf = lane >> 1, h = lane & 1;

  // ---- letters of the window and its copies (4 for none)
  if (active) {
    const int64_t start = j * stride;
    for (int s = 0; s < sp; ++s)
      for (int p = lane; p < np; p += 64)
        letters[s * np + p] = (s == 0 && p < N) ? (uint8_t)min((int)ref[start + p], 4) : (uint8_t)4;
    __builtin_amdgcn_wave_barrier();
    for (int c = 0; c < copies; ++c) {
      uint8_t* out = letters + (size_t)(c + 1) * np;
      int64_t pos = start;  // next reference letter
      int n = 0;            // letters emitted
      for (int t0 = 0; t0 < max_steps && n < N; t0 += 64) {
        const int t = t0 + lane;
        const Words4 d = philox4x32_10((uint32_t)j, (uint32_t)(j >> 32), (uint32_t)c, (uint32_t)t,
                                       seed, 0u);
        const bool live = t < max_steps;
        // 0 insertion, 1 deletion, 2 substitution, 3 match
        int kind = d.x < T1 ? 0 : d.x < 2u * T1 ? 1 : d.x < 3u * T1 ? 2 : 3;
        const uint64_t consume = __ballot(live && kind != 0);
        const int64_t p = pos + lanes_below(consume);
        if (p >= G) kind = 0;
        const bool emit = live && kind != 1;
        const uint64_t em = __ballot(emit);
        const int q = lanes_below(em);  // this step's output index in the group
        if (emit && n + q < N) {
          int L;
          if (kind == 0) {
            L = (int)(d.y & 3u);
          } else {
            const int R0 = ref[p];
            L = (kind == 3 || R0 > 3) ? R0 : (R0 + 1 + (int)(d.z % 3u)) & 3;
          }
          out[n + q] = (uint8_t)min(L, 4);
        }
        n += min(__popcll(em), N - n);
        pos += __popcll(__ballot(live && kind != 0));
      }
    }
  }

  float2 x0 = make_float2(0.f, 0.f), x1 = make_float2(0.f, 0.f);  // the window
  float X = 0.f;
  float mine = 3.0e38f;  // lane c keeps copy c's fidelity
  const uint32_t onehot_tab = 0x40u << (8 * (col & 3));
  for (int s0 = 0; s0 < S; s0 += SMAX) {
    const int SP = min(SMAX, S - s0);
    f32x16 acc[RB][2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb][0] = acc[rb][1] = f32x16{};
    for (int pb = 0; pb < N; pb += 64) {
      __syncthreads();  // the previous chunk's table parts are read (and the letters written)
      stage_table_parts(tab, pb, N, tparts, threadIdx.x, 64 * kThrWaves);
      __syncthreads();
      if (active) {
        const int steps = min(4, (N - pb + 15) >> 4);
        for (int st = 0; st < steps; ++st) {
          bf16x8 b[3][2];
#pragma unroll
          for (int pt = 0; pt < 3; ++pt)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
              b[pt][cb] = __builtin_bit_cast(bf16x8, tparts[pt][cb][2 * st + half][col]);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const int s = s0 + rb * 8 + (col >> 2);  // < sp
            const uint2 w =
                *reinterpret_cast<const uint2*>(&letters[(size_t)s * np + pb + 16 * st + 8 * half]);
            const bf16x8 a = onehot_fragment(w, onehot_tab);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
              for (int pt = 2; pt >= 0; --pt)  // small parts first
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[pt][cb], acc[rb][cb], 0, 0, 0);
          }
        }
      }
    }
    if (!active) continue;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          mat[8 * (v >> 2) + 4 * half + (v & 3)][cb * 32 + col] = 0.5f * acc[rb][cb][v];
      __builtin_amdgcn_wave_barrier();
      for (int sl = 0; sl < 8; ++sl) {
        const int sx = s0 + rb * 8 + sl;
        if (rb * 8 + sl >= SP) break;
        const float2 c0 = make_float2(mat[4 * sl + 2 * h][2 * kf], mat[4 * sl + 2 * h][2 * kf + 1]);
        const float2 c1 = make_float2(mat[4 * sl + 2 * h + 1][2 * kf], mat[4 * sl + 2 * h + 1][2 * kf + 1]);
        const float Y = wave_sum(c0.x * c0.x + c0.y * c0.y + c1.x * c1.x + c1.y * c1.y);
        if (sx == 0) {
          x0 = c0;
          x1 = c1;
          X = Y;
          continue;
        }
        const float F = fidelity32(x0, x1, X, c0, c1, Y, N);
        if (lane == sx - 1) mine = F;
      }
      __builtin_amdgcn_wave_barrier();  // before the next block overwrites mat
    }
  }
  if (!active) return;
  // ascending bitonic sort of the copies' fidelities over the 64 lanes
#pragma unroll
  for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
    for (int dd = kk >> 1; dd > 0; dd >>= 1) {
      const float other = __shfl_xor(mine, dd, 64);
      const bool up = (lane & kk) == 0;
      const bool lower = (lane & dd) == 0;
      const float lo = fminf(mine, other), hi = fmaxf(mine, other);
      mine = (lower == up) ? lo : hi;
    }
  }
  if (lane == rank) thr[j] = mine;
}

template <int PREC, int KR>
struct ThrK {
  using RF = RowFmt<PREC, KR>;
  static constexpr int NF = PREC == RM_FP32 ? 1 : 2;      // fragments (16 reads) per wavefront
  static constexpr int WAVES = 8;
  static constexpr int THREADS = WAVES * 64;
  static constexpr int READS = WAVES * NF * 16;
  static constexpr int RB = RF::RB;
  static constexpr int CPR = RF::CPR;
  static constexpr int AU4 = RF::AU4;
  static constexpr int TW = kBlkW;                          // windows per tile
  static constexpr int TILE = TW * RB;
  static constexpr int STAGES = TILE <= 16384 ? 4 : 2;     // LDS ring
  // 1 KB copies per tile: wavefronts w < NH make LH of them, the others LL;
  // each also copies the tile's thresholds (and FP8 window scales)
  static constexpr int C = TILE / 1024;
  static constexpr int LH = (C + WAVES - 1) / WAVES, LL = C / WAVES, NH = C % WAVES;
  static constexpr int EXTRA = PREC == RM_FP8_E4M3 ? 2 : 1;
  static constexpr int LTH = LH + EXTRA, LTL = LL + EXTRA;
  static_assert(C >= 1 && TILE % 1024 == 0, "tile");
};

// Wait until at most `later` tiles' copies of this wavefront (issued after the
// tile being waited for) are in flight.
template <int LT, int STAGES>
__device__ __forceinline__ void wait_tiles(int later) {
  if constexpr (STAGES >= 4) {
    if (later >= 2) {
      wait_vmcnt<2 * LT>();
      return;
    }
  }
  if (later >= 1)
    wait_vmcnt<LT>();
  else
    wait_vmcnt<0>();
}

// Product pass of the regime.  Block = (read tile, window chunk); the read
// tile sits in registers (eight wavefronts), window tiles of 32 are copied
// straight from global memory into a ring of LDS stages (rows XOR-swizzled as
// the top-k product stores them), each wavefront copying its share plus its
// own copy of the tile's thresholds (and FP8 window scales).  One barrier per
// tile: after it every wavefront's copies of the tile are in, and the stage
// read before it is free for the copies STAGES - 1 tiles ahead.  A lane holds
// one window column, so its 16 scores share one cut: their maximum is tested
// first, and only a passing lane's scores are tested one by one.
template <int PREC, int KR>
__global__ __launch_bounds__((ThrK<PREC, KR>::THREADS)) void threshold_scan_kernel(
    const uint8_t* __restrict__ index, const float* __restrict__ win_scale, int64_t W,
    const float* __restrict__ thr, float floor_f, float margin, const uint8_t* __restrict__ reads,
    const float* __restrict__ read_scale, int32_t R, int64_t chunk_windows, int n_chunks,
    uint64_t* __restrict__ pool, uint64_t pool_cap, unsigned long long* __restrict__ pool_n) {
  using K = ThrK<PREC, KR>;
  using RF = typename K::RF;
  constexpr bool kFp8 = PREC == RM_FP8_E4M3;
  constexpr int S = K::STAGES;
  __shared__ __attribute__((aligned(16))) uint8_t ring[S][K::TILE];
  __shared__ float side[S][2][K::WAVES][K::TW];  // [stage][thr, scale][wave][window]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 5, col = lane & 31;
  const int tile_r = blockIdx.x / n_chunks, chunk = blockIdx.x % n_chunks;
  const int64_t read0 = (int64_t)tile_r * K::READS;
  const int64_t wbeg = (int64_t)chunk * chunk_windows;
  const int64_t wend = min(W, wbeg + chunk_windows);
  if (wbeg >= wend) return;  // uniform over the block
  const int ntiles = (int)((wend - wbeg + K::TW - 1) / K::TW);

  // A fragments (rows past the last read are zero, so their F is 0), and for
  // FP8 the squared read scale of each of this lane's 16 score slots
  uint4 a[K::NF][K::AU4];
#pragma unroll
  for (int f = 0; f < K::NF; ++f) {
    const int64_t row = 2 * read0 + (int64_t)(wave * K::NF + f) * 32 + col;
    const uint4* src = reinterpret_cast<const uint4*>(reads + row * K::RB);
#pragma unroll
    for (int u = 0; u < K::AU4; ++u)
      a[f][u] = row < 2 * (int64_t)R ? src[RF::lane_chunk(g, u)] : make_uint4(0, 0, 0, 0);
  }
  float rsq[K::NF][8];
#pragma unroll
  for (int f = 0; f < K::NF; ++f)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t r = read0 + wave * K::NF * 16 + f * 16 + 4 * (q >> 1) + 2 * g + (q & 1);
      float sc = 1.f;
      if constexpr (kFp8) sc = r < R ? read_scale[r] : 0.f;
      rsq[f][q] = sc * sc;
    }
  __builtin_amdgcn_s_waitcnt(0);  // the fragments and scales, before any copy is in flight

  const uint32_t ring_lds = lds_offset(ring);
  const uint32_t side_lds = lds_offset(side);
  int drow[K::LH];
  uint32_t doff[K::LH];
#pragma unroll
  for (int i = 0; i < K::LH; ++i) {
    const int pos = (i * K::WAVES + wave) * 64 + lane;  // physical 16-byte chunk in the tile
    const int r = min(pos / K::CPR, K::TW - 1);  // (a wavefront's copy past C is never issued)
    drow[i] = r;
    doff[i] = (uint32_t)RF::swap(r, pos % K::CPR) * 16u;  // the logical chunk stored there
  }
  auto issue = [&](int t) {
    const int stage = t % S;
    const int64_t tb = wbeg + (int64_t)t * K::TW;
#pragma unroll
    for (int i = 0; i < K::LH; ++i) {
      if (i < K::LL || wave < K::NH) {
        const int64_t grow = min(tb + drow[i], wend - 1);  // rows past the chunk: any valid row
        dma16(index + grow * K::RB + doff[i],
              __builtin_amdgcn_readfirstlane(ring_lds + stage * K::TILE +
                                             (i * K::WAVES + wave) * 1024));
      }
    }
    const int64_t jj = min(tb + lane, wend - 1);
    if (lane < K::TW)
      dma4(thr + jj, __builtin_amdgcn_readfirstlane(
                         side_lds + (((stage * 2 + 0) * K::WAVES + wave) * K::TW) * 4));
    if constexpr (kFp8) {
      if (lane < K::TW)
        dma4(win_scale + jj, __builtin_amdgcn_readfirstlane(
                                 side_lds + (((stage * 2 + 1) * K::WAVES + wave) * K::TW) * 4));
    }
  };
  uint32_t kx, kx2;
  RF::keys(g, col, kx, kx2);

  for (int t = 0; t < S - 1 && t < ntiles; ++t) issue(t);
  for (int t = 0; t < ntiles; ++t) {
    const int stage = t % S;
    // this wavefront's copies of tile t: later tiles issued so far are t+1 .. t+S-2
    const int later = min(S - 2, ntiles - 1 - t);
    if (K::NH == 0 || wave < K::NH)
      wait_tiles<K::LTH, S>(later);
    else
      wait_tiles<K::LTL, S>(later);
    __syncthreads();  // every wavefront's copies of tile t; stage (t-1) % S is read
    if (t + S - 1 < ntiles) issue(t + S - 1);
    f32x16 acc[K::NF][1];
#pragma unroll
    for (int f = 0; f < K::NF; ++f) acc[f][0] = f32x16{};
    mfma_tile<PREC, K::NF, 1, KR>(a, &ring[stage][col * K::RB], kx, kx2, acc);
    // epilogue: this lane's window column against its cut, less the margin
    const int64_t j = wbeg + (int64_t)t * K::TW + col;
    const bool colok = j < wend;
    const float cut = fmaxf(side[stage][0][wave][col], floor_f) - margin;
    float sj2 = 1.f;
    if constexpr (kFp8) {
      const float sc = side[stage][1][wave][col];
      sj2 = sc * sc;
    }
    float F[K::NF][8];
    float fmax = 0.f;
#pragma unroll
    for (int f = 0; f < K::NF; ++f)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float re = acc[f][0][2 * q], im = acc[f][0][2 * q + 1];
        F[f][q] = fmaf(re, re, im * im);
        if constexpr (kFp8) F[f][q] *= rsq[f][q] * sj2;
        fmax = fmaxf(fmax, F[f][q]);
      }
    if (colok && fmax > 0.f && fmax >= cut) {  // rare
#pragma unroll
      for (int f = 0; f < K::NF; ++f)
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (F[f][q] > 0.f && F[f][q] >= cut) {
            const int slot = wave * K::NF * 16 + f * 16 + 4 * (q >> 1) + 2 * g + (q & 1);
            const int64_t r = read0 + slot;
            const unsigned long long p = atomicAdd(pool_n, 1ull);
            if (p < pool_cap) pool[p] = ((uint64_t)r << 32) | (uint64_t)(uint32_t)j;
          }
    }
  }
}

// ---- grouping the pool by read

__global__ void zero_u32_kernel(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void zero_counter_kernel(unsigned long long* __restrict__ p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

__global__ void pool_count_kernel(const uint64_t* __restrict__ pool,
                                  const unsigned long long* __restrict__ pool_n, uint64_t cap,
                                  uint32_t* __restrict__ cnt) {
  const uint64_t n = min((uint64_t)*pool_n, cap);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[pool[i] >> 32], 1u);
}

// Exclusive prefix sums off[0..R] of cnt[0..R) in one block: each thread
// sums a contiguous segment, the block scans the segment sums, then each
// thread writes its segment's offsets.  Also writes the untruncated pool size.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void scan_kernel(
    const uint32_t* __restrict__ cnt, int32_t R, int64_t* __restrict__ off,
    const unsigned long long* __restrict__ pool_n, int64_t* __restrict__ total) {
  __shared__ int64_t part[kScanThreads];
  const int t = threadIdx.x;
  const int64_t seg = ((int64_t)R + kScanThreads - 1) / kScanThreads;
  const int64_t b = min((int64_t)R, t * seg), e = min((int64_t)R, b + seg);
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {  // inclusive Hillis-Steele scan
    const int64_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int64_t i = b; i < e; ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == kScanThreads - 1) {
    off[R] = part[t];
    *total = (int64_t)*pool_n;
  }
}

__global__ void pool_scatter_kernel(const uint64_t* __restrict__ pool,
                                    const unsigned long long* __restrict__ pool_n, uint64_t cap,
                                    const int64_t* __restrict__ off, uint32_t* __restrict__ fill,
                                    int32_t* __restrict__ cand) {
  const uint64_t n = min((uint64_t)*pool_n, cap);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t r = (uint32_t)(pool[i] >> 32);
    const uint32_t at = atomicAdd(&fill[r], 1u);
    cand[off[r] + at] = (int32_t)(uint32_t)pool[i];
  }
}

// One wavefront per read: FP32 F of every candidate from the letters, the
// hits (F >= max(thr_j, floor), F > 0) as keys, then ranked by repeated
// wavefront maxima into the read's span of the output.
__global__ __launch_bounds__(256) void threshold_rescore_kernel(
    const uint8_t* __restrict__ ref, int N, int stride, const float2* __restrict__ phase32,
    const uint8_t* __restrict__ seq, const int64_t* __restrict__ soff, int32_t R,
    const int64_t* __restrict__ off, const int32_t* __restrict__ cand,
    const float* __restrict__ thr, float floor_f, uint64_t* __restrict__ keys,
    int32_t* __restrict__ n_found, int32_t* __restrict__ hit_idx, float* __restrict__ hit_score) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= R) return;
  const int64_t b = off[r], e = off[r + 1];
  const int64_t len = soff[r + 1] - soff[r];
  float2 x0 = make_float2(0.f, 0.f), x1 = make_float2(0.f, 0.f);
  if (len >= N) direct_sum32(seq + soff[r], N, phase32, lane, x0, x1);
  const float X = wave_sum(x0.x * x0.x + x0.y * x0.y + x1.x * x1.x + x1.y * x1.y);
  int kept = 0;
  for (int64_t i = b; i < e; ++i) {
    const int32_t j = cand[i];
    float2 c0, c1;
    direct_sum32(ref + (int64_t)j * stride, N, phase32, lane, c0, c1);
    const float C = wave_sum(c0.x * c0.x + c0.y * c0.y + c1.x * c1.x + c1.y * c1.y);
    const float F = fidelity32(x0, x1, X, c0, c1, C, N);
    if (F > 0.f && F >= fmaxf(thr[j], floor_f)) {
      if (lane == 0) keys[b + kept] = make_key(F, j);
      ++kept;
    }
  }
  // lane 0's key stores are read back by every lane: make them visible
  // (stores completed, this compute unit's cache not holding stale lines)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  uint64_t prev = ~0ull;
  for (int o = 0; o < kept; ++o) {
    uint64_t best = 0;
    for (int i = lane; i < kept; i += 64) {
      const uint64_t v = keys[b + i];
      best = (v < prev && v > best) ? v : best;
    }
    best = wave_max_u64(best);
    if (lane == 0) write_list_entry(best, &hit_idx[b + o], &hit_score[b + o]);
    prev = best;
  }
  for (int64_t i = b + kept + lane; i < e; i += 64) write_list_entry(0, &hit_idx[i], &hit_score[i]);
  if (lane == 0) n_found[r] = kept;
}

}  // namespace

hipError_t launch_window_thresholds(const rm_index& idx, const uint8_t* ref, float err,
                                    int copies, int rank, uint32_t seed, float* thr,
                                    hipStream_t s) {
  const uint32_t T1 = (uint32_t)floor((double)err / 3.0 * 4294967296.0);
  const int N = idx.p.window_len;
  const int64_t blocks = (idx.n_windows + kThrWaves - 1) / kThrWaves;
  // the product form while the letters of a block's strings fit in 64 KB of LDS
  const int S = 1 + copies;
  const int rb = min(5, (S + 7) / 8);
  const int sp = (S + 8 * rb - 1) / (8 * rb) * (8 * rb);
  const int np = (N + 63) / 64 * 64;
  const size_t lds = (size_t)kThrWaves * sp * np;
  if (copies <= 64 && lds <= 65536) {
    auto kern = rb <= 1 ? window_thresholds_mfma_kernel<1>
              : rb == 2 ? window_thresholds_mfma_kernel<2>
              : rb == 3 ? window_thresholds_mfma_kernel<3>
              : rb == 4 ? window_thresholds_mfma_kernel<4> : window_thresholds_mfma_kernel<5>;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * kThrWaves), lds, s, ref, idx.ref_len,
                       idx.n_windows, N, np, idx.p.stride,
                       reinterpret_cast<const float*>(idx.d_phase32), T1, copies, sp, rank, seed,
                       8 * N + 64, thr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(window_thresholds_kernel, dim3((unsigned)blocks), dim3(64 * kThrWaves), 0, s,
                     ref, idx.ref_len, idx.n_windows, N, idx.p.stride,
                     reinterpret_cast<const float2*>(idx.d_phase32), T1, copies, rank, seed,
                     8 * N + 64, thr);
  return hipGetLastError();
}

ThresholdWs threshold_ws_layout(int32_t n_reads, int64_t capacity) {
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  ThresholdWs L{};
  size_t o = 0;
  L.pool = o;    o += up((size_t)capacity * 8);
  L.keys = o;    o += up((size_t)capacity * 8);
  L.cand = o;    o += up((size_t)capacity * 4);
  L.cnt = o;     o += up((size_t)n_reads * 4);
  L.fill = o;    o += up((size_t)n_reads * 4);
  L.pool_n = o;  o += 256;
  L.total = o;
  return L;
}

hipError_t launch_score_threshold(const rm_index& idx, const uint8_t* ref,
                                  const void* read_emb, const float* read_scale,
                                  const uint8_t* seq, const int64_t* soff, int32_t R,
                                  const float* thr, float floor_f, int64_t* hit_off,
                                  int32_t* n_found, int32_t* hit_idx, float* hit_score,
                                  int64_t* total, int64_t capacity, void* ws, hipStream_t s) {
  const ThresholdWs L = threshold_ws_layout(R, capacity);
  uint8_t* base = static_cast<uint8_t*>(ws);
  uint64_t* pool = reinterpret_cast<uint64_t*>(base + L.pool);
  uint64_t* keys = reinterpret_cast<uint64_t*>(base + L.keys);
  int32_t* cand = reinterpret_cast<int32_t*>(base + L.cand);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(base + L.cnt);
  uint32_t* fill = reinterpret_cast<uint32_t*>(base + L.fill);
  auto* pool_n = reinterpret_cast<unsigned long long*>(base + L.pool_n);
  const int prec = idx.p.precision;
  // the product's largest error in fidelity units (FP16 / FP8 rounding of
  // unit vectors, FP32 rolling drift), so no pair at or above its cut is lost
  const float margin = prec == RM_FP8_E4M3 ? 2e-2f : prec == RM_FP16 ? 2e-3f : 1e-4f;

  hipLaunchKernelGGL(zero_u32_kernel, dim3(256), dim3(256), 0, s, cnt, (int64_t)R);
  hipLaunchKernelGGL(zero_u32_kernel, dim3(256), dim3(256), 0, s, fill, (int64_t)R);
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, pool_n);

  const int64_t W = idx.n_windows;
  auto scan = [&](auto kern, int reads_per_block, int threads) {
    const int64_t n_rt = ((int64_t)R + reads_per_block - 1) / reads_per_block;
    int64_t n_chunks = (4096 + n_rt - 1) / n_rt;
    const int64_t max_chunks = (W + 1023) / 1024;  // at least 1,024 windows per chunk
    if (n_chunks > max_chunks) n_chunks = max_chunks;
    if (n_chunks < 1) n_chunks = 1;
    int64_t cw = (W + n_chunks - 1) / n_chunks;
    cw = (cw + kBlkW - 1) / kBlkW * kBlkW;
    n_chunks = (W + cw - 1) / cw;
    hipLaunchKernelGGL(kern, dim3((unsigned)(n_rt * n_chunks)), dim3(threads), 0, s,
                       static_cast<const uint8_t*>(idx.d_emb), idx.d_scale, W, thr, floor_f,
                       margin, static_cast<const uint8_t*>(read_emb), read_scale, R, cw,
                       (int)n_chunks, pool, (uint64_t)capacity, pool_n);
  };
  const bool red = reduced_rows(idx.p);
  if (prec == RM_FP32 && red)
    scan(threshold_scan_kernel<RM_FP32, kRealReduced>, ThrK<RM_FP32, kRealReduced>::READS,
         ThrK<RM_FP32, kRealReduced>::THREADS);
  else if (prec == RM_FP32)
    scan(threshold_scan_kernel<RM_FP32, kReal>, ThrK<RM_FP32, kReal>::READS,
         ThrK<RM_FP32, kReal>::THREADS);
  else if (prec == RM_FP16 && red)
    scan(threshold_scan_kernel<RM_FP16, kRealReduced>, ThrK<RM_FP16, kRealReduced>::READS,
         ThrK<RM_FP16, kRealReduced>::THREADS);
  else if (prec == RM_FP16)
    scan(threshold_scan_kernel<RM_FP16, kReal>, ThrK<RM_FP16, kReal>::READS,
         ThrK<RM_FP16, kReal>::THREADS);
  else if (red)
    scan(threshold_scan_kernel<RM_FP8_E4M3, kRealReduced>, ThrK<RM_FP8_E4M3, kRealReduced>::READS,
         ThrK<RM_FP8_E4M3, kRealReduced>::THREADS);
  else
    scan(threshold_scan_kernel<RM_FP8_E4M3, kReal>, ThrK<RM_FP8_E4M3, kReal>::READS,
         ThrK<RM_FP8_E4M3, kReal>::THREADS);

  hipLaunchKernelGGL(pool_count_kernel, dim3(1024), dim3(256), 0, s, pool, pool_n,
                     (uint64_t)capacity, cnt);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, s, cnt, R, hit_off, pool_n,
                     total);
  hipLaunchKernelGGL(pool_scatter_kernel, dim3(1024), dim3(256), 0, s, pool, pool_n,
                     (uint64_t)capacity, hit_off, fill, cand);
  hipLaunchKernelGGL(threshold_rescore_kernel, dim3((unsigned)(((int64_t)R + 3) / 4)), dim3(256),
                     0, s, ref, idx.p.window_len, idx.p.stride,
                     reinterpret_cast<const float2*>(idx.d_phase32), seq, soff, R, hit_off, cand,
                     thr, floor_f, keys, n_found, hit_idx, hit_score);
  return hipGetLastError();
}

}  // namespace rm
