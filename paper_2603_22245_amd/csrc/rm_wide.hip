// Token encodings with 1,024 complex components (§2.1 s-mers, §2.6 compact
// versions): e.g. 8-mers mapped to 256 classes with m = 4 -- the encoding the
// paper maps with (§3.5) -- or 4-mers with m = 4.  FP16 or FP8 e4m3 storage.
//
// Lane layout: lane l owns the 16 complex components [16 l, 16 l + 16), i.e.
// factor k = 16 l / n_class and classes c0 .. c0 + 15 with c0 = 16 l mod
// n_class (n_class a multiple of 16), stored at reals [32 l, 32 l + 32) of the
// 2,048-real row (re, im interleaved per component).
//
// The product has K = 2,048, too long to keep a read tile in registers as the
// 256-real scoring kernel does, so here both operands stream through LDS:
// block tiles of 256 A rows (128 reads) x 256 windows, K in 64-byte lines per
// row copied straight from global memory into a ring of four LDS stages
// (three in flight while one is computed), eight wavefronts of 64 x 128
// outputs on 32x32x16 FP16 (32x32x64 FP8) MFMAs.  The block tile is as large
// as the 160 KB of LDS allows, since its reuse sets the bytes copied per
// flop.  Per tile the epilogue writes F = Re^2 + Im^2 of every (read, window)
// to LDS and each wavefront compares 16 reads' scores with their current
// k-th best; the (rare) hits are inserted into the read's sorted list held in
// LDS.  A block walks the window tiles of one chunk and writes each read's
// list; a merge kernel keeps the k best over the chunks.
#include "rm_tokens.h"

namespace rm {

namespace {

constexpr int kWC = 16;     // complex components per lane
constexpr int kWR = 2048;   // reals per row
constexpr int kWM = 4;              // wavefronts along the rows (64 rows each)
constexpr int kWN = 2;              // wavefronts along the windows
constexpr int kGN = 4;              // 32-window column blocks per wavefront
constexpr int kWaves = kWM * kWN;
constexpr int kThreads = 64 * kWaves;
constexpr int kTM = 64 * kWM;       // A rows per block tile (kTM / 2 reads)
constexpr int kTN = 32 * kGN * kWN; // windows per block tile
constexpr int kLine = 64;   // bytes of every row per K stage (32 FP16 or 64 FP8 elements)
constexpr int kListMax = RM_WIDE_MAX_KFETCH;
constexpr int kGroupTiles = 8;   // read tiles per group of 32 blocks on one XCD
constexpr int kGroupChunks = 4;  // window chunks per group


typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// ---- encoders ---------------------------------------------------------------

// Direct sum over the tokens at locations 0..T-1 of `str`: the lane's 16
// components (class c0 + q gets phase[loc][k] for every token of that class).
template <typename T, typename E2>
__device__ __forceinline__ void wide_direct_sum(const uint8_t* __restrict__ str, int T_, int s,
                                                const uint8_t* __restrict__ table,
                                                const E2* __restrict__ phase, int m, int k, int c0,
                                                int lane, T (&re)[kWC], T (&im)[kWC]) {
#pragma unroll
  for (int q = 0; q < kWC; ++q) re[q] = im[q] = 0;
  for (int pb = 0; pb < T_; pb += 64) {
    const int mine = (pb + lane < T_) ? token_class(str + pb + lane, s, table) : kNoToken;
    const int cnt = min(64, T_ - pb);
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      E2 e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) e[u] = phase[(int64_t)min(pb + i0 + u, T_ - 1) * m + k];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = __builtin_amdgcn_readlane(mine, i0 + u) - c0;
#pragma unroll
        for (int q = 0; q < kWC; ++q) {
          re[q] += (c == q) ? (T)e[u].x : (T)0;
          im[q] += (c == q) ? (T)e[u].y : (T)0;
        }
      }
    }
  }
}

__device__ __forceinline__ uint32_t pack_h2(float a, float b) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)a) |
         ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)b) << 16);
}

// One row of 2,048 reals: this lane's 32 (x_q re, im for q = 0..15), each
// times `mul`.  FP16: 64 bytes per lane, returns 1.  FP8: the codes of the row
// divided by 2^e, the smallest power of two with max |x| / 2^e <= 448 (32
// bytes per lane), and returns the scale that makes code x scale exactly unit
// length (1 / the norm of the codes), as the 128-component encoders do.
template <int PREC>
__device__ __forceinline__ float store_wide_row(void* __restrict__ base, int64_t row, int lane,
                                                const float (&re)[kWC], const float (&im)[kWC],
                                                float mul) {
  if constexpr (PREC == RM_FP16) {
    uint4* dst = reinterpret_cast<uint4*>(static_cast<_Float16*>(base) + row * kWR) + lane * 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = 4 * v;
      dst[v] = make_uint4(pack_h2(re[q] * mul, im[q] * mul),
                          pack_h2(re[q + 1] * mul, im[q + 1] * mul),
                          pack_h2(re[q + 2] * mul, im[q + 2] * mul),
                          pack_h2(re[q + 3] * mul, im[q + 3] * mul));
    }
    return 1.f;
  } else {
    float m = 0.f;
#pragma unroll
    for (int q = 0; q < kWC; ++q) m = fmaxf(m, fmaxf(fabsf(re[q] * mul), fabsf(im[q] * mul)));
    m = wave_max_nonneg(m);
    const float s = fp8_pow2_scale(m);
    const float inv = pow2_reciprocal(s) * mul;  // exact power of two times mul
    uint32_t w[8];
    float q2 = 0.f;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int q = 2 * v;
      w[v] = pack_fp8x2(re[q] * inv, im[q] * inv) | (pack_fp8x2(re[q + 1] * inv, im[q + 1] * inv) << 16);
      const float2 d0 = unpack_fp8x2(w[v]), d1 = unpack_fp8x2(w[v] >> 16);
      q2 += d0.x * d0.x + d0.y * d0.y + d1.x * d1.x + d1.y * d1.y;
    }
    uint4* dst = reinterpret_cast<uint4*>(static_cast<uint8_t*>(base) + row * kWR) + lane * 2;
    dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
    dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
    q2 = wave_sum(q2);
    return q2 > 0.f ? __builtin_amdgcn_rsqf(q2) : s;
  }
}

template <int PREC>
__device__ __forceinline__ void emit_wide(int64_t j, int lane, int N, const float (&re)[kWC],
                                          const float (&im)[kWC], void* __restrict__ emb,
                                          float* __restrict__ scale, float* __restrict__ norm2) {
  float acc = 0.f;
#pragma unroll
  for (int q = 0; q < kWC; ++q) acc += re[q] * re[q] + im[q] * im[q];
  const float n2 = wave_sum(acc);
  const bool deg = n2 < kDegenerateRel * (float)N;
  const float inv = deg ? 0.f : __builtin_amdgcn_rsqf(n2);
  const float sc = store_wide_row<PREC>(emb, j, lane, re, im, inv);
  if (lane == 0) {
    norm2[j] = n2;
    scale[j] = sc;
  }
}

// Rolling window encoder (§3.4) with tokens, as the 128-component token
// encoder: FP64 re-anchor at each segment start, then one-letter slides in
// FP32 (rotate by omega^-f, the token at the old start loses omega^-f after
// the rotation, the token ending at the new last letter gains omega^(f (N-s))).
template <int PREC>
__global__ __launch_bounds__(256) void encode_reference_wide_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride, int s, int m, int n_class,
    int64_t seg_len, int64_t n_seg, const double2* __restrict__ phase64,
    const float4* __restrict__ step32, const uint8_t* __restrict__ table,
    void* __restrict__ emb, float* __restrict__ scale, float* __restrict__ norm2) {
  const int lane = threadIdx.x & 63;
  const int64_t seg = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (seg >= n_seg) return;
  const int k = kWC * lane / n_class, c0 = kWC * lane - k * n_class;
  const int T = N - s + 1;
  const int64_t j0 = seg * seg_len;
  const int64_t j1 = min(W, j0 + seg_len);

  float re[kWC], im[kWC];
  {
    double dr[kWC], di[kWC];
    wide_direct_sum(ref + j0 * stride, T, s, table, phase64, m, k, c0, lane, dr, di);
#pragma unroll
    for (int q = 0; q < kWC; ++q) {
      re[q] = (float)dr[q];
      im[q] = (float)di[q];
    }
  }
  emit_wide<PREC>(j0, lane, N, re, im, emb, scale, norm2);

  const float4 st = step32[k];
  const float rr = st.x, ri = st.y;  // omega^-f
  const float ir = st.z, ii = st.w;  // omega^(f (N-s))
  const int64_t s0 = j0 * stride;
  const int64_t n_slides = (j1 - 1 - j0) * stride;
  const int64_t in_off = N - s + 1;
  int64_t j = j0;
  int until_emit = stride;
  int out_c = lane < n_slides ? token_class(ref + s0 + lane, s, table) : kNoToken;
  int in_c = lane < n_slides ? token_class(ref + s0 + lane + in_off, s, table) : kNoToken;
  for (int64_t tb = 0; tb < n_slides; tb += 64) {
    const int64_t tn = tb + 64 + lane;
    const int out_next = tn < n_slides ? token_class(ref + s0 + tn, s, table) : kNoToken;
    const int in_next =
        tn < n_slides ? token_class(ref + s0 + tn + in_off, s, table) : kNoToken;
    const int cnt = (int)min<int64_t>(64, n_slides - tb);
    for (int i = 0; i < cnt; ++i) {
      const int o = __builtin_amdgcn_readlane(out_c, i) - c0;
      const int n = __builtin_amdgcn_readlane(in_c, i) - c0;
#pragma unroll
      for (int q = 0; q < kWC; ++q) {
        const float a = re[q] * rr - im[q] * ri;
        const float b = re[q] * ri + im[q] * rr;
        re[q] = a - (o == q ? rr : 0.f) + (n == q ? ir : 0.f);
        im[q] = b - (o == q ? ri : 0.f) + (n == q ? ii : 0.f);
      }
      if (--until_emit == 0) {
        until_emit = stride;
        ++j;
        emit_wide<PREC>(j, lane, N, re, im, emb, scale, norm2);
      }
    }
    out_c = out_next;
    in_c = in_next;
  }
}

// Read heads: FP64 direct sum, normalised; rows 2r = (Re x, Im x) and
// 2r+1 = (-Im x, Re x) per component, as for the 128-component encodings.
template <int PREC>
__global__ __launch_bounds__(256) void encode_reads_wide_kernel(
    const uint8_t* __restrict__ seq, const int64_t* __restrict__ off, int32_t n_reads, int N,
    int s, int m, int n_class, const float2* __restrict__ phase32,
    const uint8_t* __restrict__ table, void* __restrict__ emb, float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= n_reads) return;
  const int k = kWC * lane / n_class, c0 = kWC * lane - k * n_class;
  const int64_t start = off[r];
  const int64_t len = off[r + 1] - start;
  float xr[kWC], xi[kWC], nxi[kWC];
#pragma unroll
  for (int q = 0; q < kWC; ++q) xr[q] = xi[q] = 0.f;
  if (len >= N) wide_direct_sum(seq + start, N - s + 1, s, table, phase32, m, k, c0, lane, xr, xi);
  float acc = 0.f;
#pragma unroll
  for (int q = 0; q < kWC; ++q) acc += xr[q] * xr[q] + xi[q] * xi[q];
  const float X = wave_sum(acc);
  const float inv = X < kDegenerateRel * N ? 0.f : 1.f / sqrtf(X);
#pragma unroll
  for (int q = 0; q < kWC; ++q) {
    xr[q] *= inv;
    xi[q] *= inv;
    nxi[q] = -xi[q];
  }
  // both rows hold the same magnitudes: the same power of two and scale
  const float sc = store_wide_row<PREC>(emb, 2 * r, lane, xr, xi, 1.f);
  store_wide_row<PREC>(emb, 2 * r + 1, lane, nxi, xr, 1.f);
  if (scale != nullptr && lane == 0) scale[r] = sc;
}

// ---- product + per-read top-k -------------------------------------------------

__device__ __forceinline__ uint64_t wide_key(float F, int64_t j) {
  return ((uint64_t)(__float_as_uint(F) + 1u) << 32) | (0xffffffffu - (uint32_t)j);
}

// LDS byte offset of a pointer into a __shared__ array.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)((__attribute__((address_space(3))) const void*)p);
}

// Asynchronous copy of 16 bytes per lane from global memory straight into LDS
// (gfx950 global_load_lds_dwordx4): lane l writes LDS bytes [lds + 16 l,
// lds + 16 l + 16).  No output register; completion is awaited with
// wait_vm<N>(), which counts this wavefront's vector-memory operations in
// issue order.  The LDS base goes in through an m0 operand.
__device__ __forceinline__ void dma16w(const void* src, uint32_t lds) {
  asm volatile("global_load_lds_dwordx4 %0, off" ::"v"(src), "{m0}"(lds) : "memory");
}
template <int N>
__device__ __forceinline__ void wait_vm() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// A stage in LDS: kTM + kTN rows (the A rows, then the window rows) of kLine
// bytes of K; row r keeps its 16-byte chunk c at position c ^ swz(r), so
// that the rows a group of lanes reads at once (the same chunk of
// consecutive rows) fall on different banks.
constexpr int kStageBytes = (kTM + kTN) * kLine;  // 32 KB
constexpr int kChunks = kLine / 16;               // 16-byte chunks per row
constexpr int kRowsPerBankRow = 256 / kLine;      // rows per 256 bytes of LDS banks
constexpr int kRing = 4;                             // stages in LDS (three in flight)
constexpr int kDmaPerWave = (kTM + kTN) * kChunks / (64 * kWaves);  // copies per lane per stage
static_assert(kDmaPerWave * 64 * kWaves == (kTM + kTN) * kChunks, "stage splits into whole copies");
static_assert((kRing - 2) * kDmaPerWave <= 63, "vmcnt range");

__device__ __forceinline__ int swz(int row) { return (row / kRowsPerBankRow) % kChunks; }
__device__ __forceinline__ uint32_t chunk_pos(int row, int c) {
  return (uint32_t)(row * kLine + 16 * (c ^ swz(row)));
}

// Work items are (read tile, window chunk); a chunk is the window tiles
// [chunk * chunk_tiles, min(n_tiles, (chunk + 1) * chunk_tiles)).  Blocks go
// to the eight XCDs in turn (block b on XCD b % 8), so the 32 blocks i =
// 32 g' .. 32 g' + 31 of XCD x (i = b / 8) run side by side and share that
// XCD's L2: they take group G = 8 g' + x of 8 read tiles x 4 chunks, so every
// read tile's rows are streamed by 4 blocks and every chunk's window rows by 8
// blocks at about the same time.  Writes the k_fetch best keys of each of the
// tile's reads over the chunk to part[read][chunk][0..k_fetch) (0 = empty).
//
// FP16: 32x32x16 MFMAs, F = Re^2 + Im^2.  FP8: 32x32x64 MFMAs on the e4m3
// codes, F = (Re^2 + Im^2) (s_r s_j)^2 with the read's and the window's
// scales.
template <int PREC>
__global__ __launch_bounds__(kThreads, 1) void score_wide_kernel(
    const uint8_t* __restrict__ A, const float* __restrict__ a_scale, int32_t n_reads,
    const uint8_t* __restrict__ B, const float* __restrict__ b_scale, int64_t W,
    int n_rt, int64_t n_tiles, int64_t chunk_tiles, int n_chunks, int n_quads, int k_fetch,
    uint64_t* __restrict__ part) {
  // the stage ring, reused by the epilogue as the F buffer [kTM / 2 reads][kTN]
  __shared__ __attribute__((aligned(1024))) uint8_t ring[kRing][kStageBytes];
  __shared__ uint64_t lists[kTM / 2][kListMax];
  static_assert(sizeof(float) * (kTM / 2) * kTN <= sizeof(ring), "F buffer fits in the ring");
  float* Fbuf = reinterpret_cast<float*>(&ring[0][0]);
  constexpr bool kFp8 = PREC == RM_FP8_E4M3;
  constexpr int64_t kRowBytes = (int64_t)kWR * (kFp8 ? 1 : 2);
  constexpr int kStages = (int)(kRowBytes / kLine);

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / kWN, wc = wave % kWN;  // this wavefront's 64 rows x 32 kGN windows
  const int xcd = blockIdx.x % 8, i_x = blockIdx.x / 8;
  const int group = (i_x / 32) * 8 + xcd, j_g = i_x % 32;
  const int rt = (group / n_quads) * kGroupTiles + j_g / kGroupChunks;
  const int chunk = (group % n_quads) * kGroupChunks + j_g % kGroupChunks;
  if (rt >= n_rt || chunk >= n_chunks) return;  // the whole block, before any barrier
  const int64_t row0 = (int64_t)rt * kTM;  // first A row (= 2 x first read)
  const int64_t M = 2 * (int64_t)n_reads;
  const int64_t t0 = (int64_t)chunk * chunk_tiles;
  const int64_t t1 = min(n_tiles, t0 + chunk_tiles);
  const uint32_t ring_lds = lds_addr(&ring[0][0]);

  for (int i = tid; i < (kTM / 2) * kListMax; i += kThreads) (&lists[0][0])[i] = 0;

  // FP8: squared scales of this lane's reads (output rows 2q, 2q+1 of a 32-row
  // block hold read q; see the epilogue) -- and, per tile, of its windows
  float sr2[2][8];
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int vv = 0; vv < 8; ++vv) {
      sr2[f][vv] = 1.f;
      if constexpr (kFp8) {
        const int v = 2 * vv;
        const int row = 64 * wr + 32 * f + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int64_t r = row0 / 2 + (row >> 1);
        const float sc = r < n_reads ? a_scale[r] : 0.f;
        sr2[f][vv] = sc * sc;
      }
    }

  // This lane's 16-byte pieces of a stage: piece p = 64 (wave + kWaves i) +
  // lane lands at LDS position p (row p / kChunks, position p % kChunks) and
  // holds chunk (p % kChunks) ^ swz(row) of that row.  Rows past the last read or
  // window re-read the last one (always in bounds); their scores are never
  // used.
  int64_t src_off[kDmaPerWave];  // byte offset of the piece's row and chunk, K stage 0
  bool is_b[kDmaPerWave];
#pragma unroll
  for (int i = 0; i < kDmaPerWave; ++i) {
    const int p = 64 * (wave + kWaves * i) + lane;
    const int row = p / kChunks;
    const int c = (p % kChunks) ^ swz(row);
    is_b[i] = row >= kTM;
    src_off[i] = (is_b[i] ? (int64_t)(row - kTM) : min(row0 + row, M - 1)) * kRowBytes + c * 16;
  }
  // Stage st of a tile holds K line st, or line kStages - 1 - st on every
  // other tile of the chunk: a tile then starts on the read rows' lines the
  // previous one ended on, which the XCD's L2 still holds.
  auto issue = [&](int64_t tile, int st) {
    const uint32_t base = ring_lds + (uint32_t)(st % kRing) * kStageBytes;
    const int64_t kl = (int64_t)(((tile - t0) & 1) ? kStages - 1 - st : st) * kLine;
#pragma unroll
    for (int i = 0; i < kDmaPerWave; ++i) {
      const uint8_t* src;
      if (is_b[i]) {
        const int64_t g = min(tile * kTN + src_off[i] / kRowBytes, W - 1);
        src = B + g * kRowBytes + (src_off[i] % kRowBytes) + kl;
      } else {
        src = A + src_off[i] + kl;
      }
      dma16w(src, __builtin_amdgcn_readfirstlane(base + 1024 * (wave + kWaves * i)));
    }
  };

  for (int64_t tile = t0; tile < t1; ++tile) {
    f32x16 acc[2][kGN];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int g = 0; g < kGN; ++g)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[f][g][v] = 0.f;
    float sj2[kGN];
#pragma unroll
    for (int g = 0; g < kGN; ++g) sj2[g] = 1.f;
    if constexpr (kFp8) {
#pragma unroll
      for (int g = 0; g < kGN; ++g) {
        const int64_t j = tile * kTN + 32 * kGN * wc + 32 * g + (lane & 31);
        const float sc = b_scale[min(j, W - 1)];
        sj2[g] = sc * sc;
      }
    }

    // stages st .. st + kRing - 2 are in flight; one barrier per stage: after
    // it every wavefront's copies of stage st have landed and every wavefront
    // has finished reading stage st - 1, whose ring slot the copies of stage
    // st + kRing - 1 then overwrite
#pragma unroll
    for (int u = 0; u < kRing - 1; ++u) issue(tile, u);
    for (int st = 0; st < kStages; ++st) {
      if (st + kRing - 2 < kStages) wait_vm<(kRing - 2) * kDmaPerWave>(); else wait_vm<0>();
      __syncthreads();
      if (st + kRing - 1 < kStages) issue(tile, st + kRing - 1);
      const uint8_t* sb = &ring[st % kRing][0];
      if constexpr (!kFp8) {
#pragma unroll
        for (int ks = 0; ks < kLine / 32; ++ks) {
          const int c = 2 * ks + (lane >> 5);  // this lane's 8 halves of the 16-K step
          half8 a[2], b[kGN];
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const int row = 64 * wr + 32 * f + (lane & 31);
            a[f] = *reinterpret_cast<const half8*>(sb + chunk_pos(row, c));
          }
#pragma unroll
          for (int g = 0; g < kGN; ++g) {
            const int row = kTM + 32 * kGN * wc + 32 * g + (lane & 31);
            b[g] = *reinterpret_cast<const half8*>(sb + chunk_pos(row, c));
          }
#pragma unroll
          for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int g = 0; g < kGN; ++g)
              acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[f], b[g], acc[f][g], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int ks = 0; ks < kLine / 64; ++ks) {
          const int c = 4 * ks + 2 * (lane >> 5);  // this lane's 32 codes of the 64-K step
          i32x8 a[2], b[kGN];
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const int row = 64 * wr + 32 * f + (lane & 31);
            const uint4 u0 = *reinterpret_cast<const uint4*>(sb + chunk_pos(row, c));
            const uint4 u1 = *reinterpret_cast<const uint4*>(sb + chunk_pos(row, c + 1));
            a[f] = i32x8{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w,
                         (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
          }
#pragma unroll
          for (int g = 0; g < kGN; ++g) {
            const int row = kTM + 32 * kGN * wc + 32 * g + (lane & 31);
            const uint4 u0 = *reinterpret_cast<const uint4*>(sb + chunk_pos(row, c));
            const uint4 u1 = *reinterpret_cast<const uint4*>(sb + chunk_pos(row, c + 1));
            b[g] = i32x8{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w,
                         (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
          }
          // formats 0/0 = FP8 e4m3 for both operands; E8M0 scales 127 = 1.0
#pragma unroll
          for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int g = 0; g < kGN; ++g)
              acc[f][g] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[f], b[g], acc[f][g], 0,
                                                                           0, 0, 127, 0, 127);
        }
      }
    }
    __syncthreads();  // every wavefront is done with the ring before it becomes the F buffer

    // ---- epilogue: F of every (read, window) of the tile into LDS.  Output
    // element v of a 32x32 block is row 8(v/4) + 4(lane/32) + v%4, column
    // lane%32; rows 2q and 2q+1 (v even, v+1) are a read's Re and Im.
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int g = 0; g < kGN; ++g)
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
          const int row = 64 * wr + 32 * f + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          const int col = 32 * kGN * wc + 32 * g + (lane & 31);
          const float re = acc[f][g][v], im = acc[f][g][v + 1];
          float F = re * re + im * im;
          if constexpr (kFp8) F *= sr2[f][v >> 1] * sj2[g];
          Fbuf[(row >> 1) * kTN + col] = F;
        }
    __syncthreads();

    // ---- per read: compare with the k-th best, insert the hits (wavefront w
    // takes reads w, w + kWaves, ...; kTN / 64 windows per lane)
    constexpr int kH = kTN / 64;
    for (int rl = wave; rl < kTM / 2; rl += kWaves) {
      const int64_t r = row0 / 2 + rl;
      if (r >= n_reads) break;  // uniform
      const uint64_t th = lists[rl][k_fetch - 1];
      uint64_t key[kH], hit[kH], any = 0;
#pragma unroll
      for (int h = 0; h < kH; ++h) {
        const int col = lane + 64 * h;
        const int64_t j = tile * kTN + col;
        key[h] = j < W ? wide_key(Fbuf[rl * kTN + col], j) : 0;
        hit[h] = __ballot(key[h] > th);
        any |= hit[h];
      }
      if (any == 0) continue;
      uint64_t cur = lane < k_fetch ? lists[rl][lane] : 0;
#pragma unroll
      for (int h = 0; h < kH; ++h) {
        uint64_t hits = hit[h];
        while (hits != 0) {
          const int src = __builtin_ctzll(hits);
          hits &= hits - 1;
          const uint64_t kn = __shfl(key[h], src, 64);
          // position = entries that beat it; shift the rest down one lane
          const int pos = __popcll(__ballot(lane < k_fetch && cur > kn));
          if (pos >= k_fetch) continue;  // uniform
          const uint64_t up = __shfl_up(cur, 1, 64);
          cur = lane < pos ? cur : (lane == pos ? kn : up);
        }
      }
      if (lane < k_fetch) lists[rl][lane] = cur;
    }
    __syncthreads();  // before the next tile's first stage overwrites Fbuf
  }

  // ---- the chunk's list of every read of the tile
  for (int rl = wave; rl < kTM / 2; rl += kWaves) {
    const int64_t r = row0 / 2 + rl;
    if (r >= n_reads) break;
    if (lane < k_fetch) part[(r * n_chunks + chunk) * k_fetch + lane] = lists[rl][lane];
  }
}

// One wavefront per read: the k_fetch best of its n_chunks lists (keys are
// distinct: the chunks hold disjoint windows).
__global__ __launch_bounds__(256) void merge_wide_kernel(const uint64_t* __restrict__ part,
                                                         int32_t n_reads, int n, int k_fetch,
                                                         int32_t* __restrict__ cand_idx,
                                                         float* __restrict__ cand_score) {
  constexpr int EMAX = 8;
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n_reads) return;
  const uint64_t* src = part + r * n;
  uint64_t mine[EMAX];
#pragma unroll
  for (int e = 0; e < EMAX; ++e) {
    const int i = e * 64 + lane;
    mine[e] = i < n ? src[i] : 0;
  }
  uint64_t res = 0;
  for (int out = 0; out < k_fetch; ++out) {
    uint64_t best = 0;
#pragma unroll
    for (int e = 0; e < EMAX; ++e) best = mine[e] > best ? mine[e] : best;
    const uint64_t g = wave_max_u64(best);
#pragma unroll
    for (int e = 0; e < EMAX; ++e)
      if (g != 0 && mine[e] == g) mine[e] = 0;
    if (lane == out) res = g;
  }
  if (lane < k_fetch)
    write_list_entry(res, &cand_idx[r * k_fetch + lane], &cand_score[r * k_fetch + lane]);
}

// ---- FP32 rescore -------------------------------------------------------------

__device__ __forceinline__ uint64_t shfl_xor64w(uint64_t v, int d) {
  const uint32_t lo = __shfl_xor((uint32_t)v, d, 64);
  const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Four wavefronts per read: the head summed a quarter of its token locations
// per wavefront (quarters added in a fixed order), the candidates
// interleaved, every encoding a direct FP32 sum over its tokens; then the
// keys are sorted and the k best written.
__global__ __launch_bounds__(256) void rescore_wide_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride, int s, int m, int n_class,
    const float2* __restrict__ phase32, const uint8_t* __restrict__ table,
    const uint8_t* __restrict__ seq, const int64_t* __restrict__ off, int32_t R, int k_fetch,
    const int32_t* __restrict__ cand, int k, int32_t* __restrict__ top_idx,
    float* __restrict__ top_score) {
  __shared__ float part[4][2 * kWC][64];
  __shared__ uint64_t keys[RM_MAX_KFETCH];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r = blockIdx.x;
  const int64_t start = off[r];
  const int64_t len = off[r + 1] - start;
  const int T = N - s + 1;
  const int kf = kWC * lane / n_class, c0 = kWC * lane - kf * n_class;

  float xr[kWC], xi[kWC];
#pragma unroll
  for (int q = 0; q < kWC; ++q) xr[q] = xi[q] = 0.f;
  if (len >= N) {
    const int q0 = wave * T / 4, q1 = (wave + 1) * T / 4;
    wide_direct_sum(seq + start + q0, q1 - q0, s, table, phase32 + (int64_t)q0 * m, m, kf, c0,
                    lane, xr, xi);
  }
#pragma unroll
  for (int q = 0; q < kWC; ++q) {
    part[wave][2 * q][lane] = xr[q];
    part[wave][2 * q + 1][lane] = xi[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kWC; ++q) {
    xr[q] = ((part[0][2 * q][lane] + part[1][2 * q][lane]) + part[2][2 * q][lane]) +
            part[3][2 * q][lane];
    xi[q] = ((part[0][2 * q + 1][lane] + part[1][2 * q + 1][lane]) + part[2][2 * q + 1][lane]) +
            part[3][2 * q + 1][lane];
  }
  float ax = 0.f;
#pragma unroll
  for (int q = 0; q < kWC; ++q) ax += xr[q] * xr[q] + xi[q] * xi[q];
  const float X = wave_sum(ax);
  const bool xdeg = X < kDegenerateRel * (float)N;

  for (int e = wave; e < k_fetch; e += 4) {
    const int32_t j = cand[r * k_fetch + e];
    uint64_t key = 0;
    if (j >= 0 && j < W) {  // uniform per wavefront
      float cr[kWC], ci[kWC];
      wide_direct_sum(ref + (int64_t)j * stride, T, s, table, phase32, m, kf, c0, lane, cr, ci);
      float ac = 0.f, pr = 0.f, pi = 0.f;
#pragma unroll
      for (int q = 0; q < kWC; ++q) {
        ac += cr[q] * cr[q] + ci[q] * ci[q];
        pr += xr[q] * cr[q] + xi[q] * ci[q];  // <x|c> = sum conj(x) c
        pi += xr[q] * ci[q] - xi[q] * cr[q];
      }
      const float C = wave_sum(ac), ipr = wave_sum(pr), ipi = wave_sum(pi);
      const bool deg = xdeg || C < kDegenerateRel * (float)N;
      const float F = deg ? 0.f : (ipr * ipr + ipi * ipi) / (X * C);
      key = wide_key(F, j);
    }
    if (lane == 0) keys[e] = key;
  }
  __syncthreads();
  if (wave != 0) return;
  uint64_t key = lane < k_fetch ? keys[lane] : 0;
#pragma unroll
  for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
    for (int d = kk >> 1; d > 0; d >>= 1) {
      const uint64_t other = shfl_xor64w(key, d);
      const bool desc_block = (lane & kk) == 0;
      const bool lower = (lane & d) == 0;
      const uint64_t mx = key > other ? key : other;
      const uint64_t mn = key > other ? other : key;
      key = (lower == desc_block) ? mx : mn;
    }
  }
  if (lane < k) write_list_entry(key, &top_idx[r * k + lane], &top_score[r * k + lane]);
}

// Sums of FP32 phases in 64-bit fixed point with 2^-40 units: an FP32 value of
// magnitude 2^-17 or more is a whole number of units, a smaller one is off by
// less than one unit, and integer addition gives the same total whatever order
// the lanes' atomics land in.  |sum| <= N <= 2^14 keeps it below 2^54.
constexpr float kFixScale = 1099511627776.0f;  // 2^40
constexpr float kFixUnit = 1.0f / 1099511627776.0f;  // 2^-40
constexpr int kAccLen = kWideComplex + kWideComplex / kWC;  // one pad slot per lane's 16

// Accumulator slot of component `comp`: lane l's components 16l..16l+15 sit at
// a stride of 17 slots, so the lanes' read-back spreads over the banks.
__device__ __forceinline__ int acc_slot(int comp) { return comp + comp / kWC; }

// A running FP32 sum with its rounding error carried alongside (Knuth's
// TwoSum: hi + e equals a + b exactly), so many small additions to a large
// value lose nothing beyond the final rounding of hi + lo.
struct CompSum {
  float hi, lo;
  __device__ __forceinline__ void add(float b) {
    const float s = hi + b;
    const float bb = s - hi;
    lo += (hi - (s - bb)) + (b - bb);
    hi = s;
  }
  __device__ __forceinline__ float value() const { return hi + lo; }
};

// Orders this wavefront's LDS accesses (a compiler barrier plus a wait on them);
// no other wavefront is waited for.
__device__ __forceinline__ void lds_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// Refinement around coarse candidates (§3.4), 1,024 components, with the
// rolling inner product: O(m) work per one-token slide.  The read head as in
// rescore_wide_kernel; then per candidate (wavefront w takes candidates w,
// w + 4, ...) the first step-1 window of its neighbourhood is summed over its
// tokens with locations counted from that window's start lo: each lane takes
// every 64th token and adds phase[loc][k] to component k * n_class + class for
// each factor k in the wavefront's fixed-point accumulator u (64-bit LDS
// atomics; the exact sum of the FP32 phases).  Window lo + i is then
// omega^(-f_k i) u_i, where u_i has lost omega^(f i) at the class of each
// token that left and gained omega^(f (i + T)) at the class of each token
// that entered, so with P_k = sum over factor k's components of conj(x) u
// (lane k) and S = |u|^2 (rotation keeps norms), <x|c> = sum_k
// omega^(-f_k i) P_k and |c|^2 = S: a slide changes two components per factor
// and updates P_k and S by their changes (FP32, compensated sums).  Slot i of the candidate's
// span in `pool` receives the key of start lo + i, 0 past the clamped
// neighbourhood or for an invalid candidate.
__global__ __launch_bounds__(256) void refine_wide_kernel(
    const uint8_t* __restrict__ ref, int64_t W1, int N, int cstride, int64_t Wc, int s, int m,
    int n_class, const float2* __restrict__ phase32, const float4* __restrict__ step32,
    const uint8_t* __restrict__ table, const uint8_t* __restrict__ seq,
    const int64_t* __restrict__ off, int32_t R, int k_fetch, const int32_t* __restrict__ cand,
    int radius, uint64_t* __restrict__ pool) {
  // four wavefronts' accumulators (real and imaginary planes); the head's
  // partial sums use the front of the same memory before them
  __shared__ __attribute__((aligned(16))) unsigned long long acc[4][2][kAccLen];
  __shared__ float2 xs[kWideComplex];  // the read head's components
  static_assert(sizeof(acc) >= 4 * 2 * kWC * 64 * sizeof(float), "head partials fit");
  auto part = reinterpret_cast<float (*)[2 * kWC][64]>(&acc[0][0][0]);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r = blockIdx.x;
  const int64_t start = off[r];
  const int64_t len = off[r + 1] - start;
  const int span = 2 * radius + 1;
  const int T = N - s + 1;
  const int kf = kWC * lane / n_class, c0 = kWC * lane - kf * n_class;

  float xr[kWC], xi[kWC];
#pragma unroll
  for (int q = 0; q < kWC; ++q) xr[q] = xi[q] = 0.f;
  if (len >= N) {
    const int q0 = wave * T / 4, q1 = (wave + 1) * T / 4;
    wide_direct_sum(seq + start + q0, q1 - q0, s, table, phase32 + (int64_t)q0 * m, m, kf, c0,
                    lane, xr, xi);
  }
#pragma unroll
  for (int q = 0; q < kWC; ++q) {
    part[wave][2 * q][lane] = xr[q];
    part[wave][2 * q + 1][lane] = xi[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kWC; ++q) {
    xr[q] = ((part[0][2 * q][lane] + part[1][2 * q][lane]) + part[2][2 * q][lane]) +
            part[3][2 * q][lane];
    xi[q] = ((part[0][2 * q + 1][lane] + part[1][2 * q + 1][lane]) + part[2][2 * q + 1][lane]) +
            part[3][2 * q + 1][lane];
  }
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < kWC; ++q) xs[kWC * lane + q] = make_float2(xr[q], xi[q]);
  }
  // every wavefront has read the partials before any accumulator is cleared,
  // and the head's components are in xs
  __syncthreads();
  unsigned long long* accR = acc[wave][0];
  unsigned long long* accI = acc[wave][1];
  float ax = 0.f;
#pragma unroll
  for (int q = 0; q < kWC; ++q) ax += xr[q] * xr[q] + xi[q] * xi[q];
  const float X = wave_sum(ax);
  const bool xdeg = X < kDegenerateRel * (float)N;
  // lanes k < m carry factor k: omega^f, and omega^(f T) (T = N - s + 1)
  const int G = n_class / kWC;  // lanes per factor; m * G = 64
  const bool fl = lane < m;
  const float4 st = step32[fl ? lane : 0];
  const float2 fwd = make_float2(st.x, -st.y);             // omega^f
  const float2 adv = cmul(fwd, make_float2(st.z, st.w));  // omega^f omega^(f (N-s))

  for (int e = wave; e < k_fetch; e += 4) {
    uint64_t* out = pool + (r * k_fetch + e) * span;
    const int32_t j = cand[r * k_fetch + e];
    int64_t lo = 0, hi = -1;
    if (j >= 0 && j < Wc) {
      const int64_t c = (int64_t)j * cstride;
      lo = c - radius < 0 ? 0 : c - radius;
      hi = c + radius > W1 - 1 ? W1 - 1 : c + radius;
    }
    if (lane < span && lo + lane > hi) out[lane] = 0;
    if (hi < lo) continue;  // uniform
    // the first window, locations relative to lo: clear this lane's
    // components, scatter the tokens
    lds_order();
#pragma unroll
    for (int q = 0; q < kWC; ++q) {
      accR[acc_slot(kWC * lane + q)] = 0;
      accI[acc_slot(kWC * lane + q)] = 0;
    }
    lds_order();
    for (int loc = lane; loc < T; loc += 64) {
      const int c = token_class(ref + lo + loc, s, table);
      if (c < 0 || c >= n_class) continue;  // no token, or a class no component has
      for (int kk = 0; kk < m; ++kk) {
        const float2 e = phase32[(int64_t)loc * m + kk];
        const int slot = acc_slot(kk * n_class + c);
        atomicAdd(&accR[slot], (unsigned long long)(long long)(e.x * kFixScale));
        atomicAdd(&accI[slot], (unsigned long long)(long long)(e.y * kFixScale));
      }
    }
    lds_order();
    // u = that window's components: P_k = sum over factor k's components of
    // conj(x) u (lane k), S = |u|^2, FP32 sums
    float pr = 0.f, pi = 0.f, sq = 0.f;
#pragma unroll
    for (int q = 0; q < kWC; ++q) {
      const float ur = (float)(long long)accR[acc_slot(kWC * lane + q)] * kFixUnit;
      const float ui = (float)(long long)accI[acc_slot(kWC * lane + q)] * kFixUnit;
      pr += xr[q] * ur + xi[q] * ui;
      pi += xr[q] * ui - xi[q] * ur;
      sq += ur * ur + ui * ui;
    }
    for (int d = 1; d < G; d <<= 1) {  // a factor's G lanes are contiguous and aligned
      pr += __shfl_xor(pr, d, 64);
      pi += __shfl_xor(pi, d, 64);
    }
    // the slides' changes are added to P_k and S with compensated sums, so the
    // running values carry no more error than the first window's sums
    CompSum Pr{__shfl(pr, fl ? lane * G : 0, 64), 0.f}, Pi{__shfl(pi, fl ? lane * G : 0, 64), 0.f};
    if (!fl) Pr.hi = Pi.hi = 0.f;
    CompSum S{wave_sum(sq), 0.f};
    float2 wt = make_float2(1.f, 0.f);  // omega^(f_k i) at slide i, lanes k < m

    // lane i holds the classes of slide lo + i: the token leaving (at lo + i)
    // and the one entering (at lo + i + T, whose last letter lo + i + N <=
    // hi - 1 + N <= W1 - 2 + N = ref_len - 1)
    const int64_t tl = lo + lane;
    const int out_c = tl < hi ? token_class(ref + tl, s, table) : kNoToken;
    const int in_c = tl < hi ? token_class(ref + tl + T, s, table) : kNoToken;
    uint64_t mine = 0;
    for (int64_t t = lo; t <= hi; ++t) {
      // window t's components are omega^(-f_k (t - lo)) u: <x|c> = sum_k conj(wt_k) P_k
      const float pr_t = Pr.value(), pi_t = Pi.value(), S_t = S.value();
      const float ipr = wave_sum(wt.x * pr_t + wt.y * pi_t);
      const float ipi = wave_sum(wt.x * pi_t - wt.y * pr_t);
      const bool deg = xdeg || S_t < kDegenerateRel * N;
      const float F = deg ? 0.f : (ipr * ipr + ipi * ipi) / (X * S_t);
      if (lane == (int)(t - lo)) mine = wide_key(F, t);
      if (t < hi) {
        const int i = (int)(t - lo);
        const int oc = __builtin_amdgcn_readlane(out_c, i);
        const int ic = __builtin_amdgcn_readlane(in_c, i);
        float dS = 0.f;
        // lane k changes component k * n_class + class of each token by d:
        // P_k += conj(x) d, S += 2 Re(conj(u) d) + |d|^2, u += d (exactly)
        auto change = [&](int cls, float2 d) {
          const int comp = lane * n_class + cls;
          const int sl = acc_slot(comp);
          const float ur = (float)(long long)accR[sl] * kFixUnit;
          const float ui = (float)(long long)accI[sl] * kFixUnit;
          const float2 xv = xs[comp];
          Pr.add(xv.x * d.x + xv.y * d.y);
          Pi.add(xv.x * d.y - xv.y * d.x);
          dS += 2.f * (ur * d.x + ui * d.y) + (d.x * d.x + d.y * d.y);
          accR[sl] += (unsigned long long)(long long)(d.x * kFixScale);
          accI[sl] += (unsigned long long)(long long)(d.y * kFixScale);
        };
        // leaving: relative location i, omega^(f i); entering: i + T
        if (fl && oc >= 0 && oc < n_class) change(oc, make_float2(-wt.x, -wt.y));
        if (fl && ic >= 0 && ic < n_class) change(ic, cmul(wt, adv));
        S.add(wave_sum(dS));
        wt = cmul(wt, fwd);
      }
    }
    if (lane <= (int)(hi - lo)) out[lane] = mine;
  }
}

}  // namespace

WidePlan plan_wide(int32_t n_reads, int64_t W) {
  WidePlan p{};
  p.n_rt = (int)(((int64_t)n_reads * 2 + kTM - 1) / kTM);
  p.n_tiles = (W + kTN - 1) / kTN;
  // chunks per read tile: one group's worth (4), more when there are few read
  // tiles (enough items for the 256 compute units several times over)
  int64_t c = kGroupChunks * ((2560 / p.n_rt + kGroupChunks) / kGroupChunks);
  if (c > kWideMaxChunks) c = kWideMaxChunks;
  if (c > p.n_tiles) c = p.n_tiles;
  if (c < 1) c = 1;
  p.chunk_tiles = (p.n_tiles + c - 1) / c;
  p.n_chunks = (int)((p.n_tiles + p.chunk_tiles - 1) / p.chunk_tiles);
  p.n_quads = (p.n_chunks + kGroupChunks - 1) / kGroupChunks;
  const int64_t groups = (int64_t)((p.n_rt + kGroupTiles - 1) / kGroupTiles) * p.n_quads;
  p.n_blocks = (groups + 7) / 8 * 8 * 32;  // whole rounds of 8 groups (idle blocks return)
  return p;
}

size_t wide_workspace_bytes(int32_t n_reads, int64_t W, int32_t k_fetch) {
  const WidePlan p = plan_wide(n_reads, W);
  return ((size_t)n_reads * p.n_chunks * k_fetch * sizeof(uint64_t) + 255) / 256 * 256;
}

hipError_t launch_encode_reference_wide(const uint8_t* ref, int64_t W, const rm_params& p,
                                        const double* phase64, const float* step32,
                                        const uint8_t* table, void* emb, float* scale,
                                        float* norm2, hipStream_t st) {
  int64_t seg = p.reanchor;
  if (seg <= 0) {
    seg = (W + 8191) / 8192;
    if (seg < 256) seg = 256;
    if (seg > 4096) seg = 4096;
  }
  const int64_t n_seg = (W + seg - 1) / seg;
  const int64_t blocks = (n_seg + 3) / 4;
  auto kern = p.precision == RM_FP8_E4M3 ? encode_reference_wide_kernel<RM_FP8_E4M3>
                                          : encode_reference_wide_kernel<RM_FP16>;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, st, ref, W, p.window_len,
                     p.stride, p.mer_len > 1 ? p.mer_len : 1, p.n_freq, kWideComplex / p.n_freq,
                     seg, n_seg, reinterpret_cast<const double2*>(phase64),
                     reinterpret_cast<const float4*>(step32), table, emb, scale, norm2);
  return hipGetLastError();
}

hipError_t launch_encode_reads_wide(const rm_params& p, const float* phase32,
                                    const uint8_t* table, const uint8_t* seq, const int64_t* off,
                                    int32_t n_reads, void* emb, float* scale, hipStream_t st) {
  auto kern = p.precision == RM_FP8_E4M3 ? encode_reads_wide_kernel<RM_FP8_E4M3>
                                          : encode_reads_wide_kernel<RM_FP16>;
  hipLaunchKernelGGL(kern, dim3((unsigned)(((int64_t)n_reads + 3) / 4)), dim3(256), 0, st, seq,
                     off, n_reads, p.window_len, p.mer_len > 1 ? p.mer_len : 1, p.n_freq,
                     kWideComplex / p.n_freq, reinterpret_cast<const float2*>(phase32), table,
                     emb, scale);
  return hipGetLastError();
}

hipError_t launch_score_wide(const rm_index& idx, const void* read_emb, const float* read_scale,
                             int32_t n_reads, int32_t k_fetch, int32_t* cand_idx,
                             float* cand_score, void* ws, hipStream_t st) {
  const WidePlan p = plan_wide(n_reads, idx.n_windows);
  uint64_t* part = static_cast<uint64_t*>(ws);
  auto kern = idx.p.precision == RM_FP8_E4M3 ? score_wide_kernel<RM_FP8_E4M3>
                                              : score_wide_kernel<RM_FP16>;
  hipLaunchKernelGGL(kern, dim3((unsigned)p.n_blocks), dim3(kThreads), 0, st,
                     static_cast<const uint8_t*>(read_emb), read_scale, n_reads,
                     static_cast<const uint8_t*>(idx.d_emb), idx.d_scale, idx.n_windows, p.n_rt,
                     p.n_tiles, p.chunk_tiles, p.n_chunks, p.n_quads, k_fetch, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(merge_wide_kernel, dim3((unsigned)(((int64_t)n_reads + 3) / 4)), dim3(256), 0,
                     st, part, n_reads, p.n_chunks * k_fetch, k_fetch, cand_idx, cand_score);
  return hipGetLastError();
}

hipError_t launch_rescore_wide(const rm_index& idx, const uint8_t* ref, const uint8_t* seq,
                               const int64_t* off, int32_t n_reads, int32_t k_fetch,
                               const int32_t* cand_idx, int32_t k, int32_t* top_idx,
                               float* top_score, hipStream_t st) {
  hipLaunchKernelGGL(rescore_wide_kernel, dim3((unsigned)n_reads), dim3(256), 0, st, ref,
                     idx.n_windows, idx.p.window_len, idx.p.stride,
                     idx.p.mer_len > 1 ? idx.p.mer_len : 1, idx.p.n_freq,
                     kWideComplex / idx.p.n_freq, reinterpret_cast<const float2*>(idx.d_phase32),
                     idx.d_token_class, seq, off, n_reads, k_fetch, cand_idx, k, top_idx,
                     top_score);
  return hipGetLastError();
}

hipError_t launch_refine_wide(const rm_index& coarse, const uint8_t* ref, const uint8_t* seq,
                              const int64_t* off, int32_t n_reads, int32_t k_fetch,
                              const int32_t* cand_idx, int32_t radius, int32_t k, int32_t* top_idx,
                              float* top_score, void* ws, hipStream_t st) {
  const int N = coarse.p.window_len;
  const int64_t W1 = coarse.ref_len - N + 1;  // step-1 windows
  uint64_t* pool = static_cast<uint64_t*>(ws);
  hipLaunchKernelGGL(refine_wide_kernel, dim3((unsigned)n_reads), dim3(256), 0, st, ref, W1, N,
                     coarse.p.stride, coarse.n_windows,
                     coarse.p.mer_len > 1 ? coarse.p.mer_len : 1, coarse.p.n_freq,
                     kWideComplex / coarse.p.n_freq,
                     reinterpret_cast<const float2*>(coarse.d_phase32),
                     reinterpret_cast<const float4*>(coarse.d_step32), coarse.d_token_class, seq,
                     off, n_reads, k_fetch, cand_idx, radius, pool);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_refine_select(pool, k_fetch * (2 * radius + 1), n_reads, k, top_idx, top_score,
                              st);
}

}  // namespace rm
