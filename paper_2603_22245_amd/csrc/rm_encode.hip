// Encoders: the rolling window encoder that builds the index, and the read-head
// encoder.
//
// Lane layout (one wavefront = one string): lane l owns factor k = l >> 1 and
// the two letters 2h, 2h+1 with h = l & 1, i.e. complex components
// (k, 2h) and (k, 2h+1), stored at reals [4l, 4l+4) of the 256-real row
// (component index k*4 + letter, re/im interleaved).  One wavefront therefore
// writes a whole row with one coalesced store.
//
// Window encoder (§3.4): window j (start j*stride) follows from window j-1.
// With stride 1 a slide takes 1 from the outgoing letter's component, turns
// every component by omega^-f_k and adds omega^(f_k (N-1)) to the incoming
// letter's component.  A larger stride (up to kBlockMax, and at most N) moves
// a block at a time: E_{j+1} = omega^(-f s) (E_j - O_j + omega^(f N) I_j), where
// O_j and I_j add omega^(f q) over the s letters leaving (starts j s + q) and
// entering (j s + N + q), q < s -- one turn per window instead of one per
// letter; with integer factors and strides of 4 or more the block sums come
// from bf16 MFMA products of signed one-hot rows with the phase table.
// Longer strides slide letter by letter.  Each wavefront walks a
// segment of consecutive windows; at the segment start the state is computed
// directly from the letters in FP64 (the re-anchor), then rolled in FP32.
// Each window is normalised (§2.3) and written in the index precision.
#include <mutex>
#include <unordered_map>

#include "rm_bf16.h"
#include "rm_internal.h"
#include "rm_tokens.h"

namespace rm {

namespace {

struct Row4 {
  float v[4];
};

// Cross-lane move (DPP) with full row and bank masks; lanes without a source
// read 0.  Every lane must be active.
template <int CTRL>
__device__ __forceinline__ float mdpp(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}

// Sum over the 64 lanes as a wavefront-uniform value: row sums of 16 lanes by
// DPP (xor 1, xor 2, half-row mirror, row mirror), then each row adds the
// previous row's sum (row_bcast:15) and rows 2 and 3 add row 1's
// (row_bcast:31); lane 63 ends with (r3 + r2) + (r1 + r0), which is the
// (r0 + r1) + (r2 + r3) of wave_sum, since each addition is commutative.
// Every lane must be active.
__device__ __forceinline__ float wave_total(float v) {
  v += mdpp<0xB1>(v);
  v += mdpp<0x4E>(v);
  v += mdpp<0x141>(v);
  v += mdpp<0x140>(v);
  v += mdpp<0x142>(v);
  v += mdpp<0x143>(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Multipliers that put a letter's term on a lane's components: m0 = 1 where
// letter L is the lane's component 0 (L == 2h), m1 = 1 where it is component
// 1 (L == 2h + 1), both 0 otherwise.  The kernels keep the ten entries
// [h][min(L, 4)] in LDS (entry 4: codes above 3, no letter), so that a
// wavefront-uniform letter costs one LDS read and no branch or select.
struct LetterMul {
  float m0, m1;
};
//
// The letter-sum form (RED) keeps the rolling state in the letter-sum basis
// instead: per factor the coordinates on the orthonormal letter weights
// w_0 = (1,1,1,1)/2 (all letters), w_1 = (1,1,-1,-1)/2, w_2 = (1,-1,1,-1)/2,
// w_3 = (1,-1,-1,1)/2 over (A,C,G,T), lane h holding coordinates 2h and
// 2h + 1; a letter L then adds w_m[L] = +-1/2 of its term to every coordinate.
__device__ __forceinline__ float letter_weight(int m, int L) {
  if (L >= 4) return 0.f;
  const int neg = (m == 1 && L >= 2) || (m == 2 && (L & 1)) || (m == 3 && (L == 1 || L == 2));
  return neg ? -0.5f : 0.5f;
}
template <bool RED = false>
__device__ __forceinline__ LetterMul letter_mul_entry(int hh, int L) {
  if constexpr (RED) return LetterMul{letter_weight(2 * hh, L), letter_weight(2 * hh + 1, L)};
  return LetterMul{(L < 4 && L == 2 * hh) ? 1.f : 0.f, (L < 4 && L == 2 * hh + 1) ? 1.f : 0.f};
}
// With omega^(f N) = 1 (integer factors) a step adds the incoming letter's term
// and removes the outgoing one's with the same factor, so one entry serves both:
// [h][5 min(out, 4) + min(in, 4)] = multipliers of `in` minus those of `out`.
template <bool RED = false>
__device__ __forceinline__ LetterMul letter_pair_entry(int hh, int out, int in) {
  const LetterMul a = letter_mul_entry<RED>(hh, out), b = letter_mul_entry<RED>(hh, in);
  return LetterMul{b.m0 - a.m0, b.m1 - a.m1};
}
__device__ __forceinline__ int letter_pair_index(int packed) {  // out | in << 8
  return 5 * min(packed & 0xff, 4) + min(packed >> 8, 4);
}

// c += a m t on the lane's two components.
__device__ __forceinline__ void letter_fma(float2& c0, float2& c1, LetterMul w, float a,
                                           float2 t) {
  const float m0 = a * w.m0, m1 = a * w.m1;
  c0.x = fmaf(m0, t.x, c0.x);
  c0.y = fmaf(m0, t.y, c0.y);
  c1.x = fmaf(m1, t.x, c1.x);
  c1.y = fmaf(m1, t.y, c1.y);
}

// Write one normalised row (4 reals per lane) in the requested precision.
// Returns the FP8 scale used (1 for FP32/FP16).  FP8 codes are RNE(v / 2^e):
// a read row (WINDOW false) takes the smallest power of two 2^e with
// max |v| / 2^e <= 448; a window row takes 2^e = 2^-8 for every window (a
// unit vector's reals are at most 1, so 256 |v| <= 256 stays below 448, and
// e4m3's relative precision is the same everywhere in its normal range, so
// nothing is lost for the reals that matter).  The common exponent bounds
// every window's scale, which the product's threshold test relies on.
template <int PREC, bool WINDOW = false>
__device__ __forceinline__ float store_row(void* base, int64_t row, int lane, Row4 x) {
  if constexpr (PREC == RM_FP32) {
    float4* dst = reinterpret_cast<float4*>(static_cast<float*>(base) + row * kReal) + lane;
    *dst = make_float4(x.v[0], x.v[1], x.v[2], x.v[3]);
    return 1.f;
  } else if constexpr (PREC == RM_FP16) {
    _Float16 h0 = (_Float16)x.v[0], h1 = (_Float16)x.v[1], h2 = (_Float16)x.v[2],
             h3 = (_Float16)x.v[3];
    uint32_t lo = (uint32_t)__builtin_bit_cast(uint16_t, h0) |
                  ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
    uint32_t hi = (uint32_t)__builtin_bit_cast(uint16_t, h2) |
                  ((uint32_t)__builtin_bit_cast(uint16_t, h3) << 16);
    uint2* dst = reinterpret_cast<uint2*>(static_cast<_Float16*>(base) + row * kReal) + lane;
    *dst = make_uint2(lo, hi);
    return 1.f;
  } else {
    float s = kFp8WindowScale, inv = 1.f / kFp8WindowScale;
    if constexpr (!WINDOW) {
      float m = fmaxf(fmaxf(fabsf(x.v[0]), fabsf(x.v[1])), fmaxf(fabsf(x.v[2]), fabsf(x.v[3])));
      m = wave_max_nonneg(m);
      s = fp8_pow2_scale(m);
      inv = pow2_reciprocal(s);  // exact: s is a power of two
    }
    uint32_t w = pack_fp8x2(x.v[0] * inv, x.v[1] * inv) |
                 (pack_fp8x2(x.v[2] * inv, x.v[3] * inv) << 16);
    uint32_t* dst = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(base) + row * kReal) + lane;
    *dst = w;
    // Norm correction: the returned scale makes the dequantised row (code * scale)
    // exactly unit length.  For a pair of nearly equal vectors the first-order
    // error of F = |<x|c>|^2 is the change of squared norm Re<c, e_c> caused by
    // quantisation; renormalising removes it (phase errors only enter F at
    // second order).
    float2 d01 = unpack_fp8x2(w), d23 = unpack_fp8x2(w >> 16);
    float q2 = wave_total(d01.x * d01.x + d01.y * d01.y + d23.x * d23.x + d23.y * d23.y);
    return q2 > 0.f ? __builtin_amdgcn_rsqf(q2) : s;  // 1 ulp
  }
}

// ---- the letter-sum form (rows of kRealReduced reals)
// With integer factors (f_k = k < N, §2.2) the components of factor k of a
// window's vector sum over the four letters to sum_p omega^(k p) = 0 (each of
// the N locations holds one letter): the vector lies in the subspace
// orthogonal to the all-letters direction of every factor.  Its coordinates on
// the orthonormal basis of that subspace given by the three non-constant
// Walsh-Hadamard rows, (1,1,-1,-1)/2, (1,-1,1,-1)/2 and (1,-1,-1,1)/2 over
// the letters (A,C,G,T), keep its norm and its inner product with any read
// (the read's all-letters part meets zero), in 3 components per factor
// instead of 4.  Lane l holds letters 2h, 2h+1 (h = l & 1) of factor l/2,
// its partner l^1 the other two; the row's reals 3l .. 3l+2 are the lane's:
// (y1.re, y1.im, y2.re) for h = 0, (y2.im, y3.re, y3.im) for h = 1.
struct Row3 {
  float v[3];
};

// The lane's three reals of the projected row of (u0, u1) (its two
// components), and of the matching "Im" row (-Im y, Re y) of a read.
__device__ __forceinline__ void letter_sum_rows(float2 u0, float2 u1, int h, Row3& re, Row3& im) {
  const float2 s = make_float2(u0.x + u1.x, u0.y + u1.y);
  const float2 d = make_float2(u0.x - u1.x, u0.y - u1.y);
  // the partner lane's values (lane ^ 1), by DPP quad_perm [1,0,3,2]
  const float2 sp = make_float2(dpp<0xB1>(s.x), dpp<0xB1>(s.y));
  const float2 dp = make_float2(dpp<0xB1>(d.x), dpp<0xB1>(d.y));
  // y1 = (s01 - s23)/2, y2 = (d01 + d23)/2, y3 = (d01 - d23)/2, letters 0 and 1
  // being lane h = 0's
  const float sg = h ? -0.5f : 0.5f;
  const float2 y1 = make_float2(sg * (s.x - sp.x), sg * (s.y - sp.y));
  const float2 y2 = make_float2(0.5f * (d.x + dp.x), 0.5f * (d.y + dp.y));
  const float2 y3 = make_float2(sg * (d.x - dp.x), sg * (d.y - dp.y));
  if (h) {
    re = Row3{{y2.y, y3.x, y3.y}};
    im = Row3{{y2.x, -y3.y, y3.x}};
  } else {
    re = Row3{{y1.x, y1.y, y2.x}};
    im = Row3{{-y1.y, y1.x, -y2.y}};
  }
}

// Write the lane's three reals of a letter-sum row (reals 3 lane .. 3 lane + 2)
// in the requested precision; FP8 codes and the returned scale as for
// store_row, the scale making the dequantised row exactly as long as the
// FP32 row.  A window row (WINDOW) is the projection of a unit vector whose
// all-letters part is zero (the form is used only on references of letters
// only), so its length is 1 up to rounding and the dequantised row is made
// unit length, as store_row does; a read head may hold other codes, whose
// all-letters part the projection drops, so its length is summed.
template <int PREC, bool WINDOW = false>
__device__ __forceinline__ float store_row3(void* base, int64_t row, int lane, Row3 x) {
  if constexpr (PREC == RM_FP32) {
    float* dst = static_cast<float*>(base) + row * kRealReduced + 3 * lane;
    dst[0] = x.v[0];
    dst[1] = x.v[1];
    dst[2] = x.v[2];
    return 1.f;
  } else if constexpr (PREC == RM_FP16) {
    const uint32_t h0 = __builtin_bit_cast(uint16_t, (_Float16)x.v[0]);
    const uint32_t h1 = __builtin_bit_cast(uint16_t, (_Float16)x.v[1]);
    const uint32_t h2 = __builtin_bit_cast(uint16_t, (_Float16)x.v[2]);
    // uniform row start plus a 32-bit lane offset
    char* rowp = static_cast<char*>(base) + row * (int64_t)(kRealReduced * sizeof(uint16_t));
    uint16_t* dst = reinterpret_cast<uint16_t*>(rowp + 6 * lane);
    dst[0] = (uint16_t)h0;
    dst[1] = (uint16_t)h1;
    dst[2] = (uint16_t)h2;
    return 1.f;
  } else {
    float s = kFp8WindowScale, inv = 1.f / kFp8WindowScale;
    if constexpr (!WINDOW) {
      float m = fmaxf(fmaxf(fabsf(x.v[0]), fabsf(x.v[1])), fabsf(x.v[2]));
      m = wave_max_nonneg(m);
      s = fp8_pow2_scale(m);
      inv = pow2_reciprocal(s);
    }
    const uint32_t w01 = pack_fp8x2(x.v[0] * inv, x.v[1] * inv);
    const uint32_t w2 = pack_fp8x2(x.v[2] * inv, 0.f) & 0xffu;
    uint8_t* dst = static_cast<uint8_t*>(base) + row * kRealReduced + 3 * lane;
    dst[0] = (uint8_t)(w01 & 0xffu);
    dst[1] = (uint8_t)(w01 >> 8);
    dst[2] = (uint8_t)w2;
    const float2 d01 = unpack_fp8x2(w01), d2 = unpack_fp8x2(w2);
    const float q2 = wave_total(d01.x * d01.x + d01.y * d01.y + d2.x * d2.x);
    if constexpr (WINDOW) {
      return q2 > 0.f ? __builtin_amdgcn_rsqf(q2) : s;  // 1 ulp
    } else {
      const float y2 = wave_total(x.v[0] * x.v[0] + x.v[1] * x.v[1] + x.v[2] * x.v[2]);
      return q2 > 0.f ? __builtin_amdgcn_rsqf(q2) * sqrtf(y2) : s;
    }
  }
}

// FP64 direct sum over letters [0, n) of `str` for this lane's two components
// (letters 2h, 2h+1 of factor k).  The phase omega^(f_k p) is read from the FP64
// table at every 64th position and advanced in between by FP64 multiplication
// with omega^(f_k) (at most 63 products, relative error below 2^-45).  The
// letter is the same for the whole wavefront, so each position adds the phase
// to one of four per-letter sums by a uniform branch; the lane keeps the two
// sums of its own letters (RED: its two letter-sum coordinates, formed from
// the four sums).  Codes above 3 add nothing.
template <bool RED = false>
__device__ __forceinline__ void direct_sum(const uint8_t* __restrict__ str, int n,
                                           const double2* __restrict__ phase64, int lane,
                                           double2& a0, double2& a1) {
  const int k = lane >> 1, h = lane & 1;
  double2 s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0, s3 = s0;
  const double2 w = phase64[(n > 1 ? kM : 0) + k];  // omega^(f_k)
  for (int pb = 0; pb < n; pb += 64) {
    const int mine = (pb + lane < n) ? (int)str[pb + lane] : 255;
    const int cnt = min(64, n - pb);
    double2 t = phase64[(int64_t)pb * kM + k];
    for (int i = 0; i < cnt; ++i) {
      const int L = __builtin_amdgcn_readlane(mine, i);
      if (L == 0) {
        s0.x += t.x;
        s0.y += t.y;
      } else if (L == 1) {
        s1.x += t.x;
        s1.y += t.y;
      } else if (L == 2) {
        s2.x += t.x;
        s2.y += t.y;
      } else if (L == 3) {
        s3.x += t.x;
        s3.y += t.y;
      }
      t = make_double2(t.x * w.x - t.y * w.y, t.x * w.y + t.y * w.x);
    }
  }
  if constexpr (RED) {
    // h = 0: w_0, w_1 (s0 + s1 +- (s2 + s3)); h = 1: w_2, w_3 (s0 - s1 +- (s2 - s3))
    const double sg = h ? -1.0 : 1.0;
    const double2 u = make_double2(s0.x + sg * s1.x, s0.y + sg * s1.y);
    const double2 v = make_double2(s2.x + sg * s3.x, s2.y + sg * s3.y);
    a0 = make_double2(0.5 * (u.x + v.x), 0.5 * (u.y + v.y));
    a1 = make_double2(0.5 * (u.x - v.x), 0.5 * (u.y - v.y));
  } else {
    a0 = h ? s2 : s0;
    a1 = h ? s3 : s1;
  }
}

// A window's squared norm and scale wait in lane registers (lane j - jb
// holds window j) and go out with one store per 64 windows.  FP8: each lane
// keeps the largest (s_j / 2^-8)^2 of the windows it held, and at the end of
// the wavefront's segment `bound` (the index's d_scale[W]) receives their
// maximum by one atomic maximum (positive floats order as their bit patterns).
struct SideBuf {
  int64_t jb;  // first window held
  int n;       // windows held (uniform)
  float n2, sc;
  float* bound;  // FP8: d_scale[W]; otherwise null
  float rmax;    // FP8: this lane's largest (s_j / 2^-8)^2 so far
};

__device__ __forceinline__ void side_flush(SideBuf& b, int lane, float* norm2, float* scale) {
  if (lane < b.n) {
    norm2[b.jb + lane] = b.n2;
    scale[b.jb + lane] = b.sc;
    const float r = b.sc * (1.f / kFp8WindowScale);
    b.rmax = fmaxf(b.rmax, r * r);
  }
  b.jb += b.n;
  b.n = 0;
}

// The segment's last flush, then its share of the index-wide FP8 bound.
__device__ __forceinline__ void side_finish(SideBuf& b, int lane, float* norm2, float* scale) {
  side_flush(b, lane, norm2, scale);
  if (b.bound != nullptr) {
    const float m = wave_max_nonneg(b.rmax);
    if (lane == 0) atomicMax(reinterpret_cast<unsigned int*>(b.bound), __float_as_uint(m));
  }
}

template <int PREC, bool RED = false>
__device__ __forceinline__ void emit_window(int64_t j, int lane, int N, float2 c0, float2 c1,
                                            void* emb, SideBuf& side, float* scale,
                                            float* norm2) {
  const float n2 = wave_total(c0.x * c0.x + c0.y * c0.y + c1.x * c1.x + c1.y * c1.y);
  const bool deg = n2 < kDegenerateRel * (float)N;
  const float inv = deg ? 0.f : __builtin_amdgcn_rsqf(n2);  // 1 ulp
  float s;
  if constexpr (RED) {
    // The state is in the letter-sum basis: lane h = 0 holds (w_0, w_1) =
    // (all letters, y1), h = 1 holds (y2, y3); the row's reals are (y1.re,
    // y1.im, y2.re) for h = 0 and (y2.im, y3.re, y3.im) for h = 1.
    const float p = mdpp<0xB1>(c0.x);  // the partner's (lane ^ 1) c0.x: y2.re for h = 0
    Row3 y;
    if (lane & 1)
      y = Row3{{inv * c0.y, inv * c1.x, inv * c1.y}};
    else
      y = Row3{{inv * c1.x, inv * c1.y, inv * p}};
    s = store_row3<PREC, true>(emb, j, lane, y);
  } else {
    Row4 x{{c0.x * inv, c0.y * inv, c1.x * inv, c1.y * inv}};
    s = store_row<PREC, true>(emb, j, lane, x);
  }
  if (lane == side.n) {
    side.n2 = n2;
    side.sc = s;
  }
  if (++side.n == 64) side_flush(side, lane, norm2, scale);
}

// Strides up to this roll block by block; the table of omega^(f_k q), q < stride,
// sits in LDS (at most 64 x 32 complex FP32 = 16 KB per block of wavefronts).
constexpr int kBlockMax = 64;

__device__ __forceinline__ double2 cmul64(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

struct RollState {
  float2 c0, c1;
  int64_t j;  // last window emitted
};

// Byte offset of entry [0][i] in a table of LetterMul (lane h adds its row).
__device__ __forceinline__ const LetterMul& tab_entry(const LetterMul* row, int byte_off) {
  return *reinterpret_cast<const LetterMul*>(reinterpret_cast<const char*>(row) + byte_off);
}

// Roll a segment from its first window: `n_slides` letters t leave (ref[s0 + t])
// while ref[s0 + t + N] enters, 64 at a time (the next 64 are loaded while the
// current ones roll; each lane holds the table offsets of one letter, read out
// as wavefront-uniform values).  UZ: integer factors (omega^(f N) = 1), so the
// entering and leaving letters share one table entry.  BLOCK: strides 2..64 (at
// most N), one turn per window; otherwise one turn per letter, emitting every
// stride-th window.
template <int PREC, bool RED, bool UZ, bool BLOCK>
__device__ __forceinline__ void roll(const uint8_t* __restrict__ ref, int64_t s0, int64_t n_slides,
                                     int N, int stride, int k, int lane,
                                     const double2* __restrict__ phase64,
                                     const float4* __restrict__ step32, const float2* tq,
                                     const LetterMul (*ltab)[5], const LetterMul (*ptab)[25],
                                     RollState& st, SideBuf& side, void* emb, float* scale,
                                     float* norm2) {
  const int h = lane & 1;
  const LetterMul* lrow = ltab[h];
  const LetterMul* prow = ptab[h];
  float2 c0 = st.c0, c1 = st.c1;
  int64_t j = st.j;
  float2 rot, inc, z = make_float2(1.f, 0.f);
  if constexpr (BLOCK) {
    // omega^(f N) and omega^(-f stride) from the FP64 table, rounded once
    const double2 zN = cmul64(phase64[(int64_t)(N - 1) * kM + k], phase64[kM + k]);
    const double2 ws = stride < N ? phase64[(int64_t)stride * kM + k] : zN;
    rot = make_float2((float)ws.x, -(float)ws.y);
    z = make_float2((float)zN.x, (float)zN.y);
  } else {
    const float4 sv = step32[k];
    rot = make_float2(sv.x, sv.y);  // omega^-f
    inc = make_float2(sv.z, sv.w);  // omega^(f (N-1))
  }
  // per-lane letter offsets: UZ one pair entry, else the leaving and the
  // entering letter's entries (byte offsets into a table row)
  auto offsets = [&](int64_t t) -> int {
    const int o = t < n_slides ? (int)ref[s0 + t] : 255;
    const int n = t < n_slides ? (int)ref[s0 + t + N] : 255;
    if constexpr (UZ)
      return 8 * letter_pair_index(o | (n << 8));
    else
      return 8 * min(o, 4) | ((8 * min(n, 4)) << 8);
  };
  float2 i0 = make_float2(0.f, 0.f), i1 = i0;  // I_j (BLOCK, not UZ)
  int q = 0, until_emit = stride;
  int off_l = offsets(lane);
  for (int64_t tb = 0; tb < n_slides; tb += 64) {
    const int off_next = offsets(tb + 64 + lane);
    const int cnt = (int)min<int64_t>(64, n_slides - tb);
    for (int i = 0; i < cnt; ++i) {
      const int off = __builtin_amdgcn_readlane(off_l, i);
      if constexpr (BLOCK) {
        const float2 t = tq[q * kM + k];
        if constexpr (UZ) {
          letter_fma(c0, c1, tab_entry(prow, off), 1.f, t);
        } else {
          letter_fma(c0, c1, tab_entry(lrow, off & 0xff), -1.f, t);
          letter_fma(i0, i1, tab_entry(lrow, off >> 8), 1.f, t);
        }
        if (++q == stride) {
          q = 0;
          if constexpr (!UZ) {
            const float2 u0 = cmul(z, i0), u1 = cmul(z, i1);
            c0 = make_float2(c0.x + u0.x, c0.y + u0.y);
            c1 = make_float2(c1.x + u1.x, c1.y + u1.y);
            i0 = make_float2(0.f, 0.f);
            i1 = i0;
          }
          c0 = cmul(c0, rot);
          c1 = cmul(c1, rot);
          ++j;
          emit_window<PREC, RED>(j, lane, N, c0, c1, emb, side, scale, norm2);
        }
      } else {
        if constexpr (UZ) {  // omega^-f (E + [in] - [out])
          const LetterMul d = tab_entry(prow, off);
          c0.x += d.m0;
          c1.x += d.m1;
          c0 = cmul(c0, rot);
          c1 = cmul(c1, rot);
        } else {  // omega^-f (E - [out]) + omega^(f (N-1)) [in]
          const LetterMul wo = tab_entry(lrow, off & 0xff);
          c0.x -= wo.m0;
          c1.x -= wo.m1;
          c0 = cmul(c0, rot);
          c1 = cmul(c1, rot);
          letter_fma(c0, c1, tab_entry(lrow, off >> 8), 1.f, inc);
        }
        if (--until_emit == 0) {
          until_emit = stride;
          ++j;
          emit_window<PREC, RED>(j, lane, N, c0, c1, emb, side, scale, norm2);
        }
      }
    }
    off_l = off_next;
  }
  st = RollState{c0, c1, j};
}

// ---- block rolling on the matrix cores (integer factors, strides kMfmaStrideMin
// .. kBlockMax, at most N)
//
// With omega^(f N) = 1 the block update is E_{j+1} = omega^(-f s) (E_j + D_j),
// D_j[k][L] = sum_{q < s} omega^(f_k q) ([ref[j s + N + q] = L] - [ref[j s + q] = L]):
// the product of signed one-hot (window, letter) rows with the table [q][64
// reals] of omega^(f_k q).  Eight windows at a time, the wavefront forms it on
// 32x32x16 bf16 MFMAs (rows 4 w + L, columns 2 k + re/im, 16 positions per
// instruction): the indicators are exact in bfloat16 and the FP32 table splits
// exactly into three bfloat16 parts, so with FP32 accumulation D_j is the
// FP32 block sum up to the order of the additions.  D goes through LDS into
// the lane layout of the rolling state; the turn and the window's emission
// stay as in the letter-by-letter path.
constexpr int kMfmaStrideMin = 4;
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Eight letter codes at positions pos .. pos+7 (little-endian bytes of the
// pair), 4 for positions outside [0, len).
__device__ __forceinline__ uint2 letters8_bytes(const uint8_t* __restrict__ ref, int64_t pos,
                                                int64_t len) {
  uint32_t w[2] = {0u, 0u};
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t p = pos + i;
    const uint32_t c = (p >= 0 && p < len) ? (uint32_t)ref[p] : 4u;
    w[i >> 2] |= c << (8 * (i & 3));
  }
  return make_uint2(w[0], w[1]);
}

// The eight letters leaving (positions po ..) and entering (pi ..) as
// letters8_bytes gives them: where the aligned dwords around both runs lie
// inside the string, three dword loads each (issued together) and two byte
// alignments; bytewise otherwise.
__device__ __forceinline__ void letters8_pair(const uint8_t* __restrict__ ref, int64_t po,
                                              int64_t pi, int64_t len, uint2& out, uint2& in) {
  const uint32_t mis = (uint32_t)(reinterpret_cast<uintptr_t>(ref) & 3);
  const uint32_t so = (uint32_t)(po + mis) & 3, si = (uint32_t)(pi + mis) & 3;
  const int64_t bo = po - so, bi = pi - si;  // offsets of 4-byte aligned addresses
  if (bo >= 0 && bo + 12 <= len && bi >= 0 && bi + 12 <= len) {
    const uint32_t* d = reinterpret_cast<const uint32_t*>(ref + bo);
    const uint32_t* e = reinterpret_cast<const uint32_t*>(ref + bi);
    const uint32_t d0 = d[0], d1 = d[1], d2 = d[2];
    const uint32_t e0 = e[0], e1 = e[1], e2 = e[2];
    out = make_uint2(__builtin_amdgcn_alignbyte(d1, d0, so), __builtin_amdgcn_alignbyte(d2, d1, so));
    in = make_uint2(__builtin_amdgcn_alignbyte(e1, e0, si), __builtin_amdgcn_alignbyte(e2, e1, si));
  } else {
    out = letters8_bytes(ref, po, len);
    in = letters8_bytes(ref, pi, len);
  }
}

// Bytes of `w` clamped to at most 4 (codes above 3 are no letter).
__device__ __forceinline__ uint32_t clamp_codes(uint32_t w) {
  typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
  const u16x2 four{4, 4};
  const u16x2 ev = __builtin_elementwise_min(__builtin_bit_cast(u16x2, w & 0x00ff00ffu), four);
  const u16x2 od = __builtin_elementwise_min(__builtin_bit_cast(u16x2, (w >> 8) & 0x00ff00ffu), four);
  return __builtin_bit_cast(uint32_t, ev) | (__builtin_bit_cast(uint32_t, od) << 8);
}

// A fragment of eight positions of a signed (window, letter) row: bf16 2.0
// where only the entering letter is the row's letter, -2.0 where only the
// leaving one is, 0 otherwise (byte 0x40 / 0xc0 as the high byte; sums come out
// doubled).  `tab` has byte L = 0x40 for the row's letter L.
__device__ __forceinline__ bf16x8 signed_onehot(uint2 in, uint2 out, uint32_t tab) {
  uint32_t v[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const uint32_t bi = __builtin_amdgcn_perm(0u, tab, clamp_codes(i ? in.y : in.x));
    const uint32_t bo = __builtin_amdgcn_perm(0u, tab, clamp_codes(i ? out.y : out.x));
    const uint32_t x = bi ^ bo;
    v[i] = x | ((bo & x) << 1);  // 0x40 -> 0xc0 where the leaving letter matched
  }
  const u32x4 av{__builtin_amdgcn_perm(0u, v[0], 0x010c000cu), __builtin_amdgcn_perm(0u, v[0], 0x030c020cu),
                 __builtin_amdgcn_perm(0u, v[1], 0x010c000cu), __builtin_amdgcn_perm(0u, v[1], 0x030c020cu)};
  return __builtin_bit_cast(bf16x8, av);
}

// A fragment of eight positions of a (window, coordinate) row of the
// letter-sum form: byte L of `tab` is 0x40 or 0xc0 (bf16 +-2.0 = 4 w_m[L]) for
// the letters, codes above 3 give 0.
__device__ __forceinline__ bf16x8 weight_fragment(uint2 w, uint32_t tab) {
  const uint32_t b0 = __builtin_amdgcn_perm(0u, tab, clamp_codes(w.x));
  const uint32_t b1 = __builtin_amdgcn_perm(0u, tab, clamp_codes(w.y));
  const u32x4 av{__builtin_amdgcn_perm(0u, b0, 0x010c000cu), __builtin_amdgcn_perm(0u, b0, 0x030c020cu),
                 __builtin_amdgcn_perm(0u, b1, 0x010c000cu), __builtin_amdgcn_perm(0u, b1, 0x030c020cu)};
  return __builtin_bit_cast(bf16x8, av);
}

// NS = 16-position steps covering the stride (1, 2 or 4).  RED: rows are
// (window, letter-sum coordinate m) and the state is in that basis; the
// entering letters' rows (+4 w_m) and the leaving ones' (-4 w_m) go through
// the product separately, which returns 4 D.
template <int PREC, bool RED, int NS>
__global__ __launch_bounds__(256) void encode_reference_mfma_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride, int64_t seg_len, int64_t n_seg,
    const double2* __restrict__ phase64, void* __restrict__ emb, float* __restrict__ scale,
    float* __restrict__ norm2) {
  // per wavefront: D of 8 windows [w][column][letter, or coordinate (RED)],
  // times 2 (letters) or 4 (RED)
  __shared__ float dbuf[4][8][64][4];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t seg = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
  if (seg >= n_seg) return;
  const int k = lane >> 1, h = lane & 1;
  const int64_t j0 = seg * seg_len;
  const int64_t j1 = min(W, j0 + seg_len);
  const int64_t len = (W - 1) * (int64_t)stride + N;  // letters the windows cover

  // B fragments: column 32 cb + (lane & 31) = real (factor c >> 1, part c & 1),
  // positions 16 t + 8 (lane >> 5) + i, zero at and past the stride
  bf16x8 b[NS][3][2];
#pragma unroll
  for (int t = 0; t < NS; ++t)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int c = 32 * cb + (lane & 31);
      uint32_t hi[8], mid[8], lo[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int q = 16 * t + 8 * (lane >> 5) + i;
        float x = 0.f;
        if (q < stride) {
          const double2 e = phase64[(int64_t)q * kM + (c >> 1)];
          x = (float)((c & 1) ? e.y : e.x);
        }
        split_bf16x3(x, hi[i], mid[i], lo[i]);
      }
      const u32x4 vh{hi[0] | hi[1] << 16, hi[2] | hi[3] << 16, hi[4] | hi[5] << 16, hi[6] | hi[7] << 16};
      const u32x4 vm{mid[0] | mid[1] << 16, mid[2] | mid[3] << 16, mid[4] | mid[5] << 16,
                     mid[6] | mid[7] << 16};
      const u32x4 vl{lo[0] | lo[1] << 16, lo[2] | lo[3] << 16, lo[4] | lo[5] << 16, lo[6] | lo[7] << 16};
      b[t][0][cb] = __builtin_bit_cast(bf16x8, vh);
      b[t][1][cb] = __builtin_bit_cast(bf16x8, vm);
      b[t][2][cb] = __builtin_bit_cast(bf16x8, vl);
    }
  // omega^(-f stride), rounded once from FP64 (the table holds rows below N)
  const double2 ws = stride < N ? phase64[(int64_t)stride * kM + k]
                                : cmul64(phase64[(int64_t)(N - 1) * kM + k], phase64[kM + k]);
  const float2 rot = make_float2((float)ws.x, -(float)ws.y);

  // Re-anchor: the first window of the segment, directly, in FP64.
  double2 a0, a1;
  direct_sum<RED>(ref + j0 * stride, N, phase64, lane, a0, a1);
  float2 c0 = make_float2((float)a0.x, (float)a0.y);
  float2 c1 = make_float2((float)a1.x, (float)a1.y);
  SideBuf side{j0, 0, 0.f, 0.f, PREC == RM_FP8_E4M3 ? scale + W : nullptr, 0.f};
  emit_window<PREC, RED>(j0, lane, N, c0, c1, emb, side, scale, norm2);

  // A role: row lane & 31 = 4 w + L (window jc + w, letter L, or letter-sum
  // coordinate L), positions 8 (lane >> 5) .. + 7 of each 16-position step
  const int aw = (lane & 31) >> 2, aL = lane & 3;
  const uint32_t tab = RED ? (aL == 0 ? 0x40404040u : aL == 1 ? 0xc0c04040u
                              : aL == 2 ? 0xc040c040u : 0x40c0c040u)
                           : 0x40u << (8 * aL);
  const float dscale = RED ? 0.25f : 0.5f;  // the product returns 4 D (RED) or 2 D
  float(*db)[64][4] = dbuf[wv];
  for (int64_t jc = j0; jc < j1 - 1; jc += 8) {
    f32x16 acc[2] = {f32x16{}, f32x16{}};
    const int64_t sw = (jc + aw) * (int64_t)stride;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int q0 = 16 * t + 8 * (lane >> 5);
      bf16x8 a = __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u}), ao = a;
      if (q0 < stride) {
        uint2 lo, li;
        letters8_pair(ref, sw + q0, sw + N + q0, len, lo, li);
        if constexpr (RED) {
          a = weight_fragment(li, tab);
          ao = weight_fragment(lo, tab ^ 0x80808080u);
        } else {
          a = signed_onehot(li, lo, tab);
        }
      }
#pragma unroll
      for (int pt = 2; pt >= 0; --pt) {
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[t][pt][0], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[t][pt][1], acc[1], 0, 0, 0);
        if constexpr (RED) {
          acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ao, b[t][pt][0], acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ao, b[t][pt][1], acc[1], 0, 0, 0);
        }
      }
    }
    // D rows 8 g + 4 (lane >> 5) + L: window 2 g + (lane >> 5), letter L
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int L = 0; L < 4; ++L) db[2 * g + (lane >> 5)][32 * cb + (lane & 31)][L] = acc[cb][4 * g + L];
    __builtin_amdgcn_wave_barrier();
    const int nw = (int)min<int64_t>(8, j1 - 1 - jc);
    for (int w = 0; w < nw; ++w) {
      // rows 2h, 2h+1 (letters or coordinates) of the real parts (column 2k)
      // and imaginary parts (2k+1)
      const float* dre = &db[w][2 * k][2 * h];
      const float* dim = &db[w][2 * k + 1][2 * h];
      c0 = make_float2(fmaf(dscale, dre[0], c0.x), fmaf(dscale, dim[0], c0.y));
      c1 = make_float2(fmaf(dscale, dre[1], c1.x), fmaf(dscale, dim[1], c1.y));
      c0 = cmul(c0, rot);
      c1 = cmul(c1, rot);
      emit_window<PREC, RED>(jc + w + 1, lane, N, c0, c1, emb, side, scale, norm2);
    }
    __builtin_amdgcn_wave_barrier();
  }
  side_finish(side, lane, norm2, scale);
}

template <int PREC, bool RED>
__global__ __launch_bounds__(256) void encode_reference_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride, int unit_z, int64_t seg_len,
    int64_t n_seg, const double2* __restrict__ phase64, const float4* __restrict__ step32,
    void* __restrict__ emb, float* __restrict__ scale, float* __restrict__ norm2) {
  extern __shared__ float2 tq[];  // [stride][kM] omega^(f_k q): block rolling only
  __shared__ LetterMul ltab[2][5];
  __shared__ LetterMul ptab[2][25];
  const bool blockwise = stride > 1 && stride <= kBlockMax && stride <= N;
  if (blockwise) {
    for (int v = threadIdx.x; v < stride * kM; v += blockDim.x) {
      const double2 e = phase64[v];
      tq[v] = make_float2((float)e.x, (float)e.y);
    }
  }
  if (threadIdx.x < 10)
    ltab[threadIdx.x / 5][threadIdx.x % 5] = letter_mul_entry<RED>(threadIdx.x / 5, threadIdx.x % 5);
  if (threadIdx.x < 50) {
    const int hh = threadIdx.x / 25, e = threadIdx.x % 25;
    ptab[hh][e] = letter_pair_entry<RED>(hh, e / 5, e % 5);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // wavefront-uniform, so that the segment's bookkeeping stays in scalar registers
  const int64_t seg = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                      __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (seg >= n_seg) return;
  const int k = lane >> 1, h = lane & 1;
  const int64_t j0 = seg * seg_len;
  const int64_t j1 = min(W, j0 + seg_len);

  // Re-anchor: the first window of the segment, directly, in FP64.
  double2 a0, a1;
  direct_sum<RED>(ref + j0 * stride, N, phase64, lane, a0, a1);
  float2 c0 = make_float2((float)a0.x, (float)a0.y);
  float2 c1 = make_float2((float)a1.x, (float)a1.y);
  SideBuf side{j0, 0, 0.f, 0.f, PREC == RM_FP8_E4M3 ? scale + W : nullptr, 0.f};
  emit_window<PREC, RED>(j0, lane, N, c0, c1, emb, side, scale, norm2);

  // Letter t = 0 .. n_slides-1 of the segment leaves at start s0 + t + 1 (it
  // is ref[s0 + t]) while ref[s0 + t + N] enters.
  const int64_t s0 = j0 * stride;
  const int64_t n_slides = (j1 - 1 - j0) * stride;
  RollState st{c0, c1, j0};
  if (blockwise) {
    if (unit_z)
      roll<PREC, RED, true, true>(ref, s0, n_slides, N, stride, k, lane, phase64, step32, tq, ltab,
                                  ptab, st, side, emb, scale, norm2);
    else
      roll<PREC, RED, false, true>(ref, s0, n_slides, N, stride, k, lane, phase64, step32, tq, ltab,
                                   ptab, st, side, emb, scale, norm2);
  } else {
    if (unit_z)
      roll<PREC, RED, true, false>(ref, s0, n_slides, N, stride, k, lane, phase64, step32, tq, ltab,
                                   ptab, st, side, emb, scale, norm2);
    else
      roll<PREC, RED, false, false>(ref, s0, n_slides, N, stride, k, lane, phase64, step32, tq,
                                    ltab, ptab, st, side, emb, scale, norm2);
  }
  side_finish(side, lane, norm2, scale);
}

// Normalise a read head (this lane's two components, FP32 sums; a squared
// norm below kDegenerateRel * N gives the zero vector) and store its two real
// rows: 2r = (Re x, Im x) per component, 2r+1 = (-Im x, Re x).  A window row
// (Re c, Im c) dotted with them gives Re and Im of sum conj(x) c.
template <int PREC, bool RED = false>
__device__ __forceinline__ void emit_head(float2 a0, float2 a1, int N, int64_t r, int lane,
                                          void* __restrict__ emb, float* __restrict__ scale) {
  const float X = wave_sum(a0.x * a0.x + a0.y * a0.y + a1.x * a1.x + a1.y * a1.y);
  const float inv = X < kDegenerateRel * N ? 0.f : 1.f / sqrtf(X);
  const float xr0 = a0.x * inv, xi0 = a0.y * inv;
  const float xr1 = a1.x * inv, xi1 = a1.y * inv;
  float s;
  if constexpr (RED) {  // the letter-sum form (a window's all-letters part is zero)
    Row3 re, im;
    letter_sum_rows(make_float2(xr0, xi0), make_float2(xr1, xi1), lane & 1, re, im);
    s = store_row3<PREC>(emb, 2 * r, lane, re);
    store_row3<PREC>(emb, 2 * r + 1, lane, im);
  } else {
    Row4 re{{xr0, xi0, xr1, xi1}};
    Row4 im{{-xi0, xr0, -xi1, xr1}};
    s = store_row<PREC>(emb, 2 * r, lane, re);
    store_row<PREC>(emb, 2 * r + 1, lane, im);
  }
  if (scale != nullptr && lane == 0) scale[r] = s;
}

// Read heads (§3.1: the first N letters of each read): an FP32 direct sum of
// the FP32 phase table over the head's letters, one wavefront per read.  A
// read shorter than N is the zero vector.
template <int PREC, bool RED>
__global__ __launch_bounds__(256) void encode_reads_kernel(
    const uint8_t* __restrict__ seq, const int64_t* __restrict__ off, int32_t n_reads, int N,
    const float2* __restrict__ phase32, void* __restrict__ emb, float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                    __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (r >= n_reads) return;
  const int64_t start = off[r];
  const int64_t len = off[r + 1] - start;
  float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
  if (len >= N) direct_sum32(seq + start, N, phase32, lane, a0, a1);
  emit_head<PREC, RED>(a0, a1, N, r, lane, emb, scale);
}

// ---- learned token offsets -------------------------------------------------
// With learned offsets a window of N letters holds the N-8 tokens at
// locations p = 0..N-9; token t of the reference (9-mer w[t..t+8]) adds
// exp(i (theta_k p + delta[t][k])) to component (k, w[t+4]).  One slide moves
// the window start from s to s+1: every component is multiplied by omega^-f_k,
// token s leaves (its term, multiplied by omega^-f_k, is subtracted) and token
// s+N-8 enters at location N-9 (exp(i delta) times omega^(f_k (N-9)) is
// added).  delta is row-major [tokens][32], FP32.

// FP64 direct sum over the tokens p = 0..N-9 of a string whose token offsets
// are rows drow[p] (lane's two components).
__device__ __forceinline__ void direct_sum_learned(const uint8_t* __restrict__ str, int N,
                                                   const float* __restrict__ drow,
                                                   const double2* __restrict__ phase64, int lane,
                                                   double2& a0, double2& a1) {
  const int k = lane >> 1, h = lane & 1;
  const int L0 = 2 * h, L1 = 2 * h + 1;
  const int T = N - 8;
  a0 = make_double2(0.0, 0.0);
  a1 = make_double2(0.0, 0.0);
  for (int pb = 0; pb < T; pb += 64) {
    int mine = (pb + lane < T) ? (int)str[pb + lane + 4] : 255;
    int cnt = min(64, T - pb);
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      double2 e[8];
      float d[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int p = min(pb + i0 + u, T - 1);
        e[u] = phase64[(int64_t)p * kM + k];
        d[u] = drow[(int64_t)p * 32 + k];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int L = __builtin_amdgcn_readlane(mine, i0 + u);
        double sn, cs;
        sincos((double)d[u], &sn, &cs);
        const double er = e[u].x * cs - e[u].y * sn, ei = e[u].x * sn + e[u].y * cs;
        a0.x += (L == L0) ? er : 0.0;
        a0.y += (L == L0) ? ei : 0.0;
        a1.x += (L == L1) ? er : 0.0;
        a1.y += (L == L1) ? ei : 0.0;
      }
    }
  }
}

constexpr int kChunk = 32;  // slides whose token terms are staged in LDS at once

template <int PREC>
__global__ __launch_bounds__(256) void encode_reference_learned_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride, int64_t seg_len, int64_t n_seg,
    const double2* __restrict__ phase64, const float2* __restrict__ phase32,
    const float4* __restrict__ step32, const float* __restrict__ delta, void* __restrict__ emb,
    float* __restrict__ scale, float* __restrict__ norm2) {
  // per wavefront: exp(i delta) of the outgoing (row 0..31) and incoming
  // (rows 32..63) tokens of the current chunk of slides
  __shared__ float2 u_stage[4][2 * kChunk][32];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t seg = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (seg >= n_seg) return;
  const int k = lane >> 1, h = lane & 1;
  const int L0 = 2 * h, L1 = 2 * h + 1;
  const int64_t j0 = seg * seg_len;
  const int64_t j1 = min(W, j0 + seg_len);

  double2 a0, a1;
  const int64_t s0 = j0 * stride;
  direct_sum_learned(ref + s0, N, delta + s0 * 32, phase64, lane, a0, a1);
  float2 c0 = make_float2((float)a0.x, (float)a0.y);
  float2 c1 = make_float2((float)a1.x, (float)a1.y);
  SideBuf side{j0, 0, 0.f, 0.f, PREC == RM_FP8_E4M3 ? scale + W : nullptr, 0.f};
  emit_window<PREC>(j0, lane, N, c0, c1, emb, side, scale, norm2);

  const float4 st = step32[k];
  const float2 rot = make_float2(st.x, st.y);    // omega^-f
  const float2 inc = phase32[(int64_t)(N - 9) * kM + k];  // omega^(f (N-9))
  float2(*stage)[32] = u_stage[wave];

  const int64_t n_slides = (j1 - 1 - j0) * stride;
  int64_t j = j0;
  int until_emit = stride;
  for (int64_t tb = 0; tb < n_slides; tb += kChunk) {
    const int cnt = (int)min<int64_t>(kChunk, n_slides - tb);
    // stage exp(i delta) of tokens s0+tb+i (out) and s0+tb+i+N-8 (in), i < cnt
#pragma unroll 4
    for (int q = 0; q < 2 * kChunk * 32 / 64; ++q) {
      const int v = q * 64 + lane;
      const int row = v >> 5, kk = v & 31;
      const int i = row & (kChunk - 1);
      if (i < cnt) {
        const int64_t tok = s0 + tb + i + (row >= kChunk ? N - 8 : 0);
        float sn, cs;
        __sincosf(delta[tok * 32 + kk], &sn, &cs);  // hardware sin/cos: ~1e-6 for offsets of a few radians
        stage[row][kk] = make_float2(cs, sn);
      }
    }
    __builtin_amdgcn_wave_barrier();
    // letters: outgoing token middle ref[s0+t+4], incoming ref[s0+t+N-4]
    const int64_t t = tb + (lane & (kChunk - 1));
    const bool in_half = lane >= kChunk;
    int mine = 255;
    if ((lane & (kChunk - 1)) < cnt) mine = (int)ref[s0 + t + (in_half ? N - 4 : 4)];
    for (int i = 0; i < cnt; ++i) {
      const int o = __builtin_amdgcn_readlane(mine, i);
      const int n = __builtin_amdgcn_readlane(mine, i + kChunk);
      slide(c0, c1, rot, o, n, h, cmul(stage[i][k], rot), cmul(stage[kChunk + i][k], inc));
      if (--until_emit == 0) {
        until_emit = stride;
        ++j;
        emit_window<PREC>(j, lane, N, c0, c1, emb, side, scale, norm2);
      }
    }
    __builtin_amdgcn_wave_barrier();  // the stage is rewritten by the next chunk
  }
  side_finish(side, lane, norm2, scale);
}

// The same sum in FP32 with the FP32 table (read heads): each term is the
// table entry omega^(f_k p) turned by exp(i delta).
__device__ __forceinline__ void direct_sum_learned32(const uint8_t* __restrict__ str, int N,
                                                     const float* __restrict__ drow,
                                                     const float2* __restrict__ phase32, int lane,
                                                     float2& a0, float2& a1) {
  const int k = lane >> 1, h = lane & 1;
  const int L0 = 2 * h, L1 = 2 * h + 1;
  const int T = N - 8;
  a0 = make_float2(0.f, 0.f);
  a1 = make_float2(0.f, 0.f);
  for (int pb = 0; pb < T; pb += 64) {
    int mine = (pb + lane < T) ? (int)str[pb + lane + 4] : 255;
    int cnt = min(64, T - pb);
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      float2 e[8];
      float d[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int p = min(pb + i0 + u, T - 1);
        e[u] = phase32[(int64_t)p * kM + k];
        d[u] = drow[(int64_t)p * 32 + k];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int L = __builtin_amdgcn_readlane(mine, i0 + u);
        float sn, cs;
        sincosf(d[u], &sn, &cs);
        const float er = e[u].x * cs - e[u].y * sn, ei = e[u].x * sn + e[u].y * cs;
        a0.x += (L == L0) ? er : 0.f;
        a0.y += (L == L0) ? ei : 0.f;
        a1.x += (L == L1) ? er : 0.f;
        a1.y += (L == L1) ? ei : 0.f;
      }
    }
  }
}

template <int PREC>
__global__ __launch_bounds__(256) void encode_reads_learned_kernel(
    const uint8_t* __restrict__ seq, const int64_t* __restrict__ off, int32_t n_reads, int N,
    const float2* __restrict__ phase32, const float* __restrict__ delta, void* __restrict__ emb,
    float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                    __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (r >= n_reads) return;
  const int64_t start = off[r];
  const int64_t len = off[r + 1] - start;
  float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
  if (len >= N) direct_sum_learned32(seq + start, N, delta + start * 32, phase32, lane, a0, a1);
  emit_head<PREC>(a0, a1, N, r, lane, emb, scale);
}

// ---- token encodings (§2.1 s-mers, §2.6 compact versions) ----------------------
// The window encoder above with tokens in place of letters (lane layout of
// rm_tokens.h): the re-anchor sums the tokens at locations 0..N-s in FP64; a
// slide removes the token at the old start (location 0, -omega^-f after the
// rotation) and adds the token ending at the new window's last letter
// (location N-s, +omega^(f (N-s)), held in step32).
template <int PREC>
__global__ __launch_bounds__(256) void encode_reference_tokens_kernel(
    const uint8_t* __restrict__ ref, int64_t W, int N, int stride, int s, int m, int n_class,
    int64_t seg_len, int64_t n_seg, const double2* __restrict__ phase64,
    const float4* __restrict__ step32, const uint8_t* __restrict__ table, void* __restrict__ emb,
    float* __restrict__ scale, float* __restrict__ norm2) {
  const int lane = threadIdx.x & 63;
  const int64_t seg = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                    __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (seg >= n_seg) return;
  const int k = 2 * lane / n_class, c0 = 2 * lane - k * n_class;
  const int T = N - s + 1;  // tokens per window
  const int64_t j0 = seg * seg_len;
  const int64_t j1 = min(W, j0 + seg_len);

  double2 a0, a1;
  direct_sum_tokens(ref + j0 * stride, T, s, table, phase64, m, k, c0, lane, a0, a1);
  float2 v0 = make_float2((float)a0.x, (float)a0.y);
  float2 v1 = make_float2((float)a1.x, (float)a1.y);
  SideBuf side{j0, 0, 0.f, 0.f, PREC == RM_FP8_E4M3 ? scale + W : nullptr, 0.f};
  emit_window<PREC>(j0, lane, N, v0, v1, emb, side, scale, norm2);

  const float4 st = step32[k];
  const float2 rot = make_float2(st.x, st.y);  // omega^-f
  const float2 inc = make_float2(st.z, st.w);  // omega^(f (N-s))

  // slide t moves the start from s0+t to s0+t+1: the outgoing token starts at
  // s0+t, the incoming one at s0+t+1+N-s (its last letter is s0+t+N)
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
      // classes relative to this lane's c0: 0 or 1 is one of its components
      const int o = __builtin_amdgcn_readlane(out_c, i) - c0;
      const int n = __builtin_amdgcn_readlane(in_c, i) - c0;
      slide(v0, v1, rot, (unsigned)o < 2u ? o : 255, (unsigned)n < 2u ? n : 255, 0, rot, inc);
      if (--until_emit == 0) {
        until_emit = stride;
        ++j;
        emit_window<PREC>(j, lane, N, v0, v1, emb, side, scale, norm2);
      }
    }
    out_c = out_next;
    in_c = in_next;
  }
  side_finish(side, lane, norm2, scale);
}

// The read-head encoder with tokens: FP32 direct sum over the head's tokens.
template <int PREC>
__global__ __launch_bounds__(256) void encode_reads_tokens_kernel(
    const uint8_t* __restrict__ seq, const int64_t* __restrict__ off, int32_t n_reads, int N,
    int s, int m, int n_class, const float2* __restrict__ phase32,
    const uint8_t* __restrict__ table, void* __restrict__ emb, float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                    __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (r >= n_reads) return;
  const int k = 2 * lane / n_class, c0 = 2 * lane - k * n_class;
  const int64_t start = off[r];
  const int64_t len = off[r + 1] - start;
  float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
  if (len >= N) direct_sum_tokens(seq + start, N - s + 1, s, table, phase32, m, k, c0, lane, a0, a1);
  emit_head<PREC>(a0, a1, N, r, lane, emb, scale);
}

}  // namespace

hipError_t launch_encode_reference(const uint8_t* ref, int64_t W, const rm_params& p,
                                   const double* phase64, const float* step32, void* emb,
                                   float* scale, float* norm2, hipStream_t s) {
  const int waves = 4;
  auto* ph = reinterpret_cast<const double2*>(phase64);
  auto* st = reinterpret_cast<const float4*>(step32);
  const bool blockwise = p.stride > 1 && p.stride <= kBlockMax && p.stride <= p.window_len;
  const int unit_z = p.schedule == RM_SCHED_DEFAULT ? 1 : 0;
  if (blockwise && unit_z && p.stride >= kMfmaStrideMin) {
    const int ns = p.stride <= 16 ? 1 : p.stride <= 32 ? 2 : 4;
    auto pick = [&](auto k1, auto k2, auto k4) { return ns == 1 ? k1 : ns == 2 ? k2 : k4; };
    decltype(&encode_reference_mfma_kernel<RM_FP32, false, 1>) mk;
    if (p.precision == RM_FP16)
      mk = p.reduced ? pick(encode_reference_mfma_kernel<RM_FP16, true, 1>,
                            encode_reference_mfma_kernel<RM_FP16, true, 2>,
                            encode_reference_mfma_kernel<RM_FP16, true, 4>)
                     : pick(encode_reference_mfma_kernel<RM_FP16, false, 1>,
                            encode_reference_mfma_kernel<RM_FP16, false, 2>,
                            encode_reference_mfma_kernel<RM_FP16, false, 4>);
    else if (p.precision == RM_FP8_E4M3)
      mk = p.reduced ? pick(encode_reference_mfma_kernel<RM_FP8_E4M3, true, 1>,
                            encode_reference_mfma_kernel<RM_FP8_E4M3, true, 2>,
                            encode_reference_mfma_kernel<RM_FP8_E4M3, true, 4>)
                     : pick(encode_reference_mfma_kernel<RM_FP8_E4M3, false, 1>,
                            encode_reference_mfma_kernel<RM_FP8_E4M3, false, 2>,
                            encode_reference_mfma_kernel<RM_FP8_E4M3, false, 4>);
    else
      mk = p.reduced ? pick(encode_reference_mfma_kernel<RM_FP32, true, 1>,
                            encode_reference_mfma_kernel<RM_FP32, true, 2>,
                            encode_reference_mfma_kernel<RM_FP32, true, 4>)
                     : pick(encode_reference_mfma_kernel<RM_FP32, false, 1>,
                            encode_reference_mfma_kernel<RM_FP32, false, 2>,
                            encode_reference_mfma_kernel<RM_FP32, false, 4>);
    // Segments: the caller's value, or as few rounds of resident blocks as
    // keep a segment within 2048 starts, each round full (a window is cheap
    // here next to the segment's N-letter FP64 re-anchor, and a block left
    // over for a round of its own costs a whole segment's time), at least 256
    // starts.
    int64_t seg = p.reanchor;
    if (seg <= 0) {
      // resident blocks per CU of this instantiation, queried once (the
      // launch may be captured into a graph)
      static std::mutex mu;
      static std::unordered_map<const void*, int> per_cu_of;
      int per_cu = 0, dev = 0, cus = 0;
      {
        std::lock_guard<std::mutex> lock(mu);
        auto it = per_cu_of.find(reinterpret_cast<const void*>(mk));
        if (it != per_cu_of.end()) {
          per_cu = it->second;
        } else {
          if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mk, 64 * waves, 0) != hipSuccess ||
              per_cu < 1)
            per_cu = 1;
          per_cu_of[reinterpret_cast<const void*>(mk)] = per_cu;
        }
      }
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          cus < 1)
        cus = 256;
      const int64_t resident = (int64_t)per_cu * cus * waves;  // wavefronts in one round
      int64_t rounds = 1;
      seg = (W + resident - 1) / resident;
      while (seg > 2048) {
        ++rounds;
        seg = (W + rounds * resident - 1) / (rounds * resident);
      }
      if (seg < 256) seg = 256;
    }
    const int64_t n_seg = (W + seg - 1) / seg;
    const int64_t blocks = (n_seg + waves - 1) / waves;
    hipLaunchKernelGGL(mk, dim3((unsigned)blocks), dim3(64 * waves), 0, s, ref, W, p.window_len,
                       p.stride, seg, n_seg, ph, emb, scale, norm2);
    return hipGetLastError();
  }
  // Segment = window starts between two FP64 re-anchors: the caller's value,
  // or W / 4096 clamped to 256 .. 512 (at least about 4096 wavefronts where W
  // allows; longer segments leave a ragged last round of blocks, shorter ones
  // repeat the N-letter FP64 re-anchor more often).
  int64_t seg = p.reanchor;
  if (seg <= 0) {
    seg = W / 4096;
    if (seg < 256) seg = 256;
    if (seg > 512) seg = 512;
  }
  const int64_t n_seg = (W + seg - 1) / seg;
  const int64_t blocks = (n_seg + waves - 1) / waves;
  auto kern = p.reduced ? encode_reference_kernel<RM_FP32, true> : encode_reference_kernel<RM_FP32, false>;
  if (p.precision == RM_FP16)
    kern = p.reduced ? encode_reference_kernel<RM_FP16, true> : encode_reference_kernel<RM_FP16, false>;
  else if (p.precision == RM_FP8_E4M3)
    kern = p.reduced ? encode_reference_kernel<RM_FP8_E4M3, true>
                     : encode_reference_kernel<RM_FP8_E4M3, false>;
  // block rolling (stride 2 .. kBlockMax, at most N) takes the table of
  // omega^(f q), q < stride, in LDS; integer factors make omega^(f N) = 1
  const size_t lds = blockwise ? (size_t)p.stride * kM * sizeof(float2) : 0;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), lds, s, ref, W, p.window_len,
                     p.stride, unit_z, seg, n_seg, ph, st, emb, scale, norm2);
  return hipGetLastError();
}

hipError_t launch_encode_reads(const rm_params& p, const float* phase32, const uint8_t* seq,
                               const int64_t* off, int32_t n_reads, void* emb, float* scale,
                               hipStream_t s) {
  const int waves = 4;
  int64_t blocks = ((int64_t)n_reads + waves - 1) / waves;
  auto* ph = reinterpret_cast<const float2*>(phase32);
  auto kern = p.reduced ? encode_reads_kernel<RM_FP32, true> : encode_reads_kernel<RM_FP32, false>;
  if (p.precision == RM_FP16)
    kern = p.reduced ? encode_reads_kernel<RM_FP16, true> : encode_reads_kernel<RM_FP16, false>;
  else if (p.precision == RM_FP8_E4M3)
    kern = p.reduced ? encode_reads_kernel<RM_FP8_E4M3, true> : encode_reads_kernel<RM_FP8_E4M3, false>;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), 0, s, seq, off, n_reads,
                     p.window_len, ph, emb, scale);
  return hipGetLastError();
}

}  // namespace rm

namespace rm {

hipError_t launch_encode_reference_learned(const uint8_t* ref, int64_t W, const rm_params& p,
                                           const double* phase64, const float* phase32,
                                           const float* step32, const float* delta, void* emb,
                                           float* scale, float* norm2, hipStream_t s) {
  int64_t seg = p.reanchor;
  if (seg <= 0) {
    seg = (W + 8191) / 8192;
    if (seg < 256) seg = 256;
    if (seg > 4096) seg = 4096;
  }
  int64_t n_seg = (W + seg - 1) / seg;
  const int waves = 4;
  int64_t blocks = (n_seg + waves - 1) / waves;
  auto* ph = reinterpret_cast<const double2*>(phase64);
  auto* p32 = reinterpret_cast<const float2*>(phase32);
  auto* st = reinterpret_cast<const float4*>(step32);
  const dim3 grid((unsigned)blocks), block(64 * waves);
  switch (p.precision) {
    case RM_FP32:
      hipLaunchKernelGGL(encode_reference_learned_kernel<RM_FP32>, grid, block, 0, s, ref, W,
                         p.window_len, p.stride, seg, n_seg, ph, p32, st, delta, emb, scale, norm2);
      break;
    case RM_FP16:
      hipLaunchKernelGGL(encode_reference_learned_kernel<RM_FP16>, grid, block, 0, s, ref, W,
                         p.window_len, p.stride, seg, n_seg, ph, p32, st, delta, emb, scale, norm2);
      break;
    default:
      hipLaunchKernelGGL(encode_reference_learned_kernel<RM_FP8_E4M3>, grid, block, 0, s, ref, W,
                         p.window_len, p.stride, seg, n_seg, ph, p32, st, delta, emb, scale, norm2);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_encode_reads_learned(const rm_params& p, const float* phase32,
                                       const uint8_t* seq, const int64_t* off, int32_t n_reads,
                                       const float* delta, void* emb, float* scale,
                                       hipStream_t s) {
  const int waves = 4;
  const dim3 grid((unsigned)(((int64_t)n_reads + waves - 1) / waves)), block(64 * waves);
  auto* ph = reinterpret_cast<const float2*>(phase32);
  switch (p.precision) {
    case RM_FP32:
      hipLaunchKernelGGL(encode_reads_learned_kernel<RM_FP32>, grid, block, 0, s, seq, off,
                         n_reads, p.window_len, ph, delta, emb, scale);
      break;
    case RM_FP16:
      hipLaunchKernelGGL(encode_reads_learned_kernel<RM_FP16>, grid, block, 0, s, seq, off,
                         n_reads, p.window_len, ph, delta, emb, scale);
      break;
    default:
      hipLaunchKernelGGL(encode_reads_learned_kernel<RM_FP8_E4M3>, grid, block, 0, s, seq, off,
                         n_reads, p.window_len, ph, delta, emb, scale);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_encode_reference_tokens(const uint8_t* ref, int64_t W, const rm_params& p,
                                          const double* phase64, const float* step32,
                                          const uint8_t* table, void* emb, float* scale,
                                          float* norm2, hipStream_t st) {
  // segments as for the letter encoding
  int64_t seg = p.reanchor;
  if (seg <= 0) {
    seg = (W + 8191) / 8192;
    if (seg < 256) seg = 256;
    if (seg > 4096) seg = 4096;
  }
  const int64_t n_seg = (W + seg - 1) / seg;
  const int waves = 4;
  const int64_t blocks = (n_seg + waves - 1) / waves;
  const int s = p.mer_len > 1 ? p.mer_len : 1;
  const int C = 128 / p.n_freq;
  auto* ph = reinterpret_cast<const double2*>(phase64);
  auto* sp = reinterpret_cast<const float4*>(step32);
  auto kern = p.precision == RM_FP32   ? encode_reference_tokens_kernel<RM_FP32>
              : p.precision == RM_FP16 ? encode_reference_tokens_kernel<RM_FP16>
                                       : encode_reference_tokens_kernel<RM_FP8_E4M3>;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), 0, st, ref, W, p.window_len,
                     p.stride, s, p.n_freq, C, seg, n_seg, ph, sp, table, emb, scale, norm2);
  return hipGetLastError();
}

hipError_t launch_encode_reads_tokens(const rm_params& p, const float* phase32,
                                      const uint8_t* table, const uint8_t* seq, const int64_t* off,
                                      int32_t n_reads, void* emb, float* scale, hipStream_t st) {
  const int waves = 4;
  const int64_t blocks = ((int64_t)n_reads + waves - 1) / waves;
  const int s = p.mer_len > 1 ? p.mer_len : 1;
  const int C = 128 / p.n_freq;
  auto* ph = reinterpret_cast<const float2*>(phase32);
  auto kern = p.precision == RM_FP32   ? encode_reads_tokens_kernel<RM_FP32>
              : p.precision == RM_FP16 ? encode_reads_tokens_kernel<RM_FP16>
                                       : encode_reads_tokens_kernel<RM_FP8_E4M3>;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), 0, st, seq, off, n_reads,
                     p.window_len, s, p.n_freq, C, ph, table, emb, scale);
  return hipGetLastError();
}

}  // namespace rm
