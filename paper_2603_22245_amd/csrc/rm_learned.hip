// Learned angle offsets: forward encoding, pair fidelity, ranking loss,
// backward pass and Adam update, all FP32.
//
// The learned encoding (the paper has none; it notes that token definitions,
// initial encodings or rotations could be altered, §2.10): 9-mer tokens at
// locations p = 0..n-9 (s-mer locations, §2.1); the middle letter L picks the
// component; the 8 flanking letters, one-hot (32 inputs), go through
// o = W2 relu(W1 x + b1) + b2 (128 outputs = 4 letters x 32 factors); the
// token adds exp(i (theta_k p + o[L*32+k])) to component (k, L), theta_k =
// 2 pi (k+1) / N (§2.2) with N the nominal length.  Fidelity (§2.4) of pairs,
// and a pairwise logistic ranking loss on Levenshtein labels.
//
// Parameters: W1 [64][32], b1 [64], W2 [128][64], b2 [128], row-major, FP32.
// One wavefront per string; lanes play two roles per token: lane j = hidden
// unit j for the first layer, lane l = (factor l/2, letters 2(l&1), 2(l&1)+1)
// for the offsets and the encoding, as in the encoders.
#include "rm_internal.h"

namespace rm {

namespace {

constexpr int kIn = 32, kHid = 64, kOut = 128;
constexpr int kW1 = 0, kB1 = kHid * kIn, kW2 = kB1 + kHid, kB2 = kW2 + kOut * kHid;
constexpr int kParams = kB2 + kOut;  // 10,432
constexpr int kW2Stride = kHid + 4;  // padded LDS row of W2: conflict-free float4 reads
constexpr int kMaxLen = 256;         // letters of a string kept in LDS
constexpr int kWaves = 4;
constexpr float kTau = 0.05f;

static_assert(kParams == RM_LEARNED_PARAMS, "parameter count");

struct Weights {  // LDS copy of the network
  float w1t[kIn * kHid];         // W1 transposed: [input][hidden]
  float b1[kHid];
  float w2[kOut * kW2Stride];    // W2 rows padded
  float b2[kOut];
};

__device__ void load_weights(Weights& w, const float* __restrict__ p) {
  for (int i = threadIdx.x; i < kHid * kIn; i += blockDim.x) {
    int j = i / kIn, c = i % kIn;
    w.w1t[c * kHid + j] = p[kW1 + i];
  }
  for (int i = threadIdx.x; i < kHid; i += blockDim.x) w.b1[i] = p[kB1 + i];
  for (int i = threadIdx.x; i < kOut * kHid; i += blockDim.x) {
    int r = i / kHid, j = i % kHid;
    w.w2[r * kW2Stride + j] = p[kW2 + i];
  }
  for (int i = threadIdx.x; i < kOut; i += blockDim.x) w.b2[i] = p[kB2 + i];
}

// Per-token forward pieces for the current wavefront.
struct Token {
  int mid;      // middle letter (>= 4: no token)
  float pre;    // lane j: first-layer pre-activation of unit j
  float delta;  // lane (k, hh): offset for factor k of the middle letter
  float s, c;   // lane (k, hh): sin and cos of the phase
};

// Forward of token p of the string held in `let` (LDS letters).  hbuf: this
// wavefront's 64-float LDS scratch.
__device__ __forceinline__ Token token_forward(const Weights& w, const uint8_t* let, int p, int N,
                                               float* hbuf, int lane) {
  Token t;
  t.mid = let[p + 4];
  // first layer: lane j sums the W1 columns selected by the 8 flanking letters
  float pre = w.b1[lane];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    int f = let[p + (i < 4 ? i : i + 1)];
    if (f < 4) pre += w.w1t[(4 * i + f) * kHid + lane];
  }
  t.pre = pre;
  hbuf[lane] = fmaxf(pre, 0.f);
  __builtin_amdgcn_wave_barrier();
  const int k = lane >> 1, hh = lane & 1;
  float d = 0.f;
  if (t.mid < 4) {
    const float* wrow = &w.w2[(t.mid * 32 + k) * kW2Stride + 32 * hh];
    const float* hv = &hbuf[32 * hh];
#pragma unroll
    for (int i = 0; i < 32; i += 4) {
      float4 a = *reinterpret_cast<const float4*>(wrow + i);
      float4 b = *reinterpret_cast<const float4*>(hv + i);
      d += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
    }
  }
  d += __shfl_xor(d, 1, 64);
  if (t.mid < 4) d += w.b2[t.mid * 32 + k];
  t.delta = d;
  // phase theta_k p + delta with the integer part reduced exactly mod N
  int r = (int)(((int64_t)(k + 1) * p) % N);
  float ang = 6.283185307179586f * (float)r / (float)N + d;
  sincosf(ang, &t.s, &t.c);
  __builtin_amdgcn_wave_barrier();  // hbuf is reused by the next token
  return t;
}

// Strings come from one set (string s = seq[off[s] .. off[s+1])) or, for
// pairs, from two: string s is string s/2 of set a (s even) or of set b (s odd).
struct Strings {
  const uint8_t* a;
  const int64_t* aoff;
  const uint8_t* b;  // null: one set
  const int64_t* boff;
};

__device__ __forceinline__ int load_string(uint8_t* let, const Strings& st, int64_t sidx,
                                           int lane) {
  const uint8_t* seq = st.a;
  const int64_t* off = st.aoff;
  if (st.b != nullptr) {
    if (sidx & 1) {
      seq = st.b;
      off = st.boff;
    }
    sidx >>= 1;
  }
  const int64_t a = off[sidx];
  int n = (int)min<int64_t>(off[sidx + 1] - a, kMaxLen);
  for (int i = lane; i < n; i += 64) let[i] = seq[a + i];
  __builtin_amdgcn_wave_barrier();
  return n;
}

// Learned encodings c of n_strings strings: out[s][256] (k*4+letter, re/im).
__global__ __launch_bounds__(64 * kWaves) void learned_encode_kernel(
    const float* __restrict__ params, Strings st, int32_t n_strings, int N,
    float* __restrict__ out) {
  __shared__ Weights w;
  __shared__ uint8_t letters[kWaves][kMaxLen];
  __shared__ float hbuf[kWaves][kHid];
  load_weights(w, params);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t s = (int64_t)blockIdx.x * kWaves + wave;
  if (s >= n_strings) return;
  const int n = load_string(letters[wave], st, s, lane);
  const int hh = lane & 1;
  float2 c0 = make_float2(0.f, 0.f), c1 = make_float2(0.f, 0.f);
  for (int p = 0; p + 9 <= n; ++p) {
    Token t = token_forward(w, letters[wave], p, N, hbuf[wave], lane);
    if (t.mid == 2 * hh) { c0.x += t.c; c0.y += t.s; }
    if (t.mid == 2 * hh + 1) { c1.x += t.c; c1.y += t.s; }
  }
  reinterpret_cast<float4*>(out + s * 256)[lane] = make_float4(c0.x, c0.y, c1.x, c1.y);
}

// The plain encoding (§2.2, s = 1) of whole strings in FP32, for comparison:
// letter p adds exp(i theta_k p) to component (k, letter), p = 0..n-1.
__global__ __launch_bounds__(256) void plain_encode_kernel(const uint8_t* __restrict__ seq,
                                                           const int64_t* __restrict__ off,
                                                           int32_t n_strings, int N,
                                                           float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= n_strings) return;
  const int64_t a = off[s], n = off[s + 1] - a;
  const int k = lane >> 1, hh = lane & 1;
  const int64_t fk = k + 1;
  float2 c0 = make_float2(0.f, 0.f), c1 = make_float2(0.f, 0.f);
  for (int64_t p = 0; p < n; ++p) {
    const int L = seq[a + p];
    if ((L >> 1) != hh) continue;
    float sn, cs;
    sincospif(2.f * (float)((fk * p) % N) / (float)N, &sn, &cs);
    if (L & 1) { c1.x += cs; c1.y += sn; } else { c0.x += cs; c0.y += sn; }
  }
  reinterpret_cast<float4*>(out + s * 256)[lane] = make_float4(c0.x, c0.y, c1.x, c1.y);
}

// F of pairs of encodings ca[i * stride], cb[i * stride]; one wavefront per pair.
__global__ __launch_bounds__(256) void pair_fidelity_kernel(const float* __restrict__ ca,
                                                            const float* __restrict__ cb,
                                                            int64_t stride, int32_t n_pairs,
                                                            float* __restrict__ F) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n_pairs) return;
  float4 a = reinterpret_cast<const float4*>(ca + i * stride)[lane];
  float4 b = reinterpret_cast<const float4*>(cb + i * stride)[lane];
  // z = sum conj(a) b
  float zr = wave_sum(a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w);
  float zi = wave_sum(a.x * b.y - a.y * b.x + a.z * b.w - a.w * b.z);
  float A = wave_sum(a.x * a.x + a.y * a.y + a.z * a.z + a.w * a.w);
  float B = wave_sum(b.x * b.x + b.y * b.y + b.z * b.z + b.w * b.w);
  if (lane == 0) F[i] = (A > 0.f && B > 0.f) ? (zr * zr + zi * zi) / (A * B) : 0.f;
}

// Ranking loss, pass 1: thread (i, part) sums over its eighth of the j's the
// terms of pair (i, j): loss softplus(z) and count for d_i < d_j (z = -(F_i -
// F_j) / tau), and the unscaled dLoss/dF_i contributions -sigma(z_ij) (d_i <
// d_j) and +sigma(z_ji) (d_j < d_i).  The eight parts are summed in a fixed
// order; per-i results go to g, lossv, cntv.
constexpr int kRankI = 32, kRankParts = 8;

__global__ __launch_bounds__(kRankI * kRankParts) void ranking_pairs_kernel(
    const float* __restrict__ F, const int32_t* __restrict__ ld, int32_t n,
    float* __restrict__ g_out, float* __restrict__ loss_out, int32_t* __restrict__ cnt_out) {
  __shared__ float sF[RM_LEARNED_MAX_PAIRS];
  __shared__ int sL[RM_LEARNED_MAX_PAIRS];
  __shared__ float rg[kRankParts][kRankI], rl[kRankParts][kRankI];
  __shared__ int rc[kRankParts][kRankI];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    sF[i] = F[i];
    sL[i] = ld[i];
  }
  __syncthreads();
  const int ti = threadIdx.x % kRankI, part = threadIdx.x / kRankI;
  const int i = blockIdx.x * kRankI + ti;
  float g = 0.f, l = 0.f;
  int cnt = 0;
  if (i < n) {
    const float Fi = sF[i];
    const int Li = sL[i];
    const int per = (n + kRankParts - 1) / kRankParts;
    const int j0 = part * per, j1 = min(n, j0 + per);
    for (int j = j0; j < j1; ++j) {
      const int Lj = sL[j];
      if (Li < Lj) {  // want F_i > F_j
        const float z = -(Fi - sF[j]) / kTau;
        l += z > 20.f ? z : log1pf(expf(z));
        ++cnt;
        g -= 1.f / (1.f + expf(-z));
      } else if (Lj < Li) {
        const float z = -(sF[j] - Fi) / kTau;
        g += 1.f / (1.f + expf(-z));
      }
    }
  }
  rg[part][ti] = g;
  rl[part][ti] = l;
  rc[part][ti] = cnt;
  __syncthreads();
  if (part == 0 && i < n) {
    for (int q = 1; q < kRankParts; ++q) {
      g += rg[q][ti];
      l += rl[q][ti];
      cnt += rc[q][ti];
    }
    g_out[i] = g;
    loss_out[i] = l;
    cnt_out[i] = cnt;
  }
}

// Ranking loss, pass 2 (one block): the loss is the sum of the terms over the
// number of ordered pairs; dLoss/dF_i = g_i / (tau * count).
__global__ __launch_bounds__(1024) void ranking_finalize_kernel(
    float* __restrict__ g, const float* __restrict__ lossv, const int32_t* __restrict__ cntv,
    int32_t n, float* __restrict__ loss) {
  __shared__ float sl[1024];
  __shared__ int sc[1024];
  const int t = threadIdx.x;
  sl[t] = t < n ? lossv[t] : 0.f;
  sc[t] = t < n ? cntv[t] : 0;
  __syncthreads();
  for (int d = 512; d > 0; d >>= 1) {  // fixed-order tree
    if (t < d) {
      sl[t] += sl[t + d];
      sc[t] += sc[t + d];
    }
    __syncthreads();
  }
  const float C = (float)sc[0];
  if (t == 0) *loss = sc[0] > 0 ? sl[0] / C : 0.f;
  const float scale = sc[0] > 0 ? 1.f / (kTau * C) : 0.f;
  if (t < n) g[t] *= scale;
}

// Backward: per string, dLoss/dc = dLoss/dF * dF/dc, then through the tokens
// and the network.  Deterministic: every lane accumulates its own share of the
// gradient (lane (k, hh): dW2 rows L*32+k, columns 32hh..32hh+31, and db2 for
// hh = 0, in registers; lane j: dW1 column j in the wavefront's LDS slice and
// db1 in a register), the wavefronts of a block are summed in a fixed order
// through LDS, and the per-block partials in block order by the reduction
// kernel.
// Strings are taken in a grid-stride loop.
constexpr int kRedW1 = 0, kRedB1 = kHid * 33, kRedW2 = kRedB1 + kHid, kRedB2 = kRedW2 + kOut * 65;
constexpr int kRedSize = kRedB2 + kOut;  // padded rows: conflict-free LDS writes
static_assert(kRedSize * sizeof(float) <= sizeof(Weights), "reduction buffer reuses the weights");

__global__ __launch_bounds__(64 * kWaves, 2) void learned_backward_kernel(
    const float* __restrict__ params, Strings st, int32_t n_pairs, int N,
    const float* __restrict__ c, const float* __restrict__ dF, float* __restrict__ partial) {
  __shared__ union {
    Weights w;
    float red[kRedSize];
  } u;
  __shared__ uint8_t letters[kWaves][kMaxLen];
  __shared__ float hbuf[kWaves][kHid];
  __shared__ float dbuf[kWaves][32];         // dLoss/d delta of the current token
  __shared__ float gw1[kWaves][kIn * kHid];  // dW1 transposed, [input][hidden]
  load_weights(u.w, params);
  for (int i = threadIdx.x; i < kWaves * kIn * kHid; i += blockDim.x) (&gw1[0][0])[i] = 0.f;
  __syncthreads();
  const Weights& w = u.w;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = lane >> 1, hh = lane & 1;
  float aw2[4][32], ab2[4], ab1 = 0.f;
#pragma unroll
  for (int L = 0; L < 4; ++L) {
    ab2[L] = 0.f;
#pragma unroll
    for (int i = 0; i < 32; ++i) aw2[L][i] = 0.f;
  }

  for (int64_t s = (int64_t)blockIdx.x * kWaves + wave; s < 2 * (int64_t)n_pairs;
       s += (int64_t)gridDim.x * kWaves) {
    const int64_t pr = s >> 1;
    const bool is_b = s & 1;
    // dF/dc for this side: F = |z|^2/(AB), z = <a|b>
    float4 a = reinterpret_cast<const float4*>(c + (2 * pr) * 256)[lane];
    float4 b = reinterpret_cast<const float4*>(c + (2 * pr + 1) * 256)[lane];
    float zr = wave_sum(a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w);
    float zi = wave_sum(a.x * b.y - a.y * b.x + a.z * b.w - a.w * b.z);
    float A = wave_sum(a.x * a.x + a.y * a.y + a.z * a.z + a.w * a.w);
    float B = wave_sum(b.x * b.x + b.y * b.y + b.z * b.z + b.w * b.w);
    float g0r = 0.f, g0i = 0.f, g1r = 0.f, g1i = 0.f;
    if (A > 0.f && B > 0.f) {
      const float F = (zr * zr + zi * zi) / (A * B), d = dF[pr], AB = A * B;
      if (!is_b) {  // G_a = 2 conj(z) b / (AB) - 2 F a / A
        g0r = d * (2.f * (zr * b.x + zi * b.y) / AB - 2.f * F * a.x / A);
        g0i = d * (2.f * (zr * b.y - zi * b.x) / AB - 2.f * F * a.y / A);
        g1r = d * (2.f * (zr * b.z + zi * b.w) / AB - 2.f * F * a.z / A);
        g1i = d * (2.f * (zr * b.w - zi * b.z) / AB - 2.f * F * a.w / A);
      } else {      // G_b = 2 z a / (AB) - 2 F b / B
        g0r = d * (2.f * (zr * a.x - zi * a.y) / AB - 2.f * F * b.x / B);
        g0i = d * (2.f * (zr * a.y + zi * a.x) / AB - 2.f * F * b.y / B);
        g1r = d * (2.f * (zr * a.z - zi * a.w) / AB - 2.f * F * b.z / B);
        g1i = d * (2.f * (zr * a.w + zi * a.z) / AB - 2.f * F * b.w / B);
      }
    }
    // lane (k, hh) holds G of components (k, 2hh) and (k, 2hh+1)
    const int n = load_string(letters[wave], st, s, lane);
    for (int p = 0; p + 9 <= n; ++p) {
      Token t = token_forward(w, letters[wave], p, N, hbuf[wave], lane);
      const int Lm = __builtin_amdgcn_readfirstlane(t.mid);
      if (Lm >= 4) continue;  // uniform: no token here
      // d delta_k = Re(conj(G) i e^{i phi}) = -Gr sin + Gi cos, G of component
      // (k, Lm) from lane (k, Lm / 2)
      const int src = 2 * k + (Lm >> 1);
      const float r0 = __shfl(g0r, src, 64), i0 = __shfl(g0i, src, 64);
      const float r1 = __shfl(g1r, src, 64), i1 = __shfl(g1i, src, 64);
      const float Gr = (Lm & 1) ? r1 : r0, Gi = (Lm & 1) ? i1 : i0;
      const float dd = -Gr * t.s + Gi * t.c;
      if (hh == 0) dbuf[wave][k] = dd;
      // dW2[L*32+k][32hh+i] += dd * h_(32hh+i); h of this token is still in hbuf
      const float* hv = &hbuf[wave][32 * hh];
      const float db = hh == 0 ? dd : 0.f;
      switch (Lm) {
#define RM_ACC_W2(L)                                                      \
  case L:                                                                 \
    _Pragma("unroll") for (int i = 0; i < 32; i += 4) {                   \
      const float4 v = *reinterpret_cast<const float4*>(hv + i);          \
      aw2[L][i] += dd * v.x;                                              \
      aw2[L][i + 1] += dd * v.y;                                          \
      aw2[L][i + 2] += dd * v.z;                                          \
      aw2[L][i + 3] += dd * v.w;                                          \
    }                                                                     \
    ab2[L] += db;                                                         \
    break;
        RM_ACC_W2(0)
        RM_ACC_W2(1)
        RM_ACC_W2(2)
        RM_ACC_W2(3)
#undef RM_ACC_W2
      }
      __builtin_amdgcn_wave_barrier();
      // dh_j = sum_k W2[L*32+k][j] d delta_k  (lane j)
      float dh = 0.f;
      const float* wcol = &w.w2[(Lm * 32) * kW2Stride + lane];
#pragma unroll 8
      for (int kk = 0; kk < 32; ++kk) dh += wcol[kk * kW2Stride] * dbuf[wave][kk];
      const float dpre = t.pre > 0.f ? dh : 0.f;
      ab1 += dpre;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int f = letters[wave][p + (i < 4 ? i : i + 1)];
        if (f < 4) gw1[wave][(4 * i + f) * kHid + lane] += dpre;
      }
      __builtin_amdgcn_wave_barrier();  // dbuf and hbuf are rewritten by the next token
    }
  }
  __syncthreads();  // every wavefront is done with the weights: reuse them
  float* red = u.red;
  for (int wv = 0; wv < kWaves; ++wv) {
    if (wave == wv) {
      const bool first = wv == 0;
#pragma unroll
      for (int L = 0; L < 4; ++L) {
        float* row = &red[kRedW2 + (L * 32 + k) * 65 + 32 * hh];
#pragma unroll
        for (int i = 0; i < 32; ++i) row[i] = (first ? 0.f : row[i]) + aw2[L][i];
        if (hh == 0) {
          float& b2 = red[kRedB2 + L * 32 + k];
          b2 = (first ? 0.f : b2) + ab2[L];
        }
      }
      float* col = &red[kRedW1 + lane * 33];
#pragma unroll 8
      for (int i = 0; i < kIn; ++i) col[i] = (first ? 0.f : col[i]) + gw1[wave][i * kHid + lane];
      red[kRedB1 + lane] = (first ? 0.f : red[kRedB1 + lane]) + ab1;
    }
    __syncthreads();
  }
  // partial gradient of this block, parameter order
  float* out = partial + (int64_t)blockIdx.x * kParams;
  for (int i = threadIdx.x; i < kHid * kIn; i += blockDim.x)
    out[kW1 + i] = red[kRedW1 + (i / kIn) * 33 + (i % kIn)];
  for (int i = threadIdx.x; i < kHid; i += blockDim.x) out[kB1 + i] = red[kRedB1 + i];
  for (int i = threadIdx.x; i < kOut * kHid; i += blockDim.x)
    out[kW2 + i] = red[kRedW2 + (i / kHid) * 65 + (i % kHid)];
  for (int i = threadIdx.x; i < kOut; i += blockDim.x) out[kB2 + i] = red[kRedB2 + i];
}

// Sum of the per-block partial gradients (block: 64 parameters x 16 subsets
// of the partials, summed in a fixed order); then either the gradient is
// written (grad != nullptr) or an Adam step is applied to state = [params | m
// | v | t].
constexpr int kRedParams = 64, kRedParts = 16;

__global__ __launch_bounds__(kRedParams * kRedParts) void reduce_adam_kernel(
    const float* __restrict__ partial, int n_blocks, float* __restrict__ grad,
    float* __restrict__ state, float lr) {
  __shared__ float red[kRedParts][kRedParams];
  const int tp = threadIdx.x % kRedParams, q = threadIdx.x / kRedParams;
  const int i = blockIdx.x * kRedParams + tp;
  float g = 0.f;
  if (i < kParams) {
    int b = q;
    for (; b + 3 * kRedParts < n_blocks; b += 4 * kRedParts) {  // 4 loads in flight
      const float v0 = partial[(int64_t)b * kParams + i];
      const float v1 = partial[(int64_t)(b + kRedParts) * kParams + i];
      const float v2 = partial[(int64_t)(b + 2 * kRedParts) * kParams + i];
      const float v3 = partial[(int64_t)(b + 3 * kRedParts) * kParams + i];
      g += v0;
      g += v1;
      g += v2;
      g += v3;
    }
    for (; b < n_blocks; b += kRedParts) g += partial[(int64_t)b * kParams + i];
  }
  red[q][tp] = g;
  __syncthreads();
  if (q != 0 || i >= kParams) return;
  for (int r = 1; r < kRedParts; ++r) g += red[r][tp];
  if (grad != nullptr) {
    grad[i] = g;
    return;
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float t = state[3 * kParams] + 1.f;  // the step count is advanced by a separate kernel
  float m = b1 * state[kParams + i] + (1.f - b1) * g;
  float v = b2 * state[2 * kParams + i] + (1.f - b2) * g * g;
  state[kParams + i] = m;
  state[2 * kParams + i] = v;
  float mh = m / (1.f - powf(b1, t));
  float vh = v / (1.f - powf(b2, t));
  state[i] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void advance_step_kernel(float* __restrict__ state) {
  if (threadIdx.x == 0 && blockIdx.x == 0) state[3 * kParams] += 1.f;
}

}  // namespace

size_t learned_workspace_bytes(int32_t n_pairs) {
  int64_t strings = 2 * (int64_t)n_pairs;
  int64_t blocks = (strings + kWaves - 1) / kWaves;
  size_t bytes = 0;
  bytes += (size_t)strings * 256 * sizeof(float);  // encodings
  bytes += (size_t)n_pairs * sizeof(float) * 4;    // F, dF, per-i loss, per-i count
  bytes += 256;                                    // loss
  bytes += (size_t)blocks * kParams * sizeof(float);
  return (bytes + 255) / 256 * 256 + 1024;
}

hipError_t launch_learned_encode(const float* params, const uint8_t* seq, const int64_t* off,
                                 int32_t n_strings, int N, float* out, hipStream_t s) {
  if (params == nullptr) {
    hipLaunchKernelGGL(plain_encode_kernel, dim3((unsigned)(((int64_t)n_strings + 3) / 4)),
                       dim3(256), 0, s, seq, off, n_strings, N, out);
    return hipGetLastError();
  }
  unsigned blocks = (unsigned)(((int64_t)n_strings + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(learned_encode_kernel, dim3(blocks), dim3(64 * kWaves), 0, s, params,
                     Strings{seq, off, nullptr, nullptr}, n_strings, N, out);
  return hipGetLastError();
}

hipError_t launch_pair_fidelity(const float* ca, const float* cb, int32_t n_pairs, float* F,
                                hipStream_t s) {
  unsigned blocks = (unsigned)(((int64_t)n_pairs + 3) / 4);
  hipLaunchKernelGGL(pair_fidelity_kernel, dim3(blocks), dim3(256), 0, s, ca, cb, (int64_t)256,
                     n_pairs, F);
  return hipGetLastError();
}

// One training (or gradient-only) step over n_pairs pairs (a_i, b_i); the
// workspace holds the encodings of a_i and b_i as rows 2i and 2i+1.
hipError_t launch_learned_step(float* state, float lr, const uint8_t* a, const int64_t* aoff,
                               const uint8_t* b, const int64_t* boff, const int32_t* ld,
                               int32_t n_pairs, int N, void* ws, float* grad_out,
                               float* loss_out, hipStream_t s) {
  const int64_t strings = 2 * (int64_t)n_pairs;
  const unsigned blocks = (unsigned)((strings + kWaves - 1) / kWaves);
  const Strings st{a, aoff, b, boff};
  uint8_t* base = static_cast<uint8_t*>(ws);
  float* c = reinterpret_cast<float*>(base);
  float* F = c + strings * 256;
  float* dF = F + n_pairs;
  float* lossv = dF + n_pairs;
  int32_t* cntv = reinterpret_cast<int32_t*>(lossv + n_pairs);
  float* loss_ws = reinterpret_cast<float*>(cntv + n_pairs);
  float* partial = reinterpret_cast<float*>(
      (reinterpret_cast<uintptr_t>(loss_ws + 64) + 255) / 256 * 256);
  hipLaunchKernelGGL(learned_encode_kernel, dim3(blocks), dim3(64 * kWaves), 0, s, state, st,
                     (int32_t)strings, N, c);
  hipLaunchKernelGGL(pair_fidelity_kernel, dim3((unsigned)((n_pairs + 3) / 4)), dim3(256), 0, s, c,
                     c + 256, (int64_t)512, n_pairs, F);
  hipLaunchKernelGGL(ranking_pairs_kernel, dim3((unsigned)((n_pairs + kRankI - 1) / kRankI)),
                     dim3(kRankI * kRankParts), 0, s, F, ld, n_pairs, dF, lossv, cntv);
  hipLaunchKernelGGL(ranking_finalize_kernel, dim3(1), dim3(1024), 0, s, dF, lossv, cntv, n_pairs,
                     loss_out ? loss_out : loss_ws);
  hipLaunchKernelGGL(learned_backward_kernel, dim3(blocks), dim3(64 * kWaves), 0, s, state, st,
                     n_pairs, N, c, dF, partial);
  hipLaunchKernelGGL(reduce_adam_kernel, dim3((kParams + kRedParams - 1) / kRedParams),
                     dim3(kRedParams * kRedParts), 0, s, partial, (int)blocks, grad_out,
                     grad_out ? nullptr : state, lr);
  if (grad_out == nullptr)
    hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, s, state);
  return hipGetLastError();
}

}  // namespace rm
