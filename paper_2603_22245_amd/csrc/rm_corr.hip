// The correlation score of §2.4 on the device.  Pairs (dna, mut) are sampled
// at mutation rates err; per rate the expected fidelity E_fid is the mean of
// its pairs' fidelities; the points (E_fid(err), err), joined in order of
// E_fid, form the fitting curve; per rate the RMSE is the root mean square
// of the vertical distances (curve(fid) - err) of its pairs' points.
//
// Two launches: one block per rate takes its mean; then one block per rate
// sorts the (E_fid, err) points in LDS (rank by E_fid, ties by rate index)
// and sums its pairs' squared distances.  Past the curve's ends the nearest
// end point's rate is taken (the curve is extended flat).

#include "rm_internal.h"

namespace rm {
namespace {

constexpr int kCorrThreads = 256;

__device__ __forceinline__ float block_sum(float v, float* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(kCorrThreads) void rate_mean_kernel(const float* __restrict__ F,
                                                                 int per, float* __restrict__ E) {
  __shared__ float red[kCorrThreads / 64];
  const float* f = F + (int64_t)blockIdx.x * per;
  float s = 0.f;
  for (int i = threadIdx.x; i < per; i += kCorrThreads) s += f[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) E[blockIdx.x] = s / (float)per;
}

__global__ __launch_bounds__(kCorrThreads) void rate_rmse_kernel(
    const float* __restrict__ F, const float* __restrict__ err, const float* __restrict__ E,
    int n_rates, int per, float* __restrict__ rmse) {
  __shared__ float cE[RM_CORR_MAX_RATES], ce[RM_CORR_MAX_RATES];
  __shared__ float red[kCorrThreads / 64];
  const int t = threadIdx.x;
  if (t < n_rates) {
    const float Ei = E[t];
    int rank = 0;
    for (int j = 0; j < n_rates; ++j) {
      const float Ej = E[j];
      rank += (Ej < Ei) || (Ej == Ei && j < t);
    }
    cE[rank] = Ei;
    ce[rank] = err[t];
  }
  __syncthreads();
  const float e_rate = err[blockIdx.x];
  const float* f = F + (int64_t)blockIdx.x * per;
  float s = 0.f;
  for (int i = t; i < per; i += kCorrThreads) {
    const float x = f[i];
    float pred;
    if (x <= cE[0]) {
      pred = ce[0];
    } else if (x >= cE[n_rates - 1]) {
      pred = ce[n_rates - 1];
    } else {
      int lo = 0, hi = n_rates - 1;  // cE[lo] < x < cE[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cE[mid] <= x) lo = mid;
        else hi = mid;
      }
      const float w = (x - cE[lo]) / (cE[hi] - cE[lo]);
      pred = ce[lo] + w * (ce[hi] - ce[lo]);
    }
    const float d = pred - e_rate;
    s += d * d;
  }
  s = block_sum(s, red);
  if (t == 0) rmse[blockIdx.x] = sqrtf(s / (float)per);
}

}  // namespace

hipError_t launch_correlation_score(const float* F, const float* err, int32_t n_rates,
                                    int32_t per, float* E, float* rmse, hipStream_t s) {
  hipLaunchKernelGGL(rate_mean_kernel, dim3((unsigned)n_rates), dim3(kCorrThreads), 0, s, F, per,
                     E);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rate_rmse_kernel, dim3((unsigned)n_rates), dim3(kCorrThreads), 0, s, F, err,
                     E, n_rates, per, rmse);
  return hipGetLastError();
}

}  // namespace rm

extern "C" int rm_correlation_score(const float* d_F, const float* d_err, int32_t n_rates,
                                    int32_t per_rate, float* d_E, float* d_rmse, void* stream) {
  if (!d_F || !d_err || !d_E || !d_rmse) return RM_EINVAL;
  if (n_rates < 1 || n_rates > RM_CORR_MAX_RATES || per_rate < 1) return RM_ESIZE;
  const hipError_t e = rm::launch_correlation_score(d_F, d_err, n_rates, per_rate, d_E, d_rmse,
                                                    static_cast<hipStream_t>(stream));
  return e == hipSuccess ? RM_OK : RM_EHIP;
}
