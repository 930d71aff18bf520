// One Adam step over all Gaussian parameters (bias-corrected moments, eps added to the corrected root),
// with one learning rate per parameter group.  The paper optimises rotation, scaling, opacity and SH
// colour by minimising its loss (LVI-GS Section III-E) without naming the optimiser.
// HBM-bound: per element it reads p, g, m, v and writes p, m, v.
#include "common.h"

namespace {

// Unless *skip_flags has the overflow bit (the frame's gradients are then undefined): step <- step + 1;
// bias = {1 - beta1^step, sqrt(1 - beta2^step)} (computed in double), bias[2] = 0.  Otherwise bias[2] = 1 and
// nothing else changes; the update kernels then leave every parameter and moment as it is.
__global__ void k_adam_prep(int64_t* __restrict__ step, float* __restrict__ bias, float b1, float b2,
                            const int32_t* __restrict__ skip_flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (skip_flags && (skip_flags[0] & GS_FLAG_INSTANCE_OVERFLOW)) {
    bias[2] = 1.f;
    return;
  }
  const int64_t t = step[0] + 1;
  step[0] = t;
  bias[0] = (float)(1.0 - pow((double)b1, (double)t));
  bias[1] = (float)sqrt(1.0 - pow((double)b2, (double)t));
  bias[2] = 0.f;
}

// period > 0: element i of the group uses lr0 when (i % period) < 3 (the degree-0 SH coefficients of a
// Gaussian's colour), lr1 otherwise.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, int64_t n, float lr0,
                                             float lr1, int period, float b1, float b2, float eps,
                                             const float* __restrict__ bias) {
  if (bias[2] != 0.f) return;  // skipped step
  const float bc1 = bias[0], bc2s = bias[1];
  const float s0 = lr0 / bc1, s1 = lr1 / bc1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  const int64_t first = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  // position of element i0 inside its period, kept up to date by additions (no division per element)
  int r = period > 0 ? (int)(first % period) : 0;
  const int rstep = period > 0 ? (int)(stride % period) : 0;
  for (int64_t i0 = first; i0 < n; i0 += stride) {
    if (i0 + 4 <= n) {
      const float4 gg = *reinterpret_cast<const float4*>(g + i0);
      float4 mm = *reinterpret_cast<const float4*>(m + i0);
      float4 vv = *reinterpret_cast<const float4*>(v + i0);
      float4 pp = *reinterpret_cast<const float4*>(p + i0);
      float* pm = &mm.x;
      float* pv = &vv.x;
      float* pq = &pp.x;
      const float* pg = &gg.x;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float gk = pg[k];
        pm[k] = b1 * pm[k] + (1.f - b1) * gk;
        pv[k] = b2 * pv[k] + (1.f - b2) * gk * gk;
        int rk = r + k;  // < 2 period, since period >= 3
        if (rk >= period) rk -= period;
        const float s = (period > 0 && rk >= 3) ? s1 : s0;
        pq[k] -= s * pm[k] / (sqrtf(pv[k]) / bc2s + eps);
      }
      *reinterpret_cast<float4*>(m + i0) = mm;
      *reinterpret_cast<float4*>(v + i0) = vv;
      *reinterpret_cast<float4*>(p + i0) = pp;
    } else {
      for (int64_t i = i0; i < n; ++i) {
        const float gk = g[i];
        const float mk = b1 * m[i] + (1.f - b1) * gk;
        const float vk = b2 * v[i] + (1.f - b2) * gk * gk;
        m[i] = mk;
        v[i] = vk;
        const float s = (period > 0 && (i % period) >= 3) ? s1 : s0;
        p[i] -= s * mk / (sqrtf(vk) / bc2s + eps);
      }
    }
    if (period > 0) {
      r += rstep;
      if (r >= period) r -= period;
    }
  }
}

hipError_t group(float* p, const float* g, float* m, float* v, int64_t n, float lr0, float lr1, int period,
                 const gs_adam& a, hipStream_t st) {
  const int threads = 256;
  int64_t blocks = (n + 4 * threads - 1) / (4 * threads);
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  k_adam<<<(unsigned)blocks, threads, 0, st>>>(p, g, m, v, n, lr0, lr1, period, a.beta1, a.beta2, a.eps, a.bias);
  return hipGetLastError();
}

}  // namespace

namespace gs_launch {

hipError_t adam_prep(const gs_adam& a, const int32_t* skip_flags, hipStream_t st) {
  k_adam_prep<<<1, 64, 0, st>>>(a.step, a.bias, a.beta1, a.beta2, skip_flags);
  return hipGetLastError();
}

hipError_t adam(const gs_params& p, const gs_params& g, const gs_params& m, const gs_params& v, const gs_adam& a,
                hipStream_t st) {
  k_adam_prep<<<1, 64, 0, st>>>(a.step, a.bias, a.beta1, a.beta2, a.skip_flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = p.n;
  const int K = (p.sh_degree + 1) * (p.sh_degree + 1);
  if ((e = group(p.means, g.means, m.means, v.means, 3 * n, a.lr[0], a.lr[0], 0, a, st)) != hipSuccess) return e;
  if ((e = group(p.log_scales, g.log_scales, m.log_scales, v.log_scales, 3 * n, a.lr[1], a.lr[1], 0, a, st)) !=
      hipSuccess)
    return e;
  if ((e = group(p.quats, g.quats, m.quats, v.quats, 4 * n, a.lr[2], a.lr[2], 0, a, st)) != hipSuccess) return e;
  if ((e = group(p.opacity, g.opacity, m.opacity, v.opacity, n, a.lr[3], a.lr[3], 0, a, st)) != hipSuccess) return e;
  return group(p.sh, g.sh, m.sh, v.sh, (int64_t)3 * K * n, a.lr[4], a.lr[5], 3 * K, a, st);
}

}  // namespace gs_launch
