// Map maintenance on the GPU (LVI-GS Section III-C): opacity pruning.  The delay buffer of Section III-C exists
// so that freshly initialised Gaussians are not removed "before they can be observed" once their opacity has
// dropped to the prunable threshold; this is the removal itself: every Gaussian whose opacity sigmoid(logit)
// lies below the threshold is dropped, and the survivors' parameters and Adam moments are compacted to the
// front of the output arrays in their original order.
//
// Work: one flag per Gaussian, an exclusive scan of the flags (the library's scan), then a gather of every kept
// row of the fifteen arrays (five parameter groups x params, m, v) with one thread per element, so reads are
// coalesced and writes are coalesced runs.  HBM-bound: 3 (44 + 12K) bytes read and at most as many written per
// Gaussian.
#include "common.h"

namespace {

// keep[i] = (opacity logit >= thr): the decision is a float comparison of the logit with the threshold's logit
// (computed once on the host), so it is exact and identical wherever it is evaluated.
__global__ void k_prune_flags(const float* __restrict__ opac, int64_t n, float thr, int32_t* __restrict__ keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keep[i] = opac[i] >= thr ? 1 : 0;
}

__global__ void k_prune_total(const int32_t* __restrict__ keep, const int32_t* __restrict__ off, int64_t n,
                              int64_t* __restrict__ n_kept) {
  if (threadIdx.x == 0 && blockIdx.x == 0) n_kept[0] = (int64_t)off[n - 1] + keep[n - 1];
}

struct Rows {
  const float* in[15];
  float* out[15];
  int len[15];  // floats per Gaussian
};

// blockIdx.y selects the array; element e of it belongs to Gaussian e / len.
__global__ __launch_bounds__(256) void k_prune_gather(const Rows r, int64_t n, const int32_t* __restrict__ keep,
                                                      const int32_t* __restrict__ off) {
  const int a = blockIdx.y;
  const int len = r.len[a];
  const float* __restrict__ in = r.in[a];
  float* __restrict__ out = r.out[a];
  const int64_t total = n * len;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / len;
    if (keep[i]) out[(int64_t)off[i] * len + (e - i * len)] = in[e];
  }
}

}  // namespace

namespace gs_launch {

size_t prune_scratch_ints(int64_t n) { return 2 * (size_t)((n + 63) / 64 * 64) + scan_scratch_ints(n); }

hipError_t prune(const gs_params& p, const gs_params& m, const gs_params& v, float thr_logit, const gs_params& op,
                 const gs_params& om, const gs_params& ov, int64_t* n_kept, int32_t* scratch, hipStream_t st) {
  const int64_t n = p.n;
  const size_t na = (size_t)((n + 63) / 64 * 64);
  int32_t* keep = scratch;
  int32_t* off = scratch + na;
  int32_t* scan_scr = scratch + 2 * na;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  k_prune_flags<<<blocks, 256, 0, st>>>(p.opacity, n, thr_logit, keep);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_exclusive(keep, off, n, scan_scr, st)) != hipSuccess) return e;
  k_prune_total<<<1, 64, 0, st>>>(keep, off, n, n_kept);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int K3 = 3 * (p.sh_degree + 1) * (p.sh_degree + 1);
  Rows r;
  const gs_params* src[3] = {&p, &m, &v};
  const gs_params* dst[3] = {&op, &om, &ov};
  for (int k = 0; k < 3; ++k) {
    r.in[5 * k + 0] = src[k]->means;      r.out[5 * k + 0] = dst[k]->means;      r.len[5 * k + 0] = 3;
    r.in[5 * k + 1] = src[k]->log_scales; r.out[5 * k + 1] = dst[k]->log_scales; r.len[5 * k + 1] = 3;
    r.in[5 * k + 2] = src[k]->quats;      r.out[5 * k + 2] = dst[k]->quats;      r.len[5 * k + 2] = 4;
    r.in[5 * k + 3] = src[k]->opacity;    r.out[5 * k + 3] = dst[k]->opacity;    r.len[5 * k + 3] = 1;
    r.in[5 * k + 4] = src[k]->sh;         r.out[5 * k + 4] = dst[k]->sh;         r.len[5 * k + 4] = K3;
  }
  int64_t gx = (n * K3 + 255) / 256;
  if (gx > 16384) gx = 16384;
  k_prune_gather<<<dim3((unsigned)gx, 15), 256, 0, st>>>(r, n, keep, off);
  return hipGetLastError();
}

}  // namespace gs_launch
