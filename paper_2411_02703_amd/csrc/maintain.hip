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

// ------------------------------------------------------------------ spatial order
// Gaussians ordered along a Z-order (Morton) curve of their means: neighbouring Gaussians then sit in neighbouring
// rows, so the threads of one wave see nearly the same views in projection and its backward, records gathered by a
// tile come from nearby memory, and emission writes longer runs.  Each coordinate is quantised to 21 bits over
// the means' bounding box, q = min(2^21 - 1, floor((x - lo) * s)) with s = (2^21 - 1) / max(hi - lo, 1e-30) (FP32,
// no contraction), and the three are interleaved (x in bit 3k, y in 3k + 1, z in 3k + 2).  A stable radix sort
// of the codes gives the permutation; rows of parameters and moments are gathered through it.
namespace {

__device__ __forceinline__ uint32_t ordered_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

__global__ __launch_bounds__(256) void k_bbox(const float* __restrict__ means, int64_t n, uint32_t* __restrict__ box) {
  uint32_t lo[3] = {~0u, ~0u, ~0u}, hi[3] = {0u, 0u, 0u};
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
    for (int k = 0; k < 3; ++k) {
      const uint32_t o = ordered_bits(means[3 * g + k]);
      lo[k] = min(lo[k], o);
      hi[k] = max(hi[k], o);
    }
  for (int k = 0; k < 3; ++k) {
    for (int s = 32; s >= 1; s >>= 1) {
      lo[k] = min(lo[k], (uint32_t)__shfl_xor((int)lo[k], s));
      hi[k] = max(hi[k], (uint32_t)__shfl_xor((int)hi[k], s));
    }
    if ((threadIdx.x & 63) == 0) {
      atomicMin(box + k, lo[k]);
      atomicMax(box + 3 + k, hi[k]);
    }
  }
}

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__global__ void k_morton(const float* __restrict__ means, int64_t n, const uint32_t* __restrict__ box,
                         uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
#pragma clang fp contract(off)
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  uint64_t code = 0;
  for (int k = 0; k < 3; ++k) {
    const float lo = from_ordered(box[k]), hi = from_ordered(box[3 + k]);
    const float s = 2097151.0f / fmaxf(hi - lo, 1e-30f);
    const float t = (means[3 * g + k] - lo) * s;
    const uint32_t q = (uint32_t)fminf(floorf(t), 2097151.0f);
    code |= spread3(q) << k;
  }
  keys[g] = code;
  vals[g] = (int32_t)g;
}

// out row k = in row perm[k], for the fifteen arrays (blockIdx.y), one thread per element.
__global__ __launch_bounds__(256) void k_permute(const Rows r, int64_t n, const int32_t* __restrict__ perm) {
  const int a = blockIdx.y;
  const int len = r.len[a];
  const float* __restrict__ in = r.in[a];
  float* __restrict__ out = r.out[a];
  const int64_t total = n * len;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t k = e / len;
    out[e] = in[(int64_t)perm[k] * len + (e - k * len)];
  }
}

}  // namespace

namespace gs_launch {

// scratch: keys x2 (u64) + vals x2 + box + sort scratch
size_t order_scratch_ints(int64_t n) {
  const size_t a = (size_t)((n + 63) / 64 * 64);
  return 2 * 2 * a + 2 * a + 64 + sort_scratch_ints(n);
}

hipError_t spatial_order(const gs_params& p, const gs_params& m, const gs_params& v, const gs_params& op,
                         const gs_params& om, const gs_params& ov, int32_t* perm_out, int32_t* scratch,
                         hipStream_t st) {
  const int64_t n = p.n;
  const size_t a = (size_t)((n + 63) / 64 * 64);
  auto* k0 = reinterpret_cast<uint64_t*>(scratch);
  auto* k1 = reinterpret_cast<uint64_t*>(scratch + 2 * a);
  int32_t* v0 = scratch + 4 * a;
  int32_t* v1 = scratch + 5 * a;
  auto* box = reinterpret_cast<uint32_t*>(scratch + 6 * a);
  int32_t* sort_scr = scratch + 6 * a + 64;
  hipError_t e = fill_i32(reinterpret_cast<int32_t*>(box), -1, 3, st);  // lo = all ones
  if (e != hipSuccess) return e;
  if ((e = fill_i32(reinterpret_cast<int32_t*>(box) + 3, 0, 3, st)) != hipSuccess) return e;
  int64_t nb = (n + 255) / 256;
  if (nb > 2048) nb = 2048;
  k_bbox<<<(unsigned)nb, 256, 0, st>>>(p.means, n, box);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_morton<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p.means, n, box, k0, v0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = sort_pairs(k0, v0, k1, v1, n, nullptr, n, 64, sort_scr, st)) != hipSuccess) return e;  // back in v0
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
  k_permute<<<dim3((unsigned)gx, 15), 256, 0, st>>>(r, n, v0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (perm_out) return hipMemcpyAsync(perm_out, v0, (size_t)n * 4, hipMemcpyDeviceToDevice, st);
  return hipSuccess;
}

}  // namespace gs_launch
