// Map expansion on the GPU (LVI-GS Sections III-A, III-C, III-E): a keyframe's colourised LiDAR points become new
// Gaussians.
//   1. Visibility filter (Sec. III-C, eq. Vp): a point is projected into the keyframe (the projection's FP32
//      operation order) and kept where the visibility rendered from the current map is still at most tau_alpha
//      (the map does not yet explain that pixel); points outside the image or behind the near plane are kept.
//   2. Voxel deduplication and density cap (Sec. III-A): points live in voxels of a fixed size; a point is
//      accepted while its voxel holds fewer than `cap` points, counting the map's Gaussians and this batch's
//      earlier points (input order).  Keys are sorted (the library's stable radix sort), so each point's rank in
//      its voxel and the map's count there come from two binary searches.
//   3. Initialisation (Sec. III-E): mean = the point, log-scales = log sqrt of the mean squared distance to its 3
//      nearest accepted neighbours (>= 1e-7), identity rotation, opacity logit = inverse sigmoid of the initial
//      opacity, SH degree-0 coefficients from the colour, higher bands 0, Adam moments 0.  The neighbours come
//      from a uniform grid over the accepted points (sorted cell keys, ring search with an exact stopping rule:
//      after ring k every unvisited point is at least k cell sizes away); a point whose third neighbour is not
//      settled within kMaxRing rings is searched by brute force, a wave per point.
// Accepted points are appended after the n_old existing Gaussians in their input order.
#include "common.h"

namespace {

constexpr uint64_t kInvalid = ~0ull;
constexpr int kBias = 1 << 20;  // voxel / cell coordinates are packed as 21-bit fields (|index| < 2^20)
constexpr int kMaxRing = 3;
constexpr float kY0 = 0.28209479177387814f;

__device__ __forceinline__ bool cell_of(float x, float y, float z, float inv, float size, int c[3]) {
  // floor(x / size) with the IEEE division (the comparison value is the same everywhere)
  const float q[3] = {x / size, y / size, z / size};
  (void)inv;
  for (int k = 0; k < 3; ++k) {
    const float f = floorf(q[k]);
    if (!(f > -(float)kBias && f < (float)kBias)) return false;
    c[k] = (int)f;
  }
  return true;
}

__device__ __forceinline__ uint64_t pack(const int c[3]) {
  return (uint64_t)(c[0] + kBias) | ((uint64_t)(c[1] + kBias) << 21) | ((uint64_t)(c[2] + kBias) << 42);
}

// First index in sorted keys[0, n) whose key is >= k.
__device__ __forceinline__ int64_t lower_bound(const uint64_t* __restrict__ keys, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < k) lo = mid + 1; else hi = mid;
  }
  return lo;
}

struct ExpandCam {
  float R[9], T[3], fx, fy, cx, cy;
  int W, H;
};

// 1. visibility filter and voxel keys of the new points (kInvalid: filtered out or outside the key range)
__global__ void k_point_keys(const float* __restrict__ pts, int64_t M, ExpandCam c, const float* __restrict__ vis,
                             float tau, float near_z, float voxel, uint64_t* __restrict__ keys,
                             int32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
  bool pass = true;
  float t[3];
  for (int r = 0; r < 3; ++r)
    t[r] = __builtin_fmaf(c.R[3 * r + 2], z, __builtin_fmaf(c.R[3 * r + 1], y, __builtin_fmaf(c.R[3 * r], x, c.T[r])));
  if (t[2] >= near_z) {
    const float u = __builtin_fmaf(c.fx, t[0] / t[2], c.cx), v = __builtin_fmaf(c.fy, t[1] / t[2], c.cy);
    if (u >= 0.f && u < (float)c.W && v >= 0.f && v < (float)c.H) pass = vis[(int64_t)(int)v * c.W + (int)u] <= tau;
  }
  int cc[3];
  keys[i] = pass && cell_of(x, y, z, 0.f, voxel, cc) ? pack(cc) : kInvalid;
  vals[i] = (int32_t)i;
}

// voxel keys of the existing Gaussians
__global__ void k_map_keys(const float* __restrict__ means, int64_t N, float voxel, uint64_t* __restrict__ keys,
                           int32_t* __restrict__ vals) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  int cc[3];
  keys[j] = cell_of(means[3 * j], means[3 * j + 1], means[3 * j + 2], 0.f, voxel, cc) ? pack(cc) : kInvalid;
  vals[j] = (int32_t)j;
}

// 2. acceptance: rank of the point in its voxel (sorted, stable) plus the map's count there, against the cap
__global__ void k_accept(const uint64_t* __restrict__ pk, const int32_t* __restrict__ pv, int64_t M,
                         const uint64_t* __restrict__ mk, int64_t N, int cap, int32_t* __restrict__ accept) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= M) return;
  const uint64_t k = pk[s];
  int ok = 0;
  if (k != kInvalid) {
    const int64_t rank = s - lower_bound(pk, s, k);
    const int64_t have = N > 0 ? lower_bound(mk, N, k + 1) - lower_bound(mk, N, k) : 0;
    ok = have + rank < cap;
  }
  accept[pv[s]] = ok;
}

__global__ void k_accept_total(const int32_t* __restrict__ accept, const int32_t* __restrict__ off, int64_t M,
                               int32_t* __restrict__ count, int64_t* __restrict__ n_added) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int32_t a = off[M - 1] + accept[M - 1];
    count[0] = a;
    n_added[0] = a;
  }
}

// 3a. grid cell keys of the accepted points, compacted to their output order
__global__ void k_cell_keys(const float* __restrict__ pts, const int32_t* __restrict__ accept,
                            const int32_t* __restrict__ off, int64_t M, float cell, uint64_t* __restrict__ keys,
                            int32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M || !accept[i]) return;
  int cc[3];
  const bool ok = cell_of(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], 0.f, cell, cc);
  keys[off[i]] = ok ? pack(cc) : kInvalid;
  vals[off[i]] = (int32_t)i;
}

__device__ __forceinline__ void push3(float d, float b[3]) {
  if (d < b[2]) {
    b[2] = d;
    if (b[2] < b[1]) { const float t = b[1]; b[1] = b[2]; b[2] = t; }
    if (b[1] < b[0]) { const float t = b[0]; b[0] = b[1]; b[1] = t; }
  }
}

__device__ __forceinline__ float spacing_log_scale(const float b[3]) {
  int found = 0;
  float sum = 0.f;
  for (int k = 0; k < 3; ++k)
    if (b[k] < INFINITY) { sum += b[k]; ++found; }
  const float d2 = fmaxf(found ? sum / (float)found : 0.f, 1e-7f);
  return 0.5f * logf(d2);
}

// 3b. ring search over the sorted cells; the log-scale goes to the new Gaussian's row, unsettled points to a list
__global__ void k_knn(const float* __restrict__ pts, const uint64_t* __restrict__ ck, const int32_t* __restrict__ cv,
                      const int32_t* __restrict__ count, float cell, const int32_t* __restrict__ off,
                      float* __restrict__ out_ls, int32_t* __restrict__ brute, int32_t* __restrict__ n_brute) {
  const int64_t A = count[0];
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A) return;
  const int i = cv[s];
  const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
  int c0[3];
  if (!cell_of(x, y, z, 0.f, cell, c0)) {
    brute[atomicAdd(n_brute, 1)] = (int)s;
    return;
  }
  float b[3] = {INFINITY, INFINITY, INFINITY};
  for (int ring = 0; ring <= kMaxRing; ++ring) {
    for (int dz = -ring; dz <= ring; ++dz)
      for (int dy = -ring; dy <= ring; ++dy)
        for (int dx = -ring; dx <= ring; ++dx) {
          if (max(abs(dx), max(abs(dy), abs(dz))) != ring) continue;  // the shell of this ring only
          const int cc[3] = {c0[0] + dx, c0[1] + dy, c0[2] + dz};
          if (abs(cc[0]) >= kBias || abs(cc[1]) >= kBias || abs(cc[2]) >= kBias) continue;
          const uint64_t key = pack(cc);
          for (int64_t j = lower_bound(ck, A, key); j < A && ck[j] == key; ++j) {
            if (j == s) continue;
            const int q = cv[j];
            const float ex = pts[3 * q] - x, ey = pts[3 * q + 1] - y, ez = pts[3 * q + 2] - z;
            push3(ex * ex + ey * ey + ez * ez, b);
          }
        }
    const float reach = (float)ring * cell;
    if (b[2] <= reach * reach) {
      const float ls = spacing_log_scale(b);
      float* o = out_ls + 3 * (int64_t)off[i];
      o[0] = o[1] = o[2] = ls;
      return;
    }
  }
  brute[atomicAdd(n_brute, 1)] = (int)s;
}

// 3c. brute force for the unsettled points: a wave per point over every accepted point, then a wave reduction
__global__ __launch_bounds__(256) void k_knn_brute(const float* __restrict__ pts, const int32_t* __restrict__ cv,
                                                   const int32_t* __restrict__ count,
                                                   const int32_t* __restrict__ brute,
                                                   const int32_t* __restrict__ n_brute,
                                                   const int32_t* __restrict__ off, float* __restrict__ out_ls) {
  const int64_t A = count[0];
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t w = wave; w < n_brute[0]; w += n_waves) {
    const int64_t s = brute[w];
    const int i = cv[s];
    const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    float b[3] = {INFINITY, INFINITY, INFINITY};
    for (int64_t j = lane; j < A; j += 64) {
      if (j == s) continue;
      const int q = cv[j];
      const float ex = pts[3 * q] - x, ey = pts[3 * q + 1] - y, ez = pts[3 * q + 2] - z;
      push3(ex * ex + ey * ey + ez * ez, b);
    }
    // merge the lanes' three smallest: three rounds of a wave minimum, removing the winner each time
    float best[3];
    for (int r = 0; r < 3; ++r) {
      float m = b[0];
      for (int sh = 32; sh >= 1; sh >>= 1) m = fminf(m, __shfl_xor(m, sh));
      best[r] = m;
      // the lowest lane holding the minimum drops it
      const uint64_t hold = __ballot(b[0] == m && m < INFINITY);
      if (hold && lane == __builtin_ctzll(hold)) {
        b[0] = b[1];
        b[1] = b[2];
        b[2] = INFINITY;
      }
    }
    if (lane == 0) {
      const float ls = spacing_log_scale(best);
      float* o = out_ls + 3 * (int64_t)off[i];
      o[0] = o[1] = o[2] = ls;
    }
  }
}

// 3d. the other parameters and zero moments of every new Gaussian
struct NewRows {
  float* means; float* quats; float* opac; float* sh;
  float* m[5]; float* v[5];  // means, log_scales, quats, opacity, sh of the moments
};

__global__ void k_expand_write(const float* __restrict__ pts, const float* __restrict__ rgb,
                               const int32_t* __restrict__ accept, const int32_t* __restrict__ off, int64_t M,
                               int64_t n_old, int K3, float logit, NewRows r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M || !accept[i]) return;
  const int64_t g = n_old + off[i];
  for (int k = 0; k < 3; ++k) r.means[3 * g + k] = pts[3 * i + k];
  r.quats[4 * g] = 1.f;
  r.quats[4 * g + 1] = r.quats[4 * g + 2] = r.quats[4 * g + 3] = 0.f;
  r.opac[g] = logit;
  float* f = r.sh + g * K3;
  for (int k = 0; k < 3; ++k) f[k] = (rgb[3 * i + k] - 0.5f) / kY0;
  for (int k = 3; k < K3; ++k) f[k] = 0.f;
  const int len[5] = {3, 3, 4, 1, K3};
  for (int a = 0; a < 5; ++a)
    for (int k = 0; k < len[a]; ++k) {
      r.m[a][g * len[a] + k] = 0.f;
      r.v[a][g * len[a] + k] = 0.f;
    }
}

}  // namespace

namespace gs_launch {

// Scratch layout (int32 units, 64-aligned pieces): point keys/vals x2, map keys/vals x2, accept, off, brute list,
// counters, sort scratch (reused by the three sorts), scan scratch.
struct ExpandLayout {
  size_t pk0, pk1, pv0, pv1, mk0, mk1, mv0, mv1, acc, off, brute, cnt, sort, scan, total;
};

static size_t a64(size_t x) { return (x + 63) / 64 * 64; }

static ExpandLayout expand_layout(int64_t N, int64_t M) {
  ExpandLayout L;
  size_t o = 0;
  const size_t m2 = a64(2 * (size_t)M), n2 = a64(2 * (size_t)(N > 0 ? N : 1));
  L.pk0 = o; o += m2; L.pk1 = o; o += m2; L.pv0 = o; o += a64(M); L.pv1 = o; o += a64(M);
  L.mk0 = o; o += n2; L.mk1 = o; o += n2; L.mv0 = o; o += a64(N > 0 ? N : 1); L.mv1 = o; o += a64(N > 0 ? N : 1);
  L.acc = o; o += a64(M); L.off = o; o += a64(M); L.brute = o; o += a64(M); L.cnt = o; o += 64;
  const int64_t big = M > N ? M : N;
  L.sort = o; o += a64(sort_scratch_ints(big > 0 ? big : 1));
  L.scan = o; o += a64(scan_scratch_ints(M > 0 ? M : 1));
  L.total = o;
  return L;
}

size_t expand_scratch_ints(int64_t n_old, int64_t M) { return expand_layout(n_old, M).total; }

hipError_t expand(const gs_params& p, const gs_params& m, const gs_params& v, int64_t n_old, const float* pts,
                  const float* rgb, int64_t M, const gs_camera& cam, const float* vis, float tau, float near_z,
                  float voxel, int cap, float cell, float init_logit, int64_t* n_added, int32_t* scratch,
                  hipStream_t st) {
  const ExpandLayout L = expand_layout(n_old, M);
  auto u64 = [&](size_t o) { return reinterpret_cast<uint64_t*>(scratch + o); };
  int32_t* cnt = scratch + L.cnt;
  hipError_t e = fill_i32(cnt, 0, 64, st);
  if (e != hipSuccess) return e;
  ExpandCam c;
  for (int k = 0; k < 9; ++k) c.R[k] = cam.R[k];
  for (int k = 0; k < 3; ++k) c.T[k] = cam.T[k];
  c.fx = cam.fx; c.fy = cam.fy; c.cx = cam.cx; c.cy = cam.cy; c.W = cam.width; c.H = cam.height;
  const unsigned bm = (unsigned)((M + 255) / 256), bn = (unsigned)((n_old + 255) / 256);
  // 1. filter + voxel keys, sorted (stable: input order inside a voxel)
  k_point_keys<<<bm, 256, 0, st>>>(pts, M, c, vis, tau, near_z, voxel, u64(L.pk0), scratch + L.pv0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = sort_pairs(u64(L.pk0), scratch + L.pv0, u64(L.pk1), scratch + L.pv1, M, nullptr, M, 64,
                      scratch + L.sort, st)) != hipSuccess)
    return e;  // 8 passes: the sorted pairs are back in the first buffers
  if (n_old > 0) {
    k_map_keys<<<bn, 256, 0, st>>>(p.means, n_old, voxel, u64(L.mk0), scratch + L.mv0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = sort_pairs(u64(L.mk0), scratch + L.mv0, u64(L.mk1), scratch + L.mv1, n_old, nullptr, n_old, 64,
                        scratch + L.sort, st)) != hipSuccess)
      return e;
  }
  // 2. acceptance, and the output order
  k_accept<<<bm, 256, 0, st>>>(u64(L.pk0), scratch + L.pv0, M, u64(L.mk0), n_old, cap, scratch + L.acc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_exclusive(scratch + L.acc, scratch + L.off, M, scratch + L.scan, st)) != hipSuccess) return e;
  k_accept_total<<<1, 64, 0, st>>>(scratch + L.acc, scratch + L.off, M, cnt, n_added);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 3. cells of the accepted points (sorted, sized by M, counted on the device), spacing, the new rows
  k_cell_keys<<<bm, 256, 0, st>>>(pts, scratch + L.acc, scratch + L.off, M, cell, u64(L.pk1), scratch + L.pv1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = sort_pairs(u64(L.pk1), scratch + L.pv1, u64(L.pk0), scratch + L.pv0, M, cnt, M, 64, scratch + L.sort,
                      st)) != hipSuccess)
    return e;
  float* ls_new = p.log_scales + 3 * n_old;
  k_knn<<<bm, 256, 0, st>>>(pts, u64(L.pk1), scratch + L.pv1, cnt, cell, scratch + L.off, ls_new,
                            scratch + L.brute, cnt + 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_knn_brute<<<256, 256, 0, st>>>(pts, scratch + L.pv1, cnt, scratch + L.brute, cnt + 1, scratch + L.off, ls_new);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  NewRows r;
  r.means = p.means; r.quats = p.quats; r.opac = p.opacity; r.sh = p.sh;
  const gs_params* mv[2] = {&m, &v};
  for (int k = 0; k < 2; ++k) {
    float** d = k == 0 ? r.m : r.v;
    d[0] = mv[k]->means; d[1] = mv[k]->log_scales; d[2] = mv[k]->quats; d[3] = mv[k]->opacity; d[4] = mv[k]->sh;
  }
  const int K3 = 3 * (p.sh_degree + 1) * (p.sh_degree + 1);
  k_expand_write<<<bm, 256, 0, st>>>(pts, rgb, scratch + L.acc, scratch + L.off, M, n_old, K3, init_logit, r);
  return hipGetLastError();
}

}  // namespace gs_launch
