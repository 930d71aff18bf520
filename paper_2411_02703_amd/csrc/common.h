// Internal device helpers of libgs (HIP, gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/libgs.h"

namespace gsk {

constexpr int kWave = 64;
// Partial sums of the loss (frame->loss[1 .. kLossSlots]); the frame holds 64 floats for the loss.
constexpr int kLossSlots = 32;

// Options as the kernels see them (passed by value).
struct DevOpts {
  float near_z, lowpass, alpha_min, alpha_max, t_min;
  float bg[3];
  int tile_w, tile_h;
};

inline DevOpts dev_opts(const gs_opts& o) {
  DevOpts d;
  d.near_z = o.near_z;
  d.lowpass = o.lowpass;
  d.alpha_min = o.alpha_min;
  d.alpha_max = o.alpha_max;
  d.t_min = o.t_min;
  d.bg[0] = o.bg[0];
  d.bg[1] = o.bg[1];
  d.bg[2] = o.bg[2];
  d.tile_w = o.tile_w;
  d.tile_h = o.tile_h;
  return d;
}

// ------------------------------------------------------------------ wave primitives
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// DPP move of a float with control CTRL; lanes without a valid source (bound_ctrl) or in a masked row read 0.
// bound_ctrl lets the move fold into the consuming add (v_add_f32_dpp).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true));
}

// Sum over the 64 lanes of a wave; the total lands in lane 63.  Six DPP adds:
// pairs, quads, half rows, rows (mirrors), then row broadcasts 15 and 31 across rows.
__device__ __forceinline__ float wave_sum_last(float x) {
  x += dpp_f<0xB1>(x);        // quad_perm [1,0,3,2]
  x += dpp_f<0x4E>(x);        // quad_perm [2,3,0,1]
  x += dpp_f<0x141>(x);       // row_half_mirror
  x += dpp_f<0x140>(x);       // row_mirror
  x += dpp_f<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_f<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Maximum over the 64 lanes of a non-negative int, returned to every lane (same DPP pattern as above).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xf, true);
}

__device__ __forceinline__ int wave_max_nonneg(int x) {
  x = max(x, dpp_i<0xB1>(x));
  x = max(x, dpp_i<0x4E>(x));
  x = max(x, dpp_i<0x141>(x));
  x = max(x, dpp_i<0x140>(x));
  x = max(x, dpp_i<0x142, 0xa>(x));
  x = max(x, dpp_i<0x143, 0xc>(x));
  return __builtin_amdgcn_readlane(x, 63);
}

// A value known to be the same in every lane, moved to scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Exclusive prefix sum over the 64 lanes (lane order) of a non-negative int; total = the wave's sum.
__device__ __forceinline__ int wave_excl_scan(int x, int& total) {
  int incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d);
    if (__lane_id() >= d) incl += y;
  }
  total = __builtin_amdgcn_readlane(incl, 63);
  return incl - x;
}

__device__ __forceinline__ float read_lane(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Records with more tile instances than this are wide: binning emits them a tile per lane of a wave and lists
// them (frame counters[198], big_rec), and their instance partials are summed by a wave per record before the
// projection backward, which then reads one pre-summed partial for them.
constexpr int kWideRecord = 32;

// Hardware float atomic add without return (global_atomic_add_f32).
__device__ __forceinline__ void atomic_add_f32(float* p, float v) { unsafeAtomicAdd(p, v); }

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous range of work items
// so neighbouring tiles (which share Gaussians) meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  const int per = (nblocks + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// View of a global tile: largest v with tile_offset <= tile (uniform scalar loop, n_views <= 64).
__device__ __forceinline__ int view_of_tile(const gs_camera* __restrict__ cams, int n_views, int tile) {
  int v = 0;
  for (int i = 1; i < n_views; ++i)
    if (cams[i].tile_offset <= tile) v = i;
  return v;
}

__device__ __forceinline__ float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

}  // namespace gsk

// ------------------------------------------------------------------ host launchers (one per file)
namespace gs_launch {
hipError_t project(const gs_params& p, const gs_frame& f, const gs_opts& o, hipStream_t s);
hipError_t project_bwd(const gs_params& p, const gs_frame& f, const gs_opts& o, const gs_params& g,
                       hipStream_t s);
size_t scan_scratch_ints(int64_t n);
// An element count read on the device: min(n_sized, mul * ceil(min(max(*p, 0), cap) / div)); p == NULL: n_sized.
struct DevCount {
  const int32_t* p = nullptr;
  int64_t cap = 0;
  int div = 1, mul = 1;
};
__device__ __forceinline__ int64_t dev_count(const DevCount& c, int64_t n_sized) {
  if (!c.p) return n_sized;
  int64_t k = c.p[0];
  k = k < 0 ? 0 : (k > c.cap ? c.cap : k);
  k = (k + c.div - 1) / c.div * c.mul;
  return k < n_sized ? k : n_sized;
}
// Exclusive scan of in[0, n) into out (in place allowed); with a device count only its first dev_count items.
hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch, hipStream_t s,
                          DevCount dc = DevCount{});
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_f32(float* p, float v, int64_t n, hipStream_t s);
// Binning up to the instance total: the records' first partial slots, visible records sorted by depth, their
// instance counts and first emission indices, counters[0] = instances (overflow flagged).
hipError_t bin_records(const gs_frame& f, hipStream_t s);
hipError_t emit(const gs_frame& f, int64_t n_sized, hipStream_t s);
size_t sort_scratch_ints(int64_t n);
// fold_tiles: passes whose histogram scan has at most this many 4096-entry tiles (by the capacity) let the
// scatter scan the tile totals itself (one launch fewer per pass; capped at 1024)
hipError_t sort_pairs32(uint32_t* k0, int32_t* v0, uint32_t* k1, int32_t* v1, int64_t n_sized,
                        const int32_t* count_dev, int64_t cap, int key_bits, int32_t* scratch, hipStream_t s,
                        int fold_tiles);
hipError_t sort_pairs(uint64_t* k0, int32_t* v0, uint64_t* k1, int32_t* v1, int64_t n_sized,
                      const int32_t* count_dev, int64_t cap, int key_bits, int32_t* scratch, hipStream_t s);
hipError_t ranges(const gs_frame& f, const uint32_t* keys, int64_t n_sized, const int32_t* count_dev, hipStream_t s);
hipError_t tile_schedule(const gs_frame& f, hipStream_t s);
hipError_t work_items(const gs_frame& f, hipStream_t s);
hipError_t render_fwd(const gs_frame& f, const gs_opts& o, const gs_images& out, hipStream_t s);
hipError_t count_pairs(const gs_frame& f, const gs_opts& o, unsigned long long* counts, hipStream_t s);
hipError_t count_valid(const gs_frame& f, const float* tgt_depth, int64_t max_pixels, float* loss, int n_loss,
                       hipStream_t s);
// loss[0] = sum of the partial sums loss[1 .. kLossSlots]
hipError_t loss_total(float* loss, hipStream_t s);
hipError_t render_bwd(const gs_frame& f, const gs_opts& o, const gs_images* fwd, const gs_loss& l,
                      hipStream_t s);
hipError_t adam(const gs_params& p, const gs_params& g, const gs_params& m, const gs_params& v,
                const gs_adam& a, hipStream_t s);
// SSIM term of the photometric loss: gradient written to g_rgb, value to loss[0] (loss holds 1 + kLossSlots).
hipError_t ssim(const gs_camera* cams_host, const gs_camera* cams_dev, int n_views, const float* rgb,
                const float* tgt, float lambda, float* g_rgb, float* loss, hipStream_t s);
// Opacity pruning: keep flags, their scan and the gather of every kept row (scratch: prune_scratch_ints(n)).
size_t prune_scratch_ints(int64_t n);
hipError_t prune(const gs_params& p, const gs_params& m, const gs_params& v, float thr_logit, const gs_params& op,
                 const gs_params& om, const gs_params& ov, int64_t* n_kept, int32_t* scratch, hipStream_t s);
// Map expansion: filter, voxel cap, neighbour spacing and the new rows (scratch: expand_scratch_ints(n_old, M)).
size_t expand_scratch_ints(int64_t n_old, int64_t M);
hipError_t expand(const gs_params& p, const gs_params& m, const gs_params& v, int64_t n_old, const float* pts,
                  const float* rgb, int64_t M, const gs_camera& cam, const float* vis, float tau, float near_z,
                  float voxel, int cap, float cell, float init_logit, int64_t* n_added, int32_t* scratch,
                  hipStream_t s);
// Spatial (Morton) order: out row k = in row perm[k] for params, m, v (scratch: order_scratch_ints(n)).
size_t order_scratch_ints(int64_t n);
hipError_t spatial_order(const gs_params& p, const gs_params& m, const gs_params& v, const gs_params& op,
                         const gs_params& om, const gs_params& ov, int32_t* perm_out, int32_t* scratch,
                         hipStream_t s);
// The step counter and bias corrections of one Adam step (skipped when *skip_flags has the overflow bit).
hipError_t adam_prep(const gs_adam& a, const int32_t* skip_flags, hipStream_t s);
// Projection backward fused with Adam: params, m, v updated in place; the gradient is written to grads_out
// when it is non-NULL.  The step's bias corrections come from adam_prep on the same stream.
hipError_t project_bwd_adam(const gs_params& p, const gs_frame& f, const gs_opts& o, const gs_params& m,
                            const gs_params& v, const gs_adam& a, const gs_params* grads_out, hipStream_t s);
}  // namespace gs_launch
