// Per-tile front-to-back compositing of colour, depth and visibility (LVI-GS Section III-B,
// eqs. Cp, Dp, Vp with the alpha of eq. alpha) and its backward.
//
// One wave64 per tile; each lane owns PPT pixels of the tile (a column of rows spaced 64/TW apart), so a
// record staged in LDS is read once per lane and used PPT times.  Records of a tile's depth-sorted list
// are staged 64 at a time (one per lane, coalesced by record id) into LDS and broadcast to all lanes.
//
// The backward walks the list in the same front-to-back order as the forward.  With the forward's final
// values C, D, V of a pixel and its upstream gradient g, the gradient of alpha_i is
//   dL/dalpha_i = T_i q_i - (S - P_i) / (1 - alpha_i),   q_i = g . (c_i, d_i, 1),
//   S = g . (C, D, V),  P_i = sum_{j <= i} alpha_j T_j q_j,
// i.e. what lies behind record i is S - P_i.  No per-pixel state has to be stored between the forward
// and the backward (the fused variant recomputes C, D, V with a first sweep in the same kernel), and the
// skip / stop decisions are re-evaluated with the forward's arithmetic.  Per-record gradients of a wave
// are summed with DPP before one atomic add per value.
#include "common.h"

namespace {

using gsk::DevOpts;

template <int TW, int TH>
struct Geo {
  static_assert(TW == 8 || TW == 16 || TW == 32, "tile width");
  static constexpr int RPP = 64 / TW;  // rows of the tile covered by the 64 lanes at once
  static constexpr int PPT = TH / RPP; // pixels per lane
  static_assert(PPT >= 1 && PPT * RPP == TH, "tile height");
};

struct TileCtx {
  int view, W, H, px, py0;
  int64_t pix_off;
  float weight;
};

template <int TW, int TH>
__device__ __forceinline__ bool tile_setup(const gs_camera* __restrict__ cams, int V, int n_tiles, TileCtx& t,
                                           int& tile) {
  tile = gsk::xcd_remap(blockIdx.x, gridDim.x);
  if (tile >= n_tiles) return false;
  t.view = gsk::view_of_tile(cams, V, tile);
  const gs_camera& c = cams[t.view];
  const int lt = tile - c.tile_offset;
  const int tyi = lt / c.tiles_x, txi = lt - tyi * c.tiles_x;
  const int lane = threadIdx.x;
  t.W = c.width;
  t.H = c.height;
  t.px = txi * TW + (lane % TW);
  t.py0 = tyi * TH + lane / TW;
  t.pix_off = c.pixel_offset;
  t.weight = c.loss_weight;
  return true;
}

// One record at one pixel: returns false if skipped (power > 0 or alpha < alpha_min).
__device__ __forceinline__ bool eval_pair(const float4& A, const float4& B, float fx, float fy, const DevOpts& op,
                                          float& alpha, float& G, bool& clamped, float& dx, float& dy) {
  dx = A.x - fx;
  dy = A.y - fy;
  const float power = -0.5f * (B.x * dx * dx + B.z * dy * dy) - B.y * dx * dy;
  if (power > 0.f) return false;
  G = __expf(power);
  const float oG = A.w * G;
  clamped = oG > op.alpha_max;
  alpha = clamped ? op.alpha_max : oG;
  return alpha >= op.alpha_min;
}

struct Stage {
  float4 A[64], B[64], C[64];
  int32_t r[64];
};

__device__ __forceinline__ void stage_batch(Stage& s, const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                            int b0, int nb) {
  const int lane = threadIdx.x;
  if (lane < nb) {
    const int r = vals[b0 + lane];
    s.A[lane] = rec[3 * (int64_t)r];
    s.B[lane] = rec[3 * (int64_t)r + 1];
    s.C[lane] = rec[3 * (int64_t)r + 2];
    s.r[lane] = r;
  }
}

// Forward sweep of one tile (shared by the forward kernel and the fused backward's first phase).
template <int PPT, int RPP>
__device__ __forceinline__ void forward_sweep(Stage& s, const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                              int2 rg, const TileCtx& t, const DevOpts& op, float* T, float* Cr,
                                              float* Cg, float* Cb, float* D, float* Vs) {
  bool live[PPT];
  float fy[PPT];
  const float fx = (float)t.px + 0.5f;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int py = t.py0 + k * RPP;
    live[k] = t.px < t.W && py < t.H;
    fy[k] = (float)py + 0.5f;
    T[k] = 1.f;
    Cr[k] = Cg[k] = Cb[k] = D[k] = Vs[k] = 0.f;
  }
  for (int b0 = rg.x; b0 < rg.y; b0 += 64) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < PPT; ++k) any |= live[k];
    if (__ballot(any) == 0) break;
    const int nb = min(64, rg.y - b0);
    __syncthreads();
    stage_batch(s, rec, vals, b0, nb);
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      const float4 A = s.A[j], B = s.B[j], C = s.C[j];
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if (!live[k]) continue;
        float alpha, G, dx, dy;
        bool cl;
        if (!eval_pair(A, B, fx, fy[k], op, alpha, G, cl, dx, dy)) continue;
        const float Tn = T[k] * (1.f - alpha);
        if (Tn < op.t_min) {
          live[k] = false;
          continue;
        }
        const float w = alpha * T[k];
        Cr[k] += w * B.w;
        Cg[k] += w * C.x;
        Cb[k] += w * C.y;
        D[k] += w * A.z;
        Vs[k] += w;
        T[k] = Tn;
      }
    }
  }
}

template <int TW, int TH>
__global__ __launch_bounds__(64) void k_render_fwd(const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                                   const int2* __restrict__ range, const gs_camera* __restrict__ cams,
                                                   int V, int n_tiles, DevOpts op, float* __restrict__ out_rgb,
                                                   float* __restrict__ out_depth, float* __restrict__ out_vis) {
  using Gm = Geo<TW, TH>;
  constexpr int PPT = Gm::PPT, RPP = Gm::RPP;
  __shared__ Stage s;
  TileCtx t;
  int tile;
  if (!tile_setup<TW, TH>(cams, V, n_tiles, t, tile)) return;
  float T[PPT], Cr[PPT], Cg[PPT], Cb[PPT], D[PPT], Vs[PPT];
  forward_sweep<PPT, RPP>(s, rec, vals, range[tile], t, op, T, Cr, Cg, Cb, D, Vs);
  const int64_t P = (int64_t)t.W * t.H;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int py = t.py0 + k * RPP;
    if (t.px < t.W && py < t.H) {
      const int64_t i = (int64_t)py * t.W + t.px;
      out_rgb[3 * t.pix_off + i] = Cr[k] + T[k] * op.bg[0];
      out_rgb[3 * t.pix_off + P + i] = Cg[k] + T[k] * op.bg[1];
      out_rgb[3 * t.pix_off + 2 * P + i] = Cb[k] + T[k] * op.bg[2];
      out_depth[t.pix_off + i] = D[k];
      out_vis[t.pix_off + i] = Vs[k];
    }
  }
}

struct BwdArgs {
  const float* fwd_rgb;
  const float* fwd_depth;
  const float* fwd_vis;
  const float* g_rgb;
  const float* g_depth;
  const float* g_vis;
  const float* tgt_rgb;
  const float* tgt_depth;
  const int32_t* n_valid;  // per view
  float lambda_d;
  float* rgrad;
  float* loss;
};

template <int TW, int TH, bool HAVE_FWD, bool LOSS>
__global__ __launch_bounds__(64) void k_render_bwd(const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                                   const int2* __restrict__ range, const gs_camera* __restrict__ cams,
                                                   int V, int n_tiles, DevOpts op, BwdArgs a) {
  using Gm = Geo<TW, TH>;
  constexpr int PPT = Gm::PPT, RPP = Gm::RPP;
  __shared__ Stage s;
  TileCtx t;
  int tile;
  if (!tile_setup<TW, TH>(cams, V, n_tiles, t, tile)) return;
  const int2 rg = range[tile];
  const int64_t P = (int64_t)t.W * t.H;
  // final values of each pixel
  float Cf[PPT], Gf[PPT], Bf[PPT], Df[PPT], Vf[PPT];
  if (HAVE_FWD) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int py = t.py0 + k * RPP;
      Cf[k] = Gf[k] = Bf[k] = Df[k] = Vf[k] = 0.f;
      if (t.px < t.W && py < t.H) {
        const int64_t i = (int64_t)py * t.W + t.px;
        Cf[k] = a.fwd_rgb[3 * t.pix_off + i];
        Gf[k] = a.fwd_rgb[3 * t.pix_off + P + i];
        Bf[k] = a.fwd_rgb[3 * t.pix_off + 2 * P + i];
        Df[k] = a.fwd_depth[t.pix_off + i];
        Vf[k] = a.fwd_vis[t.pix_off + i];
      }
    }
  } else {
    float T[PPT];
    forward_sweep<PPT, RPP>(s, rec, vals, rg, t, op, T, Cf, Gf, Bf, Df, Vf);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      Cf[k] += T[k] * op.bg[0];
      Gf[k] += T[k] * op.bg[1];
      Bf[k] += T[k] * op.bg[2];
    }
  }
  // upstream gradient of each pixel
  float gr[PPT], gg[PPT], gb[PPT], gd[PPT], gv[PPT], S[PPT];
  float loss_acc = 0.f;
  float wrgb = 0.f, wd = 0.f;
  if (LOSS) {
    wrgb = t.weight / (3.f * (float)P);
    const int M = a.n_valid[t.view];
    wd = M > 0 ? t.weight * a.lambda_d / (float)M : 0.f;
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int py = t.py0 + k * RPP;
    gr[k] = gg[k] = gb[k] = gd[k] = gv[k] = 0.f;
    if (t.px < t.W && py < t.H) {
      const int64_t i = (int64_t)py * t.W + t.px;
      if (LOSS) {
        const float er = Cf[k] - a.tgt_rgb[3 * t.pix_off + i];
        const float eg = Gf[k] - a.tgt_rgb[3 * t.pix_off + P + i];
        const float eb = Bf[k] - a.tgt_rgb[3 * t.pix_off + 2 * P + i];
        gr[k] = wrgb * gsk::sgnf(er);
        gg[k] = wrgb * gsk::sgnf(eg);
        gb[k] = wrgb * gsk::sgnf(eb);
        loss_acc += wrgb * (fabsf(er) + fabsf(eg) + fabsf(eb));
        const float dt = a.tgt_depth[t.pix_off + i];
        if (dt > 0.f) {
          const float ed = Df[k] - dt;
          gd[k] = wd * gsk::sgnf(ed);
          loss_acc += wd * fabsf(ed);
        }
      } else {
        if (a.g_rgb) {
          gr[k] = a.g_rgb[3 * t.pix_off + i];
          gg[k] = a.g_rgb[3 * t.pix_off + P + i];
          gb[k] = a.g_rgb[3 * t.pix_off + 2 * P + i];
        }
        if (a.g_depth) gd[k] = a.g_depth[t.pix_off + i];
        if (a.g_vis) gv[k] = a.g_vis[t.pix_off + i];
      }
    }
    S[k] = gr[k] * Cf[k] + gg[k] * Gf[k] + gb[k] * Bf[k] + gd[k] * Df[k] + gv[k] * Vf[k];
  }
  if (LOSS) {
    const float ls = gsk::wave_sum_last(loss_acc);
    if (threadIdx.x == 63) gsk::atomic_add_f32(a.loss, ls);
  }
  // second sweep, front to back
  bool live[PPT];
  float fy[PPT], T[PPT], Pp[PPT];
  const float fx = (float)t.px + 0.5f;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int py = t.py0 + k * RPP;
    live[k] = t.px < t.W && py < t.H;
    fy[k] = (float)py + 0.5f;
    T[k] = 1.f;
    Pp[k] = 0.f;
  }
  for (int b0 = rg.x; b0 < rg.y; b0 += 64) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < PPT; ++k) any |= live[k];
    if (__ballot(any) == 0) break;
    const int nb = min(64, rg.y - b0);
    __syncthreads();
    stage_batch(s, rec, vals, b0, nb);
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      const float4 A = s.A[j], B = s.B[j], C = s.C[j];
      float acc[10];
#pragma unroll
      for (int i = 0; i < 10; ++i) acc[i] = 0.f;
      bool hit = false;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if (!live[k]) continue;
        float alpha, G, dx, dy;
        bool cl;
        if (!eval_pair(A, B, fx, fy[k], op, alpha, G, cl, dx, dy)) continue;
        const float Tn = T[k] * (1.f - alpha);
        if (Tn < op.t_min) {
          live[k] = false;
          continue;
        }
        const float w = alpha * T[k];
        const float q = gr[k] * B.w + gg[k] * C.x + gb[k] * C.y + gd[k] * A.z + gv[k];
        Pp[k] += w * q;
        const float dalpha = T[k] * q - (S[k] - Pp[k]) * __builtin_amdgcn_rcpf(1.f - alpha);
        acc[6] += w * gr[k];
        acc[7] += w * gg[k];
        acc[8] += w * gb[k];
        acc[9] += w * gd[k];
        if (!cl) {
          acc[5] += dalpha * G;
          const float dq = dalpha * alpha;
          acc[2] += -0.5f * dx * dx * dq;
          acc[3] += -dx * dy * dq;
          acc[4] += -0.5f * dy * dy * dq;
          acc[0] += -(B.x * dx + B.y * dy) * dq;
          acc[1] += -(B.z * dy + B.y * dx) * dq;
        }
        T[k] = Tn;
        hit = true;
      }
      if (__ballot(hit) != 0) {
        float* dst = a.rgrad + 12 * (int64_t)s.r[j];
#pragma unroll
        for (int i = 0; i < 10; ++i) {
          const float sum = gsk::wave_sum_last(acc[i]);
          if (threadIdx.x == 63) gsk::atomic_add_f32(dst + i, sum);
        }
      }
    }
  }
}

__global__ void k_count_valid(const float* __restrict__ tgt_depth, const gs_camera* __restrict__ cams,
                              int32_t* __restrict__ n_valid) {
  const int v = blockIdx.y;
  const gs_camera& c = cams[v];
  const int64_t P = (int64_t)c.width * c.height;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < P && tgt_depth[c.pixel_offset + i] > 0.f;
  const uint64_t b = __ballot(ok);
  if (__lane_id() == 0 && b) atomicAdd(n_valid + v, (int)__popcll(b));
}

template <int TW, int TH>
hipError_t launch_fwd(const gs_frame& f, const DevOpts& op, const gs_images& out, hipStream_t st) {
  const int nb = ((f.n_tiles + 7) / 8) * 8;
  const int sorted = f.sort_passes & 1;
  k_render_fwd<TW, TH><<<nb, 64, 0, st>>>(reinterpret_cast<const float4*>(f.rec), f.vals[sorted],
                                          reinterpret_cast<const int2*>(f.tile_range), f.cams, f.n_views, f.n_tiles,
                                          op, out.rgb, out.depth, out.vis);
  return hipGetLastError();
}

template <int TW, int TH>
hipError_t launch_bwd(const gs_frame& f, const DevOpts& op, bool have_fwd, bool loss, const BwdArgs& a,
                      hipStream_t st) {
  const int nb = ((f.n_tiles + 7) / 8) * 8;
  const int sorted = f.sort_passes & 1;
  const auto* rec = reinterpret_cast<const float4*>(f.rec);
  const auto* rng = reinterpret_cast<const int2*>(f.tile_range);
  if (have_fwd && loss)
    k_render_bwd<TW, TH, true, true><<<nb, 64, 0, st>>>(rec, f.vals[sorted], rng, f.cams, f.n_views, f.n_tiles, op, a);
  else if (have_fwd)
    k_render_bwd<TW, TH, true, false><<<nb, 64, 0, st>>>(rec, f.vals[sorted], rng, f.cams, f.n_views, f.n_tiles, op, a);
  else if (loss)
    k_render_bwd<TW, TH, false, true><<<nb, 64, 0, st>>>(rec, f.vals[sorted], rng, f.cams, f.n_views, f.n_tiles, op, a);
  else
    k_render_bwd<TW, TH, false, false><<<nb, 64, 0, st>>>(rec, f.vals[sorted], rng, f.cams, f.n_views, f.n_tiles, op,
                                                          a);
  return hipGetLastError();
}

}  // namespace

namespace gs_launch {

#define GS_TILE_DISPATCH(FN, ...)                                          \
  do {                                                                     \
    if (o.tile_w == 16 && o.tile_h == 16) return FN<16, 16>(__VA_ARGS__);  \
    if (o.tile_w == 16 && o.tile_h == 8) return FN<16, 8>(__VA_ARGS__);    \
    if (o.tile_w == 8 && o.tile_h == 8) return FN<8, 8>(__VA_ARGS__);      \
    if (o.tile_w == 32 && o.tile_h == 8) return FN<32, 8>(__VA_ARGS__);    \
    if (o.tile_w == 32 && o.tile_h == 16) return FN<32, 16>(__VA_ARGS__);  \
    return hipErrorInvalidValue;                                           \
  } while (0)

hipError_t render_fwd(const gs_frame& f, const gs_opts& o, const gs_images& out, hipStream_t st) {
  const DevOpts op = gsk::dev_opts(o);
  GS_TILE_DISPATCH(launch_fwd, f, op, out, st);
}

hipError_t count_valid(const gs_frame& f, const float* tgt_depth, int64_t max_pixels, hipStream_t st) {
  hipError_t e = fill_i32(f.counters + 2, 0, f.n_views, st);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((max_pixels + 255) / 256), (unsigned)f.n_views);
  k_count_valid<<<grid, 256, 0, st>>>(tgt_depth, f.cams, f.counters + 2);
  return hipGetLastError();
}

hipError_t render_bwd(const gs_frame& f, const gs_opts& o, const gs_images* fwd, const gs_loss& l, hipStream_t st) {
  const DevOpts op = gsk::dev_opts(o);
  BwdArgs a;
  a.fwd_rgb = fwd ? fwd->rgb : nullptr;
  a.fwd_depth = fwd ? fwd->depth : nullptr;
  a.fwd_vis = fwd ? fwd->vis : nullptr;
  a.g_rgb = l.g_rgb;
  a.g_depth = l.g_depth;
  a.g_vis = l.g_vis;
  a.tgt_rgb = l.tgt_rgb;
  a.tgt_depth = l.tgt_depth;
  a.n_valid = f.counters + 2;
  a.lambda_d = l.lambda_d;
  a.rgrad = f.rgrad;
  a.loss = f.loss;
  const bool loss = l.tgt_rgb != nullptr;
  GS_TILE_DISPATCH(launch_bwd, f, op, fwd != nullptr, loss, a, st);
}

}  // namespace gs_launch
