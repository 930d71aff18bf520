// Per-tile front-to-back compositing of colour, depth and visibility (LVI-GS Section III-B,
// eqs. Cp, Dp, Vp with the alpha of eq. alpha) and its backward.
//
// One workgroup of NW wave64s per tile.  The tile is split into NW sub-tiles (quadrants or halves), one per
// wave; each lane owns PPT pixels of its wave's sub-tile (a column of rows spaced 64/SW apart).  The tile's
// depth-sorted list is staged 64*NW records at a time into LDS (one record per thread, gathered by record
// id).  Each record carries its exact pixel rectangle, so every wave compacts the staged batch down to the
// records whose rectangle meets its sub-tile and loops over those only.  A record is skipped only where its
// rectangle misses the pixel, where alpha < exp(-1/2)/255 holds, so the result is the same bit for bit as
// walking the whole list.  This matters for coarse pyramid levels, where a tile holds tens of thousands of
// sub-pixel Gaussians of which each pixel sees a few percent.
//
// The backward walks the list in the same front-to-back order as the forward.  With the forward's final
// values C, D, V of a pixel and its upstream gradient g, the gradient of alpha_i is
//   dL/dalpha_i = T_i q_i - (S - P_i) / (1 - alpha_i),   q_i = g . (c_i, d_i, 1),
//   S = g . (C, D, V),  P_i = sum_{j <= i} alpha_j T_j q_j,
// i.e. what lies behind record i is S - P_i.  No per-pixel state is stored between the forward and the
// backward (the fused variant recomputes C, D, V with a first sweep in the same kernel), and the skip / stop
// decisions are re-evaluated with the forward's arithmetic.  Per-record gradients of a wave are summed with
// DPP before one atomic add per value, unless at most four lanes contributed (then each adds its own).
#include "common.h"

namespace {

using gsk::DevOpts;

template <int TW, int TH, int NW>
struct Geo {
  static constexpr int SX = NW == 4 ? 2 : 1;  // sub-tiles across
  static constexpr int SY = NW / SX;          // sub-tiles down
  static constexpr int SW = TW / SX;          // sub-tile width
  static constexpr int SH = TH / SY;          // sub-tile height
  static constexpr int RPP = 64 / SW;         // rows covered by the 64 lanes at once
  static constexpr int PPT = SH / RPP;        // pixels per lane
  static constexpr int BATCH = 64 * NW;       // records staged per round
  static_assert(SW == 8 || SW == 16 || SW == 32, "sub-tile width");
  static_assert(PPT >= 1 && PPT * RPP == SH, "sub-tile height");
};

template <int BATCH, int NW>
struct Stage {
  float4 A[BATCH], B[BATCH], C[BATCH];
  int32_t r[BATCH];
  uint8_t mask[BATCH];
  uint16_t list[NW][BATCH];
  int4 wbox[NW][BATCH];  // per wave, in list order: pixel box as (x0, x1 - x0, y0, y1 - y0)
  int cover[NW];         // pixels of the wave's sub-tile covered by the boxes of its list, summed
};

// Per-pixel "stream" walk, used for a wave's batch when the boxes of its records cover under a quarter of its
// (record, pixel) pairs - the coarse pyramid levels, where a tile holds tens of thousands of sub-pixel
// Gaussians.  Each lane tests the boxes of the next 64 records of its wave's list against its own pixel and
// walks only the records that cover it, in list order.  It meets exactly the records that can contribute, in
// the same order, so the result is the same bit for bit as the dense walk; it only skips work.
__device__ __forceinline__ uint64_t cover_mask(const int4* __restrict__ boxes, int nc, int px, int py) {
  uint64_t m = 0;
#pragma unroll 8
  for (int k = 0; k < nc; ++k) {
    const int4 b = boxes[k];
    const bool c = (unsigned)(px - b.x) <= (unsigned)b.y && (unsigned)(py - b.z) <= (unsigned)b.w;
    m |= (uint64_t)c << k;
  }
  return m;
}

struct TileCtx {
  int view, W, H, tx0, ty0;  // view and tile origin (pixels)
  int px, py0;               // this lane's column and first row
  int wave, lane;
  int64_t pix_off;
  float weight;
};

// Workgroup b composites tile order[b]: tiles in descending order of list length, so the longest start first
// and are dealt round-robin over the XCDs.
template <class G>
__device__ __forceinline__ bool tile_setup(const gs_camera* __restrict__ cams, int V, int n_tiles,
                                           const int32_t* __restrict__ order, TileCtx& t, int& tile) {
  if ((int)blockIdx.x >= n_tiles) return false;
  tile = order[blockIdx.x];
  t.view = gsk::view_of_tile(cams, V, tile);
  const gs_camera& c = cams[t.view];
  const int lt = tile - c.tile_offset;
  const int tyi = lt / c.tiles_x, txi = lt - tyi * c.tiles_x;
  t.wave = threadIdx.x >> 6;
  t.lane = threadIdx.x & 63;
  t.W = c.width;
  t.H = c.height;
  t.tx0 = txi * (G::SW * G::SX);
  t.ty0 = tyi * (G::SH * G::SY);
  t.px = t.tx0 + (t.wave % G::SX) * G::SW + (t.lane % G::SW);
  t.py0 = t.ty0 + (t.wave / G::SX) * G::SH + t.lane / G::SW;
  t.pix_off = c.pixel_offset;
  t.weight = c.loss_weight;
  return true;
}

// One record at one pixel: returns false if skipped (power > 0 or alpha < alpha_min).  The operation
// sequence is fixed (contraction off, explicit fma) so that every kernel and every tile shape computes the
// same bits for the same (record, pixel) pair, whatever the compiler shares between a lane's pixels.
__device__ __forceinline__ bool eval_pair(const float4& A, const float4& B, float fx, float fy, const DevOpts& op,
                                          float& alpha, float& G, bool& clamped, float& dx, float& dy) {
#pragma clang fp contract(off)
  dx = A.x - fx;
  dy = A.y - fy;
  const float adx2 = (B.x * dx) * dx;
  const float quad = __builtin_fmaf(B.z * dy, dy, adx2);  // a dx^2 + c dy^2
  const float bxy = (B.y * dx) * dy;
  const float power = __builtin_fmaf(-0.5f, quad, -bxy);  // -(a dx^2 + c dy^2)/2 - b dx dy
  if (power > 0.f) return false;
  G = __expf(power);
  const float oG = A.w * G;
  clamped = oG > op.alpha_max;
  alpha = clamped ? op.alpha_max : oG;
  return alpha >= op.alpha_min;
}

__device__ __forceinline__ void unpack_rect(const float4& C, int& x0, int& x1, int& y0, int& y1) {
  const int a = __float_as_int(C.z), b = __float_as_int(C.w);
  x0 = a & 0xffff;
  x1 = (int)((unsigned)a >> 16);
  y0 = b & 0xffff;
  y1 = (int)((unsigned)b >> 16);
}

// Stage records [b0, b0 + nb) of the tile list, then build each wave's list of the staged records whose
// pixel rectangle meets its sub-tile.  Returns the length of this wave's list.  Ends with a barrier.
template <class G, class S>
__device__ __forceinline__ int stage_and_compact(S& s, const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                                 int b0, int nb, const TileCtx& t, int& cover) {
  const int tid = threadIdx.x;
  uint32_t m = 0;
  int4 box = make_int4(0, 0, 0, 0);
  if (tid < G::SX * G::SY) s.cover[tid] = 0;
  if (tid < nb) {
    const int r = vals[b0 + tid];
    const float4 A = rec[3 * (int64_t)r], B = rec[3 * (int64_t)r + 1], C = rec[3 * (int64_t)r + 2];
    s.A[tid] = A;
    s.B[tid] = B;
    s.C[tid] = C;
    s.r[tid] = r;
    int x0, x1, y0, y1;
    unpack_rect(C, x0, x1, y0, y1);
    box = make_int4(x0, x1 - x0, y0, y1 - y0);
#pragma unroll
    for (int w = 0; w < G::SX * G::SY; ++w) {
      const int sx0 = t.tx0 + (w % G::SX) * G::SW, sy0 = t.ty0 + (w / G::SX) * G::SH;
      if (x0 <= sx0 + G::SW - 1 && x1 >= sx0 && y0 <= sy0 + G::SH - 1 && y1 >= sy0) m |= 1u << w;
    }
  }
  s.mask[tid] = (uint8_t)m;
  __syncthreads();
  if (m) {
#pragma unroll
    for (int w = 0; w < G::SX * G::SY; ++w) {
      if (!((m >> w) & 1)) continue;
      const int sx0 = t.tx0 + (w % G::SX) * G::SW, sy0 = t.ty0 + (w / G::SX) * G::SH;
      const int ox = min(box.x + box.y, sx0 + G::SW - 1) - max(box.x, sx0) + 1;
      const int oy = min(box.z + box.w, sy0 + G::SH - 1) - max(box.z, sy0) + 1;
      atomicAdd(&s.cover[w], ox * oy);
    }
  }
  int cnt = 0;
  const uint64_t lt = gsk::lanemask_lt();
#pragma unroll
  for (int c = 0; c < G::BATCH / 64; ++c) {
    const int j = c * 64 + t.lane;
    const bool bit = (s.mask[j] >> t.wave) & 1;
    const uint64_t bal = __ballot(bit);
    if (bit) {
      const int p = cnt + __popcll(bal & lt);
      s.list[t.wave][p] = (uint16_t)j;
      const float4 C = s.C[j];
      int x0, x1, y0, y1;
      unpack_rect(C, x0, x1, y0, y1);
      s.wbox[t.wave][p] = make_int4(x0, x1 - x0, y0, y1 - y0);
    }
    cnt += __popcll(bal);
  }
  __syncthreads();
  cover = s.cover[t.wave];
  return cnt;
}

// Stream walk only where one lane holds one pixel and the wave's records cover under a fraction (default a
// quarter) of its pairs.
template <class G>
__device__ __forceinline__ bool use_stream(int cnt, int cover, const DevOpts& op) {
  return G::PPT == 1 && cnt >= 64 && (float)cover < op.stream_cover * (float)(G::SW * G::SH * cnt);
}

// Forward sweep of one tile for this lane's pixels (shared by the forward kernel and the fused backward).
template <class G, class S>
__device__ __forceinline__ void forward_sweep(S& s, const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                              int2 rg, const TileCtx& t, const DevOpts& op, float* T, float* Cr,
                                              float* Cg, float* Cb, float* D, float* Vs) {
  constexpr int PPT = G::PPT, RPP = G::RPP;
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
  // one (record, pixel) step of the front-to-back walk
  auto step = [&](const float4& A, const float4& B, const float4& C, int k) {
#pragma clang fp contract(off)
    float alpha, Gv, dx, dy;
    bool cl;
    if (!eval_pair(A, B, fx, fy[k], op, alpha, Gv, cl, dx, dy)) return;
    const float Tn = T[k] * (1.f - alpha);
    if (Tn < op.t_min) {
      live[k] = false;
      return;
    }
    const float w = alpha * T[k];
    Cr[k] = __builtin_fmaf(w, B.w, Cr[k]);
    Cg[k] = __builtin_fmaf(w, C.x, Cg[k]);
    Cb[k] = __builtin_fmaf(w, C.y, Cb[k]);
    D[k] = __builtin_fmaf(w, A.z, D[k]);
    Vs[k] = Vs[k] + w;
    T[k] = Tn;
  };
  for (int b0 = rg.x; b0 < rg.y; b0 += G::BATCH) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < PPT; ++k) any |= live[k];
    if (!__syncthreads_or(any)) break;
    const int nb = min(G::BATCH, rg.y - b0);
    int cover;
    const int cnt = stage_and_compact<G>(s, rec, vals, b0, nb, t, cover);
    if (__ballot(any) == 0) continue;
    if (use_stream<G>(cnt, cover, op)) {
      const int py = t.py0;
      for (int c0 = 0; c0 < cnt; c0 += 64) {
        uint64_t m = live[0] ? cover_mask(&s.wbox[t.wave][c0], min(64, cnt - c0), t.px, py) : 0ull;
        // the next covered record is fetched while the current one is composited
        int jn = s.list[t.wave][c0 + (m ? __builtin_ctzll(m) : 0)];
        float4 An = s.A[jn], Bn = s.B[jn], Cn = s.C[jn];
        while (__ballot(m != 0)) {
          if (m) {
            const float4 A = An, B = Bn, C = Cn;
            m &= m - 1;
            jn = s.list[t.wave][c0 + (m ? __builtin_ctzll(m) : 0)];
            An = s.A[jn];
            Bn = s.B[jn];
            Cn = s.C[jn];
            step(A, B, C, 0);
            if (!live[0]) m = 0;
          }
        }
      }
    } else {
      // records i + 1 (data) and i + 2 (index) are fetched while record i is composited
      float4 An = s.A[s.list[t.wave][0]], Bn = s.B[s.list[t.wave][0]], Cn = s.C[s.list[t.wave][0]];
      int jn2 = s.list[t.wave][cnt > 1 ? 1 : 0];
      for (int i = 0; i < cnt; ++i) {
        const float4 A = An, B = Bn, C = Cn;
        An = s.A[jn2];
        Bn = s.B[jn2];
        Cn = s.C[jn2];
        jn2 = s.list[t.wave][i + 2 < cnt ? i + 2 : 0];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
          if (live[k]) step(A, B, C, k);
      }
    }
  }
}

template <int TW, int TH, int NW>
__global__ __launch_bounds__(64 * NW) void k_render_fwd(const float4* __restrict__ rec,
                                                        const int32_t* __restrict__ vals,
                                                        const int2* __restrict__ range,
                                                        const gs_camera* __restrict__ cams, int V, int n_tiles, const int32_t* __restrict__ order,
                                                        DevOpts op, float* __restrict__ out_rgb,
                                                        float* __restrict__ out_depth, float* __restrict__ out_vis) {
  using G = Geo<TW, TH, NW>;
  constexpr int PPT = G::PPT, RPP = G::RPP;
  __shared__ Stage<G::BATCH, NW> s;
  TileCtx t;
  int tile;
  if (!tile_setup<G>(cams, V, n_tiles, order, t, tile)) return;
  float T[PPT], Cr[PPT], Cg[PPT], Cb[PPT], D[PPT], Vs[PPT];
  forward_sweep<G>(s, rec, vals, range[tile], t, op, T, Cr, Cg, Cb, D, Vs);
  const int64_t P = (int64_t)t.W * t.H;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int py = t.py0 + k * RPP;
    if (t.px < t.W && py < t.H) {
      const int64_t i = (int64_t)py * t.W + t.px;
      out_rgb[3 * t.pix_off + i] = __builtin_fmaf(T[k], op.bg[0], Cr[k]);
      out_rgb[3 * t.pix_off + P + i] = __builtin_fmaf(T[k], op.bg[1], Cg[k]);
      out_rgb[3 * t.pix_off + 2 * P + i] = __builtin_fmaf(T[k], op.bg[2], Cb[k]);
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

template <int TW, int TH, int NW, bool HAVE_FWD, bool LOSS>
__global__ __launch_bounds__(64 * NW) void k_render_bwd(const float4* __restrict__ rec,
                                                        const int32_t* __restrict__ vals,
                                                        const int2* __restrict__ range,
                                                        const gs_camera* __restrict__ cams, int V, int n_tiles, const int32_t* __restrict__ order,
                                                        DevOpts op, BwdArgs a) {
  using G = Geo<TW, TH, NW>;
  constexpr int PPT = G::PPT, RPP = G::RPP;
  __shared__ Stage<G::BATCH, NW> s;
  TileCtx t;
  int tile;
  if (!tile_setup<G>(cams, V, n_tiles, order, t, tile)) return;
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
    forward_sweep<G>(s, rec, vals, rg, t, op, T, Cf, Gf, Bf, Df, Vf);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      Cf[k] = __builtin_fmaf(T[k], op.bg[0], Cf[k]);
      Gf[k] = __builtin_fmaf(T[k], op.bg[1], Gf[k]);
      Bf[k] = __builtin_fmaf(T[k], op.bg[2], Bf[k]);
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
    if (t.lane == 63) gsk::atomic_add_f32(a.loss, ls);
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
  // per-record gradient partials of the stream walk, summed in LDS and flushed once per batch
  __shared__ float gacc[G::BATCH][10];
  __shared__ int gtouch[G::BATCH];
  for (int i = threadIdx.x; i < G::BATCH; i += 64 * NW) {
    gtouch[i] = 0;
#pragma unroll
    for (int q = 0; q < 10; ++q) gacc[i][q] = 0.f;
  }
  // one (record, pixel) step of the front-to-back walk: returns true if the pair contributed, with its
  // 10 partial derivatives in acc (added, not overwritten)
  auto step = [&](const float4& A, const float4& B, const float4& C, int k, float* acc) -> bool {
    float alpha, Gv, dx, dy;
    bool cl;
    if (!eval_pair(A, B, fx, fy[k], op, alpha, Gv, cl, dx, dy)) return false;
    const float Tn = T[k] * (1.f - alpha);
    if (Tn < op.t_min) {
      live[k] = false;
      return false;
    }
    const float w = alpha * T[k];
    const float qv = gr[k] * B.w + gg[k] * C.x + gb[k] * C.y + gd[k] * A.z + gv[k];
    Pp[k] += w * qv;
    const float dalpha = T[k] * qv - (S[k] - Pp[k]) * __builtin_amdgcn_rcpf(1.f - alpha);
    acc[6] += w * gr[k];
    acc[7] += w * gg[k];
    acc[8] += w * gb[k];
    acc[9] += w * gd[k];
    if (!cl) {
      acc[5] += dalpha * Gv;
      const float dq = dalpha * alpha;
      acc[2] += -0.5f * dx * dx * dq;
      acc[3] += -dx * dy * dq;
      acc[4] += -0.5f * dy * dy * dq;
      acc[0] += -(B.x * dx + B.y * dy) * dq;
      acc[1] += -(B.z * dy + B.y * dx) * dq;
    }
    T[k] = Tn;
    return true;
  };
  for (int b0 = rg.x; b0 < rg.y; b0 += G::BATCH) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < PPT; ++k) any |= live[k];
    if (!__syncthreads_or(any)) break;
    const int nb = min(G::BATCH, rg.y - b0);
    int cover;
    const int cnt = stage_and_compact<G>(s, rec, vals, b0, nb, t, cover);
    if (__ballot(any) != 0) {
      if (use_stream<G>(cnt, cover, op)) {
        for (int c0 = 0; c0 < cnt; c0 += 64) {
          uint64_t m = live[0] ? cover_mask(&s.wbox[t.wave][c0], min(64, cnt - c0), t.px, t.py0) : 0ull;
          int jn = s.list[t.wave][c0 + (m ? __builtin_ctzll(m) : 0)];
          float4 An = s.A[jn], Bn = s.B[jn], Cn = s.C[jn];
          while (__ballot(m != 0)) {
            if (m) {
              const float4 A = An, B = Bn, C = Cn;
              const int j = jn;
              m &= m - 1;
              jn = s.list[t.wave][c0 + (m ? __builtin_ctzll(m) : 0)];
              An = s.A[jn];
              Bn = s.B[jn];
              Cn = s.C[jn];
              float acc[10];
#pragma unroll
              for (int q = 0; q < 10; ++q) acc[q] = 0.f;
              if (step(A, B, C, 0, acc)) {
#pragma unroll
                for (int q = 0; q < 10; ++q) atomicAdd(&gacc[j][q], acc[q]);
                gtouch[j] = 1;
              }
              if (!live[0]) m = 0;
            }
          }
        }
      } else {
        int jn = s.list[t.wave][0];
        float4 An = s.A[jn], Bn = s.B[jn], Cn = s.C[jn];
        int jn2 = s.list[t.wave][cnt > 1 ? 1 : 0];
        for (int i = 0; i < cnt; ++i) {
          const float4 A = An, B = Bn, C = Cn;
          const int j = jn;
          jn = jn2;
          An = s.A[jn];
          Bn = s.B[jn];
          Cn = s.C[jn];
          jn2 = s.list[t.wave][i + 2 < cnt ? i + 2 : 0];
          float acc[10];
#pragma unroll
          for (int q = 0; q < 10; ++q) acc[q] = 0.f;
          bool hit = false;
#pragma unroll
          for (int k = 0; k < PPT; ++k)
            if (live[k]) hit |= step(A, B, C, k, acc);
          const uint64_t hits = __ballot(hit);
          if (hits != 0) {
            float* dst = a.rgrad + 12 * (int64_t)s.r[j];
            if (__popcll(hits) <= 4) {
              // few contributing lanes: each adds its own partials (no wave reduction)
              if (hit) {
#pragma unroll
                for (int q = 0; q < 10; ++q) gsk::atomic_add_f32(dst + q, acc[q]);
              }
            } else {
#pragma unroll
              for (int q = 0; q < 10; ++q) {
                const float sum = gsk::wave_sum_last(acc[q]);
                if (t.lane == 63) gsk::atomic_add_f32(dst + q, sum);
              }
            }
          }
        }
      }
    }
    // flush the LDS partials of this batch (records touched by a stream walk)
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += 64 * NW) {
      if (gtouch[i]) {
        float* dst = a.rgrad + 12 * (int64_t)s.r[i];
#pragma unroll
        for (int q = 0; q < 10; ++q) {
          gsk::atomic_add_f32(dst + q, gacc[i][q]);
          gacc[i][q] = 0.f;
        }
        gtouch[i] = 0;
      }
    }
  }
}

// Work counts of the forward: pairs evaluated (pixel inside the record's pixel rectangle, up to the
// pixel's stop) and pairs contributing.  Independent of the tile shape; diagnostic.
template <int TW, int TH, int NW>
__global__ __launch_bounds__(64 * NW) void k_count_pairs(const float4* __restrict__ rec,
                                                         const int32_t* __restrict__ vals,
                                                         const int2* __restrict__ range,
                                                         const gs_camera* __restrict__ cams, int V, int n_tiles, const int32_t* __restrict__ order,
                                                         DevOpts op, unsigned long long* __restrict__ counts) {
  using G = Geo<TW, TH, NW>;
  constexpr int PPT = G::PPT, RPP = G::RPP;
  __shared__ Stage<G::BATCH, NW> s;
  TileCtx t;
  int tile;
  if (!tile_setup<G>(cams, V, n_tiles, order, t, tile)) return;
  const int2 rg = range[tile];
  bool live[PPT];
  float fy[PPT], T[PPT];
  const float fx = (float)t.px + 0.5f;
  unsigned long long ev = 0, co = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int py = t.py0 + k * RPP;
    live[k] = t.px < t.W && py < t.H;
    fy[k] = (float)py + 0.5f;
    T[k] = 1.f;
  }
  for (int b0 = rg.x; b0 < rg.y; b0 += G::BATCH) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < PPT; ++k) any |= live[k];
    if (!__syncthreads_or(any)) break;
    const int nb = min(G::BATCH, rg.y - b0);
    int cover;
    const int cnt = stage_and_compact<G>(s, rec, vals, b0, nb, t, cover);
    for (int i = 0; i < cnt; ++i) {
      const int j = s.list[t.wave][i];
      const float4 A = s.A[j], B = s.B[j], C = s.C[j];
      int x0, x1, y0, y1;
      unpack_rect(C, x0, x1, y0, y1);
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if (!live[k]) continue;
        const int py = t.py0 + k * RPP;
        if (t.px < x0 || t.px > x1 || py < y0 || py > y1) continue;
        ++ev;
        float alpha, Gv, dx, dy;
        bool cl;
        if (!eval_pair(A, B, fx, fy[k], op, alpha, Gv, cl, dx, dy)) continue;
        const float Tn = T[k] * (1.f - alpha);
        if (Tn < op.t_min) {
          live[k] = false;
          continue;
        }
        ++co;
        T[k] = Tn;
      }
    }
  }
  atomicAdd(counts, ev);
  atomicAdd(counts + 1, co);
}

// Valid LiDAR-depth pixels per view: grid-stride per view, one atomic per block.
__global__ __launch_bounds__(256) void k_count_valid(const float* __restrict__ tgt_depth,
                                                     const gs_camera* __restrict__ cams,
                                                     int32_t* __restrict__ n_valid) {
  __shared__ int sh;
  if (threadIdx.x == 0) sh = 0;
  __syncthreads();
  const int v = blockIdx.y;
  const gs_camera& c = cams[v];
  const int64_t P = (int64_t)c.width * c.height;
  int cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x)
    cnt += tgt_depth[c.pixel_offset + i] > 0.f;
  atomicAdd(&sh, cnt);
  __syncthreads();
  if (threadIdx.x == 0 && sh) atomicAdd(n_valid + v, sh);
}

template <int TW, int TH, int NW>
hipError_t launch_fwd(const gs_frame& f, const DevOpts& op, const gs_images& out, hipStream_t st) {
  const int sorted = f.sort_passes & 1;
  k_render_fwd<TW, TH, NW><<<f.n_tiles, 64 * NW, 0, st>>>(
      reinterpret_cast<const float4*>(f.rec), f.vals[sorted], reinterpret_cast<const int2*>(f.tile_range), f.cams,
      f.n_views, f.n_tiles, f.tile_order, op, out.rgb, out.depth, out.vis);
  return hipGetLastError();
}

template <int TW, int TH, int NW>
hipError_t launch_bwd(const gs_frame& f, const DevOpts& op, bool have_fwd, bool loss, const BwdArgs& a,
                      hipStream_t st) {
  const int sorted = f.sort_passes & 1;
  const auto* rec = reinterpret_cast<const float4*>(f.rec);
  const auto* rng = reinterpret_cast<const int2*>(f.tile_range);
  const int nb = f.n_tiles, bs = 64 * NW;
  const int32_t* vals = f.vals[sorted];
  if (have_fwd && loss)
    k_render_bwd<TW, TH, NW, true, true><<<nb, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, nb, f.tile_order, op, a);
  else if (have_fwd)
    k_render_bwd<TW, TH, NW, true, false><<<nb, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, nb, f.tile_order, op,
                                                             a);
  else if (loss)
    k_render_bwd<TW, TH, NW, false, true><<<nb, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, nb, f.tile_order, op,
                                                             a);
  else
    k_render_bwd<TW, TH, NW, false, false><<<nb, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, nb, f.tile_order,
                                                              op, a);
  return hipGetLastError();
}

template <int TW, int TH, int NW>
hipError_t launch_count(const gs_frame& f, const DevOpts& op, unsigned long long* counts, hipStream_t st) {
  const int sorted = f.sort_passes & 1;
  k_count_pairs<TW, TH, NW><<<f.n_tiles, 64 * NW, 0, st>>>(
      reinterpret_cast<const float4*>(f.rec), f.vals[sorted], reinterpret_cast<const int2*>(f.tile_range), f.cams,
      f.n_views, f.n_tiles, f.tile_order, op, counts);
  return hipGetLastError();
}

}  // namespace

namespace gs_launch {

// Tile shape and waves per tile (o.waves_per_tile; 0 picks 4 where the shape allows it).
#define GS_TILE_DISPATCH(FN, ...)                                 \
  do {                                                            \
    const int nw = o.waves_per_tile;                              \
    if (o.tile_w == 16 && o.tile_h == 16) {                       \
      if (nw == 1) return FN<16, 16, 1>(__VA_ARGS__);             \
      if (nw == 2) return FN<16, 16, 2>(__VA_ARGS__);             \
      return FN<16, 16, 4>(__VA_ARGS__);                          \
    }                                                             \
    if (o.tile_w == 16 && o.tile_h == 8) {                        \
      if (nw == 1) return FN<16, 8, 1>(__VA_ARGS__);              \
      return FN<16, 8, 2>(__VA_ARGS__);                           \
    }                                                             \
    if (o.tile_w == 8 && o.tile_h == 8) return FN<8, 8, 1>(__VA_ARGS__); \
    if (o.tile_w == 32 && o.tile_h == 8) {                        \
      if (nw == 1) return FN<32, 8, 1>(__VA_ARGS__);              \
      if (nw == 2) return FN<32, 8, 2>(__VA_ARGS__);              \
      return FN<32, 8, 4>(__VA_ARGS__);                           \
    }                                                             \
    if (o.tile_w == 32 && o.tile_h == 16) {                       \
      if (nw == 1) return FN<32, 16, 1>(__VA_ARGS__);             \
      if (nw == 2) return FN<32, 16, 2>(__VA_ARGS__);             \
      return FN<32, 16, 4>(__VA_ARGS__);                          \
    }                                                             \
    return hipErrorInvalidValue;                                  \
  } while (0)

hipError_t render_fwd(const gs_frame& f, const gs_opts& o, const gs_images& out, hipStream_t st) {
  const DevOpts op = gsk::dev_opts(o);
  GS_TILE_DISPATCH(launch_fwd, f, op, out, st);
}

hipError_t count_pairs(const gs_frame& f, const gs_opts& o, unsigned long long* counts, hipStream_t st) {
  const DevOpts op = gsk::dev_opts(o);
  GS_TILE_DISPATCH(launch_count, f, op, counts, st);
}

hipError_t count_valid(const gs_frame& f, const float* tgt_depth, int64_t max_pixels, hipStream_t st) {
  hipError_t e = fill_i32(f.counters + 2, 0, f.n_views, st);
  if (e != hipSuccess) return e;
  int64_t bx = (max_pixels + 256 * 32 - 1) / (256 * 32);
  if (bx < 1) bx = 1;
  dim3 grid((unsigned)bx, (unsigned)f.n_views);
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
