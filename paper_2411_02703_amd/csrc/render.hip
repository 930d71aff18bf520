// Per-tile front-to-back compositing of colour, depth and visibility (LVI-GS Section III-B,
// eqs. Cp, Dp, Vp with the alpha of eq. alpha) and its backward.
//
// One workgroup per tile.  The tile is split into 8x8 sub-tiles, one wave64 each, one pixel per lane; a
// sub-tile is walked as BW x BW blocks (BW = 2: sixteen blocks, one per quad of lanes; BW = 4: four blocks,
// one per 16-lane DPP row; BW = 8: the whole wave).  The tile's depth-sorted list is staged in rounds of
// DEPTH records per thread into LDS; the records of the next round are fetched into registers while the
// current one is composited.  Each staged record carries its exact pixel rectangle (every pixel outside it
// has alpha < exp(-1/2)/255, so it would be skipped anyway), and sets its bit in the mask of every block its
// rectangle meets.  Each block then walks the set bits of its mask in list order, in lock-step (one record
// per step for the block's lanes, read from LDS by broadcast); the result is the same bit for bit for every
// block size, since a record is skipped only where its rectangle misses the pixel.  Small blocks waste fewer
// lanes on records that cover part of a sub-tile (coarse pyramid levels hold many sub-pixel Gaussians) and
// sum gradients over fewer lanes (2 or 4 DPP steps instead of 6).
//
// The backward walks the list in the same front-to-back order as the forward.  With the forward's final
// values C, D, V of a pixel and its upstream gradient g, the gradient of alpha_i is
//   dL/dalpha_i = T_i q_i - (S - P_i) / (1 - alpha_i),   q_i = g . (c_i, d_i, 1),
//   S = g . (C, D, V),  P_i = sum_{j <= i} alpha_j T_j q_j,
// i.e. what lies behind record i is S - P_i.  No per-pixel state is stored between the forward and the
// backward (the fused variant recomputes C, D, V with a first sweep in the same kernel), and the skip / stop
// decisions are re-evaluated with the forward's arithmetic.  Per-record partial derivatives are summed in
// LDS (a DPP wave sum first when every contributing lane of the wave is on the same record) and added to
// the record's gradient in HBM once per round.
#include "common.h"

namespace {

using gsk::DevOpts;

template <int TW, int TH, int DEPTH, int BW_ = 4>
struct Geo {
  static constexpr int SX = TW / 8;            // sub-tiles across
  static constexpr int SY = TH / 8;            // sub-tiles down
  static constexpr int NW = SX * SY;           // waves per tile
  static constexpr int NT = 64 * NW;           // threads = pixels of the tile
  static constexpr int BATCH = NT * DEPTH;     // records staged per round
  static constexpr int GS = BATCH + 1;         // LDS row stride of the gradient sums (odd: rows in distinct banks)
  static constexpr int MC = BATCH / 32;        // 32-bit mask words per block
  static constexpr int BW = BW_;               // block width (pixels)
  static constexpr int BS = 8 / BW;            // blocks across a sub-tile
  static constexpr int BPW = BS * BS;          // blocks per wave
  static constexpr int BL = BW * BW;           // lanes per block
  static constexpr int NB = NW * BPW;          // blocks per tile
  static_assert(TW % 8 == 0 && TH % 8 == 0 && NW >= 1 && NW <= 4, "tile shape");
  static_assert(DEPTH == 1 || DEPTH == 2, "batch depth");
  static_assert(BW == 2 || BW == 4 || BW == 8, "block width");
};

template <class G>
struct Stage {
  float4 A[G::BATCH], B[G::BATCH], C[G::BATCH];
  int32_t slot[G::BATCH];       // backward sweeps: first partial slot of each staged record
  uint32_t bm[G::MC][G::NB];    // per block: staged records whose rectangle meets it
  int alive[G::NW];             // per wave: a pixel is still live
};

struct TileCtx {
  int view, W, H, tx0, ty0;  // view and tile origin (pixels)
  int px, py;                // this lane's pixel
  int wave, lane;
  int blk, blk_lane0;        // this lane's block in the tile, and the block's first lane in the wave
  int64_t pix_off;
  float weight;
  bool inside;               // pixel inside the image
};

// Geometry of this thread's pixel in global tile `tile`.
template <class G>
__device__ __forceinline__ void tile_at(const gs_camera* __restrict__ cams, int V, int tile, TileCtx& t) {
  t.view = gsk::view_of_tile(cams, V, tile);
  const gs_camera& c = cams[t.view];
  const int lt = tile - c.tile_offset;
  const int tyi = lt / c.tiles_x, txi = lt - tyi * c.tiles_x;
  t.wave = threadIdx.x >> 6;
  t.lane = threadIdx.x & 63;
  t.W = c.width;
  t.H = c.height;
  t.tx0 = txi * (8 * G::SX);
  t.ty0 = tyi * (8 * G::SY);
  // lanes of a block are consecutive; blocks of a wave in row-major order over its sub-tile
  const int r = t.lane / G::BL, p = t.lane % G::BL;
  t.blk = t.wave * G::BPW + r;
  t.blk_lane0 = r * G::BL;
  t.px = t.tx0 + (t.wave % G::SX) * 8 + (r % G::BS) * G::BW + p % G::BW;
  t.py = t.ty0 + (t.wave / G::SX) * 8 + (r / G::BS) * G::BW + p / G::BW;
  t.pix_off = c.pixel_offset;
  t.weight = fmaxf(c.loss_weight, 0.f);  // an inactive view (weight < 0) adds nothing to the loss
  t.inside = t.px < t.W && t.py < t.H;
}

// Workgroup b composites tile order[b]: tiles in descending order of list length, so the longest start first.
template <class G>
__device__ __forceinline__ bool tile_setup(const gs_camera* __restrict__ cams, int V, int n_tiles,
                                           const int32_t* __restrict__ order, TileCtx& t, int& tile) {
  if ((int)blockIdx.x >= n_tiles) return false;
  tile = order[blockIdx.x];
  tile_at<G>(cams, V, tile, t);
  return true;
}

// One record at one pixel: returns false if skipped (power > 0 or alpha < alpha_min).  The operation
// sequence is fixed (contraction off, explicit fma) so that every kernel and every tile shape computes the
// same bits for the same (record, pixel) pair.  Everything is computed whatever the outcome (no branch: in a
// lock-step walk some lane of the wave nearly always takes every path, and the branches only add exec-mask
// work); G and alpha are meaningful only where the result is true.
__device__ __forceinline__ bool eval_pair(const float4& A, const float4& B, float fx, float fy, const DevOpts& op,
                                          float& alpha, float& G, bool& clamped, float& dx, float& dy) {
#pragma clang fp contract(off)
  dx = A.x - fx;
  dy = A.y - fy;
  const float adx2 = (B.x * dx) * dx;
  const float quad = __builtin_fmaf(B.z * dy, dy, adx2);  // a dx^2 + c dy^2
  const float bxy = (B.y * dx) * dy;
  const float power = __builtin_fmaf(-0.5f, quad, -bxy);  // -(a dx^2 + c dy^2)/2 - b dx dy
  G = __expf(power);
  const float oG = A.w * G;
  clamped = oG > op.alpha_max;
  alpha = fminf(oG, op.alpha_max);  // the same value as clamped ? alpha_max : oG (oG is finite)
  return !(power > 0.f) && alpha >= op.alpha_min;
}

__device__ __forceinline__ void unpack_rect(const float4& C, int& x0, int& x1, int& y0, int& y1) {
  const int a = __float_as_int(C.z), b = __float_as_int(C.w);
  x0 = a & 0xffff;
  x1 = (int)((unsigned)a >> 16);
  y0 = b & 0xffff;
  y1 = (int)((unsigned)b >> 16);
}

// Records of the tile list in flight, per thread: the round held in registers (ids r, data A, B, C and, for a
// backward sweep, the record's first partial slot sl) and the ids of the round after it (rn, -1 past the end).
// Loads are unconditional (an absent record reads record 0, which is never used), so nothing waits on them
// until the round is written to LDS.
template <class G, int DEPTH>
__device__ __forceinline__ void fetch_records(const float4* __restrict__ rec, const int32_t* __restrict__ rec_slot,
                                              const int (&r)[DEPTH], float4 (&A)[DEPTH], float4 (&B)[DEPTH],
                                              float4 (&C)[DEPTH], int (&sl)[DEPTH]) {
#pragma unroll
  for (int k = 0; k < DEPTH; ++k) {
    const int64_t ri = max(r[k], 0);
    const float4* p = rec + 3 * ri;
    A[k] = p[0];
    B[k] = p[1];
    C[k] = p[2];
    if (rec_slot) sl[k] = rec_slot[ri];
  }
}

template <class G, int DEPTH>
__device__ __forceinline__ void fetch_ids(const int32_t* __restrict__ vals, int first, int end, int (&ids)[DEPTH]) {
#pragma unroll
  for (int k = 0; k < DEPTH; ++k) {
    const int i = first + k * G::NT + (int)threadIdx.x;
    ids[k] = i < end ? vals[i] : -1;
  }
}

// Write the round held in registers into LDS, then start fetching the round after it (its ids were fetched
// one round earlier) and the ids of the round after that.
template <class G, int DEPTH>
__device__ __forceinline__ void stage_round(Stage<G>& s, const float4* __restrict__ rec,
                                            const int32_t* __restrict__ rec_slot, const int32_t* __restrict__ vals,
                                            int b0, int end, int (&r)[DEPTH], int (&rn)[DEPTH], float4 (&A)[DEPTH],
                                            float4 (&B)[DEPTH], float4 (&C)[DEPTH], int (&sl)[DEPTH]) {
#pragma unroll
  for (int k = 0; k < DEPTH; ++k) {
    const int j = k * G::NT + (int)threadIdx.x;
    s.A[j] = A[k];
    s.B[j] = B[k];
    s.C[j] = C[k];
    if (rec_slot) s.slot[j] = sl[k];
    r[k] = rn[k];
  }
  fetch_records<G, DEPTH>(rec, rec_slot, r, A, B, C, sl);
  fetch_ids<G, DEPTH>(vals, b0 + 2 * G::BATCH, end, rn);
}

// End of a round: every wave publishes whether it still has a live pixel, then the workgroup meets.  Returns
// whether any pixel of the tile is live (the same answer in every thread).
template <class G>
__device__ __forceinline__ bool round_barrier(Stage<G>& s, const TileCtx& t, bool live) {
  const bool wl = __builtin_amdgcn_ballot_w64(live) != 0;
  if (t.lane == 0) s.alive[t.wave] = wl;
  __syncthreads();
  bool any = false;
#pragma unroll
  for (int w = 0; w < G::NW; ++w) any |= s.alive[w] != 0;
  return any;
}

// Clear the block masks.
template <class G>
__device__ __forceinline__ void clear_masks(Stage<G>& s) {
  for (int i = threadIdx.x; i < G::MC * G::NB; i += G::NT) (&s.bm[0][0])[i] = 0u;
}

// Set this thread's staged records in the masks of the blocks they can reach.  Blocks are numbered
// wave-major (the wave's sub-tile, then row-major inside it).
//
// A record passes the skip test at a pixel only where alpha = o G >= alpha_min, i.e. inside its ellipse
// q(d) = a dx^2 + 2 b dx dy + c dy^2 <= k = 2 ln(o / alpha_min).  For each pixel row of the record's rectangle
// the ellipse meets the row's line of pixel centres in an x-interval
//   [(-b dy - sqrt(a k - det dy^2)) / a, (-b dy + sqrt(a k - det dy^2)) / a],   det = a c - b^2,
// and a block is marked iff one of its rows holds a pixel centre in that interval (the union over the block's
// rows is taken as one interval, a superset).  k is widened by 1% + 0.01: with det > 1e-3 a c (else the whole
// rectangle is kept) the FP32 power of the walk is within 0.1% of q, so no pair the walk would accept is
// pruned and the result does not change (the hardware square root and logarithm used here err by a few ulp,
// far inside that widening).
template <class G, int DEPTH>
__device__ __forceinline__ void scatter(Stage<G>& s, const TileCtx& t, const DevOpts& op, int nb) {
  constexpr int GX = 8 * G::SX / G::BW, GY = 8 * G::SY / G::BW;  // blocks across and down the tile
#pragma unroll
  for (int k = 0; k < DEPTH; ++k) {
    const int j = k * G::NT + (int)threadIdx.x;
    if (j >= nb) continue;
    int x0, x1, y0, y1;
    unpack_rect(s.C[j], x0, x1, y0, y1);
    const int gx0 = max(x0 - t.tx0, 0) / G::BW, gx1 = min(x1 - t.tx0, 8 * G::SX - 1) / G::BW;
    const int gy0 = max(y0 - t.ty0, 0) / G::BW, gy1 = min(y1 - t.ty0, 8 * G::SY - 1) / G::BW;
    if (x1 < t.tx0 || y1 < t.ty0 || gx0 >= GX || gy0 >= GY) continue;
    const float4 A = s.A[j], B = s.B[j];
    const float ca = B.x, cb = B.y, cc = B.z;
    const float kq = 2.f * __logf(A.w / op.alpha_min) * 1.01f + 0.01f;
    const float det = ca * cc - cb * cb;
    const bool cull = det > 1e-3f * ca * cc;  // else the whole rectangle is kept
    const float inv_a = 1.f / ca, ak = ca * kq;
    const uint32_t bit = 1u << (j & 31);
    const int wd = j >> 5;
    for (int gy = gy0; gy <= gy1; ++gy) {
      int cx0 = gx0, cx1 = gx1;
      if (cull) {
        // pixel rows of this block row inside the record's rectangle
        const int r0 = max(t.ty0 + gy * G::BW, y0), r1 = min(t.ty0 + gy * G::BW + G::BW - 1, y1);
        int lo = 1 << 30, hi = -(1 << 30);
        for (int yy = r0; yy <= r1; ++yy) {
          const float dy = (float)yy + 0.5f - A.y;
          const float disc = ak - det * dy * dy;
          if (disc < 0.f) continue;
          const float sq = __builtin_amdgcn_sqrtf(disc);  // the hardware root (~1 ulp): k is widened far more
          // pixel columns whose centres px + 0.5 lie in [A.x + xl, A.x + xr]
          const float xl = A.x + (-cb * dy - sq) * inv_a - 0.5f, xr = A.x + (-cb * dy + sq) * inv_a - 0.5f;
          lo = min(lo, (int)ceilf(fminf(fmaxf(xl, -1.f), 65536.f)));
          hi = max(hi, (int)floorf(fminf(fmaxf(xr, -1.f), 65536.f)));
        }
        if (lo > hi) continue;
        cx0 = max(gx0, (max(lo, t.tx0) - t.tx0) / G::BW);
        cx1 = min(gx1, (hi - t.tx0) / G::BW);
        if (hi < t.tx0) continue;
      }
      for (int gx = cx0; gx <= cx1; ++gx) {
        const int b = ((gy / G::BS) * G::SX + gx / G::BS) * G::BPW + (gy % G::BS) * G::BS + gx % G::BS;
        atomicOr(&s.bm[wd][b], bit);
      }
    }
  }
}

// Sum over the lanes of this lane's block (BW = 2: its quad, BW = 4: its 16-lane row, total in every lane of
// the block; BW = 8: the wave, total in lane 63).
template <class G>
__device__ __forceinline__ float block_sum(float x) {
  if (G::BW == 8) return gsk::wave_sum_last(x);
  x += gsk::dpp_f<0xB1>(x);   // quad_perm [1,0,3,2]
  x += gsk::dpp_f<0x4E>(x);   // quad_perm [2,3,0,1]
  if (G::BW == 2) return x;
  x += gsk::dpp_f<0x141>(x);  // row_half_mirror
  x += gsk::dpp_f<0x140>(x);  // row_mirror
  return x;
}

// Index of the lowest set bit of m, 31 if m is 0 (v_ffbl_b32 gives -1 for 0; a plain count of trailing zeros
// adds a clamp to 32).
__device__ __forceinline__ int low_bit_or_31(uint32_t m) {
  int r;
  asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(m));
  return r & 31;
}

// Walk one staged round: every block walks the set bits of its mask in order, its lanes in lock-step, and
// stops once all its pixels have ended.
//   step(j, active, A, B, C, acc) -> contributed   (per lane, branch-free; active = this lane has a record
//                                                   and a live pixel; clears live at the stop)
//   post(j, hit, acc)                              (whole wave, once per step, only if SYNC)
// A lane whose block has run out of records reads slot c * 32 + 31 (every slot of the round is staged, absent
// records as record 0, so its data are finite) and is inactive.
// ENDS: the step can end pixels (stop rule); without it a block's liveness is only checked per mask word.
template <class G, bool SYNC, bool ENDS, class Step, class Post>
__device__ __forceinline__ void walk_round(const Stage<G>& s, const TileCtx& t, bool& live, Step step, Post post) {
  constexpr uint64_t BMASK = G::BL == 64 ? ~0ull : ((1ull << G::BL) - 1);
#pragma unroll 1
  for (int c = 0; c < G::MC; ++c) {
    uint32_t m = ((__builtin_amdgcn_ballot_w64(live) >> t.blk_lane0) & BMASK) ? s.bm[c][t.blk] : 0u;
    if (__builtin_amdgcn_ballot_w64(m != 0) == 0) continue;
    // The block's next record is fetched from LDS while the current one is composited; two register sets
    // take turns (the loop is unrolled by two), so nothing is copied between them.
    int j0 = c * 32 + low_bit_or_31(m), j1 = 0;
    float4 A0 = s.A[j0], B0 = s.B[j0], C0 = s.C[j0], A1, B1, C1;
    auto one = [&](int j, const float4& A, const float4& B, const float4& C, int& jn, float4& An, float4& Bn,
                   float4& Cn, bool check) {
      const bool active = m != 0 && live;
      m &= m - 1;
      jn = c * 32 + low_bit_or_31(m);
      An = s.A[jn];
      Bn = s.B[jn];
      Cn = s.C[jn];
      float acc[10];
      const bool hit = step(j, active, A, B, C, acc);
      if (SYNC) post(j, hit, acc);
      if (ENDS && check && ((__builtin_amdgcn_ballot_w64(live) >> t.blk_lane0) & BMASK) == 0) m = 0;
    };
    auto more = [&]() { return SYNC ? __builtin_amdgcn_ballot_w64(m != 0) != 0 : m != 0; };
    while (more()) {
      one(j0, A0, B0, C0, j1, A1, B1, C1, false);
      if (!more()) break;
      one(j1, A1, B1, C1, j0, A0, B0, C0, true);
    }
  }
}

// All rounds of one tile list: stage (with the next round in flight), hand out, walk.  at_round(b0, go) runs
// in every thread after each round barrier, before the round's LDS is rewritten: b0 is the first record of
// the round about to be staged, go whether it will be (false once the list or every pixel has ended).
// rec_slot: the records' first partial slots, staged with them (backward sweeps), or NULL.
template <class G, int DEPTH, bool SYNC, bool ENDS, class AtRound, class Step, class Post>
__device__ __forceinline__ void sweep(Stage<G>& s, const float4* __restrict__ rec, const int32_t* __restrict__ rec_slot,
                                      const int32_t* __restrict__ vals, int2 rg, const TileCtx& t, const DevOpts& op,
                                      bool& live, AtRound at_round, Step step, Post post) {
  int fr[DEPTH], frn[DEPTH], fs[DEPTH];
  float4 fA[DEPTH], fB[DEPTH], fC[DEPTH];
  fetch_ids<G, DEPTH>(vals, rg.x, rg.y, fr);
  fetch_ids<G, DEPTH>(vals, rg.x + G::BATCH, rg.y, frn);
  fetch_records<G, DEPTH>(rec, rec_slot, fr, fA, fB, fC, fs);
  for (int b0 = rg.x;; b0 += G::BATCH) {
    const bool go = round_barrier<G>(s, t, live) && b0 < rg.y;
    at_round(b0, go);
    if (!go) break;
    const int nb = min(G::BATCH, rg.y - b0);
    clear_masks<G>(s);
    stage_round<G, DEPTH>(s, rec, rec_slot, vals, b0, rg.y, fr, frn, fA, fB, fC, fs);
    __syncthreads();
    scatter<G, DEPTH>(s, t, op, nb);
    __syncthreads();
    walk_round<G, SYNC, ENDS>(s, t, live, step, post);
  }
}

// Forward walk of records [rg.x, rg.y) for this lane's pixel from transmittance T (in/out), adding to the
// partial sums.  STOP applies the stop rule (the pixel ends before a pair would take T below t_min);
// without it the walk multiplies on (the transmittance product of a depth segment).
template <class G, int DEPTH, bool STOP>
__device__ __forceinline__ void forward_walk(Stage<G>& s, const float4* __restrict__ rec,
                                             const int32_t* __restrict__ vals, int2 rg, const TileCtx& t,
                                             const DevOpts& op, bool live, float& T, float& Cr, float& Cg,
                                             float& Cb, float& D, float& Vs) {
  const float fx = (float)t.px + 0.5f, fy = (float)t.py + 0.5f;
  auto step = [&](int, bool active, const float4& A, const float4& B, const float4& C, float*) -> bool {
#pragma clang fp contract(off)
    float alpha, Gv, dx, dy;
    bool cl;
    const bool ok = eval_pair(A, B, fx, fy, op, alpha, Gv, cl, dx, dy) && active;
    const float Tn = T * (1.f - alpha);
    const bool stop = STOP && ok && Tn < op.t_min;
    const bool hit = ok && !stop;
    if (STOP) live = live && !stop;
    // a pair that does not contribute adds w = 0 (colours, depth and T are finite and the sums non-negative,
    // so adding 0 leaves every sum's bits unchanged)
    const float w = hit ? alpha * T : 0.f;
    Cr = __builtin_fmaf(w, B.w, Cr);
    Cg = __builtin_fmaf(w, C.x, Cg);
    Cb = __builtin_fmaf(w, C.y, Cb);
    D = __builtin_fmaf(w, A.z, D);
    Vs = Vs + w;
    T = hit ? Tn : T;
    return hit;
  };
  sweep<G, DEPTH, false, STOP>(s, rec, nullptr, vals, rg, t, op, live, [](int, bool) {}, step,
                               [](int, bool, const float*) {});
}

// Forward sweep of one whole tile for this lane's pixel (forward kernel and fused backward).
template <class G, int DEPTH>
__device__ __forceinline__ void forward_sweep(Stage<G>& s, const float4* __restrict__ rec,
                                              const int32_t* __restrict__ vals, int2 rg, const TileCtx& t,
                                              const DevOpts& op, float& T, float& Cr, float& Cg, float& Cb,
                                              float& D, float& Vs) {
  T = 1.f;
  Cr = Cg = Cb = D = Vs = 0.f;
  forward_walk<G, DEPTH, true>(s, rec, vals, rg, t, op, t.inside, T, Cr, Cg, Cb, D, Vs);
}

// Final values of this lane's pixel (background behind transmittance T) into the planar images.
__device__ __forceinline__ void write_pixel(const TileCtx& t, const DevOpts& op, float T, float Cr, float Cg, float Cb,
                                            float D, float Vs, float* __restrict__ out_rgb,
                                            float* __restrict__ out_depth, float* __restrict__ out_vis) {
  if (!t.inside) return;
  const int64_t P = (int64_t)t.W * t.H;
  const int64_t i = (int64_t)t.py * t.W + t.px;
  out_rgb[3 * t.pix_off + i] = __builtin_fmaf(T, op.bg[0], Cr);
  out_rgb[3 * t.pix_off + P + i] = __builtin_fmaf(T, op.bg[1], Cg);
  out_rgb[3 * t.pix_off + 2 * P + i] = __builtin_fmaf(T, op.bg[2], Cb);
  out_depth[t.pix_off + i] = D;
  out_vis[t.pix_off + i] = Vs;
}

template <int TW, int TH, int DEPTH, int BW>
__global__ __launch_bounds__(TW * TH) void k_render_fwd(const float4* __restrict__ rec,
                                                        const int32_t* __restrict__ vals,
                                                        const int2* __restrict__ range,
                                                        const gs_camera* __restrict__ cams, int V, int n_tiles,
                                                        const int32_t* __restrict__ order, DevOpts op,
                                                        float* __restrict__ out_rgb, float* __restrict__ out_depth,
                                                        float* __restrict__ out_vis) {
  using G = Geo<TW, TH, DEPTH, BW>;
  __shared__ Stage<G> s;
  TileCtx t;
  int tile;
  if (!tile_setup<G>(cams, V, n_tiles, order, t, tile)) return;
  float T, Cr, Cg, Cb, D, Vs;
  forward_sweep<G, DEPTH>(s, rec, vals, range[tile], t, op, T, Cr, Cg, Cb, D, Vs);
  write_pixel(t, op, T, Cr, Cg, Cb, D, Vs, out_rgb, out_depth, out_vis);
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
  float lambda_ssim;  // loss mode: the L1 colour term takes 1 - lambda_ssim; g_rgb (if given) is added
  float* ipart;              // [slot][12]: instance partials, each record's instances one run
  const int32_t* rec_slot;   // first slot of each record; a record's tiles follow row by row
  int64_t capacity;          // slots stored (a slot at or past it belongs to an overflowed frame)
  float* loss;
};

// Depth segments of the fused backward (see k_fused_main).
struct SegArgs {
  const int4* items;        // {tile, segment, first slot of the tile or -1, schedule position}
  const int32_t* counters;  // [192] items, [193] slots of split tiles, [194] split tiles
  const int32_t* order;
  const int32_t* seg_count;
  const int32_t* seg_first;
  float* seg;               // [slot][6][NT]
  float* split;             // [split tile][12][NT]
  int len;                  // records per segment
};

// Upstream gradient of this pixel from its final values: the L1 loss gradient (eqs. Lc, Ld, L) or the
// given image gradients.  Adds the pixel's loss to loss_acc.
template <bool LOSS>
__device__ __forceinline__ void pixel_upstream(const TileCtx& t, const BwdArgs& a, float Cf, float Gf, float Bf,
                                               float Df, float& gr, float& gg, float& gb, float& gd, float& gv,
                                               float& loss_acc) {
  gr = gg = gb = gd = gv = 0.f;
  if (!t.inside) return;
  const int64_t P = (int64_t)t.W * t.H;
  const int64_t pi = (int64_t)t.py * t.W + t.px;
  if (LOSS) {
    const float wrgb = t.weight * (1.f - a.lambda_ssim) / (3.f * (float)P);
    const int M = a.n_valid[t.view];
    const float wd = M > 0 ? t.weight * a.lambda_d / (float)M : 0.f;
    const float er = Cf - a.tgt_rgb[3 * t.pix_off + pi];
    const float eg = Gf - a.tgt_rgb[3 * t.pix_off + P + pi];
    const float eb = Bf - a.tgt_rgb[3 * t.pix_off + 2 * P + pi];
    gr = wrgb * gsk::sgnf(er);
    gg = wrgb * gsk::sgnf(eg);
    gb = wrgb * gsk::sgnf(eb);
    loss_acc += wrgb * (fabsf(er) + fabsf(eg) + fabsf(eb));
    if (a.g_rgb) {  // the gradient of a further colour term (the SSIM term of gs_ssim)
      gr += a.g_rgb[3 * t.pix_off + pi];
      gg += a.g_rgb[3 * t.pix_off + P + pi];
      gb += a.g_rgb[3 * t.pix_off + 2 * P + pi];
    }
    const float dt = a.tgt_depth[t.pix_off + pi];
    if (dt > 0.f) {
      const float ed = Df - dt;
      gd = wd * gsk::sgnf(ed);
      loss_acc += wd * fabsf(ed);
    }
  } else {
    if (a.g_rgb) {
      gr = a.g_rgb[3 * t.pix_off + pi];
      gg = a.g_rgb[3 * t.pix_off + P + pi];
      gb = a.g_rgb[3 * t.pix_off + 2 * P + pi];
    }
    if (a.g_depth) gd = a.g_depth[t.pix_off + pi];
    if (a.g_vis) gv = a.g_vis[t.pix_off + pi];
  }
}

// Adds the workgroup's loss to one of the partial sums loss[1 .. kLossSlots] (every thread must call it):
// one atomic per workgroup, spread over the slots, since atomics on one address serialise; k_loss_total
// adds the slots into loss[0].
template <class G>
__device__ __forceinline__ void add_loss(const TileCtx& t, const BwdArgs& a, float loss_acc) {
  __shared__ float part[G::NW];
  const float ls = gsk::wave_sum_last(loss_acc);
  if (t.lane == 63) part[t.wave] = ls;
  __syncthreads();
  if (threadIdx.x == 0) {
    float sum = part[0];
#pragma unroll
    for (int w = 1; w < G::NW; ++w) sum += part[w];
    gsk::atomic_add_f32(a.loss + 1 + (blockIdx.x % gsk::kLossSlots), sum);
  }
}

__global__ void k_loss_total(float* __restrict__ loss) {
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 1; i <= gsk::kLossSlots; ++i) s += loss[i];
    loss[0] = s;
  }
}

// Partial slot of the instance of a record (pixel rectangle in C) in the tile at pixel origin (tx0, ty0): the
// record's first slot plus the tile's index in the record's tile rectangle, row by row (the emission order).
template <class G>
__device__ __forceinline__ int64_t inst_slot(int first, const float4& C, const TileCtx& t) {
  constexpr int TWp = 8 * G::SX, THp = 8 * G::SY;
  int x0, x1, y0, y1;
  unpack_rect(C, x0, x1, y0, y1);
  const int rx0 = x0 / TWp, rx1 = x1 / TWp, ry0 = y0 / THp;
  return (int64_t)first + (t.ty0 / THp - ry0) * (rx1 - rx0 + 1) + (t.tx0 / TWp - rx0);
}

// Store the LDS sums of this thread's staged records of the round that started at list position b0 (nb
// records, still staged in s) as the partials of those instances (at their slots), and clear them.  The sums are, over the record's contributing pixels (d = mean - pixel centre, dq = dL/dalpha alpha):
//   dq dx, dq dy, dq dx^2, dq dx dy, dq dy^2, dL/dalpha G, w g_r, w g_g, w g_b, w g_d;
// with the conic (a, b, c) of the record, power = -(a dx^2 + c dy^2)/2 - b dx dy gives
//   dL/dmean = -(a S_x + b S_y, b S_x + c S_y),  dL/d(a, b, c) = -(S_xx / 2, S_xy, S_yy / 2).
// Plain stores: every instance has exactly one writer (its tile or depth segment), so nothing is accumulated
// in HBM.
// LDS row of per-record sum q (0 S_x, 1 S_y, 2 S_xx, 3 S_xy, 4 S_yy, 5 opacity, 6..9 w g_(r,g,b,d)).  The rows
// are ordered so that the three sums a lane of the block reduce-scatter ends with lie 4 rows apart (rows
// r, r + 4, r + 8 with r = c0 + 2 c1, see backward_walk): one address serves its three LDS atomics.
__device__ __forceinline__ constexpr int lds_row(int q) {
  return q == 0 ? 0 : q == 1 ? 1 : q == 2 ? 4 : q == 3 ? 8 : q == 4 ? 5 : q == 5 ? 9 : q == 6 ? 2 : q == 7 ? 3
       : q == 8 ? 6 : 7;
}

template <class G, int DEPTH>
__device__ __forceinline__ void flush_grads(const Stage<G>& s, float (*gacc)[G::GS], const TileCtx& t,
                                            float* __restrict__ ipart, int64_t capacity, int nb) {
#pragma unroll
  for (int k = 0; k < DEPTH; ++k) {
    const int j = k * G::NT + (int)threadIdx.x;
    if (j >= nb) continue;
    float v[10];
    bool any = false;
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      v[q] = gacc[lds_row(q)][j];
      any |= v[q] != 0.f;
    }
    {
      const float4 B = s.B[j];
      const float sx = v[0], sy = v[1];
      v[0] = -(B.x * sx + B.y * sy);
      v[1] = -(B.y * sx + B.z * sy);
      v[2] = -0.5f * v[2];
      v[3] = -v[3];
      v[4] = -0.5f * v[4];
    }
    const int64_t q = inst_slot<G>(s.slot[j], s.C[j], t);
    if (q < capacity) {
      float4* dst = reinterpret_cast<float4*>(ipart) + 3 * q;
      dst[0] = make_float4(v[0], v[1], v[2], v[3]);
      dst[1] = make_float4(v[4], v[5], v[6], v[7]);
      dst[2] = make_float4(v[8], v[9], 0.f, 0.f);
    }
    if (any) {
#pragma unroll
      for (int q = 0; q < 10; ++q) gacc[q][j] = 0.f;
    }
  }
}

// Zero partials for the instances [b0, end) that the walk never staged (every pixel ended before them).
template <class G>
__device__ __forceinline__ void zero_grads(const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                           const TileCtx& t, float* __restrict__ ipart,
                                           const int32_t* __restrict__ rec_slot, int64_t capacity, int b0, int end) {
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int p = b0 + (int)threadIdx.x; p < end; p += G::NT) {
    const int64_t r = vals[p];
    const int64_t q = inst_slot<G>(rec_slot[r], rec[3 * r + 2], t);
    if (q >= capacity) continue;
    float4* dst = reinterpret_cast<float4*>(ipart) + 3 * q;
    dst[0] = z;
    dst[1] = z;
    dst[2] = z;
  }
}

// Backward walk of records [rg.x, rg.y) for this lane's pixel, front to back, from transmittance T and
// prefix P (the pixel's state at rg.x), with upstream gradient g and S = g . (C, D, V) of the final values.
// Per-record partial derivatives are summed in LDS and stored as the instances' partials once per round;
// instances after the walk's end get zero partials.
template <class G, int DEPTH>
__device__ __forceinline__ void backward_walk(Stage<G>& s, float (*gacc)[G::GS], const float4* __restrict__ rec,
                                              const int32_t* __restrict__ vals, int2 rg, const TileCtx& t,
                                              const DevOpts& op, bool live, float T, float Pp, float gr, float gg,
                                              float gb, float gd, float gv, float S, const BwdArgs& a) {
  const float fx = (float)t.px + 0.5f, fy = (float)t.py + 0.5f;
#pragma unroll
  for (int k = 0; k < DEPTH; ++k)
#pragma unroll
    for (int q = 0; q < 10; ++q) gacc[q][k * G::NT + threadIdx.x] = 0.f;
  // The ten per-record sums are numbered 0 S_x, 1 S_y, 2 S_xx, 3 S_xy, 4 S_yy, 5 opacity, 6..9 w g_(r,g,b,d)
  // (S_* are moments of dq, see flush_grads; sum q lives in LDS row lds_row(q)).  Each lane computes them as a kept half acc[0..4] and a sent
  // half acc[5..9] for the first exchange of the block reduce-scatter; which half is kept is the lane's share
  // c0 (c1 for the second exchange): lanes of share 0 keep S_x, S_xx, S_xy, w g_r, w g_b (sums 0, 2, 3, 6,
  // 8), lanes of share 1 keep S_y, S_yy, opacity, w g_g, w g_d (sums 1, 4, 5, 7, 9).  The colour halves
  // depend on the lane only, so their selection is made once here.  With BW = 4 the shares are c0 = b0^b2,
  // c1 = b1^b2 of the lane's row index (b_k its bits): the quad exchanges (lane^1, lane^2) flip c0 resp. c1,
  // the row mirrors flip all four bits and keep both shares.  With BW = 2 they are the quad bits b0, b1.
  const int lr = t.lane & 15;
  const bool c0 = G::BW == 4 ? ((lr ^ (lr >> 2)) & 1) != 0 : G::BW == 2 ? (lr & 1) != 0 : false;
  const bool c1 = G::BW == 4 ? (((lr >> 1) ^ (lr >> 2)) & 1) != 0 : G::BW == 2 ? (lr & 2) != 0 : false;
  const float gK0 = c0 ? gg : gr, gS0 = c0 ? gr : gg, gK1 = c0 ? gd : gb, gS1 = c0 ? gb : gd;
  auto step = [&](int, bool active, const float4& A, const float4& B, const float4& C, float* acc) -> bool {
    float alpha, Gv, dx, dy;
    bool cl;
    const bool ok = eval_pair(A, B, fx, fy, op, alpha, Gv, cl, dx, dy) && active;
    const float Tn = T * (1.f - alpha);
    const bool stop = ok && Tn < op.t_min;
    const bool hit = ok && !stop;
    live = live && !stop;
    const float wh = hit ? alpha * T : 0.f;  // w of a contributing pair, else 0
    const float qv = __builtin_fmaf(gd, A.z, __builtin_fmaf(gb, C.y, __builtin_fmaf(gg, C.x, __builtin_fmaf(gr, B.w, gv))));
    const float Pn = Pp + wh * qv;
    const float dalpha = T * qv - (S - Pn) * __builtin_amdgcn_rcpf(1.f - alpha);
    const bool shape = hit && !cl;  // a clamped alpha passes no gradient to opacity or shape
    // Every operand is finite (staged records only), so zeroing dq, w and the opacity term zeroes the
    // partials of a lane that does not contribute.
    const float dq = shape ? dalpha * alpha : 0.f;
    const float so = shape ? dalpha * Gv : 0.f;
    const float dK = c0 ? dy : dx, dS = c0 ? dx : dy;
    const float kA = dq * dK, sA = dq * dS;
    const float sxy = kA * dS;
    acc[0] = kA;       // S_x  | S_y
    acc[1] = kA * dK;  // S_xx | S_yy
    acc[2] = c0 ? so : sxy;
    acc[3] = wh * gK0;
    acc[4] = wh * gK1;
    acc[5] = sA;
    acc[6] = sA * dS;
    acc[7] = c0 ? sxy : so;
    acc[8] = wh * gS0;
    acc[9] = wh * gS1;
    Pp = Pn;
    T = hit ? Tn : T;
    return hit;
  };
  auto slot_kept = [&](int k) { return c0 ? (k == 0 ? 1 : k == 1 ? 4 : k == 2 ? 5 : k == 3 ? 7 : 9)
                                          : (k == 0 ? 0 : k == 1 ? 2 : k == 2 ? 3 : k == 3 ? 6 : 8); };
  auto slot_sent = [&](int k) { return c0 ? (k == 0 ? 0 : k == 1 ? 2 : k == 2 ? 3 : k == 3 ? 6 : 8)
                                          : (k == 0 ? 1 : k == 1 ? 4 : k == 2 ? 5 : k == 3 ? 7 : 9); };
  // After both exchanges lane (c0, c1) holds the block sums x0, x1 and (c1 = 0 only) x2 of sums
  // (0, 2, 3) for (0, 0), (1, 4, 5) for (1, 0), (6, 8) for (0, 1) and (7, 9) for (1, 1): LDS rows r, r + 4,
  // r + 8 with r = c0 + 2 c1.
  const int x_row = (c0 ? 1 : 0) + (c1 ? 2 : 0);
  // Sum the partials of one step into the records' LDS accumulators (whole wave; one record per block).  The
  // block reduction runs whenever any lane contributed: letting each contributing lane add its own ten
  // partials when few do costs more in LDS atomics than the reduction (measured).
  auto post = [&](int j, bool hit, const float* acc) {
    const uint64_t hits = __builtin_amdgcn_ballot_w64(hit);
    if (hits == 0) return;
    constexpr uint64_t BMASK = G::BL == 64 ? ~0ull : ((1ull << G::BL) - 1);
    const bool block_hit = ((hits >> t.blk_lane0) & BMASK) != 0;
    if (G::BW == 2 || G::BW == 4) {
      // Reduce-scatter: the exchange with lane^1 adds the partner's sent half to the kept half (10 -> 5
      // values per lane), the one with lane^2 halves them again (5 -> 3), and with BW = 4 the two row
      // mirrors add plain.  Lanes 0..3 of the block then hold the block sums of all ten slots: 3 LDS atomics
      // per lane instead of 10.
      float w[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) w[k] = acc[k] + gsk::dpp_f<0xB1>(acc[5 + k]);  // quad_perm [1,0,3,2]
      float x0 = (c1 ? w[3] : w[0]) + gsk::dpp_f<0x4E>(c1 ? w[0] : w[3]);         // quad_perm [2,3,0,1]
      float x1 = (c1 ? w[4] : w[1]) + gsk::dpp_f<0x4E>(c1 ? w[1] : w[4]);
      float x2 = w[2] + gsk::dpp_f<0x4E>(w[2]);
      if (G::BW == 4) {
        x0 += gsk::dpp_f<0x141>(x0);  // row_half_mirror
        x1 += gsk::dpp_f<0x141>(x1);
        x2 += gsk::dpp_f<0x141>(x2);
        x0 += gsk::dpp_f<0x140>(x0);  // row_mirror
        x1 += gsk::dpp_f<0x140>(x1);
        x2 += gsk::dpp_f<0x140>(x2);
      }
      float* dst = &gacc[x_row][j];
      if (G::BW == 4) {
        // lanes 0..3 of the blocks with a contributing lane, as a wave mask formed with scalar operations
        // (lanes 0 and 1 hold the third sum, c1 = 0)
        uint64_t rows = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (((uint32_t)(hits >> (16 * r)) & 0xffffu) != 0u) rows |= 0xfull << (16 * r);
        if (__builtin_amdgcn_inverse_ballot_w64(rows)) {
          atomicAdd(dst, x0);
          atomicAdd(dst + 4 * G::GS, x1);
        }
        if (__builtin_amdgcn_inverse_ballot_w64(rows & 0x0003000300030003ull)) atomicAdd(dst + 8 * G::GS, x2);
      } else if (block_hit) {
        atomicAdd(dst, x0);
        atomicAdd(dst + 4 * G::GS, x1);
        if (!c1) atomicAdd(dst + 8 * G::GS, x2);
      }
      return;
    }
    float sum[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) sum[q] = block_sum<G>(acc[q]);
    if ((t.lane % G::BL) == G::BL - 1 && block_hit) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        atomicAdd(&gacc[lds_row(slot_kept(k))][j], sum[k]);
        atomicAdd(&gacc[lds_row(slot_sent(k))][j], sum[5 + k]);
      }
    }
  };
  sweep<G, DEPTH, true, true>(s, rec, a.rec_slot, vals, rg, t, op, live,
                        [&](int b0, bool go) {
                          if (b0 != rg.x)
                            flush_grads<G, DEPTH>(s, gacc, t, a.ipart, a.capacity, min(G::BATCH, rg.y - (b0 - G::BATCH)));
                          if (!go) zero_grads<G>(rec, vals, t, a.ipart, a.rec_slot, a.capacity, b0, rg.y);
                        },
                        step, post);
}

// Forward sweep (or the forward images), upstream gradient, then the backward walk of one whole tile.
template <class G, int DEPTH, bool HAVE_FWD, bool LOSS>
__device__ __forceinline__ void tile_backward(Stage<G>& s, float (*gacc)[G::GS], const float4* __restrict__ rec,
                                              const int32_t* __restrict__ vals, int2 rg, const TileCtx& t,
                                              const DevOpts& op, const BwdArgs& a) {
  float Cf = 0.f, Gf = 0.f, Bf = 0.f, Df = 0.f, Vf = 0.f;
  if (HAVE_FWD) {
    if (t.inside) {
      const int64_t P = (int64_t)t.W * t.H;
      const int64_t pi = (int64_t)t.py * t.W + t.px;
      Cf = a.fwd_rgb[3 * t.pix_off + pi];
      Gf = a.fwd_rgb[3 * t.pix_off + P + pi];
      Bf = a.fwd_rgb[3 * t.pix_off + 2 * P + pi];
      Df = a.fwd_depth[t.pix_off + pi];
      Vf = a.fwd_vis[t.pix_off + pi];
    }
  } else {
    float T;
    forward_sweep<G, DEPTH>(s, rec, vals, rg, t, op, T, Cf, Gf, Bf, Df, Vf);
    Cf = __builtin_fmaf(T, op.bg[0], Cf);
    Gf = __builtin_fmaf(T, op.bg[1], Gf);
    Bf = __builtin_fmaf(T, op.bg[2], Bf);
  }
  float gr, gg, gb, gd, gv, loss_acc = 0.f;
  pixel_upstream<LOSS>(t, a, Cf, Gf, Bf, Df, gr, gg, gb, gd, gv, loss_acc);
  const float S = gr * Cf + gg * Gf + gb * Bf + gd * Df + gv * Vf;
  if (LOSS) add_loss<G>(t, a, loss_acc);
  backward_walk<G, DEPTH>(s, gacc, rec, vals, rg, t, op, t.inside, 1.f, 0.f, gr, gg, gb, gd, gv, S, a);
}

template <int TW, int TH, int DEPTH, int BW, bool HAVE_FWD, bool LOSS>
__global__ __launch_bounds__(TW * TH) void k_render_bwd(const float4* __restrict__ rec,
                                                        const int32_t* __restrict__ vals,
                                                        const int2* __restrict__ range,
                                                        const gs_camera* __restrict__ cams, int V, int n_tiles,
                                                        const int32_t* __restrict__ order, DevOpts op, BwdArgs a) {
  using G = Geo<TW, TH, DEPTH, BW>;
  __shared__ Stage<G> s;
  __shared__ float gacc[10][G::GS];
  TileCtx t;
  int tile;
  if (!tile_setup<G>(cams, V, n_tiles, order, t, tile)) return;
  tile_backward<G, DEPTH, HAVE_FWD, LOSS>(s, gacc, rec, vals, range[tile], t, op, a);
}

// ---------------------------------------------------------------------------------------------------------
// Fused backward with depth segments.  A tile list longer than L records is split into segments of L,
// each its own workgroup, so the few huge tiles of coarse pyramid levels no longer serialise the launch.
// Compositing is a product of transmittances, so per pixel:
//   1. each segment k walks its records from T = 1 without the stop rule: its transmittance product T_k and
//      local sums (C, D, V)_k (k_fused_main, alongside the unsplit tiles);
//   2. T_start,k = T_0 T_1 ... T_{k-1} (left to right, k_seg_prefix); the pixel's last live segment k* is the
//      last with T_start,k >= t_min, and only there can the stop rule end the walk: that segment is walked
//      again from T_start,k* with the stop rule (k_seg_stop);
//   3. the final values are sum_{k<k*} T_start,k (C, D, V)_k plus segment k*'s stopped sums plus the
//      background; from them the upstream gradient g, S and each segment's start state (T_start,k,
//      P_start,k = g . sum_{j<k} contribution_j) (k_seg_combine);
//   4. each live segment runs the backward walk from its start state (k_seg_bwd).
// The result equals the unsplit walk up to FP32 rounding of the transmittance product (the association of
// the product differs), which can move a stop decision that lies within that rounding of t_min.
template <class G>
__device__ __forceinline__ int2 segment_range(int2 rg, int k, int L) {
  const int lo = rg.x + k * L;
  return make_int2(lo, min(rg.y, lo + L));
}

// Step 1 for one depth segment: its transmittance product and local sums, from T = 1 without the stop rule.
template <class G, int DEPTH>
__device__ __forceinline__ void segment_sums(Stage<G>& s, const float4* __restrict__ rec,
                                             const int32_t* __restrict__ vals, int2 rg, int4 it, const TileCtx& t,
                                             const DevOpts& op, const SegArgs& g) {
  float T = 1.f, Cr = 0.f, Cg = 0.f, Cb = 0.f, D = 0.f, Vs = 0.f;
  forward_walk<G, DEPTH, false>(s, rec, vals, segment_range<G>(rg, it.y, g.len), t, op, t.inside, T, Cr, Cg, Cb, D,
                                Vs);
  float* o = g.seg + (size_t)(it.z + it.y) * 6 * G::NT + threadIdx.x;
  o[0 * G::NT] = T;
  o[1 * G::NT] = Cr;
  o[2 * G::NT] = Cg;
  o[3 * G::NT] = Cb;
  o[4 * G::NT] = D;
  o[5 * G::NT] = Vs;
}

// The work items of a launch: one per workgroup (item blockIdx.x while it is below count), or with PERSIST a
// grid sized to what the GPU holds at once, whose workgroups take items in schedule order from the counter
// *ctr (zeroed before the launch) until count is reached; every workgroup then leaves the loop.
template <bool PERSIST, class Body>
__device__ __forceinline__ void for_items(int count, int32_t* ctr, Body body) {
  if constexpr (!PERSIST) {
    if ((int)blockIdx.x < count) body((int)blockIdx.x);
  } else {
    __shared__ int s_item;
    while (true) {
      __syncthreads();  // the previous item's LDS is no longer read
      if (threadIdx.x == 0) s_item = atomicAdd(ctr, 1);
      __syncthreads();
      const int b = s_item;
      if (b >= count) return;
      body(b);
    }
  }
}

// Backward over the work items: whole tiles run the forward sweep (or read the forward images), the upstream
// gradient and the backward walk; segments of split tiles run step 1.
template <int TW, int TH, int DEPTH, int BW, bool HAVE_FWD, bool LOSS, bool PERSIST = false>
__global__ __launch_bounds__(TW * TH) void k_fused_main(const float4* __restrict__ rec,
                                                        const int32_t* __restrict__ vals,
                                                        const int2* __restrict__ range,
                                                        const gs_camera* __restrict__ cams, int V, DevOpts op,
                                                        BwdArgs a, SegArgs g, int32_t* ctr) {
  using G = Geo<TW, TH, DEPTH, BW>;
  __shared__ Stage<G> s;
  __shared__ float gacc[10][G::GS];
  for_items<PERSIST>(g.counters[192], ctr, [&](int b) {
    const int4 it = g.items[b];
    TileCtx t;
    tile_at<G>(cams, V, it.x, t);
    const int2 rg = range[it.x];
    if (it.z < 0)
      tile_backward<G, DEPTH, HAVE_FWD, LOSS>(s, gacc, rec, vals, rg, t, op, a);
    else
      segment_sums<G, DEPTH>(s, rec, vals, rg, it, t, op, g);
  });
}

// Forward over the work items: whole tiles are composited and written; segments of split tiles run step 1.
template <int TW, int TH, int DEPTH, int BW>
__global__ __launch_bounds__(TW * TH) void k_fwd_main(const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                                      const int2* __restrict__ range,
                                                      const gs_camera* __restrict__ cams, int V, DevOpts op,
                                                      SegArgs g, float* __restrict__ out_rgb,
                                                      float* __restrict__ out_depth, float* __restrict__ out_vis) {
  using G = Geo<TW, TH, DEPTH, BW>;
  __shared__ Stage<G> s;
  if ((int)blockIdx.x >= g.counters[192]) return;
  const int4 it = g.items[blockIdx.x];
  TileCtx t;
  tile_at<G>(cams, V, it.x, t);
  const int2 rg = range[it.x];
  if (it.z >= 0) {
    segment_sums<G, DEPTH>(s, rec, vals, rg, it, t, op, g);
    return;
  }
  float T, Cr, Cg, Cb, D, Vs;
  forward_sweep<G, DEPTH>(s, rec, vals, rg, t, op, T, Cr, Cg, Cb, D, Vs);
  write_pixel(t, op, T, Cr, Cg, Cb, D, Vs, out_rgb, out_depth, out_vis);
}

template <int TW, int TH, int DEPTH, int BW, bool PERSIST = false>
__global__ __launch_bounds__(TW * TH) void k_seg_stop(const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                                      const int2* __restrict__ range,
                                                      const gs_camera* __restrict__ cams, int V, DevOpts op,
                                                      SegArgs g, int32_t* ctr) {
  using G = Geo<TW, TH, DEPTH, BW>;
  __shared__ Stage<G> s;
  for_items<PERSIST>(g.counters[193], ctr, [&](int b) {
    const int4 it = g.items[b];
    TileCtx t;
    tile_at<G>(cams, V, it.x, t);
    const int2 rg = range[it.x];
    const int n = (rg.y - rg.x + g.len - 1) / g.len;
    // start transmittances of this segment and the next (k_seg_prefix)
    const float* sp = g.seg + (size_t)(it.z + it.y) * 6 * G::NT + threadIdx.x;
    const float Ts = sp[0];
    const bool last = t.inside && Ts >= op.t_min && (it.y == n - 1 || sp[6 * G::NT] < op.t_min);
    float T = Ts, Cr = 0.f, Cg = 0.f, Cb = 0.f, D = 0.f, Vs = 0.f;
    forward_walk<G, DEPTH, true>(s, rec, vals, segment_range<G>(rg, it.y, g.len), t, op, last, T, Cr, Cg, Cb, D, Vs);
    if (last) {
      float* o = g.split + (size_t)it.w * 12 * G::NT + threadIdx.x;
      o[0 * G::NT] = T;
      o[1 * G::NT] = Cr;
      o[2 * G::NT] = Cg;
      o[3 * G::NT] = Cb;
      o[4 * G::NT] = D;
      o[5 * G::NT] = Vs;
    }
  });
}

// Segments of a split tile whose loads the combine steps keep in flight together (a tile may have a hundred
// segments, and the running products make each pixel's pass serial).
constexpr int kSegBatch = 4;
constexpr int kPrefixBatch = 16;

// Step 2, first half: per pixel, the start transmittance T_start,k = T_0 T_1 ... T_{k-1} of every segment of a
// split tile (the left-to-right product), written over the segment's own product T_k.  Once it is below
// t_min, so is every later one (each T_k <= 1), and only that comparison is used: those are written as 0.
template <int TW, int TH, int BW>
__global__ __launch_bounds__(TW * TH) void k_seg_prefix(SegArgs g, DevOpts op) {
  using G = Geo<TW, TH, 1, BW>;
  const int l = blockIdx.x;
  if (l >= g.counters[194]) return;
  const int n = g.seg_count[l];
  constexpr size_t SS = 6 * G::NT;
  float* sp = g.seg + (size_t)g.seg_first[l] * SS + threadIdx.x;
  float Tr = 1.f;
  for (int k0 = 0; k0 < n; k0 += kPrefixBatch) {
    const bool live = Tr >= op.t_min;
    float v[kPrefixBatch];
#pragma unroll
    for (int i = 0; i < kPrefixBatch; ++i) v[i] = live ? sp[(size_t)min(k0 + i, n - 1) * SS] : 0.f;
#pragma unroll
    for (int i = 0; i < kPrefixBatch; ++i) {
      if (k0 + i >= n) break;
      sp[(size_t)(k0 + i) * SS] = Tr >= op.t_min ? Tr : 0.f;
      Tr = Tr * v[i];
    }
  }
}

// Step 3, first half: the pixel's last live segment ks (the last whose start transmittance, from
// k_seg_prefix, is at least t_min) and its final sums (C, D, V) and transmittance.  One pass: while the start
// transmittance of segment k is at least t_min, k is the candidate and the weighted sum of the segments
// before it is kept aside; the sums are formed in segment order.
template <class G>
__device__ __forceinline__ void split_final(const float* sp, const float* xp, int n, const TileCtx& t,
                                            const DevOpts& op, int& ks, float& Tf, float& Cr, float& Cg, float& Cb,
                                            float& D, float& Vs) {
  constexpr size_t SS = 6 * G::NT;
  ks = 0;
  bool more = true;
  float Rr = 0.f, Rg = 0.f, Rb = 0.f, RD = 0.f, RV = 0.f;  // weighted sums of the segments before k
  Cr = Cg = Cb = D = Vs = 0.f;
  for (int k0 = 0; k0 < n && more; k0 += kSegBatch) {
    float v[kSegBatch][6];
#pragma unroll
    for (int i = 0; i < kSegBatch; ++i) {
      const float* q = sp + (size_t)min(k0 + i, n - 1) * SS;
#pragma unroll
      for (int c = 0; c < 6; ++c) v[i][c] = q[c * G::NT];
    }
#pragma unroll
    for (int i = 0; i < kSegBatch; ++i) {
      const float Ts = v[i][0];
      if (k0 + i < n && Ts >= op.t_min) {
        ks = k0 + i;
        Cr = Rr;
        Cg = Rg;
        Cb = Rb;
        D = RD;
        Vs = RV;
        Rr = __builtin_fmaf(Ts, v[i][1], Rr);
        Rg = __builtin_fmaf(Ts, v[i][2], Rg);
        Rb = __builtin_fmaf(Ts, v[i][3], Rb);
        RD = __builtin_fmaf(Ts, v[i][4], RD);
        RV = __builtin_fmaf(Ts, v[i][5], RV);
      } else {
        more = false;
      }
    }
  }
  Tf = 1.f;
  if (t.inside) {
    Tf = xp[0];
    Cr += xp[1 * G::NT];
    Cg += xp[2 * G::NT];
    Cb += xp[3 * G::NT];
    D += xp[4 * G::NT];
    Vs += xp[5 * G::NT];
  }
}

// Forward of split tiles, step 3: write the final values.
template <int TW, int TH, int BW>
__global__ __launch_bounds__(TW * TH) void k_seg_fwd_out(const gs_camera* __restrict__ cams, int V, DevOpts op,
                                                         SegArgs g, float* __restrict__ out_rgb,
                                                         float* __restrict__ out_depth, float* __restrict__ out_vis) {
  using G = Geo<TW, TH, 1, BW>;
  const int l = blockIdx.x;
  if (l >= g.counters[194]) return;
  TileCtx t;
  tile_at<G>(cams, V, g.order[l], t);
  const float* sp = g.seg + (size_t)g.seg_first[l] * 6 * G::NT + threadIdx.x;
  const float* xp = g.split + (size_t)l * 12 * G::NT + threadIdx.x;
  int ks;
  float T, Cr, Cg, Cb, D, Vs;
  split_final<G>(sp, xp, g.seg_count[l], t, op, ks, T, Cr, Cg, Cb, D, Vs);
  write_pixel(t, op, T, Cr, Cg, Cb, D, Vs, out_rgb, out_depth, out_vis);
}

// Backward of split tiles, step 3: final values (or the forward images), upstream gradient, S and the start
// state (T_start, P_start) of every segment; T_start = 0 marks a segment after the pixel's end.
template <int TW, int TH, int BW, bool HAVE_FWD, bool LOSS>
__global__ __launch_bounds__(TW * TH) void k_seg_combine(const gs_camera* __restrict__ cams, int V, DevOpts op,
                                                         BwdArgs a, SegArgs g) {
  using G = Geo<TW, TH, 1, BW>;
  const int l = blockIdx.x;
  if (l >= g.counters[194]) return;
  const int n = g.seg_count[l];
  TileCtx t;
  tile_at<G>(cams, V, g.order[l], t);
  float* sp = g.seg + (size_t)g.seg_first[l] * 6 * G::NT + threadIdx.x;
  float* xp = g.split + (size_t)l * 12 * G::NT + threadIdx.x;
  constexpr size_t SS = 6 * G::NT;
  int ks;
  float Tf, Cr, Cg, Cb, D, Vs;
  split_final<G>(sp, xp, n, t, op, ks, Tf, Cr, Cg, Cb, D, Vs);
  float Cf = __builtin_fmaf(Tf, op.bg[0], Cr), Gf = __builtin_fmaf(Tf, op.bg[1], Cg);
  float Bf = __builtin_fmaf(Tf, op.bg[2], Cb), Df = D, Vf = Vs;
  if (HAVE_FWD && t.inside) {
    const int64_t P = (int64_t)t.W * t.H;
    const int64_t pi = (int64_t)t.py * t.W + t.px;
    Cf = a.fwd_rgb[3 * t.pix_off + pi];
    Gf = a.fwd_rgb[3 * t.pix_off + P + pi];
    Bf = a.fwd_rgb[3 * t.pix_off + 2 * P + pi];
    Df = a.fwd_depth[t.pix_off + pi];
    Vf = a.fwd_vis[t.pix_off + pi];
  }
  float gr, gg, gb, gd, gv, loss_acc = 0.f;
  pixel_upstream<LOSS>(t, a, Cf, Gf, Bf, Df, gr, gg, gb, gd, gv, loss_acc);
  const float S = gr * Cf + gg * Gf + gb * Bf + gd * Df + gv * Vf;
  if (LOSS) add_loss<G>(t, a, loss_acc);
  float Pr = 0.f;
  for (int k0 = 0; k0 < n; k0 += kSegBatch) {
    // segments up to ks are read (batched); later ones only get T_start = 0
    float v[kSegBatch][6];
#pragma unroll
    for (int i = 0; i < kSegBatch; ++i) {
      const float* q = sp + (size_t)min(k0 + i, n - 1) * SS;
#pragma unroll
      for (int c = 0; c < 6; ++c) v[i][c] = k0 + i <= ks ? q[c * G::NT] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < kSegBatch; ++i) {
      const int k = k0 + i;
      if (k >= n) break;
      float* q = sp + (size_t)k * SS;
      const float Ts = v[i][0];
      const float dot =
          k < ks ? Ts * (gr * v[i][1] + gg * v[i][2] + gb * v[i][3] + gd * v[i][4] + gv * v[i][5]) : 0.f;
      q[0] = k <= ks ? Ts : 0.f;
      q[1 * G::NT] = Pr;
      Pr += dot;
    }
  }
  xp[6 * G::NT] = gr;
  xp[7 * G::NT] = gg;
  xp[8 * G::NT] = gb;
  xp[9 * G::NT] = gd;
  xp[10 * G::NT] = gv;
  xp[11 * G::NT] = S;
}

template <int TW, int TH, int DEPTH, int BW, bool PERSIST = false>
__global__ __launch_bounds__(TW * TH) void k_seg_bwd(const float4* __restrict__ rec, const int32_t* __restrict__ vals,
                                                     const int2* __restrict__ range,
                                                     const gs_camera* __restrict__ cams, int V, DevOpts op,
                                                     BwdArgs a, SegArgs g, int32_t* ctr) {
  using G = Geo<TW, TH, DEPTH, BW>;
  __shared__ Stage<G> s;
  __shared__ float gacc[10][G::GS];
  for_items<PERSIST>(g.counters[193], ctr, [&](int b) {
    const int4 it = g.items[b];
    TileCtx t;
    tile_at<G>(cams, V, it.x, t);
    const float* sp = g.seg + (size_t)(it.z + it.y) * 6 * G::NT + threadIdx.x;
    const float* xp = g.split + (size_t)it.w * 12 * G::NT + threadIdx.x;
    const float Ts = sp[0], Ps = sp[1 * G::NT];
    backward_walk<G, DEPTH>(s, gacc, rec, vals, segment_range<G>(range[it.x], it.y, g.len), t, op,
                            t.inside && Ts >= op.t_min, Ts, Ps, xp[6 * G::NT], xp[7 * G::NT], xp[8 * G::NT],
                            xp[9 * G::NT], xp[10 * G::NT], xp[11 * G::NT], a);
  });
}

// Work counts of the forward: pairs evaluated (pixel inside the record's pixel rectangle, up to the
// pixel's stop) and pairs contributing.  Independent of the tile shape; diagnostic.
template <int TW, int TH>
__global__ __launch_bounds__(TW * TH) void k_count_pairs(const float4* __restrict__ rec,
                                                         const int32_t* __restrict__ vals,
                                                         const int2* __restrict__ range,
                                                         const gs_camera* __restrict__ cams, int V, int n_tiles,
                                                         const int32_t* __restrict__ order, DevOpts op,
                                                         unsigned long long* __restrict__ counts) {
  using G = Geo<TW, TH, 1>;
  __shared__ Stage<G> s;
  TileCtx t;
  int tile;
  if (!tile_setup<G>(cams, V, n_tiles, order, t, tile)) return;
  const int2 rg = range[tile];
  bool live = t.inside;
  const float fx = (float)t.px + 0.5f, fy = (float)t.py + 0.5f;
  float T = 1.f;
  unsigned long long ev = 0, co = 0;
  for (int b0 = rg.x; b0 < rg.y; b0 += G::BATCH) {
    if (!__syncthreads_or(live)) break;
    const int nb = min(G::BATCH, rg.y - b0);
    if ((int)threadIdx.x < nb) {
      const int r = vals[b0 + threadIdx.x];
      s.A[threadIdx.x] = rec[3 * (int64_t)r];
      s.B[threadIdx.x] = rec[3 * (int64_t)r + 1];
      s.C[threadIdx.x] = rec[3 * (int64_t)r + 2];
    }
    __syncthreads();
    for (int j = 0; j < nb && live; ++j) {
      int x0, x1, y0, y1;
      unpack_rect(s.C[j], x0, x1, y0, y1);
      if (t.px < x0 || t.px > x1 || t.py < y0 || t.py > y1) continue;
      ++ev;
      float alpha, Gv, dx, dy;
      bool cl;
      if (!eval_pair(s.A[j], s.B[j], fx, fy, op, alpha, Gv, cl, dx, dy)) continue;
      const float Tn = T * (1.f - alpha);
      if (Tn < op.t_min) {
        live = false;
        continue;
      }
      ++co;
      T = Tn;
    }
  }
  // one atomic per wave (sums over the lanes first)
  for (int d = 32; d >= 1; d >>= 1) {
    ev += __shfl_xor(ev, d);
    co += __shfl_xor(co, d);
  }
  if (t.lane == 0) {
    atomicAdd(counts, ev);
    atomicAdd(counts + 1, co);
  }
}

// Valid LiDAR-depth pixels per view: grid-stride per view, one atomic per block.
__global__ __launch_bounds__(256) void k_count_valid(const float* __restrict__ tgt_depth,
                                                     const gs_camera* __restrict__ cams,
                                                     int32_t* __restrict__ n_valid, float* __restrict__ loss,
                                                     int n_loss) {
  __shared__ int sh;
  // the loss slots are cleared here too (the compositing that follows adds into them)
  if (blockIdx.x == 0 && blockIdx.y == 0 && (int)threadIdx.x < n_loss) loss[threadIdx.x] = 0.f;
  if (threadIdx.x == 0) sh = 0;
  __syncthreads();
  const int v = blockIdx.y;
  const gs_camera& c = cams[v];
  const int64_t P = (int64_t)c.width * c.height;
  int cnt = 0;
  // eight independent loads in flight per thread and pass
  const int64_t step = (int64_t)gridDim.x * blockDim.x * 8;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x * 8 + threadIdx.x; b < P; b += step) {
    float d[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t i = b + k * (int64_t)blockDim.x;
      d[k] = i < P ? tgt_depth[c.pixel_offset + i] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) cnt += d[k] > 0.f;
  }
  for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d);
  if ((threadIdx.x & 63) == 0) atomicAdd(&sh, cnt);
  __syncthreads();
  if (threadIdx.x == 0 && sh) atomicAdd(n_valid + v, sh);
}

SegArgs seg_args(const gs_frame& f) {
  SegArgs g;
  g.items = reinterpret_cast<const int4*>(f.items);
  g.counters = f.counters;
  g.order = f.tile_order;
  g.seg_count = f.seg_count;
  g.seg_first = f.seg_first;
  g.seg = f.seg;
  g.split = f.split;
  g.len = f.seg_len;
  return g;
}

// Workgroups of a persistent launch: what the GPU holds at once (compute units x resident workgroups of the
// kernel per unit), at most cap.
template <class K>
int resident_grid(K kernel, int block, int64_t cap) {
  int dev = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, 0) != hipSuccess || occ < 1) occ = 1;
  const int64_t g = (int64_t)cus * occ;
  return (int)(g < cap ? g : (cap > 0 ? cap : 1));
}

template <int TW, int TH, int DEPTH, int BW>
hipError_t launch_fwd(const gs_frame& f, const DevOpts& op, const gs_images& out, hipStream_t st) {
  const int sorted = f.sort_passes & 1;
  const auto* rec = reinterpret_cast<const float4*>(f.rec);
  const auto* rng = reinterpret_cast<const int2*>(f.tile_range);
  const int bs = TW * TH;
  if (f.seg_len > 0) {
    // long lists split into depth segments
    const SegArgs g = seg_args(f);
    k_fwd_main<TW, TH, DEPTH, BW><<<f.item_cap, bs, 0, st>>>(rec, f.vals[sorted], rng, f.cams, f.n_views, op, g, out.rgb,
                                                          out.depth, out.vis);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_seg_prefix<TW, TH, BW><<<f.long_cap, bs, 0, st>>>(g, op);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_seg_stop<TW, TH, DEPTH, BW><<<f.seg_cap, bs, 0, st>>>(rec, f.vals[sorted], rng, f.cams, f.n_views, op, g,
                                                            nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_seg_fwd_out<TW, TH, BW><<<f.long_cap, bs, 0, st>>>(f.cams, f.n_views, op, g, out.rgb, out.depth, out.vis);
    return hipGetLastError();
  }
  k_render_fwd<TW, TH, DEPTH, BW><<<f.n_tiles, bs, 0, st>>>(rec, f.vals[sorted], rng, f.cams, f.n_views, f.n_tiles,
                                                        f.tile_order, op, out.rgb, out.depth, out.vis);
  return hipGetLastError();
}

template <int TW, int TH, int DEPTH, int BW, bool HAVE_FWD, bool LOSS>
hipError_t launch_split_bwd(const gs_frame& f, const DevOpts& op, const BwdArgs& a, bool persist, hipStream_t st) {
  const int sorted = f.sort_passes & 1;
  const auto* rec = reinterpret_cast<const float4*>(f.rec);
  const auto* rng = reinterpret_cast<const int2*>(f.tile_range);
  const int32_t* vals = f.vals[sorted];
  const int bs = TW * TH;
  const SegArgs g = seg_args(f);
  hipError_t e;
  // persistent: the three walking kernels take their items from counters[199..201]
  int32_t* ctr = f.counters + 199;
  if (persist) {
    if ((e = gs_launch::fill_i32(ctr, 0, 3, st)) != hipSuccess) return e;
    auto* kf = k_fused_main<TW, TH, DEPTH, BW, HAVE_FWD, LOSS, true>;
    kf<<<resident_grid(kf, bs, f.item_cap), bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, op, a, g, ctr);
  } else {
    k_fused_main<TW, TH, DEPTH, BW, HAVE_FWD, LOSS><<<f.item_cap, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, op,
                                                                                a, g, nullptr);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_seg_prefix<TW, TH, BW><<<f.long_cap, bs, 0, st>>>(g, op);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (persist) {
    auto* ks = k_seg_stop<TW, TH, DEPTH, BW, true>;
    ks<<<resident_grid(ks, bs, f.seg_cap), bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, op, g, ctr + 1);
  } else {
    k_seg_stop<TW, TH, DEPTH, BW><<<f.seg_cap, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, op, g, nullptr);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_seg_combine<TW, TH, BW, HAVE_FWD, LOSS><<<f.long_cap, bs, 0, st>>>(f.cams, f.n_views, op, a, g);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (persist) {
    auto* kb = k_seg_bwd<TW, TH, DEPTH, BW, true>;
    kb<<<resident_grid(kb, bs, f.seg_cap), bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, op, a, g, ctr + 2);
  } else {
    k_seg_bwd<TW, TH, DEPTH, BW><<<f.seg_cap, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, op, a, g, nullptr);
  }
  return hipGetLastError();
}

template <int TW, int TH, int DEPTH, int BW>
hipError_t launch_bwd(const gs_frame& f, const DevOpts& op, bool have_fwd, bool loss, const BwdArgs& a, bool persist,
                      hipStream_t st) {
  if (f.seg_len > 0) {
    // long lists split into depth segments
    if (have_fwd && loss) return launch_split_bwd<TW, TH, DEPTH, BW, true, true>(f, op, a, persist, st);
    if (have_fwd) return launch_split_bwd<TW, TH, DEPTH, BW, true, false>(f, op, a, persist, st);
    if (loss) return launch_split_bwd<TW, TH, DEPTH, BW, false, true>(f, op, a, persist, st);
    return launch_split_bwd<TW, TH, DEPTH, BW, false, false>(f, op, a, persist, st);
  }
  const int sorted = f.sort_passes & 1;
  const auto* rec = reinterpret_cast<const float4*>(f.rec);
  const auto* rng = reinterpret_cast<const int2*>(f.tile_range);
  const int nb = f.n_tiles, bs = TW * TH;
  const int32_t* vals = f.vals[sorted];
  if (have_fwd && loss)
    k_render_bwd<TW, TH, DEPTH, BW, true, true><<<nb, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, nb, f.tile_order,
                                                               op, a);
  else if (have_fwd)
    k_render_bwd<TW, TH, DEPTH, BW, true, false><<<nb, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, nb,
                                                                f.tile_order, op, a);
  else if (loss)
    k_render_bwd<TW, TH, DEPTH, BW, false, true><<<nb, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, nb,
                                                                f.tile_order, op, a);
  else
    k_render_bwd<TW, TH, DEPTH, BW, false, false><<<nb, bs, 0, st>>>(rec, vals, rng, f.cams, f.n_views, nb,
                                                                 f.tile_order, op, a);
  return hipGetLastError();
}

template <int TW, int TH>
hipError_t launch_count(const gs_frame& f, const DevOpts& op, unsigned long long* counts, hipStream_t st) {
  const int sorted = f.sort_passes & 1;
  k_count_pairs<TW, TH><<<f.n_tiles, TW * TH, 0, st>>>(
      reinterpret_cast<const float4*>(f.rec), f.vals[sorted], reinterpret_cast<const int2*>(f.tile_range), f.cams,
      f.n_views, f.n_tiles, f.tile_order, op, counts);
  return hipGetLastError();
}

}  // namespace

namespace gs_launch {

// Tile shape (one wave per 8x8 sub-tile), records staged per thread (o.batch_depth; 0 means 1) and block
// width (o.block_w; 0 means 4).
#define GS_TILE_DISPATCH_B(FN, TW, TH, DP, ...)                     \
  do {                                                              \
    if (o.block_w == 8) return FN<TW, TH, DP, 8>(__VA_ARGS__);      \
    if (o.block_w == 2) return FN<TW, TH, DP, 2>(__VA_ARGS__);      \
    return FN<TW, TH, DP, 4>(__VA_ARGS__);                          \
  } while (0)
#define GS_TILE_DISPATCH_D(FN, TW, TH, ...)                                       \
  do {                                                                            \
    if (o.batch_depth == 2) GS_TILE_DISPATCH_B(FN, TW, TH, 2, __VA_ARGS__);      \
    GS_TILE_DISPATCH_B(FN, TW, TH, 1, __VA_ARGS__);                              \
  } while (0)
#define GS_TILE_DISPATCH(FN, ...)                                                      \
  do {                                                                                 \
    if (o.tile_w == 16 && o.tile_h == 16) GS_TILE_DISPATCH_D(FN, 16, 16, __VA_ARGS__); \
    if (o.tile_w == 16 && o.tile_h == 8) GS_TILE_DISPATCH_D(FN, 16, 8, __VA_ARGS__);   \
    if (o.tile_w == 8 && o.tile_h == 8) GS_TILE_DISPATCH_D(FN, 8, 8, __VA_ARGS__);     \
    if (o.tile_w == 32 && o.tile_h == 8) GS_TILE_DISPATCH_D(FN, 32, 8, __VA_ARGS__);   \
    return hipErrorInvalidValue;                                                       \
  } while (0)

hipError_t render_fwd(const gs_frame& f, const gs_opts& o, const gs_images& out, hipStream_t st) {
  const DevOpts op = gsk::dev_opts(o);
  GS_TILE_DISPATCH(launch_fwd, f, op, out, st);
}

hipError_t count_pairs(const gs_frame& f, const gs_opts& o, unsigned long long* counts, hipStream_t st) {
  const DevOpts op = gsk::dev_opts(o);
  if (o.tile_w == 16 && o.tile_h == 16) return launch_count<16, 16>(f, op, counts, st);
  if (o.tile_w == 16 && o.tile_h == 8) return launch_count<16, 8>(f, op, counts, st);
  if (o.tile_w == 8 && o.tile_h == 8) return launch_count<8, 8>(f, op, counts, st);
  if (o.tile_w == 32 && o.tile_h == 8) return launch_count<32, 8>(f, op, counts, st);
  return hipErrorInvalidValue;
}

hipError_t loss_total(float* loss, hipStream_t st) {
  k_loss_total<<<1, 64, 0, st>>>(loss);
  return hipGetLastError();
}

hipError_t count_valid(const gs_frame& f, const float* tgt_depth, int64_t max_pixels, float* loss, int n_loss,
                       hipStream_t st) {
  hipError_t e = fill_i32(f.counters + 2, 0, f.n_views, st);
  if (e != hipSuccess) return e;
  int64_t bx = (max_pixels + 256 * 32 - 1) / (256 * 32);
  if (bx < 1) bx = 1;
  dim3 grid((unsigned)bx, (unsigned)f.n_views);
  k_count_valid<<<grid, 256, 0, st>>>(tgt_depth, f.cams, f.counters + 2, loss, n_loss);
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
  a.lambda_ssim = l.lambda_ssim;
  a.ipart = f.ipart;
  a.rec_slot = f.rec_slot;
  a.capacity = f.capacity;
  a.loss = f.loss;
  const bool loss = l.tgt_rgb != nullptr;
  GS_TILE_DISPATCH(launch_bwd, f, op, fwd != nullptr, loss, a, o.persistent != 0, st);
}

}  // namespace gs_launch
