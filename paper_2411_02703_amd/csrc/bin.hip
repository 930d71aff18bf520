// Tile binning (integer work, bit-exact by construction).  The order inside a tile is ascending depth bits, ties
// by record index, so the sorted order is unique.  Two stable LSD radix sorts (8-bit digits) reach it:
//   1. the visible records, listed wave by wave and view by view (Gaussians ascending inside a view), are sorted
//      by their 32-bit depth bits (4 passes over the records, not the instances);
//   2. the records are emitted in that order, each as its run of tile instances (key = global tile id, value =
//      record id), and the instances are sorted by tile (2 passes at up to 65,536 tiles).
// A stable sort by tile of a depth-ordered sequence is the (tile, depth, record) order; ties in depth keep
// ascending Gaussian index inside a view (the records of one view are listed in Gaussian order), and records
// of different views never share a tile.  The sorted value of an instance is its record id.
//
// The compositing backward stores each instance's partial derivatives at a slot of its own, laid out Gaussian by
// Gaussian (the exclusive scan of the per-Gaussian instance counts), views ascending inside a Gaussian, a
// record's tiles row by row: each record's first slot is written here, in Gaussian order, so that the projection
// backward reads one contiguous run per Gaussian.
#include "common.h"

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;  // 2048 keys per block
constexpr int kWaveItems = kSortTile / 4;              // 512 keys per wave

// Exclusive scan of 256 values, one per thread; returns the exclusive prefix, *total = sum.
__device__ __forceinline__ int block_scan_256(int x, int* sh_wave, int* total) {
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  int incl = x;
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d);
    if (lane >= d) incl += y;
  }
  if (lane == 63) sh_wave[wave] = incl;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wave; ++w) base += sh_wave[w];
  *total = sh_wave[0] + sh_wave[1] + sh_wave[2] + sh_wave[3];
  __syncthreads();
  return base + incl - x;
}

// Each block scans kScanTile consecutive items (exclusive) and writes its total.  The items scanned are the
// first dev_count(dc, n): blocks past them only write a zero total.  A launch with gridDim.y = 2 scans a second
// array of the same length in its second row of blocks (in_b, out_b, sums_b).
__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const int32_t* in, int32_t* out, int64_t n_sized,
                                                          int32_t* sums, gs_launch::DevCount dc,
                                                          const int32_t* in_b = nullptr, int32_t* out_b = nullptr,
                                                          int32_t* sums_b = nullptr) {
  if (blockIdx.y) {
    in = in_b;
    out = out_b;
    sums = sums_b;
  }
  __shared__ int sh_wave[4];
  const int64_t n = gs_launch::dev_count(dc, n_sized);
  if ((int64_t)blockIdx.x * kScanTile >= n) {
    if (threadIdx.x == 0) sums[blockIdx.x] = 0;
    return;
  }
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  // a thread's 16 items as four 16-byte loads and stores when they are all in range and the arrays are aligned
  const bool vec = base + kScanItems <= n &&
                   ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  int v[kScanItems];
  if (vec) {
    const int4* p = reinterpret_cast<const int4*>(in + base);
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
      const int4 x = p[q];
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const int64_t idx = base + i;
      v[i] = idx < n ? in[idx] : 0;
    }
  }
  int acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) acc += v[i];
  int total;
  int run = block_scan_256(acc, sh_wave, &total);
  int o[kScanItems];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    o[i] = run;
    run += v[i];
  }
  if (vec) {
    int4* p = reinterpret_cast<int4*>(out + base);
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) p[q] = make_int4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const int64_t idx = base + i;
      if (idx < n) out[idx] = o[i];
    }
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t* out, int64_t n_sized, const int32_t* sums,
                                                         gs_launch::DevCount dc, int32_t* out_b = nullptr,
                                                         const int32_t* sums_b = nullptr) {
  if (blockIdx.y) {
    out = out_b;
    sums = sums_b;
  }
  const int64_t n = gs_launch::dev_count(dc, n_sized);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n) return;
  const int add = sums[blockIdx.x];
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
    const int64_t idx = base + i;
    if (idx < n) out[idx] += add;
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// Two int32 ranges set to v in one launch: [p, p + n) and [q, q + m).
__global__ void k_fill2_i32(int32_t* __restrict__ p, int64_t n, int32_t* __restrict__ q, int64_t m, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
  if (i < m) q[i] = v;
}
__global__ void k_fill_f32(float* __restrict__ p, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__device__ __forceinline__ int64_t sort_count(const int32_t* count_dev, int64_t n_sized, int64_t cap) {
  if (count_dev == nullptr) return n_sized;
  const int64_t c = count_dev[0];
  return c < cap ? c : cap;
}

template <class KeyT>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const KeyT* __restrict__ keys,
                                                           const int32_t* __restrict__ count_dev, int64_t n_sized,
                                                           int64_t cap, int shift, int32_t* __restrict__ hist) {
  __shared__ int h[256];
  const int64_t n = sort_count(count_dev, n_sized, cap);
  // digit-major histogram over the blocks that hold keys: hist[d * nb + b]
  const int nb = (int)((n + kSortTile - 1) / kSortTile);
  if ((int)blockIdx.x >= nb) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t idx = base + i * kSortThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(int)((keys[idx] >> shift) & 255u)], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one 8-bit digit.  Each wave ranks its 512 keys (8 rounds of 64) with ballot-based
// digit matching, the block orders them in LDS (digit-major, stable), then writes runs to their global
// offsets from the scanned digit-major histogram (entry d * nb + b over the nb blocks that hold keys: the
// tile-local scan hist_scan plus the scanned total of its scan tile, tile_scan).
// Histogram scans of at most this many tiles can be finished inside the scatter (each block scans the tile
// totals itself, four per thread); whether they are is the caller's choice (fold_tiles), since with many keys
// per pass the scatter's extra phase costs more than the separate pass it saves.
constexpr int kFoldTiles = 4 * kSortThreads;

template <class KeyT, bool FOLD>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const KeyT* __restrict__ kin,
                                                              const int32_t* __restrict__ vin,
                                                              KeyT* __restrict__ kout, int32_t* __restrict__ vout,
                                                              const int32_t* __restrict__ count_dev, int64_t n_sized,
                                                              int64_t cap, int shift,
                                                              const int32_t* __restrict__ hist_scan,
                                                              const int32_t* __restrict__ tile_scan) {
  __shared__ KeyT sk[kSortTile];
  __shared__ int32_t sv[kSortTile];
  __shared__ int32_t wcnt[4][256];
  __shared__ int32_t dstart[256];
  __shared__ int32_t gofs[256];
  __shared__ int sh_wave[4];
  __shared__ int32_t tsc[FOLD ? kFoldTiles : 1];
  const int64_t n = sort_count(count_dev, n_sized, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= n) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = __lane_id();
  for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
  if (FOLD) {
    // tile_scan holds the scan tiles' raw totals: every block forms their exclusive scan itself (at most
    // kFoldTiles values, four per thread), in place of a separate pass over them
    const int nbt = (int)((256 * ((n + kSortTile - 1) / kSortTile) + kScanTile - 1) / kScanTile);
    int t[4], sum = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = 4 * tid + i;
      t[i] = idx < nbt ? tile_scan[idx] : 0;
      sum += t[i];
    }
    int total;
    int run = block_scan_256(sum, sh_wave, &total);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      tsc[4 * tid + i] = run;
      run += t[i];
    }
  }
  __syncthreads();
  KeyT key[kSortItems];
  int32_t val[kSortItems];
  int pos[kSortItems];
  const uint64_t lt = gsk::lanemask_lt();
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t idx = base + (int64_t)wave * kWaveItems + k * 64 + lane;
    const bool valid = idx < n;
    key[k] = valid ? kin[idx] : KeyT(0);
    val[k] = valid ? vin[idx] : 0;
    const int d = (int)((key[k] >> shift) & 255u);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const int rank = __popcll(peers & lt);
    int before = 0;
    if (valid) before = wcnt[wave][d];
    pos[k] = before + rank;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) wcnt[wave][d] = before + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {
    const int c0 = wcnt[0][tid], c1 = wcnt[1][tid], c2 = wcnt[2][tid], c3 = wcnt[3][tid];
    int total;
    const int ds = block_scan_256(c0 + c1 + c2 + c3, sh_wave, &total);
    dstart[tid] = ds;
    wcnt[0][tid] = ds;
    wcnt[1][tid] = ds + c0;
    wcnt[2][tid] = ds + c0 + c1;
    wcnt[3][tid] = ds + c0 + c1 + c2;
    const int hi = tid * (int)((n + kSortTile - 1) / kSortTile) + blockIdx.x;
    gofs[tid] = hist_scan[hi] + (FOLD ? tsc[hi / kScanTile] : tile_scan[hi / kScanTile]);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t idx = base + (int64_t)wave * kWaveItems + k * 64 + lane;
    if (idx < n) {
      const int d = (int)((key[k] >> shift) & 255u);
      const int p = wcnt[wave][d] + pos[k];
      sk[p] = key[k];
      sv[p] = val[k];
    }
  }
  __syncthreads();
  const int64_t rem = n - base;
  const int nvalid = rem < kSortTile ? (int)rem : kSortTile;
  for (int p = tid; p < nvalid; p += kSortThreads) {
    const KeyT kk = sk[p];
    const int d = (int)((kk >> shift) & 255u);
    const int64_t o = (int64_t)gofs[d] + (p - dstart[d]);
    kout[o] = kk;
    vout[o] = sv[p];
  }
}

// ------------------------------------------------------------------ the record list and the emission
// Visible records listed wave by wave (64 consecutive Gaussians), view by view inside a wave, Gaussians ascending
// inside a view: key = depth bits, value = record id.  The count
// R goes to counters[kRecCount] (entries past the record capacity are not written; R > capacity implies more
// instances than the instance capacity, which the instance total flags).
constexpr int kRecCount = 196;
// The instance total: the end of the exclusive scan of the per-Gaussian instance counts (the full count even
// when the record list itself overflowed), set by the record list's first thread.
constexpr int kInstSum = 197;

__device__ __forceinline__ int rect_area(const short4 rc) { return (rc.y - rc.x + 1) * (rc.w - rc.z + 1); }

// ... and each visible record's first partial slot.  The instances of a wave's 64 Gaussians occupy one run of
// slots from inst_first[g0] (g0 the wave's first Gaussian), laid out in the record list's order: view by view,
// Gaussians ascending within a view; so the projection backward, which takes the views together, reads each
// view's partials of the wave as one contiguous run.  Wide records (more than kWideRecord tiles) are appended
// to big_rec (count in counters[kBigCount], one atomic per wave; the list order is not fixed, which nothing
// depends on).
constexpr int kBigCount = 198;

__global__ __launch_bounds__(256) void k_record_list(const uint64_t* __restrict__ vis_mask,
                                                    const int32_t* __restrict__ n_rec,
                                                    const int32_t* __restrict__ first,
                                                    const int32_t* __restrict__ inst_first,
                                                    const int32_t* __restrict__ n_inst,
                                                    const short4* __restrict__ rect,
                                                    const uint32_t* __restrict__ zbits, int V, int64_t n, int64_t rcap,
                                                    uint32_t* __restrict__ rkeys, int32_t* __restrict__ rvals,
                                                    int32_t* __restrict__ rec_slot, int32_t* __restrict__ big_rec,
                                                    int32_t* __restrict__ counters, int64_t capacity) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) {
    // the record count R, and counters[0] = the instance total (the end of the per-Gaussian instance scan; the
    // full count) with the overflow flag if it is above the capacity
    counters[kRecCount] = first[n - 1] + n_rec[n - 1];
    const int64_t total = (int64_t)inst_first[n - 1] + n_inst[n - 1];
    counters[kInstSum] = (int32_t)total;
    counters[0] = (int32_t)total;
    if (total > capacity) atomicOr(counters + 1, GS_FLAG_INSTANCE_OVERFLOW);
  }
  const bool here = g < n;
  const uint64_t m = here ? vis_mask[g] : 0ull;
  // The wave's records start where its first Gaussian's do (the scan of the record counts) and are listed view
  // by view, each view's records in lane (Gaussian) order, so that every read and write of a view is one
  // coalesced run.  Within a view the list keeps ascending Gaussian index, which is all the depth sort's tie rule
  // needs (records of different views never share a tile).
  const int64_t g0 = g - __lane_id();
  int64_t c = __builtin_amdgcn_readfirstlane((int)(g0 < n ? first[g0] : 0));
  int32_t slot_c = __builtin_amdgcn_readfirstlane((int)(g0 < n ? inst_first[g0] : 0));
  const uint64_t lt = gsk::lanemask_lt();
  for (int v = 0; v < V; ++v) {
    const bool vis = (m >> v) & 1ull;
    const uint64_t vb = __ballot(vis);
    if (vb == 0) continue;
    const int64_t pos = c + __popcll(vb & lt);
    c += __popcll(vb);
    const int64_t r = (int64_t)v * n + g;
    const int area = vis ? rect_area(rect[r]) : 0;
    int view_total;
    const int before = gsk::wave_excl_scan(area, view_total);
    const int32_t slot = slot_c + before;
    slot_c += view_total;
    if (!vis) continue;
    if (pos < rcap) {
      rkeys[pos] = zbits[r];
      rvals[pos] = (int32_t)r;
    }
    rec_slot[r] = slot;
    const bool wide = area > gsk::kWideRecord;
    const uint64_t wb = __ballot(wide);
    if (wb) {
      const int lead = __builtin_ctzll(wb);
      int base = 0;
      if (__lane_id() == lead) base = atomicAdd(counters + kBigCount, __popcll(wb));
      base = __builtin_amdgcn_readlane(base, lead);
      const int bpos = base + __popcll(wb & lt);
      if (wide && bpos < rcap) big_rec[bpos] = (int32_t)r;
    }
  }
}

// Instance count of each depth-sorted record (its tile rectangle's area), and the rectangle itself in sorted
// order (tx0 | tx1 << 16 in rx[j], ty0 | ty1 << 16 in ry[j]) so that the emission reads it in coalesced runs.
__global__ void k_record_counts(const int32_t* __restrict__ rvals, const short4* __restrict__ rect,
                                const int32_t* __restrict__ counters, int64_t rcap, int32_t* __restrict__ cnt,
                                uint32_t* __restrict__ rx, uint32_t* __restrict__ ry) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= sort_count(counters + kRecCount, rcap, rcap)) return;
  const short4 rc = rect[rvals[j]];
  cnt[j] = rect_area(rc);
  rx[j] = (uint32_t)(uint16_t)rc.x | ((uint32_t)(uint16_t)rc.y << 16);
  ry[j] = (uint32_t)(uint16_t)rc.z | ((uint32_t)(uint16_t)rc.w << 16);
}

// Records with more tiles than this are emitted by a whole wave, a tile per lane.
constexpr int kSolo = gsk::kWideRecord;

__device__ __forceinline__ int64_t read_lane64(int64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One thread per depth-sorted record: its run of instances (tiles row by row) starts at eo[j]; key = global tile
// id, value = record id.  Records with more than kSolo tiles are written by the whole wave, a tile per lane.  The
// runs of a wave's records are consecutive (eo is their exclusive scan), so the other records are first laid out
// in a per-wave LDS window of kEmitWin instances and then stored by the wave in coalesced runs, a window at a
// time; positions of wide records in a window are marked empty and skipped by the copy.
constexpr int kEmitWin = 512;
constexpr uint32_t kEmitEmpty = 0xffffffffu;  // no tile id takes this value

__global__ __launch_bounds__(256) void k_emit(const int32_t* __restrict__ rvals, const int32_t* __restrict__ eo,
                                             const uint32_t* __restrict__ rx, const uint32_t* __restrict__ ry,
                                             const gs_camera* __restrict__ cams,
                                             int V, int64_t n, const int32_t* __restrict__ counters, int64_t rcap,
                                             int64_t capacity, uint32_t* __restrict__ keys,
                                             int32_t* __restrict__ vals) {
  __shared__ uint32_t wkey[4][kEmitWin];
  __shared__ int32_t wval[4][kEmitWin];
  const int64_t R = sort_count(counters + kRecCount, rcap, rcap);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool here = j < R;
  int64_t r = 0, o = 0;
  short4 rc = make_short4(0, -1, 0, -1);
  int toff = 0, tx_n = 1;
  if (here) {
    r = rvals[j];
    o = eo[j];
    const uint32_t x = rx[j], y = ry[j];
    rc = make_short4((short)(x & 0xffffu), (short)(x >> 16), (short)(y & 0xffffu), (short)(y >> 16));
    const int v = (int)((uint32_t)r / (uint32_t)n);  // r < 2^31
    toff = cams[v].tile_offset;
    tx_n = cams[v].tiles_x;
  }
  const int w = rc.y - rc.x + 1, cnt = here ? w * (rc.w - rc.z + 1) : 0;
  const uint64_t present = __ballot(here);
  if (present == 0) return;  // the same in every lane of the wave
  uint64_t big = __ballot(cnt > kSolo);
  // the wave's instances are [lo, hi): the records of lanes 0 .. last are consecutive in the sorted list
  const int last = 63 - __builtin_clzll(present);
  const int64_t lo = read_lane64(o, 0), hi = read_lane64(o + cnt, last);
  uint32_t* wk = wkey[wv];
  int32_t* wvv = wval[wv];
  for (int64_t win = lo; win < hi; win += kEmitWin) {
    if (big) {
      for (int i = lane; i < kEmitWin; i += 64) wk[i] = kEmitEmpty;
    }
    if (here && cnt <= kSolo) {
      const int64_t k0 = max(o, win) - o, k1 = min(o + cnt, win + kEmitWin) - o;
      if (k0 < k1) {
        int ty = rc.z + (int)k0 / w, tx = rc.x + (int)k0 % w;
        for (int64_t k = k0; k < k1; ++k) {
          const int i = (int)(o + k - win);
          wk[i] = (uint32_t)(toff + ty * tx_n + tx);
          wvv[i] = (int32_t)r;
          if (++tx > rc.y) {
            tx = rc.x;
            ++ty;
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // the wave's LDS writes land before its reads
    const int m = (int)min<int64_t>(kEmitWin, hi - win);
    for (int i = lane; i < m; i += 64) {
      const uint32_t kk = wk[i];
      const int64_t q = win + i;
      if (kk != kEmitEmpty && q < capacity) {
        keys[q] = kk;
        vals[q] = wvv[i];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // and its reads before the next window's writes
  }
  while (big) {
    const int L = __builtin_ctzll(big);
    big &= big - 1;
    const int64_t oL = read_lane64(o, L), rL = read_lane64(r, L);
    const int cL = __builtin_amdgcn_readlane(cnt, L), wL = __builtin_amdgcn_readlane(w, L);
    const int x0 = __builtin_amdgcn_readlane((int)rc.x, L), y0 = __builtin_amdgcn_readlane((int)rc.z, L);
    const int toL = __builtin_amdgcn_readlane(toff, L), txL = __builtin_amdgcn_readlane(tx_n, L);
    for (int k = lane; k < cL; k += 64) {
      const int64_t q = oL + k;
      if (q < capacity) {
        const int ty = y0 + k / wL, tx = x0 + k % wL;
        keys[q] = (uint32_t)(toL + ty * txL + tx);
        vals[q] = (int32_t)rL;
      }
    }
  }
}

__global__ void k_ranges(const uint32_t* __restrict__ keys, const int32_t* __restrict__ count_dev, int64_t n_sized,
                         int64_t cap, int2* __restrict__ range) {
  const int64_t n = sort_count(count_dev, n_sized, cap);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = keys[i];
  if (i == 0 || keys[i - 1] != t) range[t].x = (int)i;
  if (i == n - 1 || keys[i + 1] != t) range[t].y = (int)(i + 1);
}

// Compositing schedule: tiles in descending order of their list length, bucketed by floor(log2(len + 1))
// (32 buckets, longest first; the order inside a bucket does not matter).  Tiles longer than the segment
// length (split into depth segments by the fused backward) all go to bucket 0, so they lead the schedule.
__device__ __forceinline__ int len_bucket(const int2* range, int t, int seg_len) {
  const int len = range[t].y - range[t].x;
  if (seg_len > 0 && len > seg_len) return 0;
  return __clz((unsigned)len + 1u);  // 31 - floor(log2(len + 1)): longer lists get smaller bucket ids
}

__global__ __launch_bounds__(256) void k_sched_hist(const int2* __restrict__ range, int n_tiles, int seg_len,
                                                    int32_t* __restrict__ bucket_cnt) {
  __shared__ int h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_tiles) atomicAdd(&h[len_bucket(range, t, seg_len)], 1);
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(bucket_cnt + threadIdx.x, h[threadIdx.x]);
}

__global__ void k_sched_scan(const int32_t* __restrict__ bucket_cnt, int32_t* __restrict__ bucket_off) {
  if (threadIdx.x != 0) return;
  int run = 0;
  for (int b = 0; b < 32; ++b) {
    bucket_off[b] = run;
    run += bucket_cnt[b];
  }
}

__global__ __launch_bounds__(256) void k_sched_scatter(const int2* __restrict__ range, int n_tiles, int seg_len,
                                                       int32_t* __restrict__ bucket_off, int32_t* __restrict__ order) {
  __shared__ int h[32], base[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0, rank = 0;
  if (t < n_tiles) {
    b = len_bucket(range, t, seg_len);
    rank = atomicAdd(&h[b], 1);
  }
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x]) base[threadIdx.x] = atomicAdd(bucket_off + threadIdx.x, h[threadIdx.x]);
  __syncthreads();
  if (t < n_tiles) order[base[b] + rank] = t;
}

// Work items of the fused backward, in schedule order: one per tile, or one per depth segment of a tile
// longer than seg_len (those lead the schedule, so their segments take item indices 0 .. slots - 1, which
// are also their segment-state slots).
__global__ __launch_bounds__(256) void k_seg_count(const int2* __restrict__ range, const int32_t* __restrict__ order,
                                                   int n_tiles, int seg_len, int32_t* __restrict__ seg_count) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_tiles) return;
  const int2 r = range[order[p]];
  const int len = r.y - r.x;
  seg_count[p] = len > seg_len ? (len + seg_len - 1) / seg_len : 1;
}

__global__ __launch_bounds__(256) void k_seg_emit(const int32_t* __restrict__ order, int n_tiles,
                                                  const int32_t* __restrict__ seg_count,
                                                  const int32_t* __restrict__ seg_first, int4* __restrict__ items,
                                                  int32_t* __restrict__ counters) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) {
    const int nl = counters[128];  // bucket 0: split tiles
    counters[194] = nl;
    counters[193] = nl > 0 ? seg_first[nl - 1] + seg_count[nl - 1] : 0;
    counters[192] = seg_first[n_tiles - 1] + seg_count[n_tiles - 1];
  }
  if (p >= n_tiles) return;
  const int n = seg_count[p], first = seg_first[p], t = order[p];
  for (int k = 0; k < n; ++k) items[first + k] = make_int4(t, k, n > 1 ? first : -1, p);
}

// Frames of at most kSchedOneBlock tiles: the schedule and the work items in one workgroup, each phase a loop
// over the tiles between barriers (bucket histogram; its scan; the scatter into schedule order, which also
// stores each position's segment count; the scan of the segment counts with the items), in place of the seven
// launches above, whose fixed cost dominates there.  The results are those of the launches above (the order
// inside a bucket is again that of the LDS atomics).  Without segments (seg_len <= 0) only the schedule.
constexpr int kSchedOneBlock = 16384;

__global__ __launch_bounds__(1024) void k_schedule_small(const int2* __restrict__ range, int n_tiles, int seg_len,
                                                         int32_t* __restrict__ order, int32_t* __restrict__ seg_count,
                                                         int32_t* __restrict__ seg_first, int4* __restrict__ items,
                                                         int32_t* __restrict__ counters) {
  __shared__ int h[32], base[32], wsum[16];
  const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  if (tid < 32) h[tid] = 0;
  __syncthreads();
  // each thread's list lengths, loaded once (all loads in flight together) and kept for the scatter
  constexpr int kPer = kSchedOneBlock / 1024;
  int lens[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int t = j * 1024 + tid;
    lens[j] = t < n_tiles ? range[t].y - range[t].x : -1;
  }
  auto bucket = [&](int len) { return len < 0 ? 32 : (seg_len > 0 && len > seg_len ? 0 : __clz((unsigned)len + 1u)); };
  // the LDS atomics are taken once per distinct bucket of a wave (a wave's tiles fall into a few buckets, and
  // atomics of many lanes on one address serialise)
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (j * 1024 >= n_tiles) break;
    const int b = bucket(lens[j]);
    for (uint64_t rest = __builtin_amdgcn_ballot_w64(b < 32); rest;) {
      const int lb = __builtin_amdgcn_readlane(b, __builtin_ctzll(rest));
      const uint64_t m = __builtin_amdgcn_ballot_w64(b == lb);
      if (lane == 0) atomicAdd(&h[lb], __popcll(m));
      rest &= ~m;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int b = 0; b < 32; ++b) {
      base[b] = run;
      counters[128 + b] = h[b];
      run += h[b];
      counters[160 + b] = run;
    }
  }
  __syncthreads();
  const uint64_t lt = gsk::lanemask_lt();
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (j * 1024 >= n_tiles) break;
    const int t = j * 1024 + tid, len = lens[j], b = bucket(len);
    int pos = 0;
    for (uint64_t rest = __builtin_amdgcn_ballot_w64(b < 32); rest;) {
      const int lb = __builtin_amdgcn_readlane(b, __builtin_ctzll(rest));
      const uint64_t m = __builtin_amdgcn_ballot_w64(b == lb);
      int at = 0;
      if (lane == 0) at = atomicAdd(&base[lb], __popcll(m));
      at = __builtin_amdgcn_readlane(at, 0);
      if (b == lb) pos = at + __popcll(m & lt);
      rest &= ~m;
    }
    if (b < 32) {
      order[pos] = t;
      if (seg_len > 0) seg_count[pos] = len > seg_len ? (len + seg_len - 1) / seg_len : 1;
    }
  }
  if (seg_len <= 0) return;
  __syncthreads();  // order and seg_count of this workgroup visible to all its threads
  const int nl = h[0];
  int carry = 0;
  for (int c0 = 0; c0 < n_tiles; c0 += 4096) {  // four consecutive positions per thread
    const int p0 = c0 + 4 * tid;
    int cnt[4], til[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cnt[j] = p0 + j < n_tiles ? seg_count[p0 + j] : 0;
      til[j] = p0 + j < n_tiles ? order[p0 + j] : 0;
      sum += cnt[j];
    }
    int wt;
    const int ex = gsk::wave_excl_scan(sum, wt);
    if (lane == 0) wsum[wave] = wt;
    __syncthreads();
    int before = 0, chunk = 0;
    for (int w = 0; w < 16; ++w) {
      before += w < wave ? wsum[w] : 0;
      chunk += wsum[w];
    }
    int first = carry + before + ex;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int p = p0 + j, n = cnt[j];
      if (p < n_tiles) {
        seg_first[p] = first;
        for (int k = 0; k < n; ++k) items[first + k] = make_int4(til[j], k, n > 1 ? first : -1, p);
        if (p == nl - 1) counters[193] = first + n;
      }
      first += n;
    }
    carry += chunk;
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (tid == 0) {
    counters[194] = nl;
    if (nl == 0) counters[193] = 0;
    counters[192] = carry;
  }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t align64(int64_t a) { return (a + 63) & ~int64_t(63); }

}  // namespace

namespace gs_launch {

size_t scan_scratch_ints(int64_t n) {
  size_t total = 0;
  while (n > 1) {
    n = cdiv(n, kScanTile);
    total += (size_t)align64(n);
  }
  return total + 64;
}

hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch, hipStream_t st, DevCount dc) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = cdiv(n, kScanTile);
  int32_t* sums = scratch;
  k_scan_tile<<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, n, sums, dc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nb > 1) {
    e = scan_exclusive(sums, sums, nb, scratch + align64(nb), st, DevCount{});
    if (e != hipSuccess) return e;
    k_scan_add<<<(unsigned)nb, kScanThreads, 0, st>>>(out, n, sums, dc);
    return hipGetLastError();
  }
  return hipSuccess;
}

// Two exclusive scans of arrays of the same length in the launches of one (each kernel covers both).  Scratch:
// 2 * scan_scratch_ints(n).
static hipError_t scan_exclusive_pair(const int32_t* in0, int32_t* out0, const int32_t* in1, int32_t* out1,
                                      int64_t n, int32_t* scratch, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = cdiv(n, kScanTile);
  int32_t* sums0 = scratch;
  int32_t* sums1 = scratch + align64(nb);
  k_scan_tile<<<dim3((unsigned)nb, 2), kScanThreads, 0, st>>>(in0, out0, n, sums0, DevCount{}, in1, out1, sums1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 1) return e;
  if ((e = scan_exclusive_pair(sums0, sums0, sums1, sums1, nb, scratch + 2 * align64(nb), st)) != hipSuccess)
    return e;
  k_scan_add<<<dim3((unsigned)nb, 2), kScanThreads, 0, st>>>(out0, n, sums0, DevCount{}, out1, sums1);
  return hipGetLastError();
}

// The first two phases of scan_exclusive: out holds each kScanTile tile's exclusive scan and scratch[0 ..) the
// exclusive scan of the tile totals, so the exclusive scan at i is out[i] + scratch[i / kScanTile] (for a
// consumer that reads each entry once, in place of the pass that would add them).
static hipError_t scan_exclusive_tiles(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch, hipStream_t st,
                                       DevCount dc) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = cdiv(n, kScanTile);
  k_scan_tile<<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, n, scratch, dc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return scan_exclusive(scratch, scratch, nb, scratch + align64(nb), st, DevCount{});
}

hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill_i32<<<(unsigned)cdiv(n, 256), 256, 0, st>>>(p, v, n);
  return hipGetLastError();
}

hipError_t fill_f32(float* p, float v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill_f32<<<(unsigned)cdiv(n, 256), 256, 0, st>>>(p, v, n);
  return hipGetLastError();
}

size_t sort_scratch_ints(int64_t n) {
  const int64_t nb = cdiv(n > 0 ? n : 1, kSortTile);
  return (size_t)align64(256 * nb) + scan_scratch_ints(256 * nb);
}

template <class KeyT>
static hipError_t sort_impl(KeyT* k0, int32_t* v0, KeyT* k1, int32_t* v1, int64_t n_sized, const int32_t* count_dev,
                            int64_t cap, int key_bits, int32_t* scratch, hipStream_t st, int fold_tiles) {
  if (n_sized <= 0) return hipSuccess;
  const int64_t nb = cdiv(n_sized, kSortTile);
  int32_t* hist = scratch;
  int32_t* scan_scr = scratch + align64(256 * nb);
  const int passes = (key_bits + 7) / 8;
  KeyT* kb[2] = {k0, k1};
  int32_t* vb[2] = {v0, v1};
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    const int src = p & 1, dst = src ^ 1;
    k_sort_hist<KeyT><<<(unsigned)nb, kSortThreads, 0, st>>>(kb[src], count_dev, n_sized, cap, shift, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the histogram holds 256 * cdiv(count, kSortTile) entries; the scatter adds the scanned tile totals itself
    // (and, for at most kFoldTiles scan tiles, scans those totals itself too)
    const DevCount dc{count_dev, cap, kSortTile, 256};
    if (cdiv(256 * nb, kScanTile) <= fold_tiles) {
      k_scan_tile<<<(unsigned)cdiv(256 * nb, kScanTile), kScanThreads, 0, st>>>(hist, hist, 256 * nb, scan_scr, dc);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      k_sort_scatter<KeyT, true><<<(unsigned)nb, kSortThreads, 0, st>>>(kb[src], vb[src], kb[dst], vb[dst],
                                                                        count_dev, n_sized, cap, shift, hist,
                                                                        scan_scr);
    } else {
      e = scan_exclusive_tiles(hist, hist, 256 * nb, scan_scr, st, dc);
      if (e != hipSuccess) return e;
      k_sort_scatter<KeyT, false><<<(unsigned)nb, kSortThreads, 0, st>>>(kb[src], vb[src], kb[dst], vb[dst],
                                                                         count_dev, n_sized, cap, shift, hist,
                                                                         scan_scr);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t sort_pairs(uint64_t* k0, int32_t* v0, uint64_t* k1, int32_t* v1, int64_t n_sized, const int32_t* count_dev,
                      int64_t cap, int key_bits, int32_t* scratch, hipStream_t st) {
  return sort_impl<uint64_t>(k0, v0, k1, v1, n_sized, count_dev, cap, key_bits, scratch, st, kFoldTiles);
}

hipError_t sort_pairs32(uint32_t* k0, int32_t* v0, uint32_t* k1, int32_t* v1, int64_t n_sized,
                        const int32_t* count_dev, int64_t cap, int key_bits, int32_t* scratch, hipStream_t st,
                        int fold_tiles) {
  return sort_impl<uint32_t>(k0, v0, k1, v1, n_sized, count_dev, cap, key_bits, scratch, st,
                             fold_tiles < kFoldTiles ? fold_tiles : kFoldTiles);
}

// Binning up to the instance total: the records' first partial slots, the record list sorted by depth (record ids
// in rvals[0]), each sorted record's tile rectangle (rkeys[0], rkeys[1]) and first emission index (rvals[1]), the
// instance total and the overflow flag.
hipError_t bin_records(const gs_frame& f, hipStream_t st) {
  const int64_t rcap = f.rec_cap;
  hipError_t e = fill_i32(f.counters + kInstSum, 0, 2, st);  // kInstSum, kBigCount
  if (e != hipSuccess) return e;
  if ((e = scan_exclusive_pair(f.n_rec, f.rec_first, f.n_inst, f.inst_first, f.n, f.scratch, st)) != hipSuccess)
    return e;
  k_record_list<<<(unsigned)cdiv(f.n, 256), 256, 0, st>>>(f.vis_mask, f.n_rec, f.rec_first, f.inst_first, f.n_inst,
                                                          reinterpret_cast<const short4*>(f.rect), f.zbits, f.n_views,
                                                          f.n, rcap, f.rkeys[0], f.rvals[0], f.rec_slot, f.big_rec,
                                                          f.counters, f.capacity);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = sort_pairs32(f.rkeys[0], f.rvals[0], f.rkeys[1], f.rvals[1], rcap, f.counters + kRecCount, rcap, 32,
                        f.scratch, st, kFoldTiles)) != hipSuccess)
    return e;  // 4 passes: the sorted records are back in rkeys[0] / rvals[0]
  // counts straight into rvals[1], scanned in place into the emission offsets; the sorted rectangles take the
  // depth keys' buffers, which are no longer needed
  k_record_counts<<<(unsigned)cdiv(rcap, 256), 256, 0, st>>>(f.rvals[0], reinterpret_cast<const short4*>(f.rect),
                                                             f.counters, rcap, f.rvals[1], f.rkeys[0], f.rkeys[1]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_exclusive(f.rvals[1], f.rvals[1], rcap, f.scratch, st,
                          DevCount{f.counters + kRecCount, rcap, 1, 1})) != hipSuccess)
    return e;
  return hipSuccess;
}

hipError_t emit(const gs_frame& f, int64_t /*n_sized*/, hipStream_t st) {
  k_emit<<<(unsigned)cdiv(f.rec_cap, 256), 256, 0, st>>>(f.rvals[0], f.rvals[1], f.rkeys[0], f.rkeys[1], f.cams,
                                                         f.n_views, f.n, f.counters, f.rec_cap, f.capacity, f.keys[0],
                                                         f.vals[0]);
  return hipGetLastError();
}

// The longest-first schedule; its 32 bucket counts (counters[128..160)) were cleared by ranges(), which runs
// just before it.
hipError_t tile_schedule(const gs_frame& f, hipStream_t st) {
  int32_t* cnt = f.counters + 128;
  int32_t* off = f.counters + 160;
  hipError_t e = hipSuccess;
  const auto* rng = reinterpret_cast<const int2*>(f.tile_range);
  if (f.n_tiles <= kSchedOneBlock) {  // with the work items
    k_schedule_small<<<1, 1024, 0, st>>>(rng, f.n_tiles, f.seg_len, f.tile_order, f.seg_count, f.seg_first,
                                         reinterpret_cast<int4*>(f.items), f.counters);
    return hipGetLastError();
  }
  const unsigned nb = (unsigned)cdiv(f.n_tiles, 256);
  k_sched_hist<<<nb, 256, 0, st>>>(rng, f.n_tiles, f.seg_len, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_sched_scan<<<1, 64, 0, st>>>(cnt, off);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_sched_scatter<<<nb, 256, 0, st>>>(rng, f.n_tiles, f.seg_len, off, f.tile_order);
  return hipGetLastError();
}

hipError_t work_items(const gs_frame& f, hipStream_t st) {
  if (f.seg_len <= 0 || f.n_tiles <= kSchedOneBlock) return hipSuccess;  // small frames: by tile_schedule
  const auto* rng = reinterpret_cast<const int2*>(f.tile_range);
  const unsigned nb = (unsigned)cdiv(f.n_tiles, 256);
  k_seg_count<<<nb, 256, 0, st>>>(rng, f.tile_order, f.n_tiles, f.seg_len, f.seg_count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_exclusive(f.seg_count, f.seg_first, f.n_tiles, f.scratch, st)) != hipSuccess) return e;
  k_seg_emit<<<nb, 256, 0, st>>>(f.tile_order, f.n_tiles, f.seg_count, f.seg_first, reinterpret_cast<int4*>(f.items),
                                 f.counters);
  return hipGetLastError();
}

// Tile ranges; the schedule's bucket counts (counters[128..160)) are cleared in the same launch as the ranges.
hipError_t ranges(const gs_frame& f, const uint32_t* keys, int64_t n_sized, const int32_t* count_dev,
                  hipStream_t st) {
  const int64_t nr = 2 * (int64_t)f.n_tiles;
  k_fill2_i32<<<(unsigned)cdiv(nr > 32 ? nr : 32, 256), 256, 0, st>>>(f.tile_range, nr, f.counters + 128, 32, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_sized <= 0) return e;
  k_ranges<<<(unsigned)cdiv(n_sized, 256), 256, 0, st>>>(keys, count_dev, n_sized, f.capacity,
                                                         reinterpret_cast<int2*>(f.tile_range));
  return hipGetLastError();
}

}  // namespace gs_launch
