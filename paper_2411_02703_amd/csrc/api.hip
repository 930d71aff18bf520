// C ABI of libgs: argument checks, the frame layout and the launch sequences of the hot-path calls.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "common.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(GS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define GS_HIP(call, where)                       \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

bool tiles_supported(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 16 && th == 8) || (tw == 8 && th == 8) || (tw == 32 && th == 8);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t rec, rect, ipart, instfirst, mask, ninst, nrec, instoff, zbits, recslot, bigrec, rk[2], rv[2], k0, k1, v0, v1, range, order,
      counters, loss, scratch, total;
  int64_t rec_cap;
  size_t segcount, segfirst, items, seg, split;
  size_t scratch_ints;
  int key_bits, passes;
  int seg_len, seg_cap, long_cap, item_cap;
};

// Depth-segment length of the fused backward for these options (0: never split).
int seg_len_of(const gs_opts* o) { return o->seg_len == 0 ? 512 : (o->seg_len < 0 ? 0 : o->seg_len); }

int opts_check(const gs_opts* o) {
  if (!o) return fail(GS_ERR_ARG, "opts is NULL");
  if (!tiles_supported(o->tile_w, o->tile_h))
    return fail(GS_ERR_ARG, "unsupported tile %dx%d (16x16, 16x8, 8x8, 32x8)", o->tile_w, o->tile_h);
  const int nw = o->waves_per_tile;
  if (nw != 0 && nw != o->tile_w * o->tile_h / 64)
    return fail(GS_ERR_ARG, "waves_per_tile %d: a %dx%d tile has %d waves", nw, o->tile_w, o->tile_h,
                o->tile_w * o->tile_h / 64);
  if (o->batch_depth < 0 || o->batch_depth > 2) return fail(GS_ERR_ARG, "batch_depth %d outside [0, 2]", o->batch_depth);
  if (o->block_w != 0 && o->block_w != 2 && o->block_w != 4 && o->block_w != 8)
    return fail(GS_ERR_ARG, "block_w %d (0, 2, 4 or 8)", o->block_w);
  if (o->seg_len > 0 && o->seg_len < 64) return fail(GS_ERR_ARG, "seg_len %d below 64", o->seg_len);
  if (!(o->near_z > 0.f) || !(o->guard >= 1.f) || !(o->lowpass >= 0.f) || !(o->alpha_min > 0.f) ||
      !(o->alpha_max > o->alpha_min) || !(o->alpha_max < 1.f) || !(o->t_min > 0.f))
    return fail(GS_ERR_ARG, "invalid option values");
  return GS_OK;
}

int views_info(const gs_camera* cams, int32_t V, const gs_opts* o, int* n_tiles, int64_t* n_pixels,
               int64_t* max_view = nullptr) {
  if (!cams) return fail(GS_ERR_ARG, "cameras are NULL");
  if (V < 1 || V > GS_MAX_VIEWS) return fail(GS_ERR_ARG, "n_views %d outside [1, %d]", V, GS_MAX_VIEWS);
  int64_t tiles = 0, px = 0;
  for (int v = 0; v < V; ++v) {
    const gs_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384)
      return fail(GS_ERR_ARG, "view %d: size %dx%d", v, c.width, c.height);
    tiles += (int64_t)((c.width + o->tile_w - 1) / o->tile_w) * ((c.height + o->tile_h - 1) / o->tile_h);
    px += (int64_t)c.width * c.height;
    if (max_view && (int64_t)c.width * c.height > *max_view) *max_view = (int64_t)c.width * c.height;
  }
  if (tiles >= (int64_t(1) << 30)) return fail(GS_ERR_ARG, "too many tiles");
  if (3 * px >= (int64_t(1) << 31)) return fail(GS_ERR_ARG, "too many pixels");
  *n_tiles = (int)tiles;
  *n_pixels = px;
  return GS_OK;
}

Layout make_layout(int64_t n, int V, int n_tiles, int64_t cap, const gs_opts* opts) {
  Layout L;
  L.seg_len = seg_len_of(opts);
  L.seg_cap = L.seg_len > 0 ? (int)(2 * cap / L.seg_len + 2) : 0;
  L.long_cap = L.seg_len > 0 ? (int)(cap / L.seg_len + 1) : 0;
  L.item_cap = n_tiles + L.seg_cap;
  const size_t NT = (size_t)opts->tile_w * opts->tile_h;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  const size_t R = (size_t)V * (size_t)n;
  L.rec = take(R * 48);
  L.rect = take(R * 8);
  L.ipart = take((size_t)cap * 48);
  L.instfirst = take((size_t)n * 4);
  L.mask = take((size_t)n * 8);
  L.ninst = take((size_t)n * 4);
  L.nrec = take((size_t)n * 4);
  L.instoff = take((size_t)n * 4);
  L.zbits = take(R * 4);
  L.recslot = take(R * 4);
  L.rec_cap = (int64_t)R < cap ? (int64_t)R : cap;
  L.bigrec = take((size_t)L.rec_cap * 4);
  for (int k = 0; k < 2; ++k) {
    L.rk[k] = take((size_t)L.rec_cap * 4);
    L.rv[k] = take((size_t)L.rec_cap * 4);
  }
  L.k0 = take((size_t)cap * 4);
  L.k1 = take((size_t)cap * 4);
  L.v0 = take((size_t)cap * 4);
  L.v1 = take((size_t)cap * 4);
  L.range = take((size_t)n_tiles * 8);
  L.order = take((size_t)n_tiles * 4);
  L.counters = take(256 * 4);
  L.loss = take(64 * 4);
  L.segcount = take((size_t)n_tiles * 4);
  L.segfirst = take((size_t)n_tiles * 4);
  L.items = take((size_t)L.item_cap * 16);
  L.seg = take((size_t)L.seg_cap * 6 * NT * 4);
  L.split = take((size_t)L.long_cap * 12 * NT * 4);
  int64_t big = n > n_tiles ? n : n_tiles;
  if (L.rec_cap > big) big = L.rec_cap;
  // (the per-Gaussian count scans run as one pair: twice a scan's scratch over n)
  size_t s1 = gs_launch::scan_scratch_ints(big);
  if (2 * gs_launch::scan_scratch_ints(n) > s1) s1 = 2 * gs_launch::scan_scratch_ints(n);
  const size_t s2 = gs_launch::sort_scratch_ints(cap);
  L.scratch_ints = s1 > s2 ? s1 : s2;
  L.scratch = take(L.scratch_ints * 4);
  L.total = o;
  int tb = 1;
  while ((int64_t(1) << tb) < n_tiles) ++tb;
  L.key_bits = tb;
  L.passes = (L.key_bits + 7) / 8;
  return L;
}

int params_check(const gs_params* p, const char* what) {
  if (!p) return fail(GS_ERR_ARG, "%s is NULL", what);
  if (!p->means || !p->log_scales || !p->quats || !p->opacity || !p->sh)
    return fail(GS_ERR_ARG, "%s has a NULL array", what);
  if (p->n < 1) return fail(GS_ERR_ARG, "%s: n = %lld", what, (long long)p->n);
  if (p->sh_degree < 0 || p->sh_degree > 3) return fail(GS_ERR_ARG, "%s: sh_degree %d", what, p->sh_degree);
  return GS_OK;
}

int frame_check(const gs_frame* f) {
  if (!f || !f->block || !f->cams) return fail(GS_ERR_ARG, "frame not initialised");
  return GS_OK;
}

// ------------------------------------------------------------------ static sort scratch (no allocation)
// Ping-pong key/value buffers and digit histograms of gs_sort_pairs_static, for callers that cannot allocate.
// Each GPU the library runs on holds its own copy of this array until the process ends.
constexpr int64_t kStaticSortMax = int64_t(1) << 20;             // pairs
constexpr size_t kStaticKeysOff = 0;                             // uint64_t[kStaticSortMax]
constexpr size_t kStaticValsOff = kStaticKeysOff + 8 * kStaticSortMax;  // int32_t[kStaticSortMax]
constexpr size_t kStaticHistOff = kStaticValsOff + 4 * kStaticSortMax;  // int32_t histograms and scan partials
constexpr size_t kStaticBytes = kStaticHistOff + (size_t(1) << 20);

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device with that device current.
int static_scratch(hipStream_t st, unsigned char** out) {
  int dev = -1;
  GS_HIP(hipGetDevice(&dev), "gs_sort_pairs_static: current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_UNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
  if (st != nullptr) {
    hipDevice_t sdev = -1;
    GS_HIP(hipStreamGetDevice(st, &sdev), "gs_sort_pairs_static: stream device");
    if (sdev != dev) return fail(GS_ERR_ARG, "the stream belongs to device %d, the current device is %d", sdev, dev);
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    GS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "gs_sort_pairs_static: scratch address");
    if (!p) return fail(GS_ERR_HIP, "gs_sort_pairs_static: no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return GS_OK;
}

}  // namespace

extern "C" {

void gs_default_opts(gs_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tile_w = 16;
  o->tile_h = 16;
  o->near_z = 0.2f;
  o->guard = 1.3f;
  o->lowpass = 0.3f;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->t_min = 1e-4f;
}

int gs_plan_cameras(gs_camera* cams, int32_t V, const gs_opts* o) {
  int rc = opts_check(o);
  if (rc) return rc;
  int nt;
  int64_t np;
  if ((rc = views_info(cams, V, o, &nt, &np))) return rc;
  int toff = 0, poff = 0;
  for (int v = 0; v < V; ++v) {
    gs_camera& c = cams[v];
    if (!(c.fx > 0.f) || !(c.fy > 0.f) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
      return fail(GS_ERR_ARG, "view %d: invalid intrinsics", v);
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(c.R[i])) return fail(GS_ERR_ARG, "view %d: non-finite rotation", v);
    c.tiles_x = (c.width + o->tile_w - 1) / o->tile_w;
    c.tiles_y = (c.height + o->tile_h - 1) / o->tile_h;
    c.tile_offset = toff;
    c.pixel_offset = poff;
    toff += c.tiles_x * c.tiles_y;
    poff += c.width * c.height;
    // guard band: the image widened by (guard - 1)/2 of its size on each side
    const float gm = (o->guard - 1.0f) * 0.5f;
    const float mxw = gm * (float)c.width;
    const float myw = gm * (float)c.height;
    c.guard_lo_x = -mxw;
    c.guard_hi_x = (float)c.width + mxw;
    c.guard_lo_y = -myw;
    c.guard_hi_y = (float)c.height + myw;
  }
  return GS_OK;
}

size_t gs_frame_bytes(int64_t n, const gs_camera* cams, int32_t V, const gs_opts* o, int64_t capacity) {
  if (opts_check(o)) return 0;
  int nt;
  int64_t np;
  if (views_info(cams, V, o, &nt, &np)) return 0;
  if (n < 1 || capacity < 1 || capacity > INT32_MAX) return 0;
  return make_layout(n, V, nt, capacity, o).total;
}

int gs_frame_init(gs_frame* f, void* block, size_t bytes, int64_t n, const gs_camera* cams_host,
                  const gs_camera* cams_dev, int32_t V, const gs_opts* o, int64_t capacity) {
  if (!f) return fail(GS_ERR_ARG, "frame is NULL");
  int rc = opts_check(o);
  if (rc) return rc;
  int nt;
  int64_t np, mv = 0;
  if ((rc = views_info(cams_host, V, o, &nt, &np, &mv))) return rc;
  if (!cams_dev) return fail(GS_ERR_ARG, "device cameras are NULL");
  if (n < 1) return fail(GS_ERR_ARG, "n = %lld", (long long)n);
  if ((int64_t)V * n > INT32_MAX) return fail(GS_ERR_ARG, "n_views * n exceeds 2^31 - 1 records");
  if (capacity < 1 || capacity > INT32_MAX) return fail(GS_ERR_ARG, "capacity %lld", (long long)capacity);
  for (int v = 0; v < V; ++v)
    if (cams_host[v].tiles_x != (cams_host[v].width + o->tile_w - 1) / o->tile_w)
      return fail(GS_ERR_ARG, "view %d is not planned for these options (call gs_plan_cameras)", v);
  if (!block) return fail(GS_ERR_ARG, "block is NULL");
  if (((uintptr_t)block & 255) != 0) return fail(GS_ERR_ARG, "block is not 256-byte aligned");
  const Layout L = make_layout(n, V, nt, capacity, o);
  if (bytes < L.total) return fail(GS_ERR_WORKSPACE, "frame block of %zu bytes, %zu needed", bytes, L.total);
  char* b = static_cast<char*>(block);
  std::memset(f, 0, sizeof(*f));
  f->n = n;
  f->n_views = V;
  f->n_tiles = nt;
  f->n_pixels = np;
  f->max_view_pixels = mv;
  f->capacity = capacity;
  f->key_bits = L.key_bits;
  f->sort_passes = L.passes;
  f->tile_w = o->tile_w;
  f->tile_h = o->tile_h;
  f->seg_len = L.seg_len;
  f->seg_cap = L.seg_cap;
  f->long_cap = L.long_cap;
  f->item_cap = L.item_cap;
  f->cams = cams_dev;
  f->block = block;
  f->bytes = bytes;
  f->rec = reinterpret_cast<float*>(b + L.rec);
  f->rect = reinterpret_cast<int16_t*>(b + L.rect);
  f->ipart = reinterpret_cast<float*>(b + L.ipart);
  f->inst_first = reinterpret_cast<int32_t*>(b + L.instfirst);
  f->vis_mask = reinterpret_cast<uint64_t*>(b + L.mask);
  f->n_inst = reinterpret_cast<int32_t*>(b + L.ninst);
  f->n_rec = reinterpret_cast<int32_t*>(b + L.nrec);
  f->rec_first = reinterpret_cast<int32_t*>(b + L.instoff);
  f->zbits = reinterpret_cast<uint32_t*>(b + L.zbits);
  f->rec_slot = reinterpret_cast<int32_t*>(b + L.recslot);
  f->big_rec = reinterpret_cast<int32_t*>(b + L.bigrec);
  f->rec_cap = L.rec_cap;
  for (int k = 0; k < 2; ++k) {
    f->rkeys[k] = reinterpret_cast<uint32_t*>(b + L.rk[k]);
    f->rvals[k] = reinterpret_cast<int32_t*>(b + L.rv[k]);
  }
  f->keys[0] = reinterpret_cast<uint32_t*>(b + L.k0);
  f->keys[1] = reinterpret_cast<uint32_t*>(b + L.k1);
  f->vals[0] = reinterpret_cast<int32_t*>(b + L.v0);
  f->vals[1] = reinterpret_cast<int32_t*>(b + L.v1);
  f->tile_range = reinterpret_cast<int32_t*>(b + L.range);
  f->tile_order = reinterpret_cast<int32_t*>(b + L.order);
  f->counters = reinterpret_cast<int32_t*>(b + L.counters);
  f->loss = reinterpret_cast<float*>(b + L.loss);
  f->scratch = reinterpret_cast<int32_t*>(b + L.scratch);
  f->scratch_ints = L.scratch_ints;
  f->seg_count = reinterpret_cast<int32_t*>(b + L.segcount);
  f->seg_first = reinterpret_cast<int32_t*>(b + L.segfirst);
  f->items = reinterpret_cast<int32_t*>(b + L.items);
  f->seg = reinterpret_cast<float*>(b + L.seg);
  f->split = reinterpret_cast<float*>(b + L.split);
  return GS_OK;
}

int gs_project(const gs_params* p, const gs_frame* f, const gs_opts* o, void* stream) {
  int rc;
  if ((rc = params_check(p, "params")) || (rc = frame_check(f)) || (rc = opts_check(o))) return rc;
  if (p->n != f->n) return fail(GS_ERR_ARG, "params n %lld != frame n %lld", (long long)p->n, (long long)f->n);
  if (o->tile_w != f->tile_w || o->tile_h != f->tile_h) return fail(GS_ERR_ARG, "tile size differs from the frame");
  hipStream_t st = static_cast<hipStream_t>(stream);
  GS_HIP(gs_launch::fill_i32(f->counters, 0, 2, st), "gs_project: clear counters");
  GS_HIP(gs_launch::project(*p, *f, *o, st), "gs_project");
  return GS_OK;
}

int gs_bin_tiles(const gs_frame* f, const gs_opts* o, int32_t sync_count, int64_t* n_instances, void* stream) {
  int rc;
  if ((rc = frame_check(f)) || (rc = opts_check(o))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  GS_HIP(gs_launch::bin_records(*f, st), "gs_bin_tiles: records by depth");
  int64_t n_sized = f->capacity;
  const int32_t* count_dev = f->counters;
  if (sync_count) {
    int32_t c = 0;
    GS_HIP(hipMemcpyAsync(&c, f->counters, sizeof(int32_t), hipMemcpyDeviceToHost, st), "gs_bin_tiles: count");
    GS_HIP(hipStreamSynchronize(st), "gs_bin_tiles: sync");
    if (n_instances) *n_instances = c;
    n_sized = c < f->capacity ? c : f->capacity;
    count_dev = nullptr;
  }
  GS_HIP(gs_launch::emit(*f, n_sized, st), "gs_bin_tiles: emit");
  // the instance sort folds its histogram scans only for small frames (a few M instances): with ~20 M the
  // scatter's extra scan costs more than the launch it saves (measured)
  GS_HIP(gs_launch::sort_pairs32(f->keys[0], f->vals[0], f->keys[1], f->vals[1], n_sized, count_dev, f->capacity,
                                 f->key_bits, f->scratch, st, 256),
         "gs_bin_tiles: sort by tile");
  GS_HIP(gs_launch::ranges(*f, f->keys[f->sort_passes & 1], n_sized, count_dev, st), "gs_bin_tiles: ranges");
  GS_HIP(gs_launch::tile_schedule(*f, st), "gs_bin_tiles: schedule");
  GS_HIP(gs_launch::work_items(*f, st), "gs_bin_tiles: work items");
  return GS_OK;
}

int gs_render_fwd(const gs_frame* f, const gs_opts* o, const gs_images* out, void* stream) {
  int rc;
  if ((rc = frame_check(f)) || (rc = opts_check(o))) return rc;
  if (!out || !out->rgb || !out->depth || !out->vis) return fail(GS_ERR_ARG, "output images are NULL");
  if (o->tile_w != f->tile_w || o->tile_h != f->tile_h) return fail(GS_ERR_ARG, "tile size differs from the frame");
  GS_HIP(gs_launch::render_fwd(*f, *o, *out, static_cast<hipStream_t>(stream)), "gs_render_fwd");
  return GS_OK;
}

int gs_composite_bwd(const gs_frame* f, const gs_opts* o, const gs_images* fwd, const gs_loss* l, void* stream) {
  int rc;
  if ((rc = frame_check(f)) || (rc = opts_check(o))) return rc;
  if (!l) return fail(GS_ERR_ARG, "loss is NULL");
  if (fwd && (!fwd->rgb || !fwd->depth || !fwd->vis)) return fail(GS_ERR_ARG, "forward images incomplete");
  if (l->tgt_rgb && !l->tgt_depth) return fail(GS_ERR_ARG, "loss mode needs tgt_depth");
  if (!(l->lambda_ssim >= 0.f && l->lambda_ssim <= 1.f)) return fail(GS_ERR_ARG, "lambda_ssim outside [0, 1]");
  if (o->tile_w != f->tile_w || o->tile_h != f->tile_h) return fail(GS_ERR_ARG, "tile size differs from the frame");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (l->tgt_rgb) {
    // counts the valid target depths per view and clears the loss slots
    GS_HIP(gs_launch::count_valid(*f, l->tgt_depth, f->max_view_pixels, f->loss, 1 + gsk::kLossSlots, st),
           "gs_composite_bwd: valid depth");
  }
  GS_HIP(gs_launch::render_bwd(*f, *o, fwd, *l, st), "gs_composite_bwd");
  if (l->tgt_rgb) GS_HIP(gs_launch::loss_total(f->loss, st), "gs_composite_bwd: loss total");
  return GS_OK;
}

int gs_project_bwd(const gs_params* p, const gs_frame* f, const gs_opts* o, const gs_params* grads, void* stream) {
  int rc;
  if ((rc = params_check(p, "params")) || (rc = params_check(grads, "grads")) || (rc = frame_check(f)) ||
      (rc = opts_check(o)))
    return rc;
  if (p->n != f->n || grads->n != f->n || grads->sh_degree != p->sh_degree)
    return fail(GS_ERR_ARG, "params / grads / frame sizes differ");
  GS_HIP(gs_launch::project_bwd(*p, *f, *o, *grads, static_cast<hipStream_t>(stream)), "gs_project_bwd");
  return GS_OK;
}

int gs_render_bwd(const gs_params* p, const gs_frame* f, const gs_opts* o, const gs_images* fwd, const gs_loss* l,
                  const gs_params* grads, void* stream) {
  int rc;
  if ((rc = params_check(p, "params")) || (rc = params_check(grads, "grads")) || (rc = frame_check(f))) return rc;
  if (p->n != f->n || grads->n != f->n || grads->sh_degree != p->sh_degree)
    return fail(GS_ERR_ARG, "params / grads / frame sizes differ");
  if ((rc = gs_composite_bwd(f, o, fwd, l, stream))) return rc;
  return gs_project_bwd(p, f, o, grads, stream);
}

int gs_ssim(const gs_camera* cams_host, const gs_camera* cams_dev, int32_t V, const float* rgb, const float* tgt,
            float lambda, float* g_rgb, float* loss_out, void* stream) {
  if (!cams_host || !cams_dev || !rgb || !tgt || !g_rgb || !loss_out) return fail(GS_ERR_ARG, "NULL pointer");
  if (V < 1 || V > GS_MAX_VIEWS) return fail(GS_ERR_ARG, "n_views = %d", V);
  if (!(lambda >= 0.f && lambda <= 1.f)) return fail(GS_ERR_ARG, "lambda_ssim = %g", (double)lambda);
  for (int v = 0; v < V; ++v)
    if (cams_host[v].width < 1 || cams_host[v].height < 1) return fail(GS_ERR_ARG, "view %d has no pixels", v);
  GS_HIP(gs_launch::ssim(cams_host, cams_dev, V, rgb, tgt, lambda, g_rgb, loss_out, static_cast<hipStream_t>(stream)),
         "gs_ssim");
  return GS_OK;
}

size_t gs_prune_scratch_bytes(int64_t n) { return n < 1 ? 0 : 4 * gs_launch::prune_scratch_ints(n); }

int gs_prune(const gs_params* p, const gs_params* m, const gs_params* v, float min_opacity, const gs_params* op,
             const gs_params* om, const gs_params* ov, int64_t* n_kept, void* scratch, void* stream) {
  int rc;
  if ((rc = params_check(p, "params")) || (rc = params_check(m, "m")) || (rc = params_check(v, "v")) ||
      (rc = params_check(op, "out_params")) || (rc = params_check(om, "out_m")) || (rc = params_check(ov, "out_v")))
    return rc;
  const gs_params* all[5] = {m, v, op, om, ov};
  for (const gs_params* q : all)
    if (q->n != p->n || q->sh_degree != p->sh_degree) return fail(GS_ERR_ARG, "prune: sizes differ");
  if (!n_kept || !scratch) return fail(GS_ERR_ARG, "prune: NULL n_kept or scratch");
  if (!(min_opacity > 0.f && min_opacity < 1.f)) return fail(GS_ERR_ARG, "min_opacity = %g", (double)min_opacity);
  const float thr = (float)std::log((double)min_opacity / (1.0 - (double)min_opacity));
  GS_HIP(gs_launch::prune(*p, *m, *v, thr, *op, *om, *ov, n_kept, static_cast<int32_t*>(scratch),
                          static_cast<hipStream_t>(stream)),
         "gs_prune");
  return GS_OK;
}

size_t gs_expand_scratch_bytes(int64_t n_old, int64_t M) {
  return (n_old < 0 || M < 1) ? 0 : 4 * gs_launch::expand_scratch_ints(n_old, M);
}

int gs_expand(const gs_params* p, const gs_params* m, const gs_params* v, int64_t n_old, const float* pts,
              const float* rgb, int64_t M, const gs_camera* cam, const float* vis, const gs_expand_opts* o,
              int64_t* n_added, void* scratch, void* stream) {
  int rc;
  if ((rc = params_check(p, "params")) || (rc = params_check(m, "m")) || (rc = params_check(v, "v"))) return rc;
  if (m->n != p->n || v->n != p->n || m->sh_degree != p->sh_degree || v->sh_degree != p->sh_degree)
    return fail(GS_ERR_ARG, "expand: params / moments sizes differ");
  if (!pts || !rgb || !cam || !vis || !o || !n_added || !scratch) return fail(GS_ERR_ARG, "expand: NULL pointer");
  if (M < 1 || M > INT32_MAX || n_old < 0 || n_old + M > p->n)
    return fail(GS_ERR_ARG, "expand: %lld points after %lld Gaussians need room for %lld rows, have %lld",
                (long long)M, (long long)n_old, (long long)(n_old + M), (long long)p->n);
  if (cam->width < 1 || cam->height < 1 || !(cam->fx > 0.f) || !(cam->fy > 0.f))
    return fail(GS_ERR_ARG, "expand: bad camera");
  if (!(o->voxel > 0.f) || !(o->knn_cell > 0.f) || o->cap < 1 || !(o->tau_alpha >= 0.f) ||
      !(o->init_opacity > 0.f && o->init_opacity < 1.f) || !(o->near_z > 0.f))
    return fail(GS_ERR_ARG, "expand: bad options");
  const float logit = (float)std::log((double)o->init_opacity / (1.0 - (double)o->init_opacity));
  GS_HIP(gs_launch::expand(*p, *m, *v, n_old, pts, rgb, M, *cam, vis, o->tau_alpha, o->near_z, o->voxel, o->cap,
                           o->knn_cell, logit, n_added, static_cast<int32_t*>(scratch),
                           static_cast<hipStream_t>(stream)),
         "gs_expand");
  return GS_OK;
}

size_t gs_spatial_order_scratch_bytes(int64_t n) { return n < 1 ? 0 : 4 * gs_launch::order_scratch_ints(n); }

int gs_spatial_order(const gs_params* p, const gs_params* m, const gs_params* v, const gs_params* op,
                     const gs_params* om, const gs_params* ov, int32_t* perm_out, void* scratch, void* stream) {
  int rc;
  if ((rc = params_check(p, "params")) || (rc = params_check(m, "m")) || (rc = params_check(v, "v")) ||
      (rc = params_check(op, "out_params")) || (rc = params_check(om, "out_m")) || (rc = params_check(ov, "out_v")))
    return rc;
  const gs_params* all[5] = {m, v, op, om, ov};
  for (const gs_params* q : all)
    if (q->n != p->n || q->sh_degree != p->sh_degree) return fail(GS_ERR_ARG, "spatial order: sizes differ");
  if (p->n > INT32_MAX) return fail(GS_ERR_ARG, "spatial order: n above 2^31 - 1");
  if (!scratch) return fail(GS_ERR_ARG, "spatial order: scratch is NULL");
  GS_HIP(gs_launch::spatial_order(*p, *m, *v, *op, *om, *ov, perm_out, static_cast<int32_t*>(scratch),
                                  static_cast<hipStream_t>(stream)),
         "gs_spatial_order");
  return GS_OK;
}

static int adam_check(const gs_adam* a) {
  if (!a || !a->step || !a->bias) return fail(GS_ERR_ARG, "adam state is NULL");
  if (a->flags & ~GS_ADAM_SPARSE) return fail(GS_ERR_ARG, "unknown Adam flags %d", a->flags);
  if (!(a->beta1 >= 0.f && a->beta1 < 1.f) || !(a->beta2 >= 0.f && a->beta2 < 1.f) || !(a->eps >= 0.f))
    return fail(GS_ERR_ARG, "invalid Adam hyper-parameters");
  return GS_OK;
}

int gs_render_bwd_adam(const gs_params* p, const gs_frame* f, const gs_opts* o, const gs_images* fwd,
                       const gs_loss* l, const gs_params* m, const gs_params* v, const gs_adam* a,
                       const gs_params* grads_out, void* stream) {
  int rc;
  if ((rc = params_check(p, "params")) || (rc = params_check(m, "m")) || (rc = params_check(v, "v")) ||
      (grads_out && (rc = params_check(grads_out, "grads_out"))) || (rc = frame_check(f)) || (rc = opts_check(o)) ||
      (rc = adam_check(a)))
    return rc;
  if (p->n != f->n || m->n != f->n || v->n != f->n || m->sh_degree != p->sh_degree || v->sh_degree != p->sh_degree)
    return fail(GS_ERR_ARG, "params / moments / frame sizes differ");
  if (grads_out && (grads_out->n != f->n || grads_out->sh_degree != p->sh_degree))
    return fail(GS_ERR_ARG, "grads_out / frame sizes differ");
  if ((rc = gs_composite_bwd(f, o, fwd, l, stream))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  GS_HIP(gs_launch::adam_prep(*a, f->counters + 1, st), "gs_render_bwd_adam: step");
  GS_HIP(gs_launch::project_bwd_adam(*p, *f, *o, *m, *v, *a, grads_out, st), "gs_render_bwd_adam");
  return GS_OK;
}

int gs_count_pairs(const gs_frame* f, const gs_opts* o, uint64_t* counts, void* stream) {
  int rc;
  if ((rc = frame_check(f)) || (rc = opts_check(o))) return rc;
  if (!counts) return fail(GS_ERR_ARG, "counts is NULL");
  if (o->tile_w != f->tile_w || o->tile_h != f->tile_h) return fail(GS_ERR_ARG, "tile size differs from the frame");
  GS_HIP(gs_launch::count_pairs(*f, *o, reinterpret_cast<unsigned long long*>(counts),
                                static_cast<hipStream_t>(stream)),
         "gs_count_pairs");
  return GS_OK;
}

int gs_adam_step(const gs_params* p, const gs_params* g, const gs_params* m, const gs_params* v, const gs_adam* a,
                 void* stream) {
  int rc;
  if ((rc = params_check(p, "params")) || (rc = params_check(g, "grads")) || (rc = params_check(m, "m")) ||
      (rc = params_check(v, "v")))
    return rc;
  if (g->n != p->n || m->n != p->n || v->n != p->n || g->sh_degree != p->sh_degree ||
      m->sh_degree != p->sh_degree || v->sh_degree != p->sh_degree)
    return fail(GS_ERR_ARG, "params / grads / moments sizes differ");
  if ((rc = adam_check(a))) return rc;
  if (a->flags & GS_ADAM_SPARSE) return fail(GS_ERR_ARG, "gs_adam_step has no visibility: sparse Adam is a flag of "
                                                        "gs_render_bwd_adam");
  GS_HIP(gs_launch::adam(*p, *g, *m, *v, *a, static_cast<hipStream_t>(stream)), "gs_adam_step");
  return GS_OK;
}

int gs_read_counters(const gs_frame* f, int64_t* n_instances, int32_t* flags, void* stream) {
  int rc;
  if ((rc = frame_check(f))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t c[2] = {0, 0};
  GS_HIP(hipMemcpyAsync(c, f->counters, sizeof(c), hipMemcpyDeviceToHost, st), "gs_read_counters");
  GS_HIP(hipStreamSynchronize(st), "gs_read_counters: sync");
  if (n_instances) *n_instances = c[0];
  if (flags) *flags = c[1];
  return GS_OK;
}

size_t gs_sort_scratch_ints(int64_t n) { return gs_launch::sort_scratch_ints(n); }

int gs_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* keys_tmp, int32_t* vals_tmp, int64_t n, int32_t key_bits,
                  int32_t* scratch, void* stream) {
  if (!keys || !vals || !keys_tmp || !vals_tmp || !scratch) return fail(GS_ERR_ARG, "NULL buffer");
  if (n < 0 || n > INT32_MAX) return fail(GS_ERR_ARG, "n = %lld", (long long)n);
  if (key_bits < 1 || key_bits > 64) return fail(GS_ERR_ARG, "key_bits = %d", key_bits);
  if (n == 0) return GS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int passes = (key_bits + 7) / 8;
  GS_HIP(gs_launch::sort_pairs(keys, vals, keys_tmp, vals_tmp, n, nullptr, n, key_bits, scratch, st), "gs_sort_pairs");
  if (passes & 1) {
    GS_HIP(hipMemcpyAsync(keys, keys_tmp, (size_t)n * 8, hipMemcpyDeviceToDevice, st), "gs_sort_pairs: copy keys");
    GS_HIP(hipMemcpyAsync(vals, vals_tmp, (size_t)n * 4, hipMemcpyDeviceToDevice, st), "gs_sort_pairs: copy vals");
  }
  return GS_OK;
}

int64_t gs_sort_static_max(void) { return kStaticSortMax; }

int gs_sort_pairs_static(uint64_t* keys, int32_t* vals, int64_t n, int32_t key_bits, void* stream) {
  if (!keys || !vals) return fail(GS_ERR_ARG, "NULL buffer");
  if (n < 0 || n > kStaticSortMax)
    return fail(GS_ERR_ARG, "n = %lld outside [0, %lld] (the static scratch holds %lld pairs)", (long long)n,
                (long long)kStaticSortMax, (long long)kStaticSortMax);
  if (key_bits < 1 || key_bits > 64) return fail(GS_ERR_ARG, "key_bits = %d", key_bits);
  if (gs_launch::sort_scratch_ints(kStaticSortMax) * 4 > kStaticBytes - kStaticHistOff)
    return fail(GS_ERR_UNSUPPORTED, "static sort scratch too small for its histograms");
  if (n == 0) return GS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* base = nullptr;
  int rc = static_scratch(st, &base);
  if (rc) return rc;
  auto* ktmp = reinterpret_cast<uint64_t*>(base + kStaticKeysOff);
  auto* vtmp = reinterpret_cast<int32_t*>(base + kStaticValsOff);
  auto* hist = reinterpret_cast<int32_t*>(base + kStaticHistOff);
  const int passes = (key_bits + 7) / 8;
  GS_HIP(gs_launch::sort_pairs(keys, vals, ktmp, vtmp, n, nullptr, n, key_bits, hist, st), "gs_sort_pairs_static");
  if (passes & 1) {
    GS_HIP(hipMemcpyAsync(keys, ktmp, (size_t)n * 8, hipMemcpyDeviceToDevice, st), "gs_sort_pairs_static: keys");
    GS_HIP(hipMemcpyAsync(vals, vtmp, (size_t)n * 4, hipMemcpyDeviceToDevice, st), "gs_sort_pairs_static: vals");
  }
  return GS_OK;
}

const char* gs_status_string(int s) {
  switch (s) {
    case GS_OK: return "ok";
    case GS_ERR_ARG: return "invalid argument";
    case GS_ERR_HIP: return "HIP error";
    case GS_ERR_WORKSPACE: return "workspace too small";
    case GS_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* gs_last_error(void) { return g_err.c_str(); }

int gs_version(void) { return GS_VERSION; }

}  // extern "C"
