/*
 * libgs — differentiable 3D Gaussian splatting for AMD Instinct MI355X (gfx950).
 *
 * The hot path of LVI-GS's mapping back-end (Section III-B and III-E of the paper):
 *   project  : 3D Gaussians (mean, log-scale, rotation, opacity logit, SH colour) to 2D conics
 *              per view, Sigma = R S S^T R^T (eq. Sigma), mu_I = [Q|T] mu_W and
 *              Sigma_I = J Q Sigma Q^T J^T (eq. muI);
 *   bin      : tile lists ordered by depth, by an own stable LSD radix sort of
 *              (global tile << 32 | depth bits) keys;
 *   render   : front-to-back compositing of colour, depth and visibility per pixel
 *              (eqs. Cp, Dp, Vp with the alpha of eq. alpha);
 *   backward : the L1 colour + lambda_d L1 depth loss (eqs. L, Lc with the SSIM weight 0, Ld)
 *              and its gradient to every Gaussian parameter;
 *   adam     : one bias-corrected Adam step (the paper optimises rotation, scaling, opacity
 *              and SH by minimising L, Section III-E; it names no optimiser).
 *
 * Conventions (readings of what the paper leaves open):
 *   camera   : world -> camera t = R mu + T, x right, y down, z forward; pixel (u, v) has its centre
 *              at (u + 0.5, v + 0.5); depth of a Gaussian = camera z of its centre;
 *   culling  : t_z < near_z; pixel mean outside the image widened by (guard - 1)/2 of its size per
 *              side; opacity < alpha_min; det(Sigma_I) <= 0; empty pixel rectangle;
 *   EWA      : exact pinhole Jacobian at t, lowpass px^2 added to the diagonal of Sigma_I;
 *   alpha    : alpha = min(alpha_max, o exp(power)); skipped if alpha < alpha_min; a pixel stops before
 *              the first record whose T (1 - alpha) < t_min;
 *   extent   : pixel rectangle from the opacity-aware radius sqrt((2 ln(255 o) + 1) Sigma_I,diag);
 *   colour   : max(0, sum_k f_k Y_k(dir) + 0.5) with real orthonormal SH up to degree 3, dir the unit
 *              vector from the camera centre to the mean.
 *
 * Memory and ownership: every pointer is a device pointer unless marked (host).  The caller owns all
 * memory.  The library never allocates or frees device memory and keeps no device state (apart from the
 * static scratch array of gs_sort_pairs_static); the per-iteration intermediates live in a caller-provided
 * "frame" block that gs_frame_init carves.
 * Every call is asynchronous on `stream` (a hipStream_t) and can be captured in a HIP graph, except the
 * two calls documented as synchronising.  Calls on different streams need disjoint frames.
 *
 * Errors: invalid arguments are detected on the host before anything is enqueued and return
 * GS_ERR_ARG (text from gs_last_error()).  A failed HIP launch returns GS_ERR_HIP.  Conditions found
 * on the device (instance capacity exceeded, non-finite parameters) set bits in frame->counters[1]
 * without synchronising; the caller reads them after the stream completes.
 */
#ifndef LIBGS_H
#define LIBGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_VERSION 4
#define GS_MAX_VIEWS 64

typedef enum {
  GS_OK = 0,
  GS_ERR_ARG = -1,
  GS_ERR_HIP = -2,
  GS_ERR_WORKSPACE = -3,
  GS_ERR_UNSUPPORTED = -4
} gs_status;

/* bits of frame->counters[1] */
#define GS_FLAG_INSTANCE_OVERFLOW 1 /* more tile instances than the frame's capacity; outputs undefined */
#define GS_FLAG_NONFINITE 2         /* some parameter was NaN/Inf; that Gaussian was culled */

/* One view.  128 bytes, the same layout on host and device. */
typedef struct gs_camera {
  float R[9];          /* world -> camera rotation, row-major ([Q_iw] of eq. muI) */
  float T[3];          /* translation ([T_iw] of eq. muI): t = R mu + T */
  float fx, fy, cx, cy;
  float campos[3];     /* camera centre in world coordinates (-R^T T), for SH view directions */
  float loss_weight;   /* w_v: weight of this view (keyframe x pyramid level) in the loss; a negative weight
                          marks an inactive view: gs_project culls every Gaussian in it (it renders as background
                          and adds nothing to the loss or the gradient), so a schedule can switch views of a
                          captured frame off and on without re-planning it */
  int32_t width, height;
  /* filled by gs_plan_cameras: */
  int32_t tiles_x, tiles_y;
  int32_t tile_offset;  /* first global tile id of this view */
  int32_t pixel_offset; /* first pixel of this view in the concatenated image planes */
  float guard_lo_x, guard_hi_x, guard_lo_y, guard_hi_y; /* guard band, pixels */
  int32_t reserved[2];
} gs_camera;

typedef struct gs_opts {
  int32_t tile_w, tile_h; /* 16x16 (default), 8x8, 16x8 or 32x8; one wave64 per 8x8 sub-tile */
  float near_z;           /* 0.2 */
  float guard;            /* 1.3 */
  float lowpass;          /* 0.3 px^2 */
  float alpha_min;        /* 1/255 */
  float alpha_max;        /* 0.99 */
  float t_min;            /* 1e-4 */
  float bg[3];            /* background colour, 0 */
  int32_t waves_per_tile; /* 0 or tile_w * tile_h / 64 (fixed by the tile shape) */
  int32_t block_w;        /* each wave's 8x8 sub-tile is walked as blocks of block_w x block_w pixels, each in
                             lock-step over the staged records whose pixel rectangle meets it: 2, 4 or 8 (0 = 4).
                             Results are identical (a record is skipped only where its rectangle misses the
                             pixel) */
  int32_t batch_depth;    /* records staged per thread per round: 1 or 2 (0 = 1); results identical */
  int32_t seg_len;        /* compositing (gs_render_fwd, gs_render_bwd): a tile list longer than this is split
                             into depth segments of this many records, composited by separate workgroups and
                             joined per pixel (transmittance products, then prefix sums); 0 = default 512,
                             < 0 = never split.  Fixed per frame by gs_frame_init.  Results agree with the
                             unsplit walk up to FP32 rounding of the transmittance product */
  int32_t persistent;     /* compositing backward with split lists: 0 = one workgroup per work item (default);
                             1 = persistent grids (compute units x resident workgroups) whose workgroups take the
                             work items in schedule order from an atomic counter (frame counters[199..201]).
                             Results identical; offered to time the two launch schemes against each other */
} gs_opts;

/* Gaussian parameters, or gradients / Adam moments in the same layout.  Row-major float32:
 * means [n,3], log_scales [n,3], quats [n,4] (w,x,y,z, any norm > 0), opacity [n] (logits),
 * sh [n,K,3] with K = (sh_degree+1)^2 ordered by l then m = -l..l. */
typedef struct gs_params {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity;
  float* sh;
  int64_t n;
  int32_t sh_degree;
  int32_t reserved;
} gs_params;

/* Per-iteration intermediates of one batch of views, carved from one caller-owned device block.
 * Records are dense over r = v * n + g (view-major); only visible ones are written. */
typedef struct gs_frame {
  int64_t n;            /* Gaussians */
  int32_t n_views;
  int32_t n_tiles;      /* global tiles over all views */
  int64_t n_pixels;     /* pixels over all views */
  int64_t max_view_pixels; /* pixels of the largest view */
  int64_t capacity;     /* tile-instance capacity (<= 2^31 - 1) */
  int32_t key_bits;     /* bits of a global tile id (the instance sort key) */
  int32_t sort_passes;  /* 8-bit LSD passes of the instance sort */
  int32_t tile_w, tile_h;
  int32_t seg_len;      /* depth-segment length of the compositing calls (0: lists are never split) */
  int32_t seg_cap;      /* capacity of segment slots: 2 * capacity / seg_len + 2 */
  int32_t long_cap;     /* capacity of split tiles: capacity / seg_len + 1 */
  int32_t item_cap;     /* work items of the compositing calls: n_tiles + seg_cap */
  const gs_camera* cams;  /* device copy of the planned cameras (caller-owned) */
  void* block;
  size_t bytes;
  /* carved device arrays (library layout; read-only for callers except where noted) */
  float* rec;           /* [n_views*n][12]: {mu_x, mu_y, z, o}, {conic a, b, c, red},
                           {green, blue, px0 | px1 << 16, py0 | py1 << 16} (pixel rectangle as int16 pairs) */
  int16_t* rect;        /* [n_views*n][4]: tile rectangle tx0, tx1, ty0, ty1 (valid when visible) */
  float* ipart;         /* [capacity][12]: per tile instance, at its partial slot (64 Gaussians at a time from
                           inst_first of the first of them; within them view by view, Gaussians ascending in a
                           view; each record's tiles row by row from rec_slot of the record), the compositing
                           backward's partial
                           dL/d{mu_x, mu_y, a, b, c, o, red, green, blue, z} of its record summed over the
                           pixels of its tile (or depth segment); 2 words of padding.  Every backward call
                           writes every stored instance once (plain stores, no atomics).  The projection
                           backward first sums each record of big_rec into its first slot and sets that slot's
                           last word to 1 */
  int32_t* inst_first;  /* [n]: exclusive scan of n_inst; for g a multiple of 64, the first partial slot of the
                           64 Gaussians from g */
  uint64_t* vis_mask;   /* [n]: bit v set if Gaussian g is visible in view v */
  int32_t* n_inst;      /* [n]: tile instances of Gaussian g over all views */
  int32_t* n_rec;       /* [n]: visible records (views) of Gaussian g */
  int32_t* rec_first;   /* [n]: exclusive scan of n_rec; the records of the 64 Gaussians from g (g a multiple of
                           64) start at rec_first[g] in the record list */
  uint32_t* zbits;      /* [n_views*n]: IEEE bits of the camera depth of each visible record */
  int32_t* rec_slot;    /* [n_views*n]: first partial slot of each visible record */
  int32_t* big_rec;     /* [rec_cap]: the records with more than 32 tile instances (count in counters[198]); the
                           projection backward first sums each one's partials into its first slot */
  int64_t rec_cap;      /* capacity of the record list: min(n_views * n, capacity) */
  uint32_t* rkeys[2];   /* [rec_cap] record list: depth bits while sorting; then each sorted record's tile
                           rectangle, tx0 | tx1 << 16 in rkeys[0] and ty0 | ty1 << 16 in rkeys[1] */
  int32_t* rvals[2];    /* [rec_cap] record list: record ids (sorted into rvals[0]); rvals[1] then holds each
                           sorted record's first emission index */
  uint32_t* keys[2];    /* [capacity] instance keys: global tile ids (sorted into keys[sort_passes & 1]) */
  int32_t* vals[2];     /* [capacity] record id of each instance (sorted into vals[sort_passes & 1]; the other
                           buffer is sort scratch) */
  int32_t* tile_range;  /* [n_tiles][2]: [begin, end) of each tile's instances in the sorted list */
  int32_t* tile_order;  /* [n_tiles]: tiles by descending list length (the compositing schedule) */
  int32_t* counters;    /* [256]: [0] instance count, [1] flags, [2..2+n_views) valid depth pixels per view,
                           [128..192) tile-length bucket counts and offsets, [192] work items,
                           [193] segment slots of split tiles, [194] split tiles, [196] visible records,
                           [197] instances summed per Gaussian, [198] records with more than 32 instances,
                           [199..201] work-item counters of the persistent compositing launches */
  int32_t* seg_count;   /* [n_tiles]: segments of the tile at each schedule position */
  int32_t* seg_first;   /* [n_tiles]: exclusive scan of seg_count = first work item of that tile */
  int32_t* items;       /* [item_cap][4]: work items of the compositing calls, split tiles first:
                           {tile, segment, first slot of the tile or -1, schedule position} */
  float* seg;           /* [seg_cap][6][tile_w * tile_h]: per-segment pixel state of split tiles */
  float* split;         /* [long_cap][12][tile_w * tile_h]: per-pixel stop state and upstream gradient */
  float* loss;          /* [64]: loss[0] the loss value written by gs_render_bwd in loss mode; loss[1..32] its
                           partial sums */
  int32_t* scratch;     /* sort histograms and scan partials */
  size_t scratch_ints;
} gs_frame;

typedef struct gs_images {
  float* rgb;   /* sum_v [3][H_v][W_v] planar, view v at 3 * pixel_offset_v */
  float* depth; /* sum_v [H_v][W_v], view v at pixel_offset_v */
  float* vis;   /* sum_v [H_v][W_v] */
} gs_images;

/* Upstream of the backward: either targets (loss mode) or image gradients (autograd mode). */
typedef struct gs_loss {
  const float* g_rgb;     /* autograd mode: dL/d rgb image (layout of gs_images.rgb); NULL = 0 */
  const float* g_depth;   /* autograd mode: dL/d depth image; NULL = 0 */
  const float* g_vis;     /* autograd mode: dL/d visibility image; NULL = 0 */
  const float* tgt_rgb;   /* loss mode when non-NULL: target images, layout of gs_images.rgb */
  const float* tgt_depth; /* loss mode: LiDAR depth, layout of gs_images.depth, 0 = no measurement */
  float lambda_d;         /* loss mode: depth weight (0.1) */
  float lambda_ssim;      /* loss mode: weight lambda of the SSIM term in eq. Lc; the L1 colour term takes
                             (1 - lambda).  The SSIM term's image gradient comes from gs_ssim and is passed in
                             g_rgb, which loss mode ADDS to the L1 gradient (g_depth, g_vis are not used in loss
                             mode).  0 with g_rgb = NULL is the plain L1 loss */
} gs_loss;

#define GS_ADAM_SPARSE 1 /* gs_adam.flags: visible-only step (gs_render_bwd_adam) */

typedef struct gs_adam {
  float lr[6];          /* means, log_scales, quats, opacity, sh degree 0, sh degree >= 1 */
  float beta1, beta2, eps;
  int32_t flags;        /* GS_ADAM_SPARSE: in gs_render_bwd_adam only the Gaussians visible in at least one view
                           of the frame take the step; the others keep their parameters and moments (a flagged
                           variant of the dense torch semantics; the step counter is global).  gs_adam_step
                           rejects the flag (it has no visibility) */
  int64_t* step;        /* device counter, incremented by each step that is taken, before it is used */
  float* bias;          /* device scratch of 4 floats (bias corrections and the skip decision of the step) */
  const int32_t* skip_flags; /* gs_adam_step: nullable device pointer, typically &frame->counters[1]; when
                                GS_FLAG_INSTANCE_OVERFLOW is set there as the step runs, the step is skipped */
} gs_adam;

/* ------------------------------------------------------------------ host-side set-up */
void gs_default_opts(gs_opts* opts);

/* Fill tiles_x/y, tile_offset, pixel_offset and the guard band of cams[0..n_views) (host, in/out).
 * GS_ERR_ARG for n_views outside [1, 64], non-positive sizes, fx/fy <= 0, unsupported tiles. */
int gs_plan_cameras(gs_camera* cams, int32_t n_views, const gs_opts* opts);

/* Bytes of the frame block for n Gaussians, the planned cameras (host) and an instance capacity. */
size_t gs_frame_bytes(int64_t n, const gs_camera* cams, int32_t n_views, const gs_opts* opts,
                      int64_t capacity);

/* Carve `block` (device, >= gs_frame_bytes, 256-byte aligned) into *frame (host struct).
 * cams_host are the planned cameras, cams_dev a device copy of them that must stay valid. */
int gs_frame_init(gs_frame* frame, void* block, size_t bytes, int64_t n, const gs_camera* cams_host,
                  const gs_camera* cams_dev, int32_t n_views, const gs_opts* opts, int64_t capacity);

/* ------------------------------------------------------------------ the five hot-path calls */
/* Projection of every Gaussian into every view of the frame (Section III-B, eqs. Sigma and muI):
 * writes records, tile rectangles, depth bits, visibility masks and per-Gaussian record counts.  Reads each
 * Gaussian once. */
int gs_project(const gs_params* params, const gs_frame* frame, const gs_opts* opts, void* stream);

/* Tile binning (Section III-B: rasterisation iterates over the Gaussians rather than along camera rays, and
 * eq. Cp composites them in depth order, the product over j < i running over the Gaussians in front).  The
 * visible records are sorted by depth (stable LSD radix sort of their 32-bit depth bits, the records of each view
 * listed in Gaussian order), emitted in that order as runs of tile instances, and the instances sorted by global
 * tile id (stable): within a tile the order is ascending depth, ties by record index, which makes the sorted
 * order unique; per-tile ranges and the compositing schedule follow.  Errors: GS_ERR_ARG for an uninitialised
 * frame or options that do not match it; more instances than the capacity set GS_FLAG_INSTANCE_OVERFLOW
 * (instances past the capacity are dropped, the frame's outputs are then undefined, and counters[0] still holds
 * the full count).  sync_count != 0 synchronises the stream after the instance total to size the instance work
 * exactly and returns the instance count in *n_instances (host, nullable); otherwise the work is sized by the
 * capacity and the counts stay on the device (graph-capturable). */
int gs_bin_tiles(const gs_frame* frame, const gs_opts* opts, int32_t sync_count, int64_t* n_instances,
                 void* stream);

/* Forward compositing of colour, depth and visibility for every view (eqs. Cp, Dp, Vp, alpha). */
int gs_render_fwd(const gs_frame* frame, const gs_opts* opts, const gs_images* out, void* stream);

/* Backward: per-pixel upstream gradients (autograd mode) or the L1 colour + lambda_d L1 depth loss
 * against targets (loss mode: L = sum_v w_v [ mean_3P |C - I| + lambda_d mean_valid |D - D_lidar| ],
 * eqs. L, Lc, Ld), through the compositing to every record, then through the projection to the
 * parameters.  Gradients are ACCUMULATED into grads (+=; the caller zeroes them).  fwd holds the
 * forward images of this frame; NULL recomputes them per tile inside the kernel (no image is stored).
 * In loss mode the loss value is written to frame->loss. */
int gs_render_bwd(const gs_params* params, const gs_frame* frame, const gs_opts* opts, const gs_images* fwd,
                  const gs_loss* loss, const gs_params* grads, void* stream);

/* The two halves of gs_render_bwd, for callers that schedule them separately.
 * gs_composite_bwd: compositing backward only (the same eqs.): for every tile instance, the partial
 * dL/d{mean_I, conic, opacity, colour, depth} of its record over its tile's pixels, written to
 * frame->ipart (every instance, no accumulation across calls); in loss mode it also writes frame->loss.
 * gs_project_bwd: projection backward only (eqs. Sigma and muI): one thread per Gaussian sums the
 * partials of its instances view by view (one contiguous run of slots per Gaussian) and adds the parameter
 * gradients to grads (+=); no atomics. */
int gs_composite_bwd(const gs_frame* frame, const gs_opts* opts, const gs_images* fwd, const gs_loss* loss,
                     void* stream);
int gs_project_bwd(const gs_params* params, const gs_frame* frame, const gs_opts* opts, const gs_params* grads,
                   void* stream);

/* One Adam step over all parameters (Section III-E: the rotation, scaling, opacity and SH parameters, and here
 * the means as well, are optimised by minimising eq. L; the paper names no optimiser, so this is the
 * bias-corrected Adam of common 3DGS practice, eps added to the corrected root), with per-group learning
 * rates.  Dense: Gaussians with zero gradient still move.  params, m and v are updated in place; grads are
 * read only; *adam->step is incremented on the device and adam->bias (2 floats) receives the bias
 * corrections, so graph replays advance the step.  If adam->skip_flags is non-NULL and *skip_flags has
 * GS_FLAG_INSTANCE_OVERFLOW set when the step runs, nothing is updated and the counter does not advance (the
 * gradients of an overflowed frame are undefined). */
int gs_adam_step(const gs_params* params, const gs_params* grads, const gs_params* m, const gs_params* v,
                 const gs_adam* adam, void* stream);

/* The backward of gs_render_bwd fused with the Adam step of gs_adam_step (Sections III-B and III-E: the
 * loss of eq. L differentiated through eqs. Cp, Dp, Vp, alpha, muI and Sigma, then the parameters moved by one
 * optimiser step), in one pass per Gaussian after the compositing backward: a thread sums its Gaussian's
 * instance partials view by view, forms the parameter gradient in registers and applies Adam to its
 * parameters, m and v directly, so no gradient buffer is zeroed, written and read back.  Dense Adam: Gaussians
 * with no visible record take a zero gradient and still move.  params, m and v are updated in place.
 * grads_out (nullable): when given, the gradient of this call is WRITTEN there (not accumulated), for callers
 * that inspect it.  The step is skipped (params, m, v and *adam->step unchanged) when the frame's instance
 * capacity overflowed (GS_FLAG_INSTANCE_OVERFLOW in frame->counters[1]); adam->skip_flags is not used.
 * Arguments are checked as for gs_render_bwd and gs_adam_step. */
int gs_render_bwd_adam(const gs_params* params, const gs_frame* frame, const gs_opts* opts, const gs_images* fwd,
                       const gs_loss* loss, const gs_params* m, const gs_params* v, const gs_adam* adam,
                       const gs_params* grads_out, void* stream);

/* The SSIM term of the photometric loss (Section III-E, eq. Lc: L_c = (1 - lambda) L1 + lambda L_ssim) for every
 * view: lambda w_v (1 - mean over the three channels and the view's pixels of SSIM(rgb, tgt_rgb)), with SSIM over an
 * 11 x 11 Gaussian window (standard deviation 1.5 px, summing to 1, zero padding at the image borders),
 * C1 = 0.01^2, C2 = 0.03^2 (the readings of the 3DGS work the paper builds on; the paper gives none).
 * cams_host: the planned cameras (host, from gs_plan_cameras), cams_dev: their device copy; rgb, tgt_rgb and
 * g_rgb have the layout of gs_images.rgb.  g_rgb receives (is WRITTEN with) d(term)/d rgb, ready to be passed as
 * gs_loss.g_rgb of a loss-mode backward with lambda_ssim = lambda; loss_out (device, 64 floats) receives the
 * term's value in loss_out[0] (loss_out[1..32] are partial sums).  GS_ERR_ARG for NULL pointers, n_views
 * outside [1, 64] or lambda outside [0, 1]. */
int gs_ssim(const gs_camera* cams_host, const gs_camera* cams_dev, int32_t n_views, const float* rgb,
            const float* tgt_rgb, float lambda_ssim, float* g_rgb, float* loss_out, void* stream);

/* Opacity pruning (Section III-C: Gaussians whose opacity has fallen to the prunable threshold are removed):
 * every Gaussian with opacity sigmoid(logit) below min_opacity is dropped and the rest are compacted, in their
 * original order, to the front of out_params, out_m and out_v (each with room for params->n Gaussians, same
 * SH degree, not overlapping the inputs).  The decision compares the logit with the threshold's logit
 * (float)log(min_opacity / (1 - min_opacity)), computed on the host in double.  *n_kept (device) receives the
 * number kept; the caller reads it after the stream completes and uses the first n_kept rows.  scratch: device,
 * gs_prune_scratch_bytes(n) bytes.  GS_ERR_ARG for min_opacity outside (0, 1), NULL pointers or mismatched
 * sizes. */
size_t gs_prune_scratch_bytes(int64_t n);
int gs_prune(const gs_params* params, const gs_params* m, const gs_params* v, float min_opacity,
             const gs_params* out_params, const gs_params* out_m, const gs_params* out_v, int64_t* n_kept,
             void* scratch, void* stream);

/* Map expansion (Sections III-A, III-C, III-E): a keyframe's colourised LiDAR points become new Gaussians.
 *  1. visibility filter (Sec. III-C): a point projected into the keyframe (FP32, the projection's operation order)
 *     is kept where the keyframe's rendered visibility V at its pixel is at most tau_alpha (the map does not yet
 *     explain that pixel; the paper's sentence is garbled, this is its stated purpose); points behind the near
 *     plane or outside the image are kept;
 *  2. voxel deduplication and density cap (Sec. III-A): a point is accepted while its voxel (floor(x / voxel),
 *     FP32 IEEE division, |index| < 2^20) holds fewer than `cap` points: the map's n_old Gaussians, then this
 *     batch's accepted points in input order;
 *  3. initialisation (Sec. III-E): mean = the point; log-scales = log sqrt of the mean squared distance to its 3
 *     nearest accepted neighbours (at least 1e-7; fewer neighbours: the mean over those present); identity
 *     rotation; opacity logit = log(init_opacity / (1 - init_opacity)); SH degree-0 coefficients
 *     (rgb - 0.5) / Y_0, higher bands 0; Adam moments 0.
 * The accepted points are appended, in input order, as rows n_old .. n_old + *n_added - 1 of params, m and v,
 * whose arrays must have room for n_old + n_points rows (params->n is that room; rows below n_old are read, the
 * map's means only).  points, colours: device [n_points][3]; vis: device [H][W] visibility image of `cam` (host;
 * only R, T, fx, fy, cx, cy, width, height are read).  *n_added (device) receives the count.  scratch: device,
 * gs_expand_scratch_bytes(n_old, n_points) bytes.  GS_ERR_ARG for bad sizes or options, NULL pointers. */
typedef struct gs_expand_opts {
  float tau_alpha;    /* visibility threshold */
  float near_z;       /* 0.2 */
  float voxel;        /* voxel edge, metres (0.1) */
  float knn_cell;     /* cell edge of the neighbour grid, metres (> 0) */
  float init_opacity; /* opacity of a new Gaussian (0.1) */
  int32_t cap;        /* points per voxel (1: a voxel that holds a point takes no other) */
} gs_expand_opts;
size_t gs_expand_scratch_bytes(int64_t n_old, int64_t n_points);
int gs_expand(const gs_params* params, const gs_params* m, const gs_params* v, int64_t n_old, const float* points,
              const float* colours, int64_t n_points, const gs_camera* cam, const float* vis,
              const gs_expand_opts* opts, int64_t* n_added, void* scratch, void* stream);

/* Spatial order of the Gaussians (a memory layout for locality, not a step of the method): the permutation that
 * sorts the Gaussians along a Z-order (Morton) curve of their means (each coordinate quantised to 21 bits over
 * the means' bounding box: q = min(2^21 - 1, floor((x - lo) * (2^21 - 1) / max(hi - lo, 1e-30))) in FP32,
 * interleaved x, y, z from bit 0; stable, so equal codes keep their order), applied to params, m and v: out row k
 * = in row perm[k].  out_* must not overlap the inputs; perm_out (device, nullable, [n] int32) receives the
 * permutation.  Rendering and gradients are unchanged up to the order of equal-depth ties (by Gaussian index).
 * scratch: device, gs_spatial_order_scratch_bytes(n) bytes.  GS_ERR_ARG for mismatched sizes or NULL pointers. */
size_t gs_spatial_order_scratch_bytes(int64_t n);
int gs_spatial_order(const gs_params* params, const gs_params* m, const gs_params* v, const gs_params* out_params,
                     const gs_params* out_m, const gs_params* out_v, int32_t* perm_out, void* scratch,
                     void* stream);

/* ------------------------------------------------------------------ utilities */
/* Work counts of the frame's forward compositing at its tile shape, ADDED to counts[0..1] (device, uint64):
 * [0] pairs evaluated (each record of a pixel's tile list up to the record that stops the pixel),
 * [1] pairs contributing (alpha >= alpha_min, before the stop).  Diagnostic: these counts define the
 * algorithmic work of the compositing kernels. */
int gs_count_pairs(const gs_frame* frame, const gs_opts* opts, uint64_t* counts, void* stream);

/* Synchronises the stream and returns the instance count and flags of the frame (host outputs). */
int gs_read_counters(const gs_frame* frame, int64_t* n_instances, int32_t* flags, void* stream);

/* Stable ascending LSD radix sort of n (key, value) pairs on the low `key_bits` bits of the keys.
 * keys/vals are sorted in place through the buffers keys_tmp/vals_tmp; scratch must hold
 * gs_sort_scratch_ints(n) int32s.  The binning step uses the same sort. */
size_t gs_sort_scratch_ints(int64_t n);
int gs_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* keys_tmp, int32_t* vals_tmp, int64_t n,
                  int32_t key_bits, int32_t* scratch, void* stream);

/* The same sort for callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the ping-pong buffers and histograms live in a static device array
 * of the library (about 13.6 MB, one copy per GPU, held until the process ends), so the caller passes only
 * keys/vals, sorted in place.  n is limited to gs_sort_static_max() pairs (2^20); larger n returns
 * GS_ERR_ARG before anything is enqueued.  The call allocates nothing.  `stream` must belong to the current
 * device.  Every call on a GPU shares that GPU's array: calls that overlap on one GPU (on different streams,
 * or from several threads) race and must be serialised by the caller.  No part of the array needs clearing
 * between calls (every pass rewrites what it reads). */
int64_t gs_sort_static_max(void);
int gs_sort_pairs_static(uint64_t* keys, int32_t* vals, int64_t n, int32_t key_bits, void* stream);

const char* gs_status_string(int status);
const char* gs_last_error(void);
int gs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LIBGS_H */
