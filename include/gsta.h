/*
 * gsta.h -- C ABI of libgsta, the MI355X (gfx950) training hot path of GSta
 * ("GSta: Efficient Training Scheme with Siestaed Gaussians for Monocular 3D
 * Scene Reconstruction", arXiv 2504.06716).
 *
 * One training iteration of the paper's Algorithm 1 maps to:
 *   rasterize(G, freeze_map, cam_pose)           -> gsta_render_forward + gsta_render_backward
 *   loss_fcn(gt_image, render_image)             -> gsta_l1_loss (or fused: gsta_render_forward_l1)
 *   optimizer_step(G, lr, loss, freeze_map)      -> gsta_adam_masked
 *   update_freeze_map / reset_freeze_map         -> gsta_update_freeze_mask
 *   adaptive_densification(G)                    -> gsta_densify_prune, gsta_opacity_reset
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless marked (host).  The caller owns
 *     every argument buffer; the library owns only the scratch held in the
 *     context, allocated by gsta_create / gsta_reserve, and the fixed device
 *     array of gsta_l1_loss_noalloc.  No other call allocates device memory.
 *   - Work is enqueued on `stream` and the call returns without
 *     synchronising, except gsta_create, gsta_reserve, gsta_destroy and
 *     gsta_check.
 *   - Arguments are validated on the host before anything is enqueued; an
 *     invalid call returns GSTA_ERR_INVALID, enqueues nothing and leaves a
 *     message for gsta_last_error.  Conditions only the device can see (tile
 *     instance overflow, non-finite values) raise flags that gsta_check
 *     reports.
 *   - A context is not thread-safe.  Calls that share a context must be
 *     issued on one stream (or ordered by the caller).
 *
 * Parameter block (Section 3.1: a Gaussian is a mean, a scale, a rotation
 * quaternion, an opacity and SH colour coefficients up to 3 bands, 59
 * numbers at degree 3).  Structure of arrays, float32, R rows of stride ld:
 *   rows 0-2   mean (world x, y, z)
 *   rows 3-5   log-scale per local axis (scale = exp)
 *   rows 6-9   quaternion (w, x, y, z), normalised inside the library
 *   row  10    opacity logit (opacity = sigmoid)
 *   rows 11..  SH coefficients, row 11 + 3*k + channel, k < (D+1)^2
 * R = 11 + 3*(D+1)^2, D = sh_degree in 0..3.  Element (r, i) is at
 * block[r * ld + i]; ld >= n.
 */
#ifndef GSTA_H
#define GSTA_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSTA_OK = 0,
    GSTA_ERR_INVALID = 1,    /* bad argument; nothing was enqueued */
    GSTA_ERR_CAPACITY = 2,   /* (gsta_check) tile instances exceeded the reserved capacity */
    GSTA_ERR_HIP = 3,        /* a HIP runtime call failed; see gsta_last_error */
    GSTA_ERR_OOM = 4,        /* scratch allocation failed in create/reserve */
    GSTA_ERR_NONFINITE = 5   /* (gsta_check) a non-finite gradient reached the optimizer */
} gsta_status;

typedef struct gsta_ctx gsta_ctx;  /* opaque; owns all scratch */

/* Sizes the scratch is reserved for (host struct). */
typedef struct {
    int64_t max_gaussians;      /* N */
    int32_t max_views;          /* views per render call */
    int32_t max_height, max_width;
    int64_t instance_capacity;  /* (view, tile, Gaussian) pairs per render call; <= 2^32-1 */
    int32_t tile_w, tile_h;     /* must be 16 x 16 */
    int32_t n_slots;            /* forward states kept for a later backward (>= 1) */
} gsta_limits;

/* Pinhole camera (host struct).  Camera frame: x right, y down, z forward.
 * Pixel (px, py) has its centre at integer coordinates; a camera-space point
 * (x, y, z) lands at u = fx*x/z + cx, v = fy*y/z + cy. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float world_to_cam[12];     /* row-major [R | t]: x_cam = R x_world + t */
    float cam_pos[3];           /* camera centre in world coordinates (SH view direction) */
    float near_z;               /* Gaussians with camera depth <= near_z are culled */
} gsta_camera;

/* A parameter-shaped block (host struct holding a device pointer). */
typedef struct {
    int64_t n;                  /* Gaussians */
    int64_t ld;                 /* row stride in elements, >= n */
    int32_t sh_degree;          /* 0..3 */
    int32_t opacity_act;        /* row 10 -> opacity: 0 sigmoid(logit) (default); 1 |x|, the
                                   "absolute" activation of the finetune stage (Section 4.1),
                                   opacities above 1 allowed (alpha stays capped at 0.99) */
    float* block;               /* device, [R][ld] float32 */
    float* sh_mask;             /* device, [3][ld] float32, or NULL (no masking).  SH-band masking of
                                   the finetune stage (Section 3.3): in the parameters of a render
                                   call, one logit per Gaussian and SH band l = 1..3 (row l - 1); band
                                   l's coefficients are used where sigmoid(logit) > sh_mask_threshold
                                   (decided as logit > ln(t / (1 - t)) rounded to float32) and count
                                   as zero elsewhere; band 0 is never masked, bands above sh_degree
                                   are ignored.  In the gradient block of gsta_render_backward (g
                                   masked): receives dL/dlogit = dL/dM sigmoid'(logit), the
                                   straight-through estimate of the hard mask M, for the Gaussians
                                   whose parameter gradients it writes (NULL: not written).
                                   Densification rejects masked parameters. */
    float sh_mask_threshold;    /* gate threshold t on sigmoid(logit), in (0, 1); read with sh_mask */
} gsta_params;

/* Fields readable with gsta_get_state (after gsta_render_forward). */
typedef enum {
    GSTA_STATE_REC_GEO = 0,     /* float4 [V][N]: u, v, A, B: the conic (a, b) scaled so that the
                                   base-2 exponent is A dx^2 + B dx dy + C dy^2
                                   (A = -a log2(e)/2, B = -b log2(e))          */
    GSTA_STATE_REC_COL = 1,     /* float4 [V][N]: C = -c log2(e)/2, opacity, conservative screen
                                   half-extents x, y */
    GSTA_STATE_REC_RGB = 2,     /* float4 [V][N]: r, g, b (clamped colour), camera depth z */
    GSTA_STATE_RECT = 3,        /* uint16x4 [V][N]: tile x0, x1, y0, y1 (exclusive ends); all 0 if culled */
    GSTA_STATE_DEPTH_ORDER = 4, /* uint32 [V][N]: gid in ascending (float32 depth, gid) order, culled last */
    GSTA_STATE_INST_KEYS = 5,   /* uint32 [I]: view * T + tile of each instance, sorted */
    GSTA_STATE_INST_IDS = 6,    /* uint32 [I]: expansion index of each sorted instance (depth order within a tile) */
    GSTA_STATE_RANGES = 7,      /* uint32x2 [V*T]: [start, end) of each (view, tile) in the instance list */
    GSTA_STATE_T_FINAL = 8,     /* float [V][H][W]: transmittance left after the last member */
    GSTA_STATE_LAST = 9,        /* uint32 [V][H][W]: tile-list index + 1 of the last member (0 if none) */
    GSTA_STATE_N_INSTANCES = 10,/* uint64 [1]: instances generated (may exceed capacity) */
    GSTA_STATE_INST_GID = 11    /* uint32 [I]: gid of each expansion index (Gaussians in depth order,
                                   each one's tiles contiguous in row-major order) */
} gsta_state_field;

/* Execution options (gsta_set_option).  They change speed, not what is
 * computed: images, states and forward decisions are bit-identical for every
 * setting, and so are gradients except across GSTA_OPT_BWD_WAVES,
 * GSTA_OPT_BWD_VARIANT and GSTA_OPT_BWD_SEGMENT, which change the order of
 * the backward's float additions (agreement to rounding). */
typedef enum {
    GSTA_OPT_FWD_WAVES = 0,     /* forward compositing: 0 (default): one independent wave per 8x8
                                   quarter of each tile, each writing its quarter's backward
                                   checkpoints; or 1, 2 or 4 waves per 16x16 tile */
    GSTA_OPT_BWD_WAVES = 1,     /* waves per tile in backward compositing: 1, 2 or 4 (default 2) */
    GSTA_OPT_BWD_SEGMENT = 2,   /* splats per backward work item: 0 (one item per tile) or a power of
                                   two in [64, 65536] (default 64).  The forward checkpoints every
                                   pixel's transmittance and colour prefix at each multiple of it, so
                                   the backward of a long tile list is spread over several
                                   workgroups; gradients depend on it only through rounding. */
    GSTA_OPT_BINNING = 3,       /* how the per-tile lists are built: 0 (default) places every tile
                                   instance directly where views have at most 1408 tiles and the
                                   placement scratch was reserved for the call's views, else sorts;
                                   1 always expands and sorts the tile keys (LSD radix).  Both give
                                   the same lists (Section 3.1: splats per tile in depth order). */
    GSTA_OPT_DEPTH_SORT = 4,    /* the per-view depth sort: 0 (default) one kernel per 8-bit pass
                                   for views of at most 131072 Gaussians (2048 keys per workgroup,
                                   each pass leaving the next its per-chunk digit counts), else as
                                   2; 1 onesweep (a global digit histogram, then one kernel per
                                   pass with decoupled look-back); 2 histogram / scan / scatter
                                   kernels per pass.  All are the same stable sort: identical
                                   order. */
    GSTA_OPT_BWD_VARIANT = 5    /* backward compositing (Section 3.2.4): 0 (default) per pixel, lanes
                                   are pixels and each splat's terms are summed across the wave (a
                                   frozen splat skipped for all its pixels at once); 1 per splat, the
                                   paper's parallelisation: lanes are the splats of a 64-splat span,
                                   pixel state passed lane to lane, each lane summing its own splat.
                                   Gradients agree to rounding (the order of a splat's additions
                                   differs).  GSTA_OPT_BWD_WAVES applies to variant 0 only. */
} gsta_option;

/* ---- context ------------------------------------------------------------ */

/* Allocates the scratch for `lim` on the current HIP device. */
gsta_status gsta_create(const gsta_limits* lim, gsta_ctx** out);
/* Grows (never shrinks) the scratch; synchronises the device first. */
gsta_status gsta_reserve(gsta_ctx* ctx, const gsta_limits* lim);
void gsta_destroy(gsta_ctx* ctx);
/* Message for the last non-OK status returned on this context ("" if none);
 * with ctx NULL, that of the last failed context-free call on this thread. */
const char* gsta_last_error(const gsta_ctx* ctx);
/* Synchronises `stream`, then reports and clears the device flags:
 * GSTA_ERR_CAPACITY if a render overflowed the instance capacity,
 * GSTA_ERR_NONFINITE if the optimizer met a non-finite gradient.  The
 * largest instance count any render needed since the last check is written
 * to *max_instances (host, may be NULL). */
gsta_status gsta_check(gsta_ctx* ctx, hipStream_t stream, int64_t* max_instances);
/* Sets an execution option (gsta_option) for later calls. */
gsta_status gsta_set_option(gsta_ctx* ctx, int32_t option, int64_t value);
/* Copies `bytes` of an internal field of forward state `slot` into device
 * memory `dst` (stream-ordered).  For tests and tools. */
gsta_status gsta_get_state(gsta_ctx* ctx, int32_t slot, int32_t field, void* dst, int64_t bytes,
                           hipStream_t stream);

/* Phases timed by the profiler (gsta_set_profiling). */
typedef enum {
    GSTA_PHASE_PREPROCESS = 0,  /* per-Gaussian projection, records, depth keys */
    GSTA_PHASE_DEPTH_SORT = 1,  /* per-view radix sort of depth keys */
    GSTA_PHASE_BINNING = 2,     /* tile counts, scan, instance expansion */
    GSTA_PHASE_TILE_SORT = 3,   /* radix sort of tile keys + tile ranges */
    GSTA_PHASE_COMPOSITE = 4,   /* forward compositing */
    GSTA_PHASE_COMPOSITE_BWD = 5,
    GSTA_PHASE_PREPROCESS_BWD = 6,
    GSTA_PHASE_ADAM = 7,
    GSTA_PHASE_FREEZE = 8,
    GSTA_PHASE_LOSS = 9,
    GSTA_PHASE_DENSIFY = 10,    /* densify / prune / opacity reset */
    GSTA_N_PHASES = 11
} gsta_phase;

/* Profiling (for benchmarks; do not enable while capturing a HIP graph).
 * phase_mask bit i enables phase i (0 disables): the entry points record a
 * pair of HIP events on their stream around each enabled phase, and the
 * compositing kernels of enabled phases count the (pixel, splat) pairs they
 * evaluate.  gsta_read_profile synchronises,
 * writes per-phase totals since the last read -- ms[GSTA_N_PHASES] elapsed
 * time, launches[GSTA_N_PHASES] -- and counters[6] = (pixel, splat) pairs
 * evaluated by the forward and by the backward compositing, wave-level splat
 * iterations of the forward and of the backward, per-wave splat reductions
 * of the backward, and (pixel, splat) pairs of the backward that did
 * gradient work (all host arrays, each may be NULL), then resets the
 * totals. */
#define GSTA_PROFILE_COUNTERS (1 << 30)   /* phase_mask bit: also count pairs (slower kernels) */
gsta_status gsta_set_profiling(gsta_ctx* ctx, int32_t phase_mask);
gsta_status gsta_read_profile(gsta_ctx* ctx, double* ms, int64_t* launches, int64_t* counters);

/* ---- the hot path ------------------------------------------------------- */

/* Section 3.1, eqs. 1-2.  Renders n_views views of the Gaussians `g`:
 * per Gaussian, the EWA projection (covariance R S S^T R^T, Jacobian of the
 * perspective map with tangent ratios clamped to 1.3x the half field of view,
 * 2-D covariance + 0.3 I, conic = its inverse), SH colour + 0.5 clamped at 0,
 * opacity = sigmoid(logit); Gaussians with depth <= near_z are culled.  Each
 * Gaussian is binned to every 16x16 tile that meets the bounding box of its
 * 3-sigma ellipse; per tile the list is in ascending (float32 depth, gid)
 * order.  Each pixel composites front to back the Gaussians with
 * power = -0.5 d^T conic d >= -4.5 and alpha = min(0.99, o exp(power)) >=
 * 1/255, stopping before the one that would take the transmittance below
 * 1e-4:  C = sum c_i alpha_i T_i + T_final * bg.
 *   cams  (host) [n_views]; every view must have the same width and height.
 *   bg    (host) [3] background colour.
 *   image [n_views][3][H][W] float32 output.
 *   state_slot in [0, n_slots): the forward state (binning, T_final, last
 *   member) is kept there for gsta_render_backward.
 * Returns GSTA_ERR_INVALID for sizes beyond the reserved limits. */
gsta_status gsta_render_forward(gsta_ctx* ctx, const gsta_params* g, const gsta_camera* cams,
                                int32_t n_views, const float* bg, float* image, int32_t state_slot,
                                hipStream_t stream);

/* Algorithm 1, rasterize + loss_fcn in one pass: gsta_render_forward, and
 * the L1 loss of its image against `target` computed by the compositing
 * kernel as it writes each pixel.  dL_dimage and sums are those of
 * gsta_l1_loss(image, target, n_views*3*H*W) -- dL_dimage bit for bit, sums
 * up to the order of their double additions.
 *   target, dL_dimage [n_views][3][H][W] float32 (device); sums device double [2].
 * Same errors as gsta_render_forward; NULL target, dL_dimage or sums is
 * GSTA_ERR_INVALID. */
gsta_status gsta_render_forward_l1(gsta_ctx* ctx, const gsta_params* g, const gsta_camera* cams,
                                   int32_t n_views, const float* bg, const float* target, float* image,
                                   float* dL_dimage, double* sums, int32_t state_slot, hipStream_t stream);

/* Section 3.2.4.  Backward of gsta_render_forward for the same g, cams,
 * n_views, bg and state_slot (checked).  dL_dimage [n_views][3][H][W].
 * Per pixel the transmittance is recomputed front to back (nothing per
 * (pixel, Gaussian) is stored).  Gaussians with frozen[i] != 0 still
 * attenuate the pixels behind them, but get no gradient work: their rows of
 * `grad` are not written.  Rows of active Gaussians are overwritten with the
 * gradient summed over the views.  frozen [n] uint8 or NULL (none frozen).
 *   grad2d  optional [n_views][9][n] float32 output: dL/d(u, v, conic_a,
 *           conic_b, conic_c, opacity, r, g, b) per view, written for active
 *           Gaussians only; NULL to skip.
 * No atomics are involved: every per-tile partial has its own slot and the
 * sums run in a fixed order, so the result is bit-reproducible.
 *   ema     optional [4][n] float32 in/out: exponential moving averages of
 *           |dL/dmean|, |dL/d(DC colour)|, |dL/dlogit|, |dL/dlog-scale| for
 *           active Gaussians visible in >= 1 view: s <- b*s + (1-b)*g, and
 *           s <- g where s is FLT_MAX (never seen).  NULL to skip.
 *   ema_beta in [0, 1).
 *   dstats  optional [4][n] float32 in/out: densification statistics of
 *           active Gaussians (Section 3.1, Section 4.1).  For every view in
 *           which the Gaussian is visible, row 0 += |(dL/du W/2, dL/dv H/2)|
 *           (the gradient with respect to the normalised device coordinates
 *           of its projected mean) and row 1 += 1; once per call, if it is
 *           visible in any view, row 2 += |dL/d(DC colour)| and row 3 += 1.
 *           NULL to skip. */
gsta_status gsta_render_backward(gsta_ctx* ctx, const gsta_params* g, const gsta_camera* cams,
                                 int32_t n_views, const float* bg, int32_t state_slot,
                                 const float* dL_dimage, const uint8_t* frozen, gsta_params* grad,
                                 float* grad2d, float* ema, float ema_beta, float* dstats,
                                 hipStream_t stream);

/* Section 3.2.4 (optimizer that updates only non-frozen Gaussians).  Adam
 * with bias correction on every row of the block:
 *   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *   p <- p - lr[row] * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * Columns with frozen[i] != 0 keep p, m and v bit-unchanged.
 * p, grad, m, v share n and sh_degree (their ld may differ).
 *   lr_per_row (host) [R];  step >= 1 is the global step;  frozen [n] or NULL.
 * A non-finite gradient in an active column raises the NONFINITE flag (the
 * update is still applied). */
gsta_status gsta_adam_masked(gsta_ctx* ctx, gsta_params* p, const gsta_params* grad, gsta_params* m,
                             gsta_params* v, const float* lr_per_row, float beta1, float beta2,
                             float eps, int32_t step, const uint8_t* frozen, hipStream_t stream);

/* Device-resident Adam schedule, for iterations captured once in a HIP graph
 * and replayed: every scalar that changes from one iteration to the next is
 * read from device memory.  Position rows (0-2) use
 *   lr = pos_scale * exp((1 - t) ln(pos_lr_init) + t ln(pos_lr_final)),
 *   t = min((step - 1) / decay_iters, 1),
 * the other rows lr[row].  Bias corrections use `step`. */
typedef struct {
    int32_t step;            /* Adam step of the next update (>= 1) */
    int32_t decay_iters;
    float beta1, beta2, eps;
    float pos_lr_init, pos_lr_final, pos_scale;
    float lr[64];            /* per-row learning rate, rows >= 3 */
} gsta_adam_sched;

/* gsta_adam_masked with the scalars taken from `sched` (device pointer),
 * followed by sched->step += 1 on the device (stream-ordered). */
gsta_status gsta_adam_masked_sched(gsta_ctx* ctx, gsta_params* p, const gsta_params* grad, gsta_params* m,
                                   gsta_params* v, gsta_adam_sched* sched, const uint8_t* frozen,
                                   hipStream_t stream);

/* The same masked Adam step (Section 3.2.4) over any [rows][ld] float32 block
 * of n columns, all four arrays with the same ld: the optimizer of the
 * SH-band mask logits of the finetune stage (Section 3.3; rows = 3).  p,
 * grad, m, v device; lr_per_row host [rows], rows in [1, 64]; frozen [n] or
 * NULL (frozen columns bit-unchanged); step >= 1. */
gsta_status gsta_adam_rows(gsta_ctx* ctx, float* p, const float* grad, float* m, float* v, int64_t n,
                           int64_t ld, int32_t rows, const float* lr_per_row, float beta1, float beta2, float eps,
                           int32_t step, const uint8_t* frozen, hipStream_t stream);

/* Sparsity term of the SH-band masks (Section 3.3; the paper defers its
 * form to the masking methods it adopts; this library takes their mean
 * sigmoid): for logits [3][ld] (device) of n >= 1 Gaussians,
 *   out[0] = lambda * mean over the 3n logits of sigmoid(logit),
 *   out[1..3] = number of open gates of bands 1..3 (sigmoid(logit) > threshold,
 *               decided as for rendering),
 * and, if grad (device [3][ld]) is not NULL, grad += lambda sigmoid'(logit) /
 * (3n) for every column with frozen[i] == 0 (frozen [n] or NULL).  out:
 * device double [4].  Sums in a fixed order (deterministic). */
gsta_status gsta_sh_mask_reg(gsta_ctx* ctx, const float* logits, int64_t n, int64_t ld, float threshold,
                             float lambda, const uint8_t* frozen, float* grad, double* out, hipStream_t stream);

/* Section 3.2.1, eqs. 4 and 6, with the accumulation and reset of the freeze
 * map.  cond_i = (score_xyz[i] < eps_xyz) && (score_rgb[i] < eps_rgb)
 * (strict, float32), or proposal[i] != 0 when `proposal` is given.
 *   mode 0: frozen[i] |= cond_i  (frozen Gaussians stay frozen)
 *   mode 1: frozen[i] = 0        (reset; scores unused, may be NULL)
 *   mode 2: frozen[i] = cond_i   (overwrite)
 * n_frozen (device int64 [1]) receives the number of frozen Gaussians after
 * the update (may be NULL). */
gsta_status gsta_update_freeze_mask(gsta_ctx* ctx, const float* score_xyz, const float* score_rgb,
                                    int64_t n, float eps_xyz, float eps_rgb, int32_t mode,
                                    const uint8_t* proposal, uint8_t* frozen, int64_t* n_frozen,
                                    hipStream_t stream);

/* The naive freezing rules of the paper's ablation (Section 4.3, Table 3
 * rows "+mingrad" and "+random"), used in place of the thresholds of eqs. 4-6
 * to show what the gradient rule gains over them:
 *   GSTA_FREEZE_RULE_MINGRAD: among the Gaussians with score[i] < FLT_MAX
 *     (the positional gradient-norm average; FLT_MAX = never seen), the
 *     m = floor(fraction * count) with the smallest score (float32 order,
 *     equal scores by ascending index) are chosen.  Exact (radix select).
 *   GSTA_FREEZE_RULE_RANDOM: Gaussian i is chosen iff the top 32 bits of
 *     word 0 of Philox4x64-10(counter = (i, draw, 0, 0), key = (seed, 0)) are
 *     below floor(fraction * 2^32): independent Bernoulli(fraction) draws,
 *     fresh for every `draw` (e.g. the iteration of the update).  score unused.
 * The chosen Gaussians are applied with `mode` as in gsta_update_freeze_mask
 * (0: OR into the map, 1: reset, 2: replace); n_frozen (device int64 [1], may
 * be NULL) receives the frozen count.  fraction in [0, 1]; n <= max_gaussians. */
typedef enum { GSTA_FREEZE_RULE_MINGRAD = 1, GSTA_FREEZE_RULE_RANDOM = 2 } gsta_freeze_rule;
gsta_status gsta_update_freeze_mask_rule(gsta_ctx* ctx, int32_t rule, const float* score, int64_t n,
                                         double fraction, uint64_t seed, uint64_t draw, int32_t mode,
                                         uint8_t* frozen, int64_t* n_frozen, hipStream_t stream);

/* One per-Gaussian array for gsta_partition_frozen: `rows` rows of n
 * elements of `elem_bytes` (1, 2 or 4) bytes, row r at base + r*ld elements
 * (ld >= n; rows of one column block, an EMA block [4][n], a bf16 ring
 * [8][4][n] as 32 rows, an id array as 1 row). */
typedef struct {
    void* base;
    int64_t rows;
    int64_t ld;
    int32_t elem_bytes;
} gsta_columns;

/* Frozen Gaussians take no part in the optimizer step or the backward's
 * per-Gaussian chain (Section 3.2.4); the kernels skip them per column, so
 * a frozen set scattered over the columns saves little.  This call moves
 * them out of the way: a stable partition of columns [0, n) by the freeze
 * map, active (frozen[i] == 0) columns first, then the frozen ones, each
 * group in its former order.  The permutation is applied in place to every
 * array of `arrays` (host array of `count` descriptors; each array at most
 * once, none overlapping another or `tmp`) and to `frozen` itself, which
 * ends as n_active zeros followed by ones.  Rendering is unchanged up to the
 * order of Gaussians at exactly equal depth, which follows the column order.
 *   tmp: device scratch of at least max over arrays of rows*n*elem_bytes
 *        bytes (e.g. the gradient block between iterations).
 *   n_active (device int64 [1], may be NULL) receives the active count.
 * Not capturable into a HIP graph (it issues device-to-device copies). */
gsta_status gsta_partition_frozen(gsta_ctx* ctx, int64_t n, uint8_t* frozen, const gsta_columns* arrays,
                                  int32_t count, void* tmp, int64_t tmp_bytes, int64_t* n_active,
                                  hipStream_t stream);

/* Eq. 3 with lambda_SSIM = 0: L = mean |C - C*| over `count` values.
 *   dL_dimage[j] = sign(C_j - C*_j) / count (sign(0) = 0).
 *   sums (device double [2]) receive sum |C - C*| and sum (clamp(C,0,1) - C*)^2
 *   (the loss is sums[0] / count, the PSNR 10 log10(count / sums[1])). */
gsta_status gsta_l1_loss(gsta_ctx* ctx, const float* image, const float* target, int64_t count,
                         float* dL_dimage, double* sums, hipStream_t stream);

/* The D-SSIM term of eq. 3, L = (1 - lambda) L1 + lambda L_D-SSIM with
 * lambda_SSIM = 0.2 in the paper.  SSIM per channel with an 11 x 11 Gaussian
 * window (sigma 1.5, normalised, zero padding at the image border), C1 =
 * 0.01^2, C2 = 0.03^2; L_D-SSIM = 1 - mean of the SSIM map over the
 * n_views * 3 * height * width values.  The separable window runs as row and
 * column passes over LDS tiles, fused with the map and its derivative
 * (Section 3.3, accelerated SSIM).
 *   image, target [n_views][3][height][width] float32.
 *   dL_dimage in/out: on entry the L1 gradient (gsta_l1_loss or the fused
 *     forward), on exit (1 - lambda) dL_dimage + lambda dL_D-SSIM/dimage,
 *     the gradient of eq. 3.
 *   ssim_sum (device double [1]) receives the sum of the SSIM map (the loss
 *     is (1 - lambda) L1 + lambda (1 - ssim_sum / count)).
 * Sizes must fit the reserved limits; lambda in [0, 1]. */
gsta_status gsta_dssim_loss(gsta_ctx* ctx, const float* image, const float* target, int32_t n_views,
                            int32_t height, int32_t width, float lambda, float* dL_dimage, double* ssim_sum,
                            hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the L1
 * loss of gsta_l1_loss without a context.  Same arguments, same kernels and
 * the same fixed summation order, so dL_dimage and sums equal gsta_l1_loss's
 * bit for bit.  Its partial sums live in a library-owned device array of
 * 1024 double2 (16 KiB) per GPU, held until the process ends; the call
 * allocates nothing.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (different streams, no ordering) race and must not be
 * issued.  count in [1, GSTA_L1_NOALLOC_MAX_COUNT] (1024 workgroups x 256
 * lanes x 4096 values per lane); beyond it, or with a NULL pointer, the call
 * returns GSTA_ERR_INVALID, enqueues nothing and leaves a message for
 * gsta_last_error(NULL). */
#define GSTA_L1_NOALLOC_MAX_COUNT ((int64_t)1 << 30)
gsta_status gsta_l1_loss_noalloc(const float* image, const float* target, int64_t count, float* dL_dimage,
                                 double* sums, hipStream_t stream);

/* Adaptive densification and pruning (Section 3.1: Gaussians are densified
 * by gradient norm and pruned by opacity; Section 4.1: run every 100
 * iterations with thresholds scaled like the freezing thresholds, the
 * diffuse-colour criterion on a fifth of the steps).  The clone / split /
 * prune rules are the 3DGS conventions the paper builds on.  Decisions, all
 * float32 comparisons of the inputs:
 *   mean screen gradient  = dstats[0] / dstats[1] (0 if dstats[1] = 0),
 *   mean colour gradient  = dstats[2] / dstats[3] (0 if dstats[3] = 0),
 *   selected = (mean screen gradient >= grad_threshold
 *               || (use_rgb && mean colour gradient >= rgb_threshold)) && !frozen,
 *   split    = selected && max(log-scales) >  split_log_scale,
 *   clone    = selected && max(log-scales) <= split_log_scale,
 *   live     = logit >= prune_logit   (opacity at least sigmoid(prune_logit)). */
typedef struct {
    float grad_threshold;          /* e.g. eps_den_xyz(k) = 2e-4 scaled by the eq. 5 factor */
    float rgb_threshold;           /* e.g. eps_den_rgb(k) = 1e-6 scaled likewise */
    int32_t use_rgb;               /* 0/1: colour criterion on this step */
    float split_log_scale;         /* ln(0.01 * scene extent) */
    float prune_logit;             /* ln(0.005 / 0.995) */
    float child_log_scale_shift;   /* ln(1.6): children's scales are the parent's / 1.6 */
    uint64_t noise_seed;           /* with noise NULL: the children's normals come from Philox4x64-10 */
    int64_t noise_draw;            /* (counter (column, noise_draw, child, 0), key (noise_seed, 1)), Box-Muller
                                      on its four words u = (w >> 11 + 0.5) 2^-53: r = sqrt(-2 ln u0),
                                      n = (r cos 2 pi u1, r sin 2 pi u1, sqrt(-2 ln u2) cos 2 pi u3), in double;
                                      e.g. noise_draw = the iteration */
} gsta_densify_cfg;

/* One densify-and-prune step: a stream compaction of every per-Gaussian
 * array into the caller's output arrays (which must not overlap the inputs).
 * Output columns, in order: each live Gaussian that is not split, in input
 * order (its p, m, v, ema and frozen copied); a copy of each live
 * clone-selected Gaussian (zero m and v, ema FLT_MAX, not frozen); the first
 * child of each live split Gaussian, then the second children.  Child c of
 * Gaussian i has mean mu_i + R(q_i) (exp(log_s_i) * noise[3c + a][i])_a,
 * log-scales log_s_i - child_log_scale_shift and every other parameter of
 * i; zero m and v, ema FLT_MAX, not frozen.  Split and non-live Gaussians
 * leave the set (frozen ones are pruned by the same rule).
 *   g, m, v   [R][ld] inputs (shared n and sh_degree).
 *   ema [4][n] or NULL (then survivors get FLT_MAX); frozen [n] or NULL.
 *   dstats [4][n] as accumulated by gsta_render_backward.
 *   noise [6][n] float32 standard-normal draws (rows 3c..3c+2 for child c),
 *         or NULL to draw them in the kernel (cfg->noise_seed, noise_draw).
 *   g_out, m_out, v_out: the n field is the output capacity (columns).
 *   ema_out [4][n_out] contiguous (room for 4 * capacity floats) or NULL;
 *   frozen_out [n_out] (room for capacity) or NULL.
 *   counts (device int64 [4]) receives (n_out, kept, clones, split parents).
 * If n_out exceeds the capacity nothing is written to the outputs and
 * gsta_check reports GSTA_ERR_CAPACITY. */
gsta_status gsta_densify_prune(gsta_ctx* ctx, const gsta_params* g, const gsta_params* m,
                               const gsta_params* v, const float* ema, const uint8_t* frozen,
                               const float* dstats, const float* noise, const gsta_densify_cfg* cfg,
                               gsta_params* g_out, gsta_params* m_out, gsta_params* v_out,
                               float* ema_out, uint8_t* frozen_out, int64_t* counts,
                               hipStream_t stream);

/* Switch to the finetune stage's absolute opacity activation (Section 4.1:
 * when the finetune starts, opacity = sigmoid(x) becomes opacity = |x|).
 * For every column of g (opacity_act 0 on entry): x <- sigmoid(x), so each
 * opacity is unchanged, and the Adam moments of row 10 are zeroed (they were
 * taken in logit units).  The caller renders g with opacity_act = 1 from
 * then on.  g, m, v share n. */
gsta_status gsta_opacity_to_absolute(gsta_ctx* ctx, gsta_params* g, gsta_params* m, gsta_params* v,
                                     hipStream_t stream);

/* Opacity reset (Section 4.1, every 3K iterations): for every active
 * Gaussian logit <- min(logit, logit_cap) (opacity capped at
 * sigmoid(logit_cap), e.g. 0.01) and the Adam moments of the opacity row are
 * zeroed.  Frozen Gaussians are left untouched. */
gsta_status gsta_opacity_reset(gsta_ctx* ctx, gsta_params* g, gsta_params* m, gsta_params* v,
                               const uint8_t* frozen, float logit_cap, hipStream_t stream);

/* ---- learned freeze proposer ---------------------------------------------
 * A project extension (the paper has no such model), made for the callers
 * that want Gaussians frozen earlier than the rule of Section 3.2.1 alone
 * would: an MLP 32 -> 64 -> 64 -> 1 (ReLU, ReLU, logit) reads the last 8
 * logged gradient-norm averages of a Gaussian and proposes it for the
 * freeze map; the rule vetoes proposals whose averages are far above its
 * thresholds (gsta_mlp_propose) and accepted proposals are OR-ed into the
 * map (gsta_update_freeze_mask, `proposal`).
 *
 * Parameters: a flat float32 array of GSTA_MLP_PARAMS values, W1 [64][32]
 * (offset 0), b1 [64] (2048), W2 [64][64] (2112), b2 [64] (6208), w3 [64]
 * (6272), b3 (6336); plus a bf16 copy of W1 then W2 (GSTA_MLP_BF16 values,
 * 16-byte aligned) that the forward reads.  The hidden layers run on bf16
 * matrix cores with float32 accumulation; the first hidden layer is rounded
 * to bf16 (nearest, ties to even) before the second.
 * Trajectory ring: [8][4][n] bf16 (entry, score, Gaussian). */
#define GSTA_MLP_PARAMS 6337
#define GSTA_MLP_BF16 6144

/* ring[slot][q][i] = bf16(min(ema[q][i], 1e30)) for the 4 averages
 * (xyz, rgb, opacity, scale) of gsta_render_backward; slot in [0, 8). */
gsta_status gsta_traj_push(gsta_ctx* ctx, const float* ema, int64_t n, uint16_t* ring, int32_t slot,
                           hipStream_t stream);

/* Adds to sums (device double [64]) the per-feature sum (0..31) and sum of
 * squares (32..63) of the unstandardised features log10(r + 1e-12) of
 * gsta_mlp_features over the n Gaussians, for standardisation statistics
 * over a training set (call once per ring snapshot; the caller zeroes). */
gsta_status gsta_mlp_feature_stats(gsta_ctx* ctx, const uint16_t* ring, int64_t n, int32_t head, double* sums,
                                   hipStream_t stream);

/* x [n][32] bf16: x[i][4j + q] = bf16((log10(ring[(head - j) & 7][q][i] + 1e-12)
 * - mean[4j + q]) / std_dev[4j + q]), j = 0 the newest entry (at head).
 * mean, std_dev: device float [32]. */
gsta_status gsta_mlp_features(gsta_ctx* ctx, const uint16_t* ring, int64_t n, int32_t head, const float* mean,
                              const float* std_dev, uint16_t* x, hipStream_t stream);

/* logits [n] of the MLP for features x [n][32] bf16.  h1 ([n][64] bf16) and
 * h2 ([n][64] float32) optionally receive the hidden layers for
 * gsta_mlp_backward (NULL to skip). */
gsta_status gsta_mlp_forward(gsta_ctx* ctx, const uint16_t* w_bf16, const float* w, const uint16_t* x, int64_t n,
                             float* logits, uint16_t* h1, float* h2, hipStream_t stream);

/* Mean binary cross-entropy of logits against labels (uint8 0/1) into loss
 * (device double [1]) and dz[i] = (sigmoid(logits[i]) - labels[i]) / n. */
gsta_status gsta_mlp_bce(gsta_ctx* ctx, const float* logits, const uint8_t* labels, int64_t n, float* dz,
                         double* loss, hipStream_t stream);

/* grad [GSTA_MLP_PARAMS] = gradient of sum_i dz[i] * logit_i with respect to
 * the flat parameters, through the forward's saved h1, h2 (the bf16
 * roundings taken as identity).  Deterministic (fixed summation order). */
gsta_status gsta_mlp_backward(gsta_ctx* ctx, const uint16_t* w_bf16, const float* w, const uint16_t* x,
                              const uint16_t* h1, const float* h2, const float* dz, int64_t n, float* grad,
                              hipStream_t stream);

/* Adam on the float32 parameters (bias-corrected with `step`), then the
 * bf16 copies of W1 and W2 are refreshed. */
gsta_status gsta_mlp_adam(gsta_ctx* ctx, float* w, const float* grad, float* m, float* v, float lr, float beta1,
                          float beta2, float eps, int32_t step, uint16_t* w_bf16, hipStream_t stream);

/* w_bf16 = bf16 copies of W1 and W2 of w (after the caller sets w). */
gsta_status gsta_mlp_sync_bf16(gsta_ctx* ctx, const float* w, uint16_t* w_bf16, hipStream_t stream);

/* proposal[i] = logits[i] > logit_threshold && score_xyz[i] < veto_xyz &&
 * score_rgb[i] < veto_rgb (float32 comparisons). */
gsta_status gsta_mlp_propose(gsta_ctx* ctx, const float* logits, const float* score_xyz, const float* score_rgb,
                             int64_t n, float logit_threshold, float veto_xyz, float veto_rgb, uint8_t* proposal,
                             hipStream_t stream);

/* ---- captured iterations and the autotuner --------------------------------
 * Several views per launch, whole iterations captured in a HIP graph and an
 * autotuner over launch options are project extensions (not in the paper)
 * for the many small launches of one training iteration. */

/* A captured sequence of library calls (a training iteration), replayed
 * with gsta_graph_launch.  A graph keeps the pointers, sizes, cameras and
 * options of its capture: it is invalid after gsta_reserve, after any buffer
 * it uses is freed, or for other cameras.  Host-side scalars (e.g. Adam's
 * step) must come from device memory (gsta_adam_masked_sched). */
typedef struct gsta_graph gsta_graph;
/* Starts capturing `stream` (not the null stream): the library calls issued
 * on it until gsta_graph_end are recorded, not run.  Profiling must be off;
 * gsta_check, gsta_reserve and gsta_autotune are refused meanwhile. */
gsta_status gsta_graph_begin(gsta_ctx* ctx, hipStream_t stream);
/* Ends the capture and instantiates it into *out (release with
 * gsta_graph_destroy). */
gsta_status gsta_graph_end(gsta_ctx* ctx, hipStream_t stream, gsta_graph** out);
/* Replays a captured graph on `stream` (stream-ordered, no synchronisation). */
gsta_status gsta_graph_launch(gsta_graph* graph, hipStream_t stream);
void gsta_graph_destroy(gsta_graph* graph);

/* Result of gsta_autotune (host struct). */
typedef struct {
    int32_t fwd_waves;      /* GSTA_OPT_FWD_WAVES chosen */
    int32_t bwd_waves;      /* GSTA_OPT_BWD_WAVES chosen */
    int32_t bwd_segment;    /* GSTA_OPT_BWD_SEGMENT chosen (0: one work item per tile) */
    int32_t candidates;     /* settings timed */
    float fwd_ms;           /* forward per call with the chosen forward shape */
    float step_ms;          /* forward + backward per call with the chosen options */
    int32_t bwd_variant;    /* GSTA_OPT_BWD_VARIANT chosen (bwd_waves applies to variant 0) */
} gsta_tuning;

/* Times the execution options that do not change results on the caller's
 * own workload -- forward waves {0, 1, 2, 4} (forward calls), then the
 * backward: the per-pixel variant's waves {1, 2, 4} and the per-splat
 * variant (Section 3.2.4), each x segment length {64, 128, 256, one item per
 * tile} (forward + backward calls) -- `repeats` calls each after one untimed
 * call, and sets the fastest on the context (profiling is suspended
 * meanwhile).  Synchronises.  frozen [n] (device, or NULL): the freeze map
 * the backward calls skip, as in training.  image [n_views][3][H][W],
 * dL_dimage (same shape; any values) and grad (shaped like g) are the
 * caller's scratch; their contents afterwards are unspecified.  out (host)
 * may be NULL. */
gsta_status gsta_autotune(gsta_ctx* ctx, const gsta_params* g, const gsta_camera* cams, int32_t n_views,
                          const float* bg, float* image, float* dL_dimage, gsta_params* grad, const uint8_t* frozen,
                          int32_t repeats, gsta_tuning* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GSTA_H */
