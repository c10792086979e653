/*
 * snp.h -- C ABI of the splattable-neural-primitive rasterizer for MI355X
 * (gfx950).
 *
 * The library renders primitives made of an ellipsoid bound and a shallow
 * cosine density MLP (Splat the Net, ICLR 2026, Sec. 3.1, Eq. 5-6): for every
 * pixel ray and every primitive whose screen bounds cover the pixel it
 * intersects the ray with the ellipsoid, integrates the density exactly over
 * the chord (Eq. 7-8), turns the integral into alpha = 1 - exp(-max(0, .))
 * (Eq. 9) and blends front to back in depth order (Eq. 3-4).  The backward
 * pass is the exact adjoint of that forward pass for an L1 image loss.
 *
 * Conventions shared by every entry point
 *  - All arrays passed as `const float*` / `float*` are DEVICE pointers,
 *    owned by the caller, float32, C-contiguous.  `cams` and `cfg` are HOST
 *    pointers read during the call only.
 *  - Every call only enqueues work on `stream` (a hipStream_t; 0 = null
 *    stream).  No call allocates memory, synchronises, or keeps a pointer
 *    after it returns -- except snp_read_status and snp_read_counters
 *    (synchronise the stream), snp_kernel_timing_read (waits for its events)
 *    and the snp_graph_* calls (documented there).
 *  - Arguments are validated on the host before anything is enqueued; an
 *    invalid call returns SNP_ERR_INVALID and enqueues nothing.
 *  - Sizes that are only known on the device (the number of tile instances)
 *    are checked on the device against the workspace capacity; an overflow
 *    sets a flag that snp_read_status reports (SNP_ERR_CAPACITY); the results
 *    of that step are then incomplete and must be discarded.
 *  - Images: the V views are packed one after another, view v as a row-major
 *    H_v x W_v x 3 block (RGB); transmittances likewise as H_v x W_v.
 *  - Primitive arrays (P primitives, N hidden units): centers P x 3,
 *    scales P x 3 (semi-axis lengths, > 0), quats P x 4 (w, x, y, z; need not
 *    be normalised), w1 P x N x 3, b1 P x N, w2 P x N, b2 P, optionally wt
 *    P x N (time-conditioned density), and the colour: colors P x 3
 *    (color_mode 0), cmlp P x K with xi P x 8 (color_mode 1; K from 11
 *    network inputs), sh P x 16 x 3 (color_mode 2), colors (c_dc), cmlp
 *    (K from 14 inputs) and xi (color_mode 3), or colors (c_dc) and cmlp
 *    (K from 9 inputs; color_mode 4).
 *  - A second primitive kind (snp_config.primitive = 1) renders 3D Gaussians
 *    through the same tiling, sorting and blending, as the 3DGS splatting
 *    kernel the paper measures against (App. A, integration-cost table):
 *    scales are then standard deviations, opacity P floats, and w1..b2 are
 *    not read.  It has a forward pass only.
 */
#ifndef SNP_H_
#define SNP_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SNP_OK = 0,
  SNP_ERR_INVALID = 1,     /* bad argument; nothing was enqueued */
  SNP_ERR_CAPACITY = 2,    /* tile instances exceeded the workspace capacity */
  SNP_ERR_HIP = 3,         /* a HIP runtime call or kernel launch failed */
  SNP_ERR_UNSUPPORTED = 4, /* valid but not built (e.g. N outside {4,8,16,32}) */
  SNP_ERR_RANGE = 5,       /* density-MLP phase outside the hardware sine range */
  SNP_ERR_TOO_LARGE = 6    /* snp_step_static: the step does not fit in its static scratch */
} snp_status;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  A world point X
 * has camera coordinates R X + t (R row-major); pixel (i, j) -- column i,
 * row j -- has its centre at (i + 0.5, j + 0.5) and views the direction
 * R^-1 ((i + 0.5 - cx)/fx, (j + 0.5 - cy)/fy, 1) from the camera centre
 * -R^-1 t (Sec. 2.1: rays r(t) = o + t d, t in world length). */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float light[3]; /* world position of the view's point light (colour mode 3 only) */
} snp_camera;

/* Rendering options.  Readings of what the paper leaves open:
 *  n_hidden   N, width of the density MLP (Eq. 6); 4, 8, 16 or 32.
 *  omega0     frequency boost omega0 of Eq. 6 (multiplies W1 x + b1).
 *  color_mode 0 = constant RGB per primitive; 1 = per-(primitive, view)
 *             colour MLP: input [normalize(x_B - o_v), xi_p], cmlp_depth
 *             ReLU layers of cmlp_width units, sigmoid RGB output; weights
 *             per primitive layer after layer, each W (out x in) then b;
 *             2 = spherical harmonics of degree 3 (Sec. 3.1, four bands as
 *             in 3DGS): colour = max(0, 1/2 + sum_k Y_k(d) sh[k]) with the
 *             16 real orthonormal harmonics at d = normalize(x_B - o_v);
 *             3 = relighting colour: colors (c_dc) + the colour network of
 *             mode 1 with input [normalize(x_B - o_v), normalize(l_v - x_B),
 *             xi_p] (14 inputs; l_v = the camera's light), per (primitive,
 *             view);
 *             4 = per-ray relighting colour (the relighting application's
 *             colour per view ray): colors (c_dc) + sigmoid(MLP(input)) per
 *             (pixel, primitive) pair, input [(o + t_in d - x_B)/max(s_B),
 *             d, normalize(l_v - x_B)] (9 inputs: the ray's entry point into
 *             the ellipsoid normalised as the density's input, the unit ray
 *             direction, the light direction relative to the centre), one
 *             ReLU layer of cmlp_width = 16 units (cmlp_depth = 1), no xi;
 *             built for N = 8, 16, 16 x 16 tiles with one pixel per thread
 *             and backward batches of 8 (else SNP_ERR_UNSUPPORTED).
 *  tile_w, tile_h, px_per_lane: rasterizer tile shape and pixels per thread;
 *             supported shapes are listed by snp_supported_tiles().
 *  z_near     a primitive is culled for a view unless its whole ellipsoid
 *             lies in front of camera-space z = z_near.
 *  t_eps      a pixel takes no more primitives once its transmittance fell
 *             below t_eps (0 disables early termination).
 *  alpha_min  primitives with alpha < alpha_min are skipped (0 disables).
 *  alpha_max  alpha is clamped to at most alpha_max (< 1).
 *  bg         background colour added as T_final * bg.
 *  persistent 1 = one persistent launch over all (view, tile) work items
 *             with a device work queue (for neural primitives the queue
 *             hands out the tiles with the most instances first, so the
 *             heaviest tiles do not form the tail); 0 = one workgroup per
 *             tile.
 *  bwd_batch  instances per batch of the backward rasterizer (0 = the
 *             default for the tile shape); the tile shape is shared with the
 *             forward, and the backward runs one pixel per thread.
 *  fwd_cache  1 = the forward stores the integral (alpha-hat, Eq. 8-9) of
 *             every (pixel, instance) pair it evaluates, capacity x tile_w x
 *             tile_h floats in the workspace, and the backward reads it back
 *             instead of evaluating the density MLP again; a backward must
 *             then follow a forward of the same step on the same workspace.
 *             0 = the backward re-evaluates every pair (no extra memory).
 *  fwd_cache_instances  with fwd_cache = 1: how many leading tile instances
 *             (in sorted order) have their pairs kept, 0 = all of them
 *             (the workspace capacity); batches of the backward that reach
 *             past them re-evaluate.  Lets the cache use whatever memory is
 *             free when the whole of it does not fit.
 *  primitive  0 = neural primitives (everything above); 1 = 3D Gaussians
 *             splatted as in 3DGS (EWA): covariance R diag(s^2) R^T pushed
 *             through the Jacobian of the projection at the centre (x/z and
 *             y/z clamped to 1.3 times the view), plus 0.3 px^2 on the
 *             diagonal; kept iff the centre is in front of z_near; screen
 *             bound the square of radius ceil(3 sqrt(lambda_max)) around the
 *             projected centre; per pixel inside it alpha = min(alpha_max,
 *             opacity exp(-d^T Sigma2d^-1 d / 2)).  n_hidden, omega0 and
 *             fwd_cache are ignored; forward only (the backward, snp_step
 *             and snp_graph_create return SNP_ERR_UNSUPPORTED).
 *  bin_order  how snp_bin / snp_sort reach the (tile, depth) order; both
 *             give the same arrays bit for bit.  1 = the (view, primitive)
 *             pairs are sorted by depth first, instances are emitted in that
 *             order and sorted by their tile bits only (fewer passes over
 *             the instances, a few more launches); 2 = instances emitted in
 *             primitive order and sorted by the whole key; 0 = 1 when
 *             V * P >= 2^16, else 2.
 *  time       xi_t in [0, 1] of the dynamic-scene application: with
 *             prims.wt the phase of hidden unit k is omega0 (W1_k x + b1_k) +
 *             time * wt_k (the time term added unscaled, as the paper prints
 *             it); with prims.sh_t (color_mode 2) the zero-order SH
 *             coefficient is sh[p][0][c] + sum_{i=1..4} (a_i xi^i +
 *             b_i cos(i xi) + c_i sin(i xi)) (polynomial and Fourier series
 *             of degree 4); ignored without either. */
typedef struct {
  int32_t n_hidden;
  float omega0;
  int32_t color_mode;
  int32_t cmlp_width, cmlp_depth;
  int32_t tile_w, tile_h, px_per_lane;
  float z_near, t_eps, alpha_min, alpha_max;
  float bg[3];
  int32_t persistent;
  int32_t bwd_batch;
  int32_t fwd_cache;
  int64_t fwd_cache_instances;
  int32_t primitive;
  int32_t bin_order;
  float time;
} snp_config;

typedef struct {
  int64_t P;
  const float *centers, *scales, *quats, *w1, *b1, *w2, *b2;
  const float *colors; /* color_mode 0, or c_dc of color_mode 3 or 4, else NULL */
  const float *cmlp;   /* color_mode 1, 3 or 4, else NULL */
  const float *xi;     /* color_mode 1 or 3, else NULL */
  const float *sh;     /* color_mode 2: P x 16 x 3 (basis (l, m) in order (0,0), (1,-1), (1,0), (1,1), (2,-2) ... (3,3); channel), else NULL */
  const float *opacity; /* primitive 1: P opacities in (0, 1], used as given; else NULL */
  const float *wt;      /* P x N temporal weights of the time-conditioned density, or NULL */
  const float *sh_t;    /* color_mode 2 in the dynamic-scene application: P x 12 x 3 coefficients of the
                           time-dependent zero-order SH term (a_1..a_4 of xi_t^i, b_1..b_4 of cos(i xi_t),
                           c_1..c_4 of sin(i xi_t); channel), added to sh[p][0][c]; or NULL */
} snp_prims;

/* Gradient outputs, same shapes as the parameters.  The backward ADDS into
 * them (the caller zeroes them first); NULL skips a tensor (gradients of xi
 * are only produced when non-NULL). */
typedef struct {
  float *centers, *scales, *quats, *w1, *b1, *w2, *b2, *colors, *cmlp, *xi, *sh;
  float *wt;   /* P x N, with prims.wt */
  float *sh_t; /* P x 12 x 3, with prims.sh_t */
} snp_grads;

/* Byte offsets of the internal arrays inside a workspace (for inspection by
 * tests and tools).  All offsets are from the workspace base pointer. */
typedef struct {
  size_t bytes;           /* total workspace size */
  size_t cams;            /* per-view device constants */
  size_t table;           /* per-primitive density table, P x table_stride floats */
  size_t records;         /* per-(view, primitive) records, V*P x 24 floats */
  size_t rects;           /* per-(view, primitive) pixel rectangles, int32 x0,x1,y0,y1 */
  size_t depth_bits;      /* per-(view, primitive) uint32 depth key (0 = culled) */
  size_t tile_counts;     /* per-(view, primitive) uint32 number of tiles */
  size_t offsets;         /* uint32 exclusive scan of tile_counts over the (view, primitive) pairs (in depth order with bin_order 1) */
  size_t keys;            /* uint64 sorted keys (tile << 31 | depth bits), capacity entries */
  size_t values;          /* uint32 sorted primitive ids, capacity entries */
  size_t ranges;          /* per global tile uint32 [start, end) */
  size_t counters;        /* uint64: [0] instances, [1] overflow flag, [2] hit pairs, [3] range flag */
  size_t gview;           /* backward: per-(view, primitive) gradient records */
  size_t gtable;          /* backward: per-primitive table gradients */
  size_t loss;            /* loss partial sums (float64) */
  size_t disc_coef;       /* per-(view, primitive) 6 float64 coefficients of the ray discriminant */
  int64_t capacity;       /* tile-instance capacity */
  int32_t table_stride;   /* floats per table row */
  int32_t total_tiles;    /* tiles over all views */
  size_t ahat_cache;      /* fwd_cache = 1: float per (instance, tile pixel), else unused */
  size_t ahat_cache_bytes; /* 0 when fwd_cache = 0; cached instances x tile pixels x 4 */
  size_t tile_pairs;      /* per global tile uint32: hit pairs counted by a forward with count_pairs != 0 */
} snp_layout;

/* Size and layout of the workspace for P primitives seen by V cameras with
 * room for `max_instances` (tile, primitive) instances.  The workspace must
 * be 256-byte aligned, at least layout.bytes long, and is reused by every
 * later call of the same step.  Every call that takes a workspace also takes
 * this layout; it is recomputed from the call's arguments and must match
 * (else SNP_ERR_INVALID). */
snp_status snp_workspace_layout(const snp_config* cfg, int64_t P, int32_t V, const snp_camera* cams,
                                int64_t max_instances, snp_layout* out);

/* Per-(primitive, view) preprocessing (Sec. 3.1-3.2 quantities that do not
 * depend on the pixel): near culling, exact screen bounds of the projected
 * ellipsoid, depth key, tile counts, the ray-frame coefficients the
 * rasterizer evaluates per pixel, the per-primitive phase table of the
 * density MLP, and the colour of every (primitive, view).  The culling,
 * bounds and depth are computed in float64 in a fixed operation order. */
snp_status snp_preprocess(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                          void* ws, const snp_layout* layout, hipStream_t stream);

/* Tile binning, the "tiling" stage of the full rendering pipeline the paper
 * times (App. A, Integration Cost: preprocessing, primitive sorting/tiling,
 * integration, alpha blending); it prepares the per-ray set of intersected
 * primitives in depth order that Eq. 4 composites.  Computes the exclusive
 * scan of the tile counts and one (key, value) instance per covered tile, key = (global tile id << 31) | depth bits,
 * value = primitive id; instance count and overflow flag on the device.
 * With bin_order 1 the (view, primitive) pairs are first sorted by depth
 * bits (stably, so equal depths keep primitive order) and the scan and the
 * instances follow that order. */
snp_status snp_bin(const snp_config* cfg, int64_t P, int32_t V, const snp_camera* cams, void* ws,
                   const snp_layout* layout, hipStream_t stream);

/* The "sorting" stage (App. A, Integration Cost): Eq. 4 blends the
 * primitives met by a ray in depth order, so every tile's list is put in
 * ascending depth.  Stable device radix sort of the instances into key order
 * (equal keys in primitive order) and the [start, end) range of every global
 * tile; per tile the values are then the primitive ids in (depth bits, id)
 * order.  With
 * bin_order 1 the instances arrive from snp_bin in depth order, so the tile
 * bits of the key alone are sorted. */
snp_status snp_sort(const snp_config* cfg, int64_t P, int32_t V, const snp_camera* cams, void* ws,
                    const snp_layout* layout, hipStream_t stream);

/* Forward rasterizer (Eq. 3-4, 7-9).  images: sum_v H_v W_v 3 floats;
 * final_T: sum_v H_v W_v floats.  count_pairs != 0 also counts the hit pairs
 * (pixel, primitive with the ray meeting the ellipsoid, pixel not yet
 * terminated) into the workspace counter [2], and per tile into the
 * layout.tile_pairs array (cleared by the same call). */
snp_status snp_render_forward(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                              void* ws, const snp_layout* layout, float* images, float* final_T, int32_t count_pairs,
                              hipStream_t stream);

/* L1 loss: loss_out[0] (device double) = sum |images - targets| / n_norm and
 * dL_dimages = sign(images - targets) / n_norm.  n_norm is the element count
 * the mean is taken over (all views of the step). */
snp_status snp_loss_l1(const snp_config* cfg, int32_t V, const snp_camera* cams, const float* images,
                       const float* targets, double n_norm, void* ws, const snp_layout* layout, double* loss_out,
                       float* dL_dimages, hipStream_t stream);

/* Backward of the differentiable splatting renderer the primitives are
 * trained through (Sec. 3.3, Training: the 3DGS image loss, optimised by
 * gradient descent; Sec. 6: neural primitives in a differentiable
 * splatting-based renderer): the exact adjoint of snp_render_forward,
 * giving the gradients of the loss with respect to every primitive parameter
 * from dL/dimages, the forward's images and the workspace the forward left
 * (its sorted tile lists, records and tables).  The traversal walks each
 * tile's list in forward order and recomputes the transmittance; no per-pixel
 * history is kept.  What it reads per (pixel, instance) pair depends on
 * cfg.fwd_cache: with 1 the forward stored the integral of every pair it
 * evaluated in the workspace (layout.ahat_cache, for the leading
 * fwd_cache_instances instances) and the backward reads it back; with 0, and
 * for batches past the cached instances, it re-evaluates the density
 * integral.  Adds into `grads`. */
snp_status snp_render_backward(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                               void* ws, const snp_layout* layout, const float* images, const float* dL_dimages,
                               const snp_grads* grads, hipStream_t stream);

/* One whole training step: zero `grads`, preprocess, bin, sort, forward,
 * L1 loss against `targets` (mean over n_norm elements), backward. */
snp_status snp_step(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams, void* ws,
                    const snp_layout* layout, float* images, float* final_T, const float* targets, double n_norm,
                    double* loss_out, float* dL_dimages, const snp_grads* grads, hipStream_t stream);

/* snp_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same step with the same arguments, except that the workspace is not the
 * caller's but a static device array of 64 MiB inside the library (each GPU
 * the library runs on holds one until the process ends).  The call allocates
 * nothing.  The instance capacity is the largest whose workspace layout fits
 * in the 64 MiB, including the pair cache when cfg->fwd_cache = 1 (set
 * fwd_cache = 0 for more instances).  Returns SNP_ERR_TOO_LARGE, enqueueing
 * nothing, when even a capacity of one instance does not fit.  Every call on
 * one GPU shares its array: calls that overlap on one GPU (other streams,
 * other threads) race, and the array keeps the last call's contents (the
 * step initialises everything it reads).  counters_out (DEVICE, 8 int64, or
 * NULL) receives the workspace counters at the end of the step, as
 * snp_read_counters lists them: [0] instances, [1] overflow flag (non-zero:
 * the instances exceeded the capacity and the step's results are
 * incomplete), [3] phase-range flag. */
snp_status snp_step_static(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                           float* images, float* final_T, const float* targets, double n_norm, double* loss_out,
                           float* dL_dimages, const snp_grads* grads, int64_t* counters_out, hipStream_t stream);

/* Captures snp_step with these exact arguments into a HIP graph (the
 * pointers must stay valid while the graph lives) and returns an opaque
 * handle.  This call synchronises `stream`.  snp_graph_launch replays it on
 * `stream`; snp_graph_destroy frees it. */
snp_status snp_graph_create(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                            void* ws, const snp_layout* layout, float* images, float* final_T, const float* targets,
                            double n_norm, double* loss_out, float* dL_dimages, const snp_grads* grads,
                            hipStream_t stream, void** graph_out);
snp_status snp_graph_launch(void* graph, hipStream_t stream);
snp_status snp_graph_destroy(void* graph);

/* Captures the forward pipeline alone -- preprocess, bin, sort, forward
 * (snp_preprocess ... snp_render_forward with these arguments, no pair
 * counting) -- into a HIP graph, for callers that only render (both
 * primitive kinds).  The instance count is only known on the device: a
 * replay whose instances exceed the workspace capacity sets the overflow
 * flag that snp_read_status reports.  Synchronises `stream`; replay with
 * snp_graph_launch, free with snp_graph_destroy. */
snp_status snp_graph_create_forward(const snp_config* cfg, const snp_prims* prims, int32_t V,
                                    const snp_camera* cams, void* ws, const snp_layout* layout, float* images,
                                    float* final_T, hipStream_t stream, void** graph_out);

/* Synchronises `stream`, then reads the instance count and the flags.
 * Returns SNP_ERR_CAPACITY if the last binning overflowed and SNP_ERR_RANGE if
 * a density-MLP phase exceeded the supported range. */
snp_status snp_read_status(void* ws, const snp_layout* layout, int64_t* instances_out, int64_t* hit_pairs_out,
                           hipStream_t stream);

/* Synchronises `stream` and copies the 8 device counters of the workspace:
 * [0] instances, [1] overflow flag, [2] hit pairs and [6] pairs with a
 * positive, unclamped integral (both counted by snp_render_forward with
 * count_pairs != 0), [3] phase-range flag, [4], [5] work-queue heads,
 * [7] the number of (view, primitive) pairs the depth sort ordered. */
snp_status snp_read_counters(void* ws, const snp_layout* layout, int64_t* out8, hipStream_t stream);

/* Kernel timing for measurement: while enabled, every eager (not captured)
 * snp_render_forward / snp_render_backward records a HIP event pair on its
 * stream right around its rasterizer kernel; snp_kernel_timing_read waits
 * for the last pairs and returns their durations in milliseconds (-1 if none
 * was recorded).  Enabling clears the recorded pairs. */
snp_status snp_kernel_timing(int32_t enable);
snp_status snp_kernel_timing_read(float* fwd_ms, float* bwd_ms);

/* Tile shapes the rasterizer is built for: writes up to `max` triples
 * (tile_w, tile_h, px_per_lane) and returns how many exist. */
int32_t snp_supported_tiles(int32_t* triples, int32_t max);

const char* snp_status_string(snp_status s);

/* Device self-test of the wave-wide reduction the backward uses: `in` and
 * `out` are device arrays of 64 * waves floats; out[i] = sum of in over the
 * wave of i.  Enqueues on `stream`. */
snp_status snp_selftest_wave_sum(const float* in, float* out, int32_t waves, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Training-step extras after the backward (Sec. 3.3, "Training" and
 * "Population Control"; the appendix on hyperparameters: Adam with learning
 * rates 1.6e-4 for means, 5e-3 scales, 1e-3 quaternions, 2.5e-3 SH, 1e-3
 * MLP; densify / prune thresholds 1e-4 / 2e-6, growing scale 1e-2, pruning
 * scale 0.5).  Device pointers as above; nothing allocates.
 * ------------------------------------------------------------------------- */

/* One parameter tensor of an Adam step. */
typedef struct {
  float *param;       /* n floats, updated in place */
  const float *grad;  /* n floats */
  float *m, *v;       /* first and second moments, n floats each, zero before step 1 */
  int64_t n;
  float lr;
  int32_t log_space;  /* 1: the moments and the update are for log(param)
                         (param > 0), the 3DGS parameterisation of scales; the
                         gradient is taken as d loss / d param */
} snp_adam_group;

#define SNP_MAX_ADAM_GROUPS 32

/* One Adam step (Kingma & Ba) over up to SNP_MAX_ADAM_GROUPS tensors in one
 * launch: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2, theta -= lr
 * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  step >= 1 counts
 * the steps taken including this one.  The betas are float64 (1 - b2 for
 * b2 = 0.999 rounded to float32 would be off by 1.3e-5).  SNP_ERR_INVALID
 * for null pointers of a non-empty group, n < 0, step < 1 or betas outside
 * [0, 1). */
snp_status snp_adam_step(const snp_adam_group* groups, int32_t n_groups, int64_t step, double beta1, double beta2,
                         double eps, hipStream_t stream);

/* Geometry regulariser: loss = weight / P * sum_p std(s_p), the population
 * standard deviation of each primitive's three scale components; adds its
 * gradient into grad_scales (NULL: loss only; 0 where std = 0) and writes
 * the loss (float64, device) to loss_out.  Uses the loss scratch of a
 * workspace (any layout from snp_workspace_layout). */
snp_status snp_scale_regularizer(int64_t P, const float* scales, float weight, float* grad_scales, double* loss_out,
                                 void* ws, const snp_layout* layout, hipStream_t stream);

/* Population-control statistic, once per training step after the backward:
 * grad_acc[p] += ||d loss / d (W1, b1, W2, b2) of p||_2 (from grads w1, b1,
 * w2, b2 with N hidden units) and visible[p] += 1 if p covered a tile of any
 * of the V views in the workspace's last preprocess. */
snp_status snp_densify_accumulate(int64_t P, int32_t N, int32_t V, const snp_grads* grads, void* ws,
                                  const snp_layout* layout, float* grad_acc, float* visible, hipStream_t stream);

typedef struct {
  float densify_threshold; /* statistic above it: clone or split */
  float prune_threshold;   /* visible and statistic below it: prune */
  float grow_scale;        /* max scale <= it: clone, else split */
  float prune_scale;       /* max scale above it: prune */
  float split_shrink;      /* scales of split children: s / split_shrink (1.6 in 3DGS) */
} snp_density_control;

enum { SNP_PRUNE = 0, SNP_KEEP = 1, SNP_CLONE = 2, SNP_SPLIT = 3 };

/* Scratch bytes snp_densify_plan needs for P primitives. */
size_t snp_densify_scratch_bytes(int64_t P);

/* Decides per primitive, with statistic = grad_acc / visible (0 if never
 * visible), in this order: prune if max scale > prune_scale; prune if
 * visible and statistic < prune_threshold; clone (max scale <= grow_scale)
 * or split if statistic > densify_threshold; else keep.  Writes action[P],
 * offsets[P] (first output row of each primitive: primitives stay in index
 * order, a clone's copy follows it, a split primitive is replaced by its two
 * children) and the new primitive count (int64, device) to new_count. */
snp_status snp_densify_plan(int64_t P, const float* scales, const float* grad_acc, const float* visible,
                            const snp_density_control* dc, int32_t* action, uint32_t* offsets, int64_t* new_count,
                            void* scratch, size_t scratch_bytes, hipStream_t stream);

/* One per-primitive array to carry over: src P x width, dst new_count x
 * width (the caller sizes it from snp_densify_plan's count).  kind:
 * SNP_ROWS_PARAM copied to every output row; SNP_ROWS_CENTERS / SCALES the
 * same but split children get x + R(q) diag(s) u_k (u_k = noise[p][k], 3
 * standard normals each) / s / split_shrink; SNP_ROWS_STATE optimizer state,
 * kept on the row that continues the original (a kept primitive, the first
 * row of a clone) and zero on new rows. */
enum { SNP_ROWS_PARAM = 0, SNP_ROWS_STATE = 1, SNP_ROWS_CENTERS = 2, SNP_ROWS_SCALES = 3 };
typedef struct {
  const float *src;
  float *dst;
  int32_t width;
  int32_t kind;
} snp_row_array;

/* Writes every array's new rows (one launch per array).  centers, scales,
 * quats: the primitives' current values (for split children); noise: P x 2 x
 * 3 standard normals (may be NULL if no primitive splits). */
snp_status snp_densify_apply(int64_t P, const int32_t* action, const uint32_t* offsets, const float* centers,
                             const float* scales, const float* quats, const float* noise, float split_shrink,
                             const snp_row_array* arrays, int32_t n_arrays, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SNP_H_ */
