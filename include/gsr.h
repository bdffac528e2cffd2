/*
 * gsr.h -- C ABI of an MI355X (gfx950) differentiable tile-based Gaussian-splatting
 * rasterizer: the step GSFusion's online optimisation runs forward and backward over
 * the Gaussian map at every iteration (Sec. III-B-3 of arXiv 2408.12677).
 *
 * The library renders a set of 3D Gaussians (Eq. 1-2: mean p_g, covariance
 * Sigma = R S S^T R^T, opacity, spherical-harmonic colour) through one or more pinhole
 * cameras: it projects each Gaussian to a 2D splat (Eq. 3-5), sorts the splats by
 * depth inside every screen tile, alpha-blends them front to back (Eq. 11) into
 * colour, depth and alpha images, evaluates the L1 loss of Eq. 12 (plus an optional
 * weighted L1 depth term), and propagates the loss gradient back to every Gaussian
 * parameter in closed form (Sec. III-B-3, the optimisation paragraph).
 *
 * Conventions
 *  - Every buffer pointer handed to the library is DEVICE memory on the context's
 *    GPU unless the comment says "host".  All arrays are float32, C-contiguous.
 *  - Gaussians (structure of arrays, N entries):
 *      means [N,3]      world-space centres
 *      scales [N,3]     per-axis standard deviations (S = diag(scales)), > 0
 *      quats [N,4]      rotation as (w,x,y,z); normalised inside, need not be unit
 *      opacities [N]    activated opacity in [0,1]
 *      sh [N,K,3]       real SH coefficients per colour channel, K=(deg+1)^2, index
 *                       k = l*l+l+m; colour = max(0, 0.5 + sum_k sh_k Y_k(d)) with d the
 *                       unit direction from the camera centre to the mean and Y the
 *                       orthonormal real harmonics with Condon-Shortley phase.
 *  - Cameras (host structs): OpenCV pinhole, world->camera x_c = R x_w + t, pixel
 *    (i,j) is sampled at its integer coordinates; Gaussians with camera depth
 *    <= znear are culled.
 *  - Images: colour [3,H,W] (planar), depth [H,W] (sum of z*alpha*T, background 0),
 *    alpha [H,W] (1 - final transmittance).
 *  - Keys: (global tile id << 32) | bits(float32 depth), sorted ascending and stably;
 *    a global tile id is the view's tile offset plus ty*tiles_x+tx.
 *  - Streams: all device work is enqueued on the context's HIP stream.  Only
 *    gsr_forward (one 16-byte read-back of the pair and visible-record counts),
 *    gsr_seed (an 8-byte read-back of the Gaussian count) and gsr_debug_export
 *    synchronise with the host.  A context is not thread-safe.
 *  - Errors: every call returns a gsr_status; arguments are validated before any
 *    device work; a failing call leaves outputs unspecified but the context usable.
 *    gsr_last_error() gives a message.  NaN/Inf inputs are not rejected unless the
 *    settings ask for the check (GSR_CHECK_FINITE).
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_ABI_VERSION 1
#define GSR_MAX_VIEWS 16

typedef enum {
  GSR_OK = 0,
  GSR_EINVAL = 1,    /* invalid argument (NULL pointer, size out of range, bad enum) */
  GSR_ENOMEM = 2,    /* device allocation failed */
  GSR_EDEVICE = 3,   /* HIP runtime error or no usable device */
  GSR_ECAPACITY = 4, /* a captured graph's key capacity was exceeded; re-create it */
  GSR_EINTERNAL = 5
} gsr_status;

typedef struct gsr_ctx gsr_ctx;     /* per-stream context (owns scratch memory) */
typedef struct gsr_saved gsr_saved; /* forward state needed by the backward pass */
typedef struct gsr_graph gsr_graph; /* a captured forward+loss+backward step */

typedef struct {
  int64_t n;          /* number of Gaussians, >= 0 */
  int32_t sh_degree;  /* 0..3 */
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacities;
  const float* sh;
} gsr_gaussians;

typedef struct {
  int32_t width, height; /* 1..8192 */
  float fx, fy, cx, cy;  /* intrinsics in pixels */
  float R[9];            /* world->camera rotation, row-major (host) */
  float t[3];            /* world->camera translation (host) */
  float znear;           /* > 0 */
} gsr_camera;

/* Rendering rules.  gsr_settings_default() gives tile 16, batch 256, extent 3.33
 * standard deviations (>= sqrt(2 ln 255), so no splat value >= alpha_min is ever
 * outside its tile rectangle), low-pass 0.3 px^2 on the projected covariance,
 * alpha_min 1/255 (strictly smaller values are skipped), alpha_max 0.99 (clamp),
 * T_min 1e-4 (stop after the Gaussian that takes transmittance below it), guard 0.15
 * (only Gaussians inside the view frustum are rendered, Sec. III-B-3: the projected
 * centre must fall inside the image widened by guard x its width/height on each
 * side, and the depth must exceed znear), black background. */
typedef struct {
  int32_t tile;      /* 8, 16 or 32 */
  int32_t batch;     /* Gaussians staged in LDS per round: 128 or 256 */
  float extent_k;
  float lowpass;
  float alpha_min;
  float alpha_max;
  float T_min;
  float guard;       /* >= 0 */
  float bg[3];
  uint32_t flags;    /* GSR_EXACT_TILES | GSR_NORMALIZED_DEPTH | GSR_CHECK_FINITE, or 0 */
  float jclamp;      /* >= 0; > 0: guard-band clamp inside the projection's Jacobian (below) */
} gsr_settings;

/* settings.jclamp: with jclamp > 0 the Jacobian J of the perspective projection (Eq. 5) is
 * evaluated with x/z and y/z clamped to +-jclamp W / (2 fx) and +-jclamp H / (2 fy) (jclamp
 * times the half field of view; 1.3 is the usual choice): a Gaussian far off the optical
 * axis then gets the projected covariance it would have at the limit, instead of one
 * stretched by J's growth with x/z.  The splat centre is not clamped.  The limits are
 * binary32 jclamp ((W / 2) / fx); the clamp decision is taken on tx / tz in binary32 inside
 * the fixed discrete-stage sequence.  0 (default) is Eq. 5 as printed. */

/* settings.flags: tile lists hold, per tile row of a splat's rectangle, only the columns
 * that its ellipse d^T Q d <= extent_k^2 reaches inside the row's pixel band (the rest of
 * the rectangle holds no pixel the splat can reach).  The images, and every pixel's
 * processed contributors, are the same as with the full rectangles; the lists are shorter.
 * gsr_info.num_keys stays the rectangles' pair count (an upper bound); the pairs in use are
 * those inside the tile ranges. */
#define GSR_EXACT_TILES 1u
/* settings.flags: the depth output is D / (1 - T_final), the depth of the surface the
 * pixel sees as an opacity-weighted mean (0 where nothing is hit), instead of the
 * accumulated D = sum z alpha T; the backward takes its gradient through the division. */
#define GSR_NORMALIZED_DEPTH 2u
/* settings.flags: NaN or infinite inputs are not rejected by default (they propagate into the
 * images and gradients).  With this flag every eager forward (gsr_forward, and the forward
 * gsr_graph_create runs to size its buffers; not the captured replays) first reads every
 * Gaussian parameter once on the device and returns GSR_EINVAL, naming the smallest index of
 * a Gaussian with a non-finite value, before any rendering (one more host synchronisation). */
#define GSR_CHECK_FINITE 4u

typedef struct {
  float* color; /* [3,H,W] */
  float* depth; /* [H,W] or NULL */
  float* alpha; /* [H,W] or NULL */
} gsr_view_out;

/* dL/d(outputs) of one view; NULL means zero. */
typedef struct {
  const float* color; /* [3,H,W] */
  const float* depth; /* [H,W] */
  const float* alpha; /* [H,W] */
} gsr_view_grad;

/* L1 targets of one view (Eq. 12 and the depth term). */
typedef struct {
  const float* color; /* [3,H,W] */
  const float* depth; /* [H,W]; pixels with target depth <= 0 are left out of the depth term */
} gsr_target;

/* Output gradients in the parameter layouts; any pointer may be NULL to skip it. */
typedef struct {
  float* means;
  float* scales;
  float* quats;
  float* opacities;
  float* sh;
} gsr_gaussian_grads;

/* Sizes of a forward pass (host values). */
typedef struct {
  int64_t num_keys;      /* M: duplicated (tile, Gaussian) pairs */
  int64_t num_tiles;     /* tiles over all views */
  int64_t num_pixels;    /* pixels over all views */
  int64_t num_records;   /* V*N */
  int32_t views;
  int32_t sort_passes;   /* 8-bit radix passes run */
} gsr_info;

/* Per-kernel device time accumulated by the optional event timer (see
 * gsr_ctx_set_timing); entry i belongs to the kernel gsr_kernel_name(i). */
#define GSR_MAX_KERNELS 32
typedef struct {
  double ms[GSR_MAX_KERNELS];         /* summed launch durations, milliseconds */
  int64_t launches[GSR_MAX_KERNELS];  /* launches timed */
  int32_t count;                      /* kernels in use */
} gsr_timing;

/* Host copies of the intermediate state, for tests.  Each pointer may be NULL;
 * sizes follow gsr_info. */
typedef struct {
  uint64_t* keys;     /* [M] sorted keys */
  uint32_t* values;   /* [M] record index v*N+g of each sorted key */
  uint32_t* ranges;   /* [num_tiles,2] [start,end) per tile, [0,0) when empty */
  float* T_final;     /* [num_pixels] final transmittance, views concatenated */
  uint32_t* n_contrib;/* [num_pixels] one past the list position of the last contributor */
  uint32_t* tiles_touched; /* [V*N] tile-rectangle area, 0 when culled */
  float* mu;          /* [V*N,2] splat centres (binary32, exact op sequence) */
  float* depth;       /* [V*N] camera depth (binary32) */
  float* conic;       /* [V*N,3] inverse projected covariance (A, B, C) */
  float* color;       /* [V*N,3] SH colour */
  int32_t* rect;      /* [V*N,4] tile rectangle (tx0, tx1, ty0, ty1), inclusive */
  uint32_t* n_used;   /* [num_pixels] contributors (list entries that passed the skip rule) */
} gsr_debug;

/* Library version of this header. */
int32_t gsr_abi_version(void);

/* Fill *s with the default rules above.  EINVAL if s is NULL. */
gsr_status gsr_settings_default(gsr_settings* s);

/* A caller's device allocator.  Every device buffer the library allocates for itself
 * (scratch, saved forward state, graph buffers, TSDF maps, seeding counts) is taken from
 * alloc and returned through free:
 *   alloc(user, bytes, hip_stream) returns `bytes` (> 0) of device memory on the context's
 *     device, usable by work enqueued on hip_stream after the call (stream-ordered, like
 *     hipMallocAsync), 256-byte aligned, or NULL when it cannot (the call that needed it
 *     then fails with GSR_ENOMEM and the context stays usable);
 *   free(user, ptr, hip_stream) gives back a block once the work enqueued on hip_stream
 *     before the call is done with it (like hipFreeAsync).
 * Both are called from the thread that calls the library, never from device work. */
typedef struct gsr_alloc {
  void* (*alloc)(void* user, size_t bytes, void* hip_stream);
  void (*free)(void* user, void* ptr, void* hip_stream);
  void* user;
} gsr_alloc;

/* Create a context on HIP device `device` enqueuing on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  alloc (copied; may be NULL): the caller's allocator for the
 * library's device memory; NULL takes it from the device's stream-ordered memory pool.
 * EDEVICE when the device cannot be used; EINVAL for an allocator without both functions. */
gsr_status gsr_ctx_create(int32_t device, void* hip_stream, const gsr_alloc* alloc, gsr_ctx** out);
gsr_status gsr_ctx_destroy(gsr_ctx* ctx);
gsr_status gsr_ctx_set_stream(gsr_ctx* ctx, void* hip_stream);

/* Turn the per-kernel HIP-event timer on or off.  When on, every kernel launch is
 * bracketed by two events on the context's stream (a few microseconds of overhead). */
gsr_status gsr_ctx_set_timing(gsr_ctx* ctx, int32_t enable);

/* Synchronise the stream and report the time accumulated per kernel since the last
 * reset; reset != 0 starts a new accumulation. */
gsr_status gsr_ctx_get_timing(gsr_ctx* ctx, gsr_timing* out, int32_t reset);

/* Name of timer entry `id` ("" when out of range). */
const char* gsr_kernel_name(int32_t id);

/* Forward render (Eq. 2-5 and 11) of V views of one Gaussian map.
 * cams[V] are host structs, outs[V] device images.  With saved != NULL the state
 * the backward needs (splat records, sorted list, tile ranges, final transmittance,
 * contributor counts) is kept in *saved; the caller must then keep g's arrays
 * alive and unchanged until gsr_saved_free.  1 <= V <= GSR_MAX_VIEWS.
 * Synchronises once to read the duplicated-key count back. */
gsr_status gsr_forward(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cams, int32_t V,
                       const gsr_settings* s, const gsr_view_out* outs, gsr_saved** saved);

/* L1 loss (Eq. 12, mean over 3*P colour values) plus depth_weight times the mean
 * absolute depth error over pixels with a valid target depth, summed over views.
 * Reads the rendered images outs[V] and targets[V]; writes dL/dcolour and
 * dL/ddepth into grads_out[V] (device buffers of the image shapes; sign(0) = 0).
 * *loss_dev (device float) receives the loss. */
gsr_status gsr_loss_l1(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_out* outs,
                       const gsr_target* targets, float depth_weight, float* const* grad_color_out,
                       float* const* grad_depth_out, float* loss_dev);

#define GSR_ACCUMULATE 1u /* add into the gradient buffers instead of overwriting */

/* Backward pass (Sec. III-B-3: the closed-form gradients of the blended images of Eq. 11
 * with respect to every Gaussian parameter, taken back through the projection of Eq. 3-5
 * and the SH colour): given dL/d(outputs) per view (grads[V], device images of the view's
 * shape, NULL members = zero), write dL/d(parameters) of the Gaussians saved by
 * gsr_forward, summed over views, into out (parameter layouts; a NULL member skips that
 * group).  flags: GSR_ACCUMULATE adds into out instead of overwriting it.  Transmittance
 * is recovered per pixel from the saved final value and per-tile checkpoints; no
 * per-(pixel, Gaussian) state is stored.  Floating-point atomics make the summation order
 * (not the value) nondeterministic.  EINVAL for NULL saved/grads/out or unknown flags;
 * the saved state stays valid and may be used again. */
gsr_status gsr_backward(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_grad* grads,
                        const gsr_gaussian_grads* out, uint32_t flags);

/* ---- Allocation-free backward ------------------------------------------------------------
 * For callers that cannot allocate device memory while a step runs: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, result and
 * kernels as gsr_backward, but the per-record gradient rows that gsr_backward takes from the
 * stream-ordered pool live in one fixed device array of GSR_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends; the call allocates and frees
 * nothing.  It needs (V*N*12 + N*3)*4 bytes of that array (V views and N Gaussians of the
 * saved forward: 30 MB for one view of 500k Gaussians; one view of at most 1,118,481);
 * a larger saved state gives GSR_EINVAL before any device work.  The array is cleared by a
 * kernel on every call (never by a memset).  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (two streams, two contexts or two threads) race, so the caller
 * serialises them. */
#define GSR_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
gsr_status gsr_backward_noalloc(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_grad* grads,
                                const gsr_gaussian_grads* out, uint32_t flags);

gsr_status gsr_saved_info(const gsr_saved* saved, gsr_info* info);
gsr_status gsr_saved_free(gsr_saved* saved);

/* Copy intermediate state to host memory (synchronises the stream). */
gsr_status gsr_debug_export(gsr_ctx* ctx, const gsr_saved* saved, const gsr_debug* out);

/* ---- Optimiser step (Sec. III-B-3) -----------------------------------------------------
 * The parameters are optimised directly by gradient descent on the loss; the optimiser
 * is Adam (Kingma and Ba, Algorithm 1).  Per element with gradient g at step t:
 *   m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
 *   x <- x - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * The optimised variables are the means, log(scales), the quaternions (unnormalised),
 * logit(opacities) and the SH coefficients; the stored parameters stay activated, so a
 * step maps a scale s to u = log s with gradient s dL/ds, updates u and stores exp(u),
 * and an opacity o to w = log(o/(1-o)) with gradient o(1-o) dL/do, storing
 * 1/(1+exp(-w)) clamped to [2^-24, 1-2^-24].  SH coefficients k = 0 (DC) use lr_sh_dc,
 * the others lr_sh_rest.  Every element is updated at every step (an element without
 * gradient still moves by its momentum).  The moments are caller-owned device arrays in
 * the parameter layouts, and `state` four device words (zero before the first step) in
 * which the library keeps the step count and the step's bias corrections; the count
 * advances on the device, so a captured graph steps correctly on every replay. */
typedef struct gsr_adam {
  float lr_means;     /* 1.6e-4 */
  float lr_scales;    /* 5e-3 (on log scale) */
  float lr_quats;     /* 1e-3 */
  float lr_opacities; /* 0.05 (on the logit) */
  float lr_sh_dc;     /* 2.5e-3 */
  float lr_sh_rest;   /* 1.25e-4 */
  float beta1;        /* 0.9 */
  float beta2;        /* 0.999 */
  float eps;          /* 1e-15 */
  gsr_gaussian_grads m;  /* first moments (all five arrays required) */
  gsr_gaussian_grads v;  /* second moments */
  uint32_t* state;       /* [4] device: steps taken, then binary32 bias corrections */
} gsr_adam;

/* Default rates and betas (the 3D Gaussian splatting values above); pointers NULL. */
gsr_status gsr_adam_default(gsr_adam* a);
/* One Adam step of n Gaussians (SH degree 0..3): params are updated in place from grads
 * (both in the parameter layouts; gsr_gaussian_grads here simply names five device arrays). */
gsr_status gsr_adam_step(gsr_ctx* ctx, int64_t n, int32_t sh_degree, const gsr_gaussian_grads* params,
                         const gsr_gaussian_grads* grads, const gsr_adam* opt);
/* gsr_backward fused with one Adam step: each Gaussian's parameter gradient is formed as
 * in gsr_backward and applied at once to the Gaussian arrays given to gsr_forward (which
 * must be writable) instead of being written out. */
gsr_status gsr_backward_adam(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_grad* grads,
                             const gsr_adam* opt);

/* ---- Batched keyframes: one captured step -------------------------------------------
 * Capture forward + L1 loss + backward of V views (uneven resolutions allowed) into a
 * hipGraph: one concatenated tile space, one sort, persistent compositing kernels that
 * take tiles longest-list-first from a device work queue, all counts kept on the device
 * (keyframe replay and global optimisation, Sec. III-B-3).  Every pointer argument is
 * bound at capture: a launch re-runs the step on the current contents of the same
 * buffers (parameters, targets, images, gradients).  Buffers are sized from one eager
 * forward of the given inputs times (1 + headroom).  A launch whose key or visible-record
 * count exceeds those capacities sets a device flag that stays set for the graph's
 * lifetime; it is read back asynchronously and reported as GSR_ECAPACITY by the next
 * gsr_graph_launch that finds an earlier step complete, and by gsr_graph_sync (the graph
 * must then be re-created).  Gradients are overwritten on every launch.  With opt (may be
 * NULL) the step ends with one Adam step fused into the backward, as in
 * gsr_backward_adam: every launch is then one complete optimisation iteration that updates
 * the Gaussian arrays of g in place, and grads may be NULL; a launch that overflowed, and
 * every launch after it, leaves the parameters, the moments and the step count unchanged. */
gsr_status gsr_graph_create(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cams, int32_t V,
                            const gsr_settings* s, const gsr_view_out* outs, const gsr_target* targets,
                            float depth_weight, float* const* grad_color, float* const* grad_depth,
                            const gsr_gaussian_grads* grads, float* loss_dev, float headroom,
                            const gsr_adam* opt, gsr_graph** out);
/* Enqueue one step on the context's stream (asynchronous). */
gsr_status gsr_graph_launch(gsr_graph* gr);
/* Wait for the last launch; GSR_ECAPACITY if any launch overflowed. */
gsr_status gsr_graph_sync(gsr_graph* gr);
/* Sizes measured at creation, and the key / visible-record capacities. */
gsr_status gsr_graph_info(const gsr_graph* gr, gsr_info* info, int64_t* cap_keys, int64_t* cap_visible);
gsr_status gsr_graph_free(gsr_graph* gr);

/* ---- Launch-shape autotuner -----------------------------------------------------------
 * Time forward + backward at every (tile, batch, list kind) in {8,16,32} x {128,256} x
 * {rectangles, GSR_EXACT_TILES} and write the fastest into s->tile / s->batch and the
 * GSR_EXACT_TILES bit of s->flags (other fields and bits are kept).  Results are cached in the
 * text file named by $GSR_AUTOTUNE_CACHE (default ~/.cache/gsr_autotune.txt), keyed by
 * architecture, CU count, log2 of the total pixel count and of N, SH degree and V; a
 * cached entry is used without timing unless GSR_AUTOTUNE_NO_CACHE is set.  The forward
 * images do not depend on the choice (the extent keeps every splat value >= alpha_min
 * inside its tile rectangle).  After two warm-up steps each, the candidates take turns, one
 * eager step per turn, nine turns; each is scored by the median of its nine steps, a step's
 * time being the sum of its kernels' durations.  best_ms (may be NULL) receives that median
 * for the chosen shape. */
#define GSR_AUTOTUNE_NO_CACHE 1u
gsr_status gsr_autotune(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cams, int32_t V,
                        gsr_settings* s, uint32_t flags, float* best_ms);

/* ---- Quadtree seeding and Gaussian initialisation (Sec. III-B-2, Eq. 10) --------------
 * One RGB-D frame is cut into a quadtree: root cells of 64x64 pixels aligned at (0,0)
 * and clipped at the border split into their four quadrants while the cell's measure
 * passes `threshold` and its side exceeds `min_side`.  Measures:
 *   GSR_SEED_CONTRAST        range (max - min) of the mean of the three colour channels;
 *                            a cell splits when it is >= threshold (the paper's rule:
 *                            every leaf has contrast below the threshold, 0.1 in Sec. IV)
 *   GSR_SEED_DEPTH_VARIANCE  population variance (m^2) of the valid depths (> 0); a cell
 *                            splits when it is > threshold; cells without a valid depth
 *                            are dropped
 * Every leaf (x0, y0, w, h) whose centre pixel (x0 + w/2, y0 + h/2) has a valid depth d
 * gives one Gaussian (the paragraph after Eq. 10): mean = T_WC pi^-1(centre, d) with the
 * camera's world->camera (R, t); scales = (s, s, s) with s the distance from the
 * back-projected centre to the back-projected top-left pixel (x0, y0) at depth d;
 * rotation (1, 0, 0, 0); opacity `opacity`; SH DC coefficients (c - 0.5) / Y_00 from the
 * centre pixel's colour c (Y_00 = 1/(2 sqrt(pi))), all other coefficients 0.  Gaussians
 * are written root by root in raster order and depth-first (top-left, top-right,
 * bottom-left, bottom-right) inside a root.  The voxel-weight neighbourhood check of the
 * paper needs the TSDF map and is left to the caller.  Statistics are binary64; the
 * threshold is the binary32 value given. */
#define GSR_SEED_CONTRAST 0
#define GSR_SEED_DEPTH_VARIANCE 1
typedef struct gsr_seed_settings {
  int32_t measure;    /* GSR_SEED_CONTRAST (default) or GSR_SEED_DEPTH_VARIANCE */
  float threshold;    /* 0.1 */
  int32_t min_side;   /* smallest cell side: 1, 2, 4 (default), 8, 16, 32 or 64 */
  float opacity;      /* 0.5 */
  int32_t sh_degree;  /* 0..3: coefficients written per Gaussian (K = (deg+1)^2) */
} gsr_seed_settings;

typedef struct gsr_seed_out {  /* device buffers of `capacity` Gaussians */
  float* means;      /* [capacity,3] */
  float* scales;     /* [capacity,3] */
  float* quats;      /* [capacity,4] */
  float* opacities;  /* [capacity] */
  float* sh;         /* [capacity,K,3] */
  int32_t* leaves;   /* [capacity,4] (x0, y0, w, h) of each Gaussian's cell, or NULL */
} gsr_seed_out;

typedef struct gsr_tsdf gsr_tsdf; /* a TSDF voxel-block map (below) */

gsr_status gsr_seed_settings_default(gsr_seed_settings* s);
/* rgb [3,H,W] in [0,1] and depth [H,W] in metres (<= 0: no depth) are device images of
 * cam's size.  With map != NULL (the frame fused into it first, gsr_tsdf_integrate) a
 * leaf also needs the voxel that holds its mean to have weight exactly 1, i.e. to be seen
 * for the first time by that frame (the paper's check against duplicating primitives);
 * map == NULL skips the check.  Writes the Gaussians into `out` and their number into
 * *count (host).  When more than `capacity` would be written, writes nothing, sets
 * *count to the number needed and returns GSR_ECAPACITY.  capacity
 * ceil(W/min_side)*ceil(H/min_side) always suffices.  Synchronises once to read the count. */
gsr_status gsr_seed(gsr_ctx* ctx, const gsr_camera* cam, const float* rgb, const float* depth,
                    const gsr_seed_settings* s, const gsr_tsdf* map, const gsr_seed_out* out, int64_t capacity,
                    int64_t* count);

/* ---- TSDF fusion (Sec. III-B-1, Eq. 6-9) -----------------------------------------------
 * A map of voxel blocks (8x8x8 voxels of side `voxel`) found through a device hash table
 * of block coordinates.  Fusing a depth frame: every pixel with depth d > 0 marches its
 * viewing ray through the band [d - trunc, d + trunc] at camera depths
 * (d - trunc) + i * step, i = 0 .. floor(2 trunc / step), and allocates the blocks its
 * samples fall in; then every voxel of those blocks is projected (nearest pixel,
 * floor(u + 0.5)) and, where that pixel has depth D > 0,
 *   sdf = D - z_v (Eq. 6),  tsdf = clamp(sdf / trunc, -1, 1) (Eq. 7),
 *   w_k = min(w_max, w_(k-1) + 1) (Eq. 8),
 *   tsdf_k = (tsdf_(k-1) w_(k-1) + tsdf w_k) / (w_(k-1) + w_k)   (GSR_TSDF_EQ9, as printed)
 *         or (tsdf_(k-1) w_(k-1) + tsdf) / (w_(k-1) + 1)          (GSR_TSDF_UNIT_WEIGHT, the
 *            running average the text describes).
 * Voxels start at tsdf 0, weight 0.  Block selection and voxel projection are fixed
 * sequences of correctly rounded binary32 operations (so they are reproducible bit for
 * bit); the values are binary32.  Defaults: voxel 0.01 m (Sec. IV-A), trunc 0.08 m,
 * w_max 100, step 0.01 m, GSR_TSDF_EQ9. */
#define GSR_TSDF_EQ9 0
#define GSR_TSDF_UNIT_WEIGHT 1
typedef struct gsr_tsdf_settings {
  float voxel;        /* voxel side, metres */
  float trunc;        /* truncation band eps, metres */
  float w_max;        /* weight cap, >= 1 */
  float step;         /* ray-march step in camera depth, metres */
  int32_t weighting;  /* GSR_TSDF_EQ9 or GSR_TSDF_UNIT_WEIGHT */
} gsr_tsdf_settings;

gsr_status gsr_tsdf_settings_default(gsr_tsdf_settings* s);
/* A map with room for max_blocks blocks (1 .. 2^28; 4 KiB of device memory per block plus
 * a hash table of at least twice as many 16-byte slots), all voxels at zero. */
gsr_status gsr_tsdf_create(gsr_ctx* ctx, const gsr_tsdf_settings* s, int64_t max_blocks, gsr_tsdf** out);
gsr_status gsr_tsdf_free(gsr_tsdf* map);
/* Fuse the depth image [H,W] (device, cam's size) seen from cam.  Asynchronous.  Blocks
 * beyond the map's capacity (or a full table) are not allocated and set a flag bit that
 * gsr_tsdf_info reports (1 table full, 2 pool full, 4 coordinates out of range). */
gsr_status gsr_tsdf_integrate(gsr_ctx* ctx, gsr_tsdf* map, const gsr_camera* cam, const float* depth);
/* Allocated blocks, blocks met by the last fused frame and the flag bits (synchronises). */
gsr_status gsr_tsdf_info(gsr_ctx* ctx, const gsr_tsdf* map, int64_t* blocks, int64_t* met_last, uint32_t* flags);
/* Host copies of the allocated blocks (synchronises): coords [n,3] block coordinates
 * (a block holds voxels 8*coords + (0..7)), tsdf and weight [n,512] with x fastest, then
 * y, then z.  *count = n always; GSR_ECAPACITY when capacity < n (nothing copied); NULL
 * arrays are skipped. */
gsr_status gsr_tsdf_export(gsr_ctx* ctx, const gsr_tsdf* map, int32_t* coords, float* tsdf, float* weight,
                           int64_t capacity, int64_t* count);
/* out[i] (device) = weight of the voxel that holds points[i] (device [n,3]; the voxel index
 * is floor(p / voxel) in binary32); 0 where no block is allocated. */
gsr_status gsr_tsdf_weights(gsr_ctx* ctx, const gsr_tsdf* map, const float* points, int64_t n, float* out);

/* ---- Keyframe-list optimisation schedule (Sec. III-B-3; settings of Sec. IV-A) --------
 * Host-only bookkeeping of which view each optimisation iteration of a time step renders.
 * The number of Gaussians the seeding of a frame added measures its information gain:
 *   - count > threshold: the frame is a keyframe, joins the keyframe list and gets m
 *     iterations;
 *   - otherwise it gets n iterations, followed by one iteration on each of the first
 *     min(m - n, list length) keyframes of the list after a shuffle.
 * With store_all every frame joins the list (after its own draw) while m or n still
 * follows the threshold (the paper's ScanNet++ setting: m 10, n 1, every frame kept; its
 * Replica setting: m 5, n 3, threshold 50).  A negative threshold makes every frame a
 * keyframe.  The shuffle gives list entry i (0-based, insertion order) the key
 * h(h(seed, frame + 1), i + 1), h(s, k) being the k-th output of SplitMix64 seeded with s
 * (s + k * 0x9E3779B97F4A7C15 through its 64-bit mixing function), and orders the list
 * by (key, i).  Offline optimisation after scanning iterates over gsr_schedule_keyframes. */
typedef struct gsr_schedule gsr_schedule;
typedef struct gsr_schedule_settings {
  int32_t m;          /* iterations of a keyframe, >= n */
  int32_t n;          /* iterations of another frame, >= 0 */
  int64_t threshold;  /* keyframe when the frame's new Gaussians exceed it (50) */
  int32_t store_all;  /* nonzero: every frame joins the keyframe list */
  uint64_t seed;      /* seed of the keyframe draw */
} gsr_schedule_settings;

/* EINVAL unless 0 <= n <= m <= 10^6. */
gsr_status gsr_schedule_create(const gsr_schedule_settings* s, gsr_schedule** out);
gsr_status gsr_schedule_free(gsr_schedule* sch);
/* The iterations of time step `frame` (>= 0) whose seeding added new_gaussians (>= 0):
 * writes the frame rendered by each iteration, in order, into iters[0, *count) (host,
 * cap >= m) and whether the frame is a keyframe into *is_keyframe (may be NULL). */
gsr_status gsr_schedule_step(gsr_schedule* sch, int64_t frame, int64_t new_gaussians, int64_t* iters, int32_t cap,
                             int32_t* count, int32_t* is_keyframe);
/* The keyframe list in insertion order: *count always, out[0, count) when out != NULL
 * (EINVAL when cap is smaller). */
gsr_status gsr_schedule_keyframes(const gsr_schedule* sch, int64_t* out, int64_t cap, int64_t* count);

/* Message of the last failing call on ctx ("" if none); ctx may be NULL for
 * failures that had no context. */
const char* gsr_last_error(const gsr_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */
