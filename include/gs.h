/*
 * gs.h - C ABI of libgsmi, an MI355X (gfx950) differentiable tile-based
 * 3D Gaussian rasterizer.
 *
 * The library implements the rendering function R(M, T) that GEVO evaluates
 * to re-render past keyframes from the Gaussian map instead of storing them
 * (Sec. I; Sec. III-B2, the photometric-consistency loss E_pc over rendered
 * past views), and the gradients of a photometric loss with respect to the
 * map and the camera pose that the local and global mapping objectives
 * minimise over (Eq. 2 and Eq. 3).  The renderer itself is the Gaussian
 * splatting rasterizer the paper builds on (Sec. I, Sec. IV-C); the exact
 * definition implemented here is:
 *
 *   activations   s = exp(log_scale), q / |q|, o = sigmoid(opacity_logit)
 *   covariance    Sigma = (R(q) diag(s)) (R(q) diag(s))^T
 *   view          p = R_cw mu + t_cw; culled if p_z <= 0.2
 *   projection    u = fx p_x / p_z + cx, v = fy p_y / p_z + cy;
 *                 pixel (i, j) is sampled at its centre (i + 1/2, j + 1/2)
 *   EWA           Sigma' = J R_cw Sigma R_cw^T J^T + 0.3 I, with p_x/p_z and
 *                 p_y/p_z clamped to +-1.3 W/(2 fx), +-1.3 H/(2 fy) inside J;
 *                 conic Q = Sigma'^-1
 *   extent        r = ceil(3 sqrt(lambda_max(Sigma'))) pixels
 *   tiles         every tile holding a pixel centre in [u-r, u+r] x [v-r, v+r]
 *   colour        real spherical harmonics (degree 0..3, Condon-Shortley
 *                 phase, ordered l, m = -l..l) of the unit direction from the
 *                 camera centre to mu, plus 1/2, clamped below at 0
 *   order         per tile ascending (camera-frame depth, Gaussian index)
 *   blending      front to back: power = -1/2 d^T Q d (skip if > 0),
 *                 alpha = min(0.99, o e^power) (skip if < 1/255), stop before
 *                 the transmittance would fall below 1e-4;
 *                 C = sum_i alpha_i T_i c_i + T_final bg.
 *                 alpha_i T_i is the blending weight w(g, u) of Sec. III-B2.
 *
 * Conventions
 *   - Every entry point returns a gs_status; no exception crosses the ABI.
 *     On GS_ERR_HIP the HIP error text is available from gs_last_error()
 *     (thread-local).
 *   - The caller owns all memory.  The library allocates no device memory:
 *     scratch comes from *_workspace_size() followed by a caller pointer
 *     (device memory, 256-byte aligned).
 *   - Pointers named *_dev and every array inside the structs below are
 *     device pointers unless stated otherwise.
 *   - Work is enqueued asynchronously on the caller's stream.  The only call
 *     that synchronises is gs_bin_sort with a non-NULL n_keys_host.
 *   - Arguments are validated before anything is enqueued; a failed call
 *     enqueues nothing.
 *   - Gradient outputs are accumulated (+=) so that several calls (views)
 *     sum; the caller zeroes them.
 *   - Calls are reentrant; calls that share output or workspace buffers on
 *     different streams race.
 *   - Floating-point work is IEEE float32 (pose gradients are reduced in
 *     float64).
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t; NULL selects the null stream. */
typedef struct ihipStream_t* gs_stream_t;

typedef enum gs_status {
  GS_OK = 0,
  GS_ERR_INVALID_ARGUMENT = 1, /* null pointer, bad size, bad enum            */
  GS_ERR_CAPACITY = 2,         /* caller buffer too small; size reported      */
  GS_ERR_HIP = 3,              /* HIP runtime error; see gs_last_error()      */
  GS_ERR_UNSUPPORTED = 4       /* valid but unsupported configuration         */
} gs_status;

#define GS_MAX_VIEWS 64
#define GS_MAX_SH_DEGREE 3

/* Pinhole camera (80 bytes).  R is world->camera, row-major; (R, t) maps a
 * world point mu to p = R mu + t with x right, y down, z forward. */
typedef struct gs_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  int32_t pad[2];
} gs_camera;

/* Gaussian map, structure of arrays, component-major float32 (device):
 *   means [3][n], log_scales [3][n], quats [4][n] in (w, x, y, z) order (not
 *   necessarily normalised), opacity_logits [n], sh [3][K][n] with
 *   K = (sh_degree + 1)^2.  Non-finite parameters or a zero quaternion cull
 *   the Gaussian. */
typedef struct gs_gaussians {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* sh;
  int64_t n;
  int32_t sh_degree;
} gs_gaussians;

/* A batch of views.  cams_host (host memory) supplies image sizes, which fix
 * the tile layout; cams_dev (device memory, same contents) supplies poses and
 * intrinsics to the kernels, so a caller may update poses on the device
 * between launches as long as sizes do not change.  Views are packed in
 * order: global tile ids start at sum of previous views' tile counts, pixel
 * buffers at sum of previous views' W*H.  tile_size must be 16. */
typedef struct gs_views {
  const gs_camera* cams_host;
  const gs_camera* cams_dev;
  int32_t n_views;   /* 1 .. GS_MAX_VIEWS */
  int32_t tile_size; /* 16 */
} gs_views;

/* Per-(view, Gaussian) screen-space splats, [V][n] each (device):
 *   xy            float2: u, v
 *   conic_opacity float4: Q00, Q01, Q11, o
 *   rgb_depth     float4: r, g, b, camera-frame z
 *   radius        int32:  r in pixels, 0 = culled
 *   tiles         uint32: number of tiles the splat's rectangle covers, 0 if
 *                 it covers none (optional: NULL = not stored; gs_preprocess
 *                 writes it when non-NULL, gs_bin_sort reads it when non-NULL
 *                 and otherwise computes it from xy and radius) */
typedef struct gs_projected {
  float* xy;
  float* conic_opacity;
  float* rgb_depth;
  int32_t* radius;
  uint32_t* tiles;
} gs_projected;

/* Tile binning result (device):
 *   keys   [capacity] uint64 (global tile << 32) | float32 bits of depth,
 *          ascending; ties ordered by value.  Optional for gs_bin_sort
 *          (NULL = not written; values, ranges and order are the same, and
 *          the sort then carries 32-bit tile ids in the workspace, which
 *          moves a third less data); the compositing calls never read it.
 *   values [capacity] uint32 view * n + Gaussian index
 *   ranges [n_tiles][2] uint32 [start, end) into keys/values per global tile
 *   n_keys [1] uint32 number of keys emitted (may exceed capacity, in which
 *          case the call reported or flagged overflow and keys are partial)
 *   order  [n_tiles] uint32 (optional, NULL = not computed): every global
 *          tile id once, longest lists first: tiles are grouped by list
 *          length (0, then half-octave steps), groups in descending length,
 *          ascending tile id within a group.  gs_bin_sort writes it when
 *          non-NULL (the identity when it returns before the ranges exist);
 *          the compositing calls then start the most expensive tiles first,
 *          which shortens the tail of the launch, and their results do not
 *          depend on it.
 *   queue  [GS_QUEUE_WORDS] uint32 (optional, NULL = none): tile counters of
 *          the persistent schedule (GS_SCHEDULE_PERSISTENT).  Each
 *          compositing call owns GS_QUEUE_COUNTERS counters, GS_QUEUE_STRIDE
 *          words apart, from word GS_QUEUE_STRIDE * GS_QUEUE_COUNTERS * call
 *          (call = GS_QUEUE_FWD, GS_QUEUE_BWD or GS_QUEUE_ERROR).  Must be
 *          zero before first use: gs_bin_sort zeroes it, and every call that
 *          uses its counters leaves them zero again.  Calls of the same kind
 *          that share a queue must not overlap in time.  Without a queue the
 *          persistent schedule launches one workgroup per tile. */
enum {
  GS_QUEUE_FWD = 0,
  GS_QUEUE_BWD = 1,
  GS_QUEUE_ERROR = 2,
  GS_QUEUE_COUNTERS = 8, /* counters per call                   */
  GS_QUEUE_STRIDE = 32,  /* words between counters (128 bytes)  */
  GS_QUEUE_WORDS = 1024  /* 4 calls' worth; the fourth is spare  */
};
typedef struct gs_bins {
  uint64_t* keys;
  uint32_t* values;
  uint32_t* ranges;
  uint32_t* n_keys;
  int64_t capacity;
  uint32_t* order;
  uint32_t* queue;
} gs_bins;

/* Gradients, same layouts as gs_gaussians, accumulated (+=).  xi [V][6]
 * float32 is dL/dxi for a left perturbation T_cw <- Exp(xi) T_cw at xi = 0,
 * xi = (rho, phi), translation first.  Any pointer may be NULL only when the
 * corresponding flag excludes it (see gs_render_bwd). */
typedef struct gs_grads {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
  float* xi;
} gs_grads;

enum {
  GS_BWD_NO_POSE = 1u,   /* skip the pose gradient (xi may be NULL)            */
  GS_BWD_POSE_ONLY = 2u, /* only the pose gradient (map grads may be NULL)      */
  GS_BWD_OVERWRITE = 4u, /* store gradients instead of accumulating (+=) them   */
  GS_BWD_KEEP_CLEAR = 8u /* workspace handed over clear, returned clear (below)  */
};

/* Kernels that gs_set_kernel_events() can bracket. */
enum {
  GS_KERNEL_PREPROCESS = 0,   /* gs_preprocess's projection kernel                  */
  GS_KERNEL_BIN_SORT = 1,     /* gs_bin_sort from key emission to tile ranges       */
  GS_KERNEL_RENDER_FWD = 2,   /* gs_render_fwd's compositing kernel                 */
  GS_KERNEL_RENDER_BWD = 3,   /* gs_render_bwd's reverse tile walk                  */
  GS_KERNEL_PROJECT_BWD = 4,  /* gs_render_bwd's per-Gaussian projection backward   */
  GS_KERNEL_COUNT = 5
};

/* Short name of a status code (static string). */
const char* gs_status_string(int status);
/* Text of the last GS_ERR_* raised on this thread (static per-thread buffer). */
const char* gs_last_error(void);
/* Library version string, ending in a hash of the sources it was built from
 * (static string). */
const char* gs_version(void);

/* Kernel configuration keys for gs_set_tuning(). */
enum {
  GS_TUNE_FWD_PIXELS_PER_LANE = 0, /* gs_render_fwd: pixels per lane, 1 | 2 | 4 (default 1) */
  GS_TUNE_BWD_PIXELS_PER_LANE = 1, /* gs_render_bwd: pixels per lane, 1 | 2 | 4 (default 1) */
  GS_TUNE_FWD_SCHEDULE = 2,        /* gs_render_fwd(_l1): a GS_SCHEDULE_* value            */
  GS_TUNE_BWD_SCHEDULE = 3,        /* gs_render_bwd and gs_render_error: GS_SCHEDULE_*     */
  GS_TUNE_FWD_STAGE = 4,           /* gs_render_fwd(_l1): splats each thread stages in LDS
                                      per batch, 1 | 2 (default 0: 1, or 2 at 2 pixels per
                                      lane)                                                */
  GS_TUNE_BWD_STAGE = 5,           /* gs_render_bwd: likewise, 1 | 2 (default 0: 2, or 1 at
                                      1 pixel per lane)                                    */
  GS_TUNE_COUNT = 6
};

/* Tile schedules of the compositing kernels (GS_TUNE_*_SCHEDULE). */
enum {
  GS_SCHEDULE_HEAVIEST_FIRST = 1, /* one workgroup per tile, launched in bins->order (default;
                                     tile id order when bins->order is NULL)                  */
  GS_SCHEDULE_TILE_ID = 2,        /* one workgroup per tile, launched in tile id order        */
  GS_SCHEDULE_PERSISTENT = 3,     /* as many workgroups as the GPU holds at once, each taking
                                     tiles in bins->order from a counter in bins->queue until
                                     none is left                                              */
  GS_SCHEDULE_PERSISTENT_HALF = 4 /* the same with half as many workgroups                    */
};

/* Process-wide kernel configuration, set by an autotuner.  Pixels per lane:
 * a 16x16 tile is covered by 256 / value threads; a staging batch holds
 * (splats per thread) x 256 / (pixels per lane) splats.  value 0 restores
 * the default.  Applies to launches enqueued after the call; a captured graph
 * keeps the configuration it was captured with.  Results are identical for
 * every setting up to float32 summation order of the gradient atomics. */
int gs_set_tuning(int key, int value);
/* Current value of a tuning key (< 0 for an unknown key). */
int gs_get_tuning(int key);

/* Timing hook (thread-local): while set, every launch of `kernel` on this
 * thread is bracketed by hipEventRecord(start, stream) and
 * hipEventRecord(stop, stream) on the launch stream.  start/stop are
 * hipEvent_t handles owned by the caller; NULL clears the hook.  Meant for
 * measuring one kernel's duration in place; adds two event records per
 * launch while set. */
int gs_set_kernel_events(int kernel, void* start_event, void* stop_event);

/* Total tiles and pixels of a view batch (host-only, validates views; < 0 on
 * invalid input). */
int64_t gs_num_tiles(const gs_views* views);
int64_t gs_num_pixels(const gs_views* views);

/* Projection of every Gaussian into every view (the activations, covariance,
 * view transform, projection, EWA, extent and colour steps above).
 * out arrays hold [n_views][n] entries.  Culled entries get radius 0; their
 * other fields are left as they were (no consumer reads them). */
int gs_preprocess(const gs_gaussians* g, const gs_views* views, gs_projected* out,
                  gs_stream_t stream);

/* Scratch for gs_bin_sort (bytes). */
size_t gs_bin_sort_workspace_size(int64_t n, const gs_views* views, int64_t capacity);

/* Tile binning and sorting of the splats in p ([n_views][n]): counts the
 * tiles of each splat's rectangle, scans, emits one key per (splat, tile)
 * in splat-major, row-major order, radix-sorts keys ascending (stable, so
 * equal keys keep ascending value order) and writes per-tile ranges.
 * n_keys_host != NULL: synchronises once to read the key count; if it
 * exceeds bins->capacity, *n_keys_host holds the required capacity, nothing
 * further is enqueued and GS_ERR_CAPACITY is returned.
 * n_keys_host == NULL: no synchronisation (capture-safe); keys beyond the
 * capacity are dropped and bins->n_keys reports the full count, which the
 * caller must check against the capacity after the stream completes. */
int gs_bin_sort(const gs_projected* p, int64_t n, const gs_views* views, gs_bins* bins,
                uint32_t* n_keys_host, void* workspace, size_t workspace_bytes,
                gs_stream_t stream);

/* Forward compositing of every tile of every view.
 * image [3][H][W] per view (planar, views packed), final_T [H][W] and
 * n_contrib [H][W] (1 + list position of the last blended splat, 0 if none)
 * per view; depth (optional, may be NULL) = sum_i w_i z_i per pixel.
 * bg: host pointer to 3 floats, or NULL for black. */
int gs_render_fwd(const gs_projected* p, int64_t n, const gs_bins* bins, const gs_views* views,
                  const float* bg, float* image, float* final_T, uint32_t* n_contrib,
                  float* depth, gs_stream_t stream);

/* Scratch for gs_render_bwd (bytes). */
size_t gs_render_bwd_workspace_size(int64_t n, const gs_views* views);

/* Backward of gs_render_fwd and gs_preprocess: given dL/dimage (layout of
 * image) and the forward's final_T and n_contrib, walks each tile's list in
 * reverse recovering the transmittance, reduces per-splat gradients over each
 * wavefront and accumulates them with atomics, then chains them per Gaussian
 * to the map parameters (summed over views) and to each view's pose tangent.
 * flags: 0, GS_BWD_NO_POSE or GS_BWD_POSE_ONLY, optionally or-ed with
 * GS_BWD_OVERWRITE (gradients of culled Gaussians are then written as 0) and
 * GS_BWD_KEEP_CLEAR.  Without GS_BWD_KEEP_CLEAR the call first clears the
 * per-splat partials it accumulates into (one pass over the [V][n] entries).
 * With it the caller guarantees that the workspace is clear on entry: all
 * zero bytes (e.g. a fresh workspace the caller zeroed), or last used by a
 * completed call with this flag for the same n and views and not modified
 * since; the call then skips that pass and leaves the workspace clear again
 * (the projection backward zeroes each partial after reading it). */
int gs_render_bwd(const gs_gaussians* g, const gs_projected* p, const gs_bins* bins,
                  const gs_views* views, const float* bg, const float* dL_dimage,
                  const float* final_T, const uint32_t* n_contrib, gs_grads* grads,
                  uint32_t flags, void* workspace, size_t workspace_bytes, gs_stream_t stream);

/* One bias-corrected Adam step over n float32 parameters, in place:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * mask (optional, uint8 [n]): entries with mask 0 are left untouched (the
 * hook for optimising only an active subset of Gaussians, Sec. III-B2). */
int gs_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                 float beta1, float beta2, float eps, int32_t step, const uint8_t* mask,
                 gs_stream_t stream);

/* Capture-safe Adam step (same update as gs_adam_step) whose step number
 * lives in device memory, for use inside a captured HIP graph:
 *   t = *step_dev + 1 sets the bias correction; if commit != 0 the call then
 *   stores t into *step_dev (the last parameter group of an optimisation step
 *   commits, so all groups of one step share t).
 * guard_n_keys (optional, device): when *guard_n_keys > guard_capacity (the
 * step's tile binning overflowed and its gradients are incomplete) the call
 * leaves p, m, v and *step_dev untouched. */
int gs_adam_step_dev(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                     float beta1, float beta2, float eps, int32_t* step_dev, int32_t commit,
                     const uint8_t* mask, const uint32_t* guard_n_keys, int64_t guard_capacity,
                     gs_stream_t stream);

/* One parameter group of gs_adam_step_groups_dev (device pointers). */
typedef struct gs_adam_group {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  float lr;
} gs_adam_group;

#define GS_ADAM_MAX_GROUPS 8

/* gs_adam_step_dev over up to GS_ADAM_MAX_GROUPS parameter groups (each with
 * its own learning rate and n >= 0, no mask) in a single launch, followed by
 * the commit of *step_dev.  groups is a host array read during the call.
 * Results are identical to one gs_adam_step_dev call per group with the
 * last one committing. */
int gs_adam_step_groups_dev(const gs_adam_group* groups, int32_t n_groups, float beta1,
                            float beta2, float eps, int32_t* step_dev,
                            const uint32_t* guard_n_keys, int64_t guard_capacity,
                            gs_stream_t stream);

/* gs_render_fwd fused with gs_l1_loss_grad: composites exactly as
 * gs_render_fwd (same image, final_T, n_contrib; no depth) and, from the
 * image values it writes, dL/dC = sign(C - C*) / (3 H W) into dL_dimage
 * (identical to gs_l1_loss_grad's) and, if loss != NULL, the loss (the
 * same sum, added in a fixed order: equal up to float rounding).
 * target: [3][H][W] per view like image.  ws: gs_render_fwd_l1_workspace_size
 * bytes (one float per tile). */
size_t gs_render_fwd_l1_workspace_size(const gs_views* views);
int gs_render_fwd_l1(const gs_projected* p, int64_t n, const gs_bins* bins,
                     const gs_views* views, const float* bg, float* image, float* final_T,
                     uint32_t* n_contrib, const float* target, float* dL_dimage, double* loss,
                     void* workspace, size_t workspace_bytes, gs_stream_t stream);

/* Per-Gaussian rendering error of the global stage (Sec. III-B2, the
 * selection of the set E_t of Gaussians with high rendering error in the
 * current window): for every view k and splat g ([n_views][n] entries, the
 * layout of the projected splats)
 *   err[k][g] = sum over pixels u of w(g, u) * sum_c |image_c(u) - target_c(u)|
 * where w(g, u) = alpha T is g's blending weight at u.  p, bins, image and
 * n_contrib are those of a gs_render_fwd (or gs_render_fwd_l1) call on the
 * same views, unchanged since; target holds the views' reference images C_k
 * (layout of image).  The weights are recomputed with the forward's own
 * float32 arithmetic, so they equal the forward's bit for bit.  The RGB
 * residual's |.| is its L1 norm over the three channels (the paper leaves the
 * channel reduction open).  err (device float32 [n_views][n]) is
 * overwritten: 0 for splats that blend into no pixel.  Accumulated with
 * float32 atomics (the summation order varies between calls). */
int gs_render_error(const gs_projected* p, int64_t n, const gs_bins* bins, const gs_views* views,
                    const float* image, const float* target, const uint32_t* n_contrib,
                    float* err, gs_stream_t stream);

/* Active set of the global stage's selective optimisation (Sec. III-B2):
 *   mask[g] = 1 if max over the n_views views of err[k][g] > eps, or if
 *             always[g] != 0 (the newly inserted Gaussians, which are always
 *             optimised); 0 otherwise
 * for g < n.  err: device float32 [n_views][n] (e.g. from gs_render_error);
 * always (optional, device uint8 [n]); mask (device uint8 [n]) overwritten;
 * err_max (optional, device float32 [n]) receives the per-Gaussian maximum;
 * n_active (optional, device uint32 [1]) receives the number of set mask
 * bytes.  n_views in 1 .. GS_MAX_VIEWS, eps finite.  The comparison is done
 * in float32. */
int gs_active_set(const float* err, int64_t n, int32_t n_views, float eps, const uint8_t* always,
                  uint8_t* mask, float* err_max, uint32_t* n_active, gs_stream_t stream);

/* gs_adam_step_groups_dev restricted to an active set of Gaussians: every
 * group is laid out [C][n_gauss] (its n a multiple of n_gauss, like the
 * parameter groups of gs_gaussians), and element e of a group is updated
 * only if gauss_mask[e % n_gauss] != 0; other elements (parameter and both
 * moments) are left untouched.  The updated elements equal those of the
 * unmasked call bit for bit.  gauss_mask: device uint8 [n_gauss]. */
int gs_adam_step_groups_masked_dev(const gs_adam_group* groups, int32_t n_groups, float beta1,
                                   float beta2, float eps, int32_t* step_dev,
                                   const uint8_t* gauss_mask, int64_t n_gauss,
                                   const uint32_t* guard_n_keys, int64_t guard_capacity,
                                   gs_stream_t stream);

/* ---- map maintenance of the global stage (Sec. III-B2) -------------------
 * Structure-of-arrays data ([C][n] float32 arrays, component-major like the
 * parameter groups of gs_gaussians and their Adam moments) is moved by the
 * calls below; up to GS_SOA_MAX_ARRAYS arrays per call. */
#define GS_SOA_MAX_ARRAYS 16

/* One array of gs_concat: dst [C][n_a + n_b] = a [C][n_a] followed, per
 * component, by b [C][n_b]; when b is NULL the second part is filled with
 * `fill`.  Device pointers; dst must not overlap a or b. */
typedef struct gs_concat_array {
  const float* a;
  const float* b;
  float* dst;
  int32_t components;
  float fill;
} gs_concat_array;

/* Insertion of the local map into the global map, M'_t = M_{t-1} united with
 * the local map (Sec. III-B2), as a concatenation of every parameter array
 * (global Gaussians first); the insertion's lowered opacity is a constant
 * fill of the local part of the opacity-logit array (b = NULL, fill =
 * logit(0.2)), and new Adam moments are fills of 0.  arrays is a host array
 * read during the call; n_a, n_b >= 0. */
int gs_concat(const gs_concat_array* arrays, int32_t n_arrays, int64_t n_a, int64_t n_b,
              gs_stream_t stream);

/* Opacity rule of the pruning step (Sec. III-B2): keep[i] = 1 if the opacity
 * sigmoid(opacity_logits[i]) is at least min_opacity, else 0, decided in
 * float32 as opacity_logits[i] >= logit(min_opacity) (the threshold computed
 * in float64 and rounded to float32).  min_opacity in (0, 1); keep: device
 * uint8 [n]. */
int gs_prune_mask(const float* opacity_logits, int64_t n, float min_opacity, uint8_t* keep,
                  gs_stream_t stream);

/* One array of gs_compact: src [C][n]; dst has room for C * n floats and
 * receives the compacted [C][n_kept] array in its first C * n_kept floats. */
typedef struct gs_compact_array {
  const float* src;
  float* dst;
  int32_t components;
} gs_compact_array;

/* Scratch for gs_compact (bytes). */
size_t gs_compact_workspace_size(int64_t n);

/* Stable compaction of every array by keep (device uint8 [n]): kept entries
 * keep their order.  n_kept (device uint32 [1]) receives their count; the
 * destination component stride is that count, read on the device, so no
 * host synchronisation is needed (capture-safe).  dst must not overlap src. */
int gs_compact(const gs_compact_array* arrays, int32_t n_arrays, int64_t n, const uint8_t* keep,
               uint32_t* n_kept, void* workspace, size_t workspace_bytes, gs_stream_t stream);

/* Isotropic regulariser of the mapping objectives (Eq. 2, Eq. 3; the paper
 * only says that it keeps Gaussians from growing elongated or thin):
 *   E_iso = weight / (3 n) * sum_i sum_j |s_ij - (s_i0 + s_i1 + s_i2) / 3|
 * with s = exp(log_scales) ([3][n] device float32).  Its gradient with respect
 * to the log-scales is added (+=) to grad_log_scales ([3][n]); loss
 * (optional, device float64 [1]) is overwritten with E_iso. */
int gs_iso_loss_grad(const float* log_scales, int64_t n, float weight, float* grad_log_scales,
                     double* loss, gs_stream_t stream);

/* Pose step of the mapping objectives, which minimise over the keyframe poses
 * T_k as well as the map (Eq. 2, Eq. 3): one Adam step on each view's pose
 * tangent xi = (rho, phi) from its gradient grad_xi [n_views][6] (as written
 * by gs_render_bwd), then T_cw <- Exp(delta) T_cw with delta = -lr m_hat /
 * (sqrt(v_hat) + eps) (lr_trans for rho, lr_rot for phi), evaluated in float64
 * (closed-form SE(3) exponential) and stored back into cams_dev's R and t.
 * m, v: device float32 [n_views][6] moments; step_dev: device int32 step
 * counter (t = *step_dev + 1, then incremented); view_mask (optional, device
 * uint8 [n_views]): only views with a nonzero byte move (the past views of
 * the photometric-consistency loss keep their poses).  cams_dev: the device
 * camera records of a gs_views (sizes and intrinsics are not touched).
 * Capture-safe: no host synchronisation. */
int gs_pose_adam_step(gs_camera* cams_dev, const float* grad_xi, float* m, float* v,
                      int32_t n_views, const uint8_t* view_mask, float lr_trans, float lr_rot,
                      float beta1, float beta2, float eps, int32_t* step_dev, gs_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * gs_render_fwd_l1 without a workspace.  Same arguments, results and
 * asynchrony as gs_render_fwd_l1 (bit for bit); the per-tile loss shares go
 * to a static device array of GS_NOALLOC_MAX_TILES floats (1 MiB) that the
 * library holds on every GPU it runs on until the process ends.  The call
 * allocates nothing and synchronises nothing; a batch of more than
 * GS_NOALLOC_MAX_TILES tiles is rejected with GS_ERR_CAPACITY before any
 * work is enqueued.  The array's address is taken on the current device at
 * the first call there (the stream must belong to the current device).
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (different streams or threads) race, so serialise them.  Nothing needs
 * clearing between calls: each call writes every tile share it reads. */
#define GS_NOALLOC_MAX_TILES 262144
int gs_render_fwd_l1_noalloc(const gs_projected* p, int64_t n, const gs_bins* bins,
                             const gs_views* views, const float* bg, float* image,
                             float* final_T, uint32_t* n_contrib, const float* target,
                             float* dL_dimage, double* loss, gs_stream_t stream);

/* L1 photometric loss L = sum over views of mean |C - C*| over 3 H W, and
 * dL/dC = sign(C - C*) / (3 H W) (sign(0) = 0), for every view (layouts of
 * image).  loss (optional, device float64 [1]) is overwritten with L. */
int gs_l1_loss_grad(const float* image, const float* target, const gs_views* views,
                    float* dL_dimage, double* loss, gs_stream_t stream);

/* ---- overhead-memory ledger of the mapping loop (Sec. IV-B) ---------------
 * The paper reports a system's memory as the map plus the overhead, the
 * inputs and temporaries needed to produce the map, counting only variables
 * essential to the algorithm (caches kept solely for speed are left out) and
 * tracking them where they are created and freed.  The calls below are that
 * ledger: a driver registers each essential buffer's bytes under a category
 * when it allocates it and releases them (negative bytes) when it frees it.
 * Host-only (no device work), process-wide, thread-safe. */
enum {
  GS_MEM_MAP = 0,            /* the Gaussian map (parameters)                    */
  GS_MEM_KEYFRAMES = 1,      /* keyframe images held in the sliding window       */
  GS_MEM_POSES = 2,          /* keyframe camera records (window and past poses)  */
  GS_MEM_INIT = 3,           /* initialisation temporaries (cost volume, depth)  */
  GS_MEM_RENDER_TARGETS = 4, /* re-rendered past views of the consistency loss   */
  GS_MEM_BLEND_STATE = 5,    /* per-pixel state kept from forward to backward    */
  GS_MEM_OPTIMISER = 6,      /* optimiser state of the map and poses             */
  GS_MEM_CATEGORIES = 7
};

/* Adds bytes (negative: releases) to a category.  GS_ERR_INVALID_ARGUMENT for
 * an unknown category or a release below zero (then nothing changes). */
int gs_mem_track(int32_t category, int64_t bytes);
/* Current and peak bytes per category (arrays of GS_MEM_CATEGORIES, host,
 * each optional), and the current and peak overhead total (every category
 * but GS_MEM_MAP and GS_MEM_OPTIMISER, whose size follows the map's;
 * optional). */
int gs_mem_report(int64_t* current, int64_t* peak, int64_t* overhead_current,
                  int64_t* overhead_peak);
/* Restarts the peaks from the current values. */
int gs_mem_reset_peaks(void);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
