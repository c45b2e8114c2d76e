/*
 * amr.h -- C ABI of the MI355X octree AMR ray caster.
 *
 * The library casts one ray per pixel through an octree AMR volume truncated
 * at a camera-defined maximum level and accumulates, per ray, one of three
 * projections (Labadens et al., "Volume Rendering of AMR Simulations"):
 *   AMR_SUM    sum over the cells met of value x chord length (Sec. 2.2);
 *   AMR_MAX    maximum of the values met, a maximum-intensity projection
 *              (named in Sec. 2.1);
 *   AMR_WMEAN  weighted mean of a field along the ray, weight x chord as the
 *              measure (a mass-weighted mean when the weight is the density;
 *              the per-cell fields are those listed in Sec. 1).
 * Truncation follows Sec. 2: every cell at the maximum level is treated as a
 * leaf and carries the restricted value of its subtree.
 *
 * Conventions for every entry point:
 *  - Return an amr_status; nothing throws across the ABI.  On error,
 *    amr_last_error() (thread-local) describes it and no output is written.
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary process memory.  The caller owns every buffer it
 *    passes in; the library owns trees, batches and LOD models, which are
 *    released with the matching *_free call.
 *  - Stream-ordered calls take a hipStream_t passed as amr_stream (NULL =
 *    the null stream).  They enqueue work and return; outputs are valid
 *    after the stream is synchronised.  They allocate nothing.
 *  - Positions are integers in units of 2^-28 of the unit box [0,1)^3; the
 *    root cell is level 0; a level-l cell has side 2^-l.  Cells are
 *    half-open boxes [a, b).
 */
#ifndef AMR_H_
#define AMR_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMR_OK = 0,
  AMR_EINVAL = 1,     /* bad argument (null, range, alignment, NaN/Inf) */
  AMR_ETREE = 2,      /* leaves do not tile the box as a complete octree */
  AMR_ENOMEM = 3,     /* host or device allocation failed */
  AMR_EHIP = 4,       /* a HIP runtime call or kernel launch failed */
  AMR_ECAPACITY = 5,  /* an output buffer is too small */
  AMR_ESTALE = 6,     /* a batch refers to a tree that was freed */
  AMR_EMODEL = 7      /* LOD model shape or version mismatch */
} amr_status;

typedef enum { AMR_SUM = 0, AMR_MAX = 1, AMR_WMEAN = 2 } amr_op;
typedef enum { AMR_HOST = 0, AMR_DEVICE = 1 } amr_location;

typedef void* amr_stream; /* hipStream_t */
typedef struct amr_tree amr_tree;

/* Thread-local description of the last error (never NULL). */
const char* amr_last_error(void);

/* ------------------------------------------------------------------ tree */

/* Leaves of an octree: n leaves, leaf q at level level[q] (0..24) with
 * integer coordinates 0 <= ix,iy,iz < 2^level.  fields[f * field_stride + q]
 * is fp32 field f of leaf q (field 0 is conventionally the density, fields
 * 1..3 the velocity).  location says where the five arrays live. */
typedef struct {
  int64_t n;
  const int32_t* level;
  const int32_t* ix;
  const int32_t* iy;
  const int32_t* iz;
  const float* fields;
  int32_t nfields;       /* 1..8 */
  int32_t location;      /* amr_location */
  int64_t field_stride;  /* >= n */
} amr_leaves;

/* How interior (truncated) cells get their values (Sec. 2 leaves this open;
 * the reading taken is RAMSES-style conservative restriction):
 * restrict_weight[f] = -1: field f is the volume mean of the 8 children;
 * restrict_weight[f] = w >= 0: field f is the mean weighted by field w
 * (mass-weighted for w = density); field w must itself be a volume mean.
 * Means are taken in fp64, children summed in Morton child order 0..7
 * (bit0 = x, bit1 = y, bit2 = z), and rounded once to fp32.
 * use_defaults != 0 ignores restrict_weight: field 0 volume mean, every
 * other field weighted by field 0.  host_only != 0 keeps the tree in host
 * memory (inspection and CPU tests; such a tree cannot be rendered). */
typedef struct {
  int32_t restrict_weight[8];
  int32_t use_defaults;
  int32_t host_only;
} amr_build_opts;

/* Build the linear octree (synchronous).  Validates that the leaves tile the
 * unit box as a complete octree (AMR_ETREE on a gap, an overlap, a
 * duplicate or a coordinate out of range; AMR_EINVAL on a NaN/Inf field or a
 * level outside 0..24), sorts them in Morton order, lays every cell out
 * level by level in Morton order (the 8 children of a cell contiguous), and
 * uploads per-cell arrays: first-child index (int32, -1 for leaves), fp32
 * values [nfields][ncells] and the deepest leaf level below each cell
 * (uint8).  The caller's arrays are not retained.  *out receives a
 * library-owned tree, released by amr_tree_free. */
amr_status amr_build_linear_octree(const amr_leaves* in, const amr_build_opts* opt, amr_stream s, amr_tree** out);
void amr_tree_free(amr_tree* t);

typedef struct {
  int64_t ncells;
  int64_t nleaves;
  int32_t nfields;
  int32_t lmax;        /* deepest leaf level */
  int32_t levelmin;    /* shallowest leaf level: levels 0..levelmin are complete */
  int32_t host_only;
  int64_t cells_per_level[25];
  int64_t level_offset[26];
  int64_t device_bytes;
} amr_tree_info_t;

amr_status amr_tree_info(const amr_tree* t, amr_tree_info_t* info);

/* Per-cell arrays of the tree, in the library's layout (see
 * amr_build_linear_octree): host pointers for a host_only tree, device
 * pointers otherwise.  They stay valid until amr_tree_free. */
amr_status amr_tree_arrays(const amr_tree* t, const int32_t** child, const float** values,
                           const uint8_t** maxdepth);


/* ---------------------------------------------------------------- camera */

/* Camera description (box units).  kind 0 = perspective (fov_y, radians),
 * 1 = orthographic (ortho_height).  W x H pixels.  max_level >= 0 fixes the
 * deepest level read; -1 derives it from the pixel footprint (Sec. 2: cells
 * much smaller than a pixel are discarded). */
typedef struct {
  int32_t kind;
  int32_t W, H;
  int32_t max_level;
  int32_t level_bias;
  int32_t pad_;
  double eye[3], target[3], up[3];
  double fov_y;
  double ortho_height;
} amr_camera_desc;

/* Quantised camera: the exact integer ray contract.  For pixel (i, j)
 * (i = column, j = row, j = 0 at the bottom), with a = 2i + 1 - W and
 * b = 2j + 1 - H (rays through pixel centres, Sec. 2.2 "one ray per pixel"):
 *   perspective:  origin O,              direction F + a U + b V
 *   orthographic: origin O + a U + b V,  direction F
 * Origins lie in [-2^30, 2^30) and direction components in (-2^30, 2^30). */
typedef struct {
  int32_t kind, W, H, max_level;
  int64_t O[3], F[3], U[3], V[3];
} amr_camera;

/* Quantise a camera (host only, no GPU needed).  The record is defined on
 * the real numbers: with f = target - eye, g = up x f, h = f x g (so that
 * f / |f|, g / |g| and h / (|f| |g|) are the view, image-x and image-y unit
 * vectors) and the half-pixel step s = tan(fov_y/2) / H (perspective: the
 * field of view is vertical) or ortho_height / (2H) (orthographic),
 *   O = rne(2^28 eye), F = rne(2^28 f/|f|), U = rne(2^28 s g/|g|),
 *   V = rne(2^28 s h/(|f| |g|)),
 * rne = round to nearest, ties to even.  The library evaluates this in
 * fp64 (normalised vectors, norms as sqrt((x^2 + y^2) + z^2), no fused
 * operations), which yields these integers unless a component lies within
 * about 1e-7 of a rounding boundary.
 * Automatic max_level (Sec. 2): the smallest L >= 0 with 2^-L <= p, p the
 * pixel footprint (ortho_height / H, or 2 |f| tan(fov_y/2) / H at the
 * target), plus level_bias, clamped to [0, 24] and to the tree's deepest
 * level when t is not NULL.  AMR_EINVAL on a degenerate basis, fov_y
 * outside (0, 3), W or H outside 1..32768, origins or directions outside
 * the ranges above, or an explicit max_level outside 0..24. */
amr_status amr_set_camera(const amr_camera_desc* d, const amr_tree* t, amr_camera* out);

/* ---------------------------------------------------------------- render */

typedef struct {
  int32_t field;         /* value field for SUM / MAX; for WMEAN the scalar
                            field, or the first of 3 velocity components */
  int32_t weight_field;  /* WMEAN weight (density) */
  int32_t los_velocity;  /* WMEAN: f = (v_field, v_field+1, v_field+2) . d/|d| */
  int32_t variant;       /* kernel variant; -1 = default (see amr_variant_count) */
} amr_render_opts;

/* Render one image (Sec. 2.2: one ray per pixel, top-down descent to the
 * leaves of the truncated tree, value x chord summed in any order).
 * out: device fp32, H x W row-major (out[j*W + i]).
 *   SUM   sum of v * chord (box units); 0 for rays that miss the box.
 *   MAX   maximum of v; -inf for rays that miss the box.
 *   WMEAN sum(w f chord) / sum(w chord), 0 when the weight integral is 0.
 * aux: device fp32 H x W or NULL; for WMEAN receives sum(w chord), computed
 *   with the SUM projection's arithmetic, so it equals the SUM image of the
 *   weight field bit for bit (same variant).
 * Cell decisions are exact integer predicates, so the cell sequence of
 * every ray is deterministic; sums are fp32 Kahan-compensated; chord
 * lengths come from an exact integer numerator, in fp64 for cells at level
 * 18 and deeper.  Every variant visits the same cells and gives a
 * bit-identical MAX.  The split variants (names with "split"), among them
 * the default, cut every ray into spans at base-level planes, walk the
 * spans on different waves and merge their Kahan sums in span order: their
 * SUM and WMEAN differ from the unsplit walk by rounding only and are
 * themselves deterministic.  Variants named "center" only dispatch the
 * packet rows from the middle of the image out; their results equal those
 * of the same variant without it, bit for bit. */
amr_status amr_render(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_render_opts* opts, float* out,
                      float* aux, amr_stream s);

/* Number of kernel variants (ray-packet shape, waves per block, descent
 * mode, spans per ray, dispatch order) amr_render_opts.variant may select, a
 * short name for each, and the one used when none is selected or tuned.
 * That default holds while the camera's maximum level lies fewer than 10
 * levels below the tree's complete base level; deeper, amr_render takes
 * p8x8_w4_fastlds (the walk with an ancestor stack) instead. */
int32_t amr_variant_count(void);
const char* amr_variant_name(int32_t v);
int32_t amr_variant_default(void);

/* ---------------------------------------------------------------- batch */

/* Many images in one launch (the paper renders independent images in
 * parallel with dynamic master/worker load balancing, Sec. 3.1-3.2): image k
 * renders tree trees[pairs[2k]] through camera cams[pairs[2k+1]] with op and
 * opts into outs[k] (device fp32, H x W of that camera; auxs[k] the WMEAN
 * weight plane or auxs == NULL).  The plan copies the trees' and cameras'
 * descriptions to the device, orders the images by the length of their
 * longest ray (measured once here, one counting pass per image), then by
 * size, largest first, and owns a
 * hipGraph captured on first use: either a persistent kernel over a global
 * atomic queue of 64-ray packets (with its queue reset), or, for the "grid"
 * configurations, one block per packet of all images dispatched in order by
 * the hardware.  Output pointers are fixed at creation.  Every image is
 * bit-identical to amr_render of the same image with the matching variant:
 * variant 0 for the unsplit configurations, p8x8_split2_fast for
 * p8x8_split2_grid.  The trees must outlive the plan; amr_render_batch returns
 * AMR_ESTALE if one was freed.  Creation allocates device memory
 * (AMR_ENOMEM); rendering does not.  Concurrent launches of one plan race on
 * its queue counter; AMR_EHIP from amr_batch_set_config if a grid
 * configuration would need more than 2^31 - 1 blocks. */
typedef struct amr_batch amr_batch;
amr_status amr_batch_create(const amr_tree* const* trees, int32_t ntrees, const amr_camera* cams, int32_t ncams,
                            const int32_t* pairs, int32_t npairs, amr_op op, const amr_render_opts* opts,
                            float* const* outs, float* const* auxs, amr_batch** plan);
amr_status amr_render_batch(amr_batch* plan, amr_stream s);
void amr_batch_free(amr_batch* plan);

/* Launch configurations (packet shape, descent mode, waves per CU and
 * packets per queue pop of the persistent kernel, or one block per packet
 * with the rays split in spans), the current one, and explicit selection. */
int32_t amr_batch_config_count(void);
const char* amr_batch_config_name(int32_t c);
int32_t amr_batch_config(const amr_batch* plan);
amr_status amr_batch_set_config(amr_batch* plan, int32_t c);

/* Autotuner for a plan: runs every configuration reps times (after one
 * warm-up, synchronously on the plan's own stream), keeps the fastest and
 * returns it in *best; times_ms (NULL or amr_batch_config_count() floats)
 * receives the best time of each.  The outputs are overwritten. */
amr_status amr_batch_tune(amr_batch* plan, int32_t reps, int32_t* best, float* times_ms);

/* Autotuner for single images: times every amr_render variant on this
 * (tree, camera, op) on stream s (synchronising it), stores the fastest as
 * the tree's default for op (used when opts.variant is -1) and returns it;
 * times_ms (NULL or amr_variant_count() floats) receives each best time.
 * out/aux are overwritten. */
amr_status amr_tune(amr_tree* t, const amr_camera* cam, amr_op op, const amr_render_opts* opts, float* out,
                    float* aux, amr_stream s, int32_t reps, int32_t* best, float* times_ms);
/* Set the tree's default variant for op directly (-1: amr_variant_default),
 * e.g. from a saved tuning cache. */
amr_status amr_set_default_variant(amr_tree* t, amr_op op, int32_t v);

/* ------------------------------------------------- after the ray cast */

/* Local resolution of the image (Sec. 2.2: the post-filter's size follows
 * the local resolution of the image): per pixel, the chord-weighted mean,
 * over the cells the ray meets in the truncated tree, of the cell side in
 * pixels at the cell's depth.  A perspective record's pixel spacing at ray
 * parameter t is 2 |U| t 2^-28 box units (neighbouring pixel rays differ by
 * 2U), taken at the middle of each cell's chord; an orthographic record's
 * is 2 |U| 2^-28.  res: device fp32 H x W; 0 for rays that miss the box.
 * Sums fp32 Kahan-compensated. */
amr_status amr_render_resolution(const amr_tree* t, const amr_camera* cam, float* res, amr_stream s);

/* One walk per ray for both an image and its resolution plane: out / aux as
 * amr_render with the unsplit variant p8x8_w1_fast (bit for bit; same op,
 * field, weight_field and los_velocity; opts.variant is ignored) and res as
 * amr_render_resolution (bit for bit), for the cost of one walk with a
 * slightly heavier visitor instead of two walks.  Same arguments and errors
 * as those two calls; res: device fp32 H x W. */
amr_status amr_render_with_resolution(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_render_opts* opts,
                                      float* out, float* aux, float* res, amr_stream s);

/* Adaptive Gaussian blur (Sec. 2.2) of an image img (device fp32 H x W,
 * row-major) with standard deviation sigma = kappa * res (pixels) at each
 * output pixel, res a resolution plane as above.  The filter is a ladder of
 * 2-D Gaussians of sigma_k = 0.5 x 2^(k/2), k = 0..10, each truncated to the
 * square of radius ceil(3 sigma_k) and normalised over that square's pixels
 * inside the image; a pixel takes the blend of the two levels around its
 * sigma, linear in log2 sigma (below sigma_0, of the image itself and
 * level 0, linear in sigma; above sigma_10, level 10; sigma <= 0: the image
 * value).  out: device fp32 H x W, not aliasing img.  workspace: device,
 * 256-byte aligned, amr_blur_workspace_bytes(W, H) bytes (11 fp32 planes).
 * Sums in fp64.  AMR_EINVAL on a bad size, kappa < 0, null, misaligned or
 * aliased buffers; AMR_ECAPACITY on a small workspace. */
int64_t amr_blur_workspace_bytes(int32_t W, int32_t H);
amr_status amr_blur_adaptive(const float* img, const float* res, int32_t W, int32_t H, float kappa, float* out,
                             void* workspace, int64_t workspace_bytes, amr_stream s);

/* Slice map (Sec. 3, the "Slicemap" of the GPU trial: a simple tree
 * search): for an orthographic record, the value of field `field` of the
 * cell of the tree truncated at cam->max_level that holds the point
 * O + aU + bV of each pixel (the origins of its rays; cells half-open, so a
 * point on a face belongs to the cell above it).  out: device fp32 H x W,
 * the cell's stored value (bit for bit), NaN for points outside the box.
 * AMR_EINVAL for a perspective record or a bad field. */
amr_status amr_slice(const amr_tree* t, const amr_camera* cam, int32_t field, float* out, amr_stream s);

/* ------------------------------------------------------- learned LOD */

/* Learned per-tile level of detail.  Sec. 2 truncates the tree at one
 * camera-wide level from the pixel size; here a network predicts, for each
 * 16 x 16 pixel tile, the shallowest level L in 1..16 whose render stays
 * within rel_tol of the full-depth render.
 *   coarse_level  level at which the 16 probe rays per tile are walked (4)
 *   quantile      level = first class whose cumulative probability >= q
 *   conf_thresh   tiles whose top class probability is below it render at
 *                 full depth (>= 1 forces full depth everywhere)
 *   rel_tol       per-pixel tolerance of the audit (1e-3)
 *   audit_frac    fraction of tiles re-rendered at full depth and compared;
 *                 pixels off by more than rel_tol are overwritten and counted
 *   audit_seed    seed of the audited-tile selection */
typedef struct {
  int32_t coarse_level;
  float quantile;
  float conf_thresh;
  float rel_tol;
  float audit_frac;
  int32_t audit_seed;
} amr_lod_config;

/* Library-owned model: fp32 master parameters, bf16 copy, gradients and
 * Adam moments on the device.  32 -> 64 -> 64 -> 64 -> 16 MLP (ReLU); the
 * 16 outputs are the classes of levels 1..16. */
typedef struct amr_lod_model amr_lod_model;
int32_t amr_lod_param_count(void);
amr_status amr_lod_create(const amr_lod_config* cfg, uint64_t seed, amr_lod_model** out); /* He init, seeded */
void amr_lod_free(amr_lod_model* m);
amr_status amr_lod_save(const amr_lod_model* m, const char* path);   /* versioned binary */
amr_status amr_lod_load(const char* path, amr_lod_model** out);      /* AMR_EMODEL on format/version */
amr_status amr_lod_get_config(const amr_lod_model* m, amr_lod_config* cfg);
amr_status amr_lod_set_config(amr_lod_model* m, const amr_lod_config* cfg);
/* Host copies of the fp32 parameters / gradients (amr_lod_param_count()
 * floats: W1[32][64], b1, W2[64][64], b2, W3[64][64], b3, W4[64][16], b4). */
amr_status amr_lod_get_params(const amr_lod_model* m, float* host);
amr_status amr_lod_set_params(amr_lod_model* m, const float* host);
amr_status amr_lod_get_grads(const amr_lod_model* m, float* host);

/* Tiles of a W x H image: ceil(W/16) ceil(H/16), row-major. */
int64_t amr_lod_tiles(int32_t W, int32_t H);

/* Per-tile features (device bf16 [tiles][32]) from 16 probe rays per tile
 * walked with the tree truncated at coarse_level. */
amr_status amr_lod_features(const amr_tree* t, const amr_camera* cam, int32_t coarse_level, uint16_t* feat,
                            amr_stream s);

/* Network forward on n feature rows: logits (device fp32 [n][16]); acts
 * (device bf16 [3][n][64] or NULL) keeps the hidden activations for
 * amr_lod_backward. */
amr_status amr_lod_forward(const amr_lod_model* m, const uint16_t* feat, int64_t n, float* logits, uint16_t* acts,
                           amr_stream s);

/* Loss per sample: -log p_y + lambda * sum_{c < y} p_c over the 16 classes
 * (labels device int8 [n]); dlogits (device fp32 [n][16]) = gradient * scale;
 * loss_sum (device fp32, may be NULL) += sum of the losses. */
amr_status amr_lod_loss(const float* logits, const int8_t* labels, int64_t n, float lambda, float scale,
                        float* dlogits, float* loss_sum, amr_stream s);

/* Backward: accumulates parameter gradients (fp32, in the model) from
 * dlogits; dz is device scratch of bf16 [3][n][64] + [n][16]. */
amr_status amr_lod_backward(amr_lod_model* m, const uint16_t* feat, const uint16_t* acts, const float* dlogits,
                            int64_t n, uint16_t* dz, amr_stream s);
amr_status amr_lod_zero_grads(amr_lod_model* m, amr_stream s);
/* One Adam step with the accumulated gradients, which it then clears;
 * refreshes the bf16 weights.  beta1 = 0.9 and beta2 = 0.999 as fp32 values
 * (0.89999998 and 0.99900001), eps = 1e-8; moments and weights in fp32, the
 * bias corrections 1 - beta^t in fp64 then rounded to fp32. */
amr_status amr_lod_adam_step(amr_lod_model* m, float lr, amr_stream s);

/* Training labels: imgs[0..15] are device renders (same camera, same op) at
 * levels 1..16; the label of a tile is the first level whose render is
 * within tol of the level-16 render at every pixel of the tile (device
 * int8 [tiles], class = level - 1). */
amr_status amr_lod_labels(const float* const* imgs, int32_t W, int32_t H, float tol, int8_t* labels, amr_stream s);

/* Render with the learned per-tile levels (tiles at or above the camera's
 * max_level render exactly like amr_render; audited tiles below it are also
 * rendered at full depth when their render cut a cell, and a second launch
 * repairs their pixels).  Four launches: features, network and plan
 * (one kernel), tile render, repair.  workspace: device, 256-byte aligned,
 * at least amr_lod_workspace_bytes(W, H) (features, logits and plan of the
 * tiles, 4 KiB of counters, and two fp32 W x H planes for the audit).
 * tile_levels (device int8 [tiles] or NULL) receives the levels used;
 * forced_levels (device int8 [tiles] or NULL) replaces the network's choice
 * (tests of the audit).
 * stats: device int64[8] overwritten with tiles, fallbacks, audited tiles,
 * overwritten pixels, sum of tile levels, and audited 8 x 8 packets walked
 * again at full depth (those with a ray that stopped its descent at a cell
 * that has children; the others already are the full-depth image). */
int64_t amr_lod_workspace_bytes(int32_t W, int32_t H);
amr_status amr_render_lod(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_lod_model* m,
                          const amr_render_opts* opts, float* out, float* aux, int8_t* tile_levels,
                          const int8_t* forced_levels, void* workspace, int64_t workspace_bytes, int64_t* stats,
                          amr_stream s);

/* amr_render_lod without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): the workspace is a fixed device array
 * of amr_lod_noalloc_max_bytes() bytes (40 MiB) inside the library, one per
 * GPU, held until the process ends; the call itself allocates nothing.
 * Same arguments and results as amr_render_lod otherwise (same kernels:
 * the outputs are bit-identical to amr_render_lod's).  AMR_ECAPACITY when
 * amr_lod_workspace_bytes(W, H) exceeds that size (2048 x 2048 images fit);
 * AMR_EHIP if the array's device address cannot be obtained.  Every call on
 * one GPU shares that GPU's array and leaves its contents there: calls that
 * overlap in time on one GPU (other streams, other threads) race and must
 * be serialised by the caller. */
int64_t amr_lod_noalloc_max_bytes(void);
amr_status amr_render_lod_noalloc(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_lod_model* m,
                                  const amr_render_opts* opts, float* out, float* aux, int8_t* tile_levels,
                                  const int8_t* forced_levels, int64_t* stats, amr_stream s);

/* ------------------------------------------- trees larger than the GPU */

/* Rendering a tree held in host memory, streamed through the GPU chunk by
 * chunk.  The paper finds reading the data the dominant cost (Sec. 3) and
 * notes that the camera's depth bound means not every cell need be read
 * (Sec. 2); the order of accumulation along a ray is free (Sec. 2.2).
 *
 * A plan cuts a host_only tree (amr_build_opts.host_only) into chunks: the
 * complete subtrees under cells (cubes) of levels 0..base, base = min(the
 * tree's shallowest leaf level, 10), found by splitting cubes in Morton
 * order while a subtree holds more than max_chunk_cells cells.  Each chunk
 * keeps its cells level by level in Morton order with chunk-local
 * first-child indices, in pinned host memory owned by the plan (the tree is
 * not retained and may be freed).  The plan also owns nbuffers device
 * buffers of max_chunk_cells cells each, a copy stream and two events per
 * buffer.
 * host_only != 0 builds the chunks in ordinary host memory and nothing on
 * the device (inspection and CPU tests; such a plan cannot render).
 * AMR_EINVAL for a tree that is not host_only, max_chunk_cells outside
 * 1..2^31-1 or nbuffers outside 0, 2..8; AMR_ECAPACITY when the subtree of one base-level cell exceeds
 * max_chunk_cells; AMR_ENOMEM when host (pinned) or device memory runs out. */
typedef struct amr_stream_plan amr_stream_plan;
typedef struct {
  int64_t max_chunk_cells;
  int32_t host_only;
  int32_t nbuffers;  /* device buffers the chunks rotate through: 2..8, 0 = 4 */
} amr_stream_opts;
amr_status amr_stream_plan_create(const amr_tree* host_tree, const amr_stream_opts* opts, amr_stream_plan** out);
/* Waits for the plan's copies and kernels, then releases it. */
void amr_stream_plan_free(amr_stream_plan* p);

typedef struct {
  int32_t nchunks;
  int32_t min_chunk_level, max_chunk_level;
  int32_t nbuffers;
  int64_t max_chunk_cells;  /* the capacity asked for */
  int64_t largest_chunk;    /* cells of the largest chunk */
  int64_t cells;            /* cells over all chunks (levels above a chunk's cube are in none) */
  int64_t host_bytes;       /* the chunks' host arrays */
  int64_t device_bytes;     /* the device buffers (0 for host_only plans) */
} amr_stream_plan_info_t;
amr_status amr_stream_plan_info(const amr_stream_plan* p, amr_stream_plan_info_t* out);

/* Chunk i (0 <= i < nchunks, Morton order of the cubes): the cube (level,
 * ix, iy, iz), its ncells cells and their host arrays: records holds 2
 * int32 per cell (chunk-local first-child index or -1, and the bits of
 * field 0 as fp32), values the fields [nfields][ncells], packed fields 0..3
 * interleaved (4 fp32 per cell) or NULL for trees of fewer than 4 fields.
 * level_start[l] is the local index of the first cell of level l
 * (level_start[25] = ncells); off_local[l], for levels level..base, is the
 * local index that Morton code 0 of level l would have, so the cell of
 * Morton code m at such a level is off_local[l] + m.  first is the chunk's
 * offset in the plan's concatenated arrays.  Pointers live as long as the
 * plan. */
typedef struct {
  int32_t level, ix, iy, iz;
  int64_t ncells;
  int64_t first;
  int64_t level_start[26];
  int32_t off_local[26];
  const int32_t* records;
  const float* values;
  const float* packed;
} amr_stream_chunk_t;
amr_status amr_stream_chunk(const amr_stream_plan* p, int32_t i, amr_stream_chunk_t* out);

/* Pixel rectangle rect = {i0, j0, i1, j1} (inclusive) holding every pixel
 * of cam whose ray can meet chunk i's cube (i1 < i0 when none can): the
 * rays the streamed render walks for that chunk. */
amr_status amr_stream_chunk_rect(const amr_stream_plan* p, int32_t i, const amr_camera* cam, int32_t rect[4]);

/* Workspace of amr_render_streamed: 32 bytes per pixel (two planes of
 * per-pixel partial sums), device memory aligned to 256 bytes. */
int64_t amr_stream_workspace_bytes(int32_t W, int32_t H);

/* amr_render (same op, opts.field / weight_field / los_velocity, outputs and
 * conventions; opts.variant is ignored) of the plan's tree, streamed: for
 * each chunk whose rectangle is not empty, in chunk order, the copy stream
 * copies the chunk's cells of levels down to min(cam->max_level, lmax)
 * (only the arrays the op reads) into the next of the plan's device
 * buffers in turn, after the kernel that last read that buffer; then the
 * chunk's kernel walks each ray of the rectangle inside the chunk's cube
 * (the ray clipped exactly to the cube) and adds its fp32 Kahan partial
 * sums to the pixel's (maximum for MAX).  Chunks alternate between stream s
 * (first plane of the workspace) and the plan's second compute stream
 * (second plane), so that kernels overlap; at the end s merges the second
 * plane into the first, pixel by pixel, and writes the outputs.  Every cell
 * of the truncated tree at a chunk's level or deeper lies in one chunk, and
 * its decisions are the whole ray's, so MAX is bit-identical to amr_render
 * and SUM / WMEAN differ from it by rounding only; the order of the sums
 * depends on the chunk order and the camera alone, so results are
 * deterministic.  The calls enqueue work on s and on the plan's streams and
 * return; the outputs are valid once s is synchronised.  One plan renders
 * one image at a time (calls on one plan are ordered by its events;
 * workspaces must not be shared between calls in flight).
 * stats: host int64[3] or NULL: chunks walked, bytes copied to the device,
 * pixels covered by the rectangles.  AMR_EINVAL for a host_only plan, a bad
 * camera, op or field, misaligned buffers, or cam->max_level shallower than
 * the plan's deepest chunk level; AMR_ECAPACITY for a small workspace;
 * AMR_EHIP when a copy or launch fails. */
amr_status amr_render_streamed(amr_stream_plan* p, const amr_camera* cam, amr_op op, const amr_render_opts* opts,
                               float* out, float* aux, void* workspace, int64_t workspace_bytes, int64_t* stats,
                               amr_stream s);

/* ---------------------------------------------------------------- debug */

/* Segments (cells met) per ray for every pixel: counts (device int32 H x W,
 * may be NULL) and their total (device int64, 1 element, overwritten).
 * The counts come from the walk the renders time (the unsplit whole-ray
 * walk), so they are the segment counts of the benchmarked launches. */
amr_status amr_count_segments(const amr_tree* t, const amr_camera* cam, int32_t* counts, int64_t* total,
                              amr_stream s);

/* Distinct cells met by the rays of an image (the compulsory traffic of a
 * render is that count times the bytes read per cell).  bitmap: device
 * uint32, ceil(ncells / 32) words, bit c for cell c (the cell index of the
 * tree's layout); cells met get their bit set (bits already set stay set,
 * so several images accumulate, and the caller clears the bitmap to
 * start).  distinct: device int64, increased by the number of bits this
 * call set.  Calls that overlap on one bitmap count each cell once. */
amr_status amr_mark_cells(const amr_tree* t, const amr_camera* cam, uint32_t* bitmap, int64_t* distinct,
                          amr_stream s);

/* Cell sequences of the rays ray_ids[0..n) (pixel index j*W + i, device
 * int64).  offsets (device int64, n + 1) must already hold the exclusive
 * prefix sum of the rays' segment counts (from amr_count_segments);
 * cells (device int32, 4 per segment: level, ix, iy, iz, unmirrored) receive
 * the cells in the order the ray meets them.  AMR_ECAPACITY is not
 * detectable on the device: the caller sizes cells from offsets[n]. */
amr_status amr_trace_rays(const amr_tree* t, const amr_camera* cam, const int64_t* ray_ids, int64_t n,
                          const int64_t* offsets, int32_t* cells, amr_stream s);

/* Segment counts of the rays ray_ids[0..n) only (device int32 counts[n]). */
amr_status amr_count_rays(const amr_tree* t, const amr_camera* cam, const int64_t* ray_ids, int64_t n,
                          int32_t* counts, amr_stream s);

#ifdef __cplusplus
}
#endif
#endif /* AMR_H_ */
