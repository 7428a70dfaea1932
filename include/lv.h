/*
 * lv.h -- C ABI of the MI355X (gfx950) library for learning-free uplifting of
 * 2D feature maps onto 3D Gaussian Splatting scenes and graph diffusion over
 * the Gaussians (LUDVIG, arXiv 2410.14462).
 *
 * Method (paper references are to sections and equations):
 *   Sec. 3.1, Eq. (1)  each pixel p of view d alpha-blends an ordered set of
 *                      Gaussians; w_i(d,p) = alpha_i(d,p) prod_{j<i}(1-alpha_j).
 *   Sec. 3.2, Eq. (3)  f_i = sum_{(d,p)} w_i(d,p) F_{d,p} / sum_{(d,p)} w_i(d,p).
 *   Sec. 3.2, Eq. (5)  the same as f = diag(beta)^-1 W^T F; beta_i = sum w_i is
 *                      also the Gaussian importance (Gaussian filtering).
 *   Sec. 3.3, Eq. (8)  diffusion g_{t+1} = A g_t / ||g_t||_2.
 *
 * Conventions fixed by this library where the paper is silent:
 *   - Gaussian i: mean mu (3 floats), per-axis scale s (linear, 3 floats),
 *     rotation quaternion (w,x,y,z) (normalised by the library), opacity in
 *     (0,1).  Covariance = R diag(s)^2 R^T.
 *   - Camera: world->camera rotation R (row-major) and t, x_c = R x_w + t,
 *     x right / y down / z forward; pinhole fx, fy, cx, cy in pixels; pixel
 *     (i,j) covers [i,i+1) x [j,j+1) and is sampled at its centre.
 *   - Gaussians with z_c <= znear are culled.  The 2D footprint is the EWA
 *     projection (Jacobian with x/z, y/z clamped to 1.3 x the half-FoV
 *     tangent) plus 0.3 px^2; alpha = min(0.99, opacity * exp(-d^T C d / 2));
 *     a Gaussian with alpha < 1/255 at a pixel is skipped; a pixel stops at
 *     the Gaussian that would take its transmittance below 1e-4 (that Gaussian
 *     is not counted).  Each 16x16 tile walks the Gaussians whose tile
 *     rectangle (radius ceil(3 sqrt(lambda_max))) covers it, sorted by the
 *     FP32 bits of z_c, ties by Gaussian index.  Which Gaussians a pixel counts
 *     is decided by a fixed sequence of FP32 operations, so it is reproducible
 *     bit for bit on any IEEE-754 machine.
 *   - Feature maps are HWC: view v is [height][width][D] contiguous.
 *
 * Memory: every pointer named "device" is HIP device memory (e.g. a torch
 * tensor's data_ptr()).  Handles (lv_scene, lv_accum, lv_graph) are owned by
 * the library; free them with the matching *_destroy.  Output buffers are
 * owned by the caller.  Every call is asynchronous on the HIP stream passed
 * as `stream` (hipStream_t; NULL = the null stream) unless stated otherwise;
 * inputs must stay valid until the stream passes the call.
 *
 * Errors: every call returns an lv_status.  On a non-OK status nothing is
 * enqueued and outputs are untouched; lv_last_error() describes the failure
 * (thread-local).  No C++ exception crosses this interface.
 *
 * Threads: distinct handles may be used from different threads.  One handle
 * must not be used by two threads at once, and an accumulator must not be
 * the target of work in flight on two streams at once (calls on one stream
 * are ordered by the stream).
 */
#ifndef LV_H
#define LV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LV_OK = 0,
    LV_ERR_INVALID_ARG = 1,
    LV_ERR_OUT_OF_MEMORY = 2,
    LV_ERR_DEVICE = 3,
    LV_ERR_UNSUPPORTED = 4,
    LV_ERR_CANCELLED = 5     /* a server request cancelled before it ran */
} lv_status;

/* Storage type of feature maps / diffusion signals.  Arithmetic is FP32.
 * The _PX8 types are feature maps (uplift inputs only) of the same element
 * types in the pixel-block layout that lv_encode_map writes: element
 * (y, x, c) of a W-pixel-wide map whose pixels hold ld channels (ld = D
 * unless a channel slice of a wider map is read) is at
 * ((y ceil(W/8) + floor(x/8)) ld + c) 8 + (x mod 8), pixels past W are 0.
 * The 8 pixels of one channel that an 8-pixel row of a tile quadrant needs
 * are then contiguous: one 16-byte read per matrix-product operand for
 * BF16 (the blend, Sec. 3.2).  Maps must be aligned to their 8-pixel
 * blocks (32, 16 or 8 bytes). */
typedef enum {
    LV_F32 = 0,
    LV_BF16 = 1,       /* bfloat16, round-to-nearest-even                     */
    LV_FP8_E4M3 = 2,   /* OCP E4M3FN with a per-(view, channel) FP32 scale     */
    LV_F32_PX8 = 3,
    LV_BF16_PX8 = 4,
    LV_FP8_E4M3_PX8 = 5
} lv_dtype;

/* Pinhole camera, 80 bytes. */
typedef struct lv_camera {
    float R[9];        /* world->camera rotation, row-major                    */
    float t[3];        /* x_c = R x_w + t                                      */
    float fx, fy;      /* focal lengths in pixels                              */
    float cx, cy;      /* principal point in pixels                            */
    float znear;       /* Gaussians with z_c <= znear are culled               */
    int32_t width;     /* image size in pixels, 1..16384                       */
    int32_t height;
    int32_t reserved;  /* must be 0                                            */
} lv_camera;

typedef struct lv_scene lv_scene;
typedef struct lv_accum lv_accum;
typedef struct lv_graph lv_graph;

/* Thread-local description of the last non-OK status of this thread. */
const char* lv_last_error(void);

/* ------------------------------------------------------- device memory -- */
/* Every device buffer the library allocates -- cached scratch (structure
 * builds, pair buffers), temporary scratch (graph builds, filtering, server
 * accumulators) and the buffers its handles own -- comes from `alloc` and
 * returns through `free` once registered (e.g. a framework's caching
 * allocator); without one, hipMalloc / hipFree (hipMallocAsync /
 * hipFreeAsync for temporary scratch).  alloc(bytes, stream, ctx) returns a
 * device pointer (256-byte aligned) usable on `stream`, or NULL (the call
 * then fails with LV_ERR_OUT_OF_MEMORY); free(ptr, bytes, stream, ctx)
 * releases it after the work enqueued on `stream` (stream-ordered; NULL
 * stream: the device is idle).  The callbacks may be called from any thread
 * (the server's workers too).  lv_set_allocator(NULL, NULL, NULL) restores
 * the default.  It first releases the cached scratch (lv_release_scratch of
 * every stream) and fails with LV_ERR_INVALID_ARG while any handle still
 * owns device memory (memory must return to the allocator it came from).
 * Call it while no library work is in flight. */
typedef void* (*lv_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*lv_free_fn)(void* ptr, size_t bytes, void* stream, void* ctx);
lv_status lv_set_allocator(lv_alloc_fn alloc, lv_free_fn free, void* ctx);
/* Frees the scratch the library caches for `stream` (all_streams != 0: for
 * every stream, and the buffers kept from destroyed scenes); the scratch is
 * allocated again by the next call that needs it.  No library work may be in
 * flight on those streams. */
lv_status lv_release_scratch(void* stream, int32_t all_streams);
/* Device bytes the library holds (handles and cached scratch) and the
 * number of its live device allocations. */
lv_status lv_memory_stats(int64_t* bytes, int64_t* allocations);

/* Library version string. */
const char* lv_version(void);

/* ---------------------------------------------------------------- scenes -- */
/* Blending constants of a scene (Sec. 3.1, Eq. 1, with the rasteriser
 * conventions the paper relies on): alpha clamp, skip threshold,
 * transmittance stop, 2D dilation (px^2) and tile edge (px).  opts = NULL
 * means the defaults 0.99f, 1/255.f, 1e-4f, 0.3f, 16, which are also the
 * only values this build runs: others give LV_ERR_UNSUPPORTED (the kernels
 * and their exact FP32 decision sequence are compiled for them).
 * flags: by default the library stores the Gaussians in the Morton order
 * of their centres (10 bits per axis over the scene's bounding box, equal
 * codes in the caller's order), which gives the blend's reads of projected
 * records and its accumulator updates spatial locality.  The order is
 * internal: every per-Gaussian input and output (features, weight sums,
 * counts, render inputs, graph nodes, debug views) stays in the caller's
 * order, and Gaussians at exactly equal depth still blend in the order of
 * their caller index, so results equal those of the caller's order up to
 * the summation order of the accumulators.  LV_SCENE_CALLER_ORDER stores
 * them in the caller's order instead. */
#define LV_SCENE_CALLER_ORDER 1u
typedef struct lv_scene_opts {
    float alpha_max, alpha_min, t_eps, dilation;
    int32_t tile;
    uint32_t flags;
} lv_scene_opts;

/* Make a scene resident on the current device (Sec. 3.1 scene
 * representation).  means [n][3], scales [n][3], quats [n][4] (w,x,y,z),
 * opacity [n]: device FP32 arrays, read (not retained) by the call.  The
 * library derives the covariances R diag(s)^2 R^T and keeps its own copy
 * (48 bytes per Gaussian).  n = 0 is valid.  opts: see lv_scene_opts.
 * Errors: LV_ERR_INVALID_ARG (null pointers with n > 0, n >= 2^31),
 * LV_ERR_UNSUPPORTED (non-default opts), LV_ERR_OUT_OF_MEMORY. */
lv_status lv_scene_create(const float* means, const float* scales, const float* quats,
                          const float* opacity, int64_t n, const lv_scene_opts* opts, void* stream,
                          lv_scene** out);
lv_status lv_scene_destroy(lv_scene* scene);
int64_t lv_scene_size(const lv_scene* scene);

/* --------------------------------------------------------------- uplift -- */
/* Eq. (3) / Eq. (5): uplift m feature maps of D channels onto the scene.
 *   cams      host array [m] of cameras.
 *   maps      host array [m] of device pointers; maps[v] is [H_v][W_v][D] of
 *             `dtype` (HWC, contiguous).
 *   scales    LV_FP8_E4M3 only: device FP32 [m][D], the value of channel c of
 *             view v is scales[v*D + c] * decode(byte); NULL otherwise.
 *   out_feat  device FP32 [n][D]: f_i = U_i / beta_i, 0 where beta_i = 0.
 *   out_wsum  device FP32 [n]: beta_i = sum over views and pixels of w_i
 *             (nullable).
 * D in [1, 4096]; m >= 0 (m = 0 writes zeros).  Views are processed in
 * chunks (one host synchronisation per chunk) bounded by a scratch budget
 * (a sixteenth of the device memory, clamped to [4, 16] GiB) for the
 * per-(view, Gaussian) items and the same for the (tile, Gaussian) pairs; a
 * chunk whose pairs exceed that (or 2^31) is split and built again.  Scratch
 * is cached per (device, stream) until lv_release_scratch.  Errors:
 * LV_ERR_INVALID_ARG (bad sizes, null maps, reserved != 0),
 * LV_ERR_UNSUPPORTED (one view alone has 2^31 pairs or more),
 * LV_ERR_OUT_OF_MEMORY, LV_ERR_DEVICE. */
lv_status lv_uplift(lv_scene* scene, const lv_camera* cams, int32_t m, const void* const* maps,
                    lv_dtype dtype, const float* scales, int32_t D, float* out_feat,
                    float* out_wsum, void* stream);

/* lv_uplift for several feature sets over the same views in one pass (one
 * structure build and one blend walk; see lv_uplift_accumulate_sets).  Set k
 * has its own maps (device pointers, HWC with D_k channels), FP8 scales and
 * outputs.  1 <= nsets <= 8. */
typedef struct lv_uplift_set {
    const void* const* maps;   /* host array [m] of device pointers */
    const float* scales;       /* FP8 only: device [m][D], else NULL */
    int32_t D;
    float* out_feat;           /* device [n][D] */
    float* out_wsum;           /* device [n], nullable */
} lv_uplift_set;
lv_status lv_uplift_sets(lv_scene* scene, const lv_camera* cams, int32_t m, const lv_uplift_set* sets,
                         int32_t nsets, lv_dtype dtype, void* stream);

/* Streaming form of lv_uplift: the accumulator holds U = W^T F [n][D] (FP32)
 * and beta (exact 64-bit fixed point in units of 2^-35, at most 2^29 units of
 * weight per Gaussian), to which views are added in any grouping
 * (accumulating views [0,k) then [k,m) equals all m).  With
 * LV_ACCUM_COUNTS it also counts, per Gaussian, the (view, pixel) pairs
 * that contribute (exact integers).
 * LV_ACCUM_DETERMINISTIC: U too is 64-bit fixed point (units of 2^-35: each
 * partial sum is rounded to the nearest unit and added with an integer
 * atomic), so U, beta and the features are the same bit for bit from run to
 * run and for any grouping of the views, and a comparison with the FP32
 * accumulator exposes lost updates.  Limits: |U_ic| < 2^28, absolute
 * rounding up to 2^-36 per partial sum (against the FP32 accumulator's
 * relative 2^-24), twice the accumulator memory and the integer atomics'
 * traffic.  All accumulators of one call take the same mode (else
 * LV_ERR_INVALID_ARG). */
#define LV_ACCUM_COUNTS 1u
#define LV_ACCUM_DETERMINISTIC 2u
lv_status lv_accum_create(lv_scene* scene, int32_t D, uint32_t flags, void* stream, lv_accum** out);
lv_status lv_accum_reset(lv_accum* acc, void* stream);
lv_status lv_uplift_accumulate(lv_accum* acc, const lv_camera* cams, int32_t m,
                               const void* const* maps, lv_dtype dtype, const float* scales,
                               void* stream);
/* Several feature sets over the same views in one pass (the same weights
 * w_i(p) serve every set, Eq. 5 with F the concatenation of the sets'
 * channels): set k adds maps[k] (host array [m] of device pointers) to
 * sets[k].acc.  maps[k][v] may be NULL: set k does not take view v (nothing
 * is added to it for that view, its beta included).  A map is HWC with the
 * accumulator's D channels per pixel, consecutive pixels `stride` elements
 * apart (stride 0 means D; stride > D reads channels [0, D) of a wider map).
 * 1 <= nsets <= 8; all accumulators on the same scene and distinct; one
 * storage dtype for all sets.  Each set's result equals
 * lv_uplift_accumulate of that set alone over the views it takes (within
 * FP32 accumulation order). */
typedef struct lv_feature_set {
    lv_accum* acc;
    const void* const* maps;
    const float* scales;       /* FP8 only: device [m][D], else NULL */
    int32_t stride;            /* elements between consecutive pixels; 0 = D */
} lv_feature_set;
lv_status lv_uplift_accumulate_sets(const lv_camera* cams, int32_t m, const lv_feature_set* sets,
                                   int32_t nsets, lv_dtype dtype, void* stream);
/* f = U / beta (0 where beta = 0) into out_feat [n][D]; beta into out_wsum
 * [n] (nullable); raw U into out_sum [n][D] (nullable). */
lv_status lv_accum_finalize(lv_accum* acc, float* out_feat, float* out_wsum, float* out_sum,
                            void* stream);
/* Checkpoint / resume of an accumulator: its raw state, in the caller's
 * Gaussian order, to or from caller device buffers.  U [n][D]: FP32, or
 * int64 (units of 2^-35) for an LV_ACCUM_DETERMINISTIC accumulator; beta [n]
 * uint64 (units of 2^-35); counts [n] uint32 (accumulators with
 * LV_ACCUM_COUNTS; NULL skips them, and on import NULL zeroes them).
 * Importing what another accumulator of the same scene, D and flags
 * exported, then adding the remaining views, equals adding all views to one
 * accumulator (bit for bit for beta, counts and a deterministic U).
 * Errors: LV_ERR_INVALID_ARG (null accumulator, U or beta with n > 0;
 * counts given without LV_ACCUM_COUNTS), LV_ERR_DEVICE. */
lv_status lv_accum_export(lv_accum* acc, void* U, uint64_t* beta, uint32_t* counts, void* stream);
lv_status lv_accum_import(lv_accum* acc, const void* U, const uint64_t* beta, const uint32_t* counts,
                          void* stream);
/* Count-normalised features (appendix, comparison with GaussianEditor's
 * uplifting): f_i = U_i / c_i into out_feat [n][D], c_i the number of counted
 * (view, pixel) pairs of Gaussian i instead of the sum of their weights; 0
 * where c_i = 0.  The accumulator must have been created with
 * LV_ACCUM_COUNTS (else LV_ERR_INVALID_ARG). */
lv_status lv_accum_finalize_count(lv_accum* acc, float* out_feat, void* stream);
/* Weight-based filtering (Sec. 3.2, Gaussian filtering): beta_i estimates
 * the importance of Gaussian i; keep the k Gaussians with the largest
 * wsum[i] (device FP32 [n], e.g. the out_wsum of lv_accum_finalize), ties to
 * the lower index.  keep (device uint8 [n]) gets 1 for kept Gaussians and 0
 * for the others.  Values are ordered as IEEE floats (-0 below +0).  Scratch
 * (about 16 bytes per Gaussian) comes from the stream-ordered allocator.
 * Errors: LV_ERR_INVALID_ARG (n < 0 or n >= 2^31, k outside [0, n], null
 * buffers with n > 0), LV_ERR_DEVICE. */
lv_status lv_prune_by_weight(const float* wsum, int64_t n, int64_t k, uint8_t* keep, void* stream);
/* Anchor initialisation of a diffusion (appendix on diffusion for
 * segmentation): of the n values g (device FP32, e.g. an uplifted mask),
 * the ceil(fraction * npos) largest of the npos positive ones (ties to the
 * lower index) are copied to g0 (device FP32 [n]), every other entry of g0
 * is 0.  0 < fraction <= 1.  Scratch from the stream-ordered allocator. */
lv_status lv_anchor_init(const float* g, int64_t n, float fraction, float* g0, void* stream);
/* Reachability after diffusion (same appendix): h[i][c] = unary[i] where
 * gT[i][c] > 0, else 0 (gT, h: device FP32 [n][D]; unary: device FP32 [n]). */
lv_status lv_reach_unary(const float* gT, const float* unary, int64_t n, int32_t D, float* h,
                         void* stream);
/* Per-Gaussian contribution counts (device uint32 [n]); the accumulator must
 * have been created with LV_ACCUM_COUNTS. */
lv_status lv_accum_counts(lv_accum* acc, uint32_t* out_counts, void* stream);
lv_status lv_accum_destroy(lv_accum* acc);

/* Work statistics of an accumulator since its creation or last reset
 * (synchronous): views processed, (tile, Gaussian) pairs, visible
 * (view, Gaussian) items, and -- only with LV_ACCUM_COUNTS, else -1 --
 * pixels with at least one counted Gaussian, counted (Gaussian, view,
 * pixel) contributions (the non-zeros of W) and partial sums: (Gaussian,
 * view, 8x8 pixel block) triples with a contribution, each of which the
 * blend adds to U, beta (and counts) with one atomic update per channel. */
typedef struct lv_uplift_stats {
    int64_t views, pairs, visible, covered_pixels, contributions, partial_sums;
} lv_uplift_stats;
lv_status lv_accum_stats(lv_accum* acc, lv_uplift_stats* out);

/* Benchmark timing of the blend-and-accumulate and forward-render kernels:
 * after lv_profile_start, every blend launch (uplift) and render launch
 * (lv_render) is bracketed by HIP events on its stream; lv_profile_stop waits for them and returns the number of launches,
 * their summed duration in milliseconds and, in per_launch_ms (host, nullable,
 * `capacity` entries), each launch's duration in launch order.
 * Process-wide. */
lv_status lv_profile_start(void);
lv_status lv_profile_stop(int64_t* launches, double* total_ms, double* per_launch_ms,
                          int64_t capacity);

/* ---------------------------------------------------------- storage codec -- */
/* Encode one FP32 map src [pixels][D] (device) into dst (device) of dtype:
 * LV_BF16 rounds to nearest even; LV_FP8_E4M3 computes, per channel,
 * scale = absmax / 448 (1 where the channel is all zero) into scales [D]
 * (device FP32) and stores the saturating round-to-nearest-even E4M3 code
 * of x / scale.  LV_F32 copies. */
lv_status lv_encode(const float* src, int64_t pixels, int32_t D, lv_dtype dtype, void* dst,
                    float* scales, void* stream);
/* Encode one FP32 map src [H][W][D] (device, HWC) into dst (device) in
 * `dtype`: the element types and FP8 scales of lv_encode, in the HWC layout
 * (then the same as lv_encode with pixels = H W) or in the pixel-block
 * layout of the _PX8 types (dst then holds H ceil(W/8) D 8 elements, the
 * pixels past W zero, and must be aligned to 16 bytes (8 for FP8)).  The
 * blend reads a pixel-block map with one vector load per 8 pixels of a
 * channel instead of eight element loads.  Same errors as lv_encode, plus
 * H or W outside [0, 16384]. */
lv_status lv_encode_map(const float* src, int32_t H, int32_t W, int32_t D, lv_dtype dtype, void* dst,
                        float* scales, void* stream);

/* lv_encode without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as lv_encode, except that the
 * FP8 per-channel absmax lives in a static device array of 4096 uint32 (16 KiB,
 * held by each GPU the library runs on until the process ends): D must be in
 * [1, 4096], else LV_ERR_INVALID_ARG.  Every call on one GPU shares that array
 * (it is cleared at the start of each FP8 call, on the caller's stream), so
 * FP8 calls that overlap on one GPU (different streams, no ordering) race;
 * calls on one stream are ordered and safe.  LV_BF16 and LV_F32 use no
 * scratch. */
lv_status lv_encode_noalloc(const float* src, int64_t pixels, int32_t D, lv_dtype dtype, void* dst,
                            float* scales, void* stream);

/* -------------------------------------------------------------- diffusion -- */
/* Sec. 3.3: a graph A over the n Gaussians as CSR (row_ptr [n+1], col [nnz]
 * int32, val [nnz] of val_dtype = LV_F32 or LV_BF16), device arrays copied by
 * the call.  Columns must be in [0, n).  Errors: LV_ERR_INVALID_ARG. */
lv_status lv_graph_create_csr(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                              const void* val, lv_dtype val_dtype, void* stream, lv_graph** out);
lv_status lv_graph_destroy(lv_graph* graph);

/* The diffusion graph built on the device (Sec. 3.3: a weighted graph
 * joining each Gaussian to its spatial neighbours, symmetrised by the union
 * of the directed kNN pairs).  Each centre of the scene is joined to its k
 * nearest other centres, ordered by (squared distance, index) with squared
 * distances in FP64 as ((dx dx + dy dy) + dz dz) of the FP32 centres; a
 * pair's weight is exp(-|x_i - x_j|^2 / sigma^2) * max(0, cos(f_i, f_j))
 * (FP64), sigma the median of the n k directed distances, the larger
 * directed weight where both directions exist; the union pairs with a
 * positive weight are stored, columns ascending; rows are normalised to sum
 * 1 (FP32 values) and a row without any gets a self-loop of weight 1.
 * feats: device FP32 [n][D] (e.g. uplifted features).  Scratch (about
 * 60 + 36 k bytes per Gaussian) comes from the stream-ordered allocator; the
 * call synchronises the stream once (to size the CSR).  Errors:
 * LV_ERR_INVALID_ARG (k outside [1, 32], D outside [1, 4096], n <= k, null
 * pointers), LV_ERR_UNSUPPORTED (n (2k + 1) >= 2^31), LV_ERR_OUT_OF_MEMORY,
 * LV_ERR_DEVICE. */
typedef enum lv_graph_kind {
    LV_GRAPH_SPATIAL_COSINE = 0,  /* the weights above */
    LV_GRAPH_FEATURE_RBF = 1      /* Eq. 7 with Eq. 9, see lv_graph_opts */
} lv_graph_kind;
/* opts NULL: LV_GRAPH_SPATIAL_COSINE.  LV_GRAPH_FEATURE_RBF (the paper's
 * weights, Eq. 7 with the feature kernel of Eq. 9, appendix on diffusion
 * for segmentation): A_ij = exp(-|g_i - g_j|^2 / (b s_f^2)) (sqrt(P_i)
 * sqrt(P_j)) on the same union pairs, g the l2-normalised features (a zero
 * feature stays 0), s_f the median of |g_i - g_j| over the n k directed
 * kNN pairs, b = bandwidth > 0, P = unary (device FP32 [n], >= 0; NULL: 1);
 * FP64, stored FP32, no row normalisation, no self-loops (a row may be
 * empty); pairs with weight 0 are not stored, and with binarize > 0 only the
 * pairs whose weight exceeds binarize are stored, with value 1. */
typedef struct lv_graph_opts {
    int32_t kind;
    float bandwidth;
    const float* unary;
    float binarize;
} lv_graph_opts;
lv_status lv_graph_build_knn(lv_scene* scene, const float* feats, int32_t D, int32_t k,
                             const lv_graph_opts* opts, void* stream, lv_graph** out);
/* Size of a graph (n, nnz: nullable) and, where the pointers are not NULL,
 * copies of its CSR arrays into caller device buffers (row_ptr [n+1], col
 * [nnz] int32, val [nnz] of the graph's value dtype), on the stream. */
lv_status lv_graph_csr(const lv_graph* graph, int64_t* n, int64_t* nnz, int32_t* row_ptr, int32_t* col,
                       void* val, void* stream);

/* Eq. (8): `steps` diffusion steps g_{t+1} = A (g_t / ||g_t||_2), each of the
 * D channels normalised by its own norm (a zero-norm channel stays 0).
 * g0 and out are device [n][D] of dtype (LV_F32 or LV_BF16; sums and norms
 * are FP32).  out = g_steps (steps = 0 copies g0).  scene may be NULL; if
 * given, its size must equal the graph's.  Scratch: 2 n D FP32 + 2 D FP32. */
lv_status lv_diffuse(const lv_scene* scene, const lv_graph* graph, const void* g0, lv_dtype dtype,
                     int32_t D, int32_t steps, void* out, void* stream);

/* ---------------------------------------------------------------- render -- */
/* Eq. (4): the forward render F^ = W g of per-Gaussian features, the map the
 * uplift is the normalised transpose of.  g: device FP32 [n][D]; outs: host
 * array [m] of device FP32 [H_v][W_v][D] outputs, F^(p) = sum_i w_i(p) g_i;
 * alphas: host array [m] (nullable, entries nullable) of device FP32
 * [H_v][W_v], the accumulated opacity sum_i w_i(p).  The weights are those of
 * the uplift (same structure and walk).  D in [1, 4096]; every output pixel
 * is written (0 where no Gaussian counts).  Errors as lv_uplift. */
lv_status lv_render(lv_scene* scene, const lv_camera* cams, int32_t m, const float* g, int32_t D,
                    float* const* outs, float* const* alphas, void* stream);

/* -------------------------------------------------------------- serving -- */
/* A request server for uplift (Eq. 3 / Eq. 5) over resident scenes.  Of
 * hbm_budget, workers x scratch_bytes are set aside for the workers' scratch
 * (structure builds and pair buffers, whose chunks are sized to fit it);
 * requests are admitted first come, first served while the memory they need
 * (their accumulators, n (D + 2) x 4 bytes) fits in the rest; a request
 * larger than the rest is refused.  Each of `workers` threads runs one pass
 * at a time on its own HIP stream, so passes overlap on the device; a free
 * worker takes the oldest admitted request and merges into the same pass the
 * other admitted requests on the same scene with the same storage dtype (at
 * most max_sets requests and max_channels channels): one structure build and
 * one blend walk over the union of their views, each request adding only its
 * own views (FP8 requests with their scales rearranged to the union's
 * views).  If a merged pass fails, each of its requests runs again alone, so
 * a request's status is its own.  Memory of finished passes returns to the
 * budget at once, admitting waiting requests while other passes run.  Each
 * result equals lv_uplift of that request alone (within FP32 accumulation
 * order).  A worker's scratch is freed when the server is destroyed. */
typedef struct lv_server lv_server;
typedef struct lv_server_opts {
    int64_t hbm_budget;     /* bytes; <= 0: half of the free device memory */
    int32_t workers;        /* passes in flight, 1..8 (0: 2) */
    int32_t max_sets;       /* requests per pass, 1..8 (0: 8) */
    int32_t max_channels;   /* channels per pass (0: 1024) */
    int32_t reserved;       /* must be 0 */
    int64_t scratch_bytes;  /* per worker; <= 0: 4 GiB */
} lv_server_opts;
/* One request: as lv_uplift, plus the pixel stride of its maps (0 = D), a
 * caller tag and the stream that produces its inputs: the pass waits for the
 * work enqueued on `stream` before the submission (an event recorded at
 * submission; NULL: the null stream).  cams and the maps table are copied at
 * submission; the scene, the maps, scales and outputs must stay valid until
 * the request completes. */
typedef struct lv_request {
    lv_scene* scene;
    const lv_camera* cams;
    int32_t m;
    const void* const* maps;
    int32_t stride;
    lv_dtype dtype;
    const float* scales;
    int32_t D;
    float* out_feat;
    float* out_wsum;
    uint64_t tag;
    void* stream;
} lv_request;
/* A finished request: status, the number of requests in its pass, times in
 * ns since the server was created (submission, admission within the
 * budget, start and end of its pass; the outputs are complete at t_end;
 * t_admit is 0 for a request cancelled before admission, t_start and t_end
 * its cancellation), the memory it was admitted with, D and its number of
 * views. */
typedef struct lv_completion {
    uint64_t tag;
    int32_t status;
    int32_t batch_size;
    int64_t t_submit, t_start, t_end;
    int64_t t_admit, bytes;
    int32_t D, views;
} lv_completion;
/* peak_bytes: the most request memory admitted at once (<= budget less the
 * workers' scratch); peak_device_bytes: the largest device memory in use
 * (hipMemGetInfo, sampled at every pass's start and end) above what was in
 * use when the server was created. */
typedef struct lv_server_stats {
    int64_t submitted, completed, passes, peak_bytes, budget, cancelled, peak_device_bytes;
} lv_server_stats;
lv_status lv_server_create(const lv_server_opts* opts, lv_server** out);
/* Non-blocking.  LV_ERR_INVALID_ARG for a malformed request,
 * LV_ERR_OUT_OF_MEMORY if it can never fit the budget. */
lv_status lv_server_submit(lv_server* srv, const lv_request* req);
/* Moves up to cap completions into out (oldest first); *n receives the count. */
lv_status lv_server_poll(lv_server* srv, lv_completion* out, int32_t cap, int32_t* n);
/* Blocks until every submitted request has completed. */
lv_status lv_server_drain(lv_server* srv);
/* Cancels the request with this tag if it has not started: it completes at
 * once with status LV_ERR_CANCELLED and its memory returns to the budget.
 * LV_ERR_INVALID_ARG if no waiting request has the tag (unknown, running or
 * finished). */
lv_status lv_server_cancel(lv_server* srv, uint64_t tag);
lv_status lv_server_stats_get(lv_server* srv, lv_server_stats* out);
/* Drains, stops the workers and frees the server. */
lv_status lv_server_destroy(lv_server* srv);

/* ------------------------------------------------------------ inspection -- */
/* Per-view structure for verification; synchronous.  Host buffers (each
 * nullable): visible [n], depth [n] (FP32 bits of z_c), rect [n][4]
 * (x0,y0,x1,y1 tile rectangle), rec [n][8] (ux, uy, ux_lo, uy_lo, L11, L12,
 * L22, opacity: the centre is ux + ux_lo, uy + uy_lo, the exponent
 * -((L11 dx + L12 dy)^2 + (L22 dy)^2)), tile_start [tiles+1] and ids
 * [ids_capacity] (per tile, Gaussian indices in blending order).  *P_out
 * receives the number of (tile, Gaussian) pairs; ids is filled only when
 * ids_capacity >= P. */
typedef struct lv_view_debug {
    uint8_t* visible;
    uint32_t* depth;
    int32_t* rect;
    float* rec;
    int64_t* tile_start;
    int32_t* ids;
    int64_t ids_capacity;
} lv_view_debug;
lv_status lv_debug_view(lv_scene* scene, const lv_camera* cam, lv_view_debug* out, int64_t* P_out);

#ifdef __cplusplus
}
#endif
#endif /* LV_H */
