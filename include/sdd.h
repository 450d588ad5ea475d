/*
 * sdd.h -- spectral domain-decomposition ray tracing on MI355X (gfx950).
 *
 * C ABI of the HIP library libsdd.so.  The library renders a lit room by
 * spectral Monte-Carlo path tracing:
 *   - ray / triangle traversal over per-subdomain BVHs (inverse ray tracing,
 *     Sec. 4 of the paper: primary ray per pixel, one shadow ray per vertex
 *     toward the light, secondary reflection / refraction rays, a bounce cap);
 *   - per-wavelength light / material interaction: Lambert reflection and a
 *     glass pane whose Fresnel terms come from the complex index
 *     n(lambda) + i k(lambda) (Eq. 1), with incoherent slab transmittance and
 *     Beer-Lambert absorption (Sec. 6, "direct use of the Fresnel definition");
 *   - the paper's spatial domain decomposition (Sec. 5): the scene is split
 *     into a uniform grid of subdomains, each with its own BVH; a ray is
 *     traced inside one subdomain over the parameter interval (t_enter, t_exit]
 *     and, if it finds nothing, is handed across the interface to the
 *     neighbouring subdomain with its origin, direction and t carried
 *     unchanged (the interface condition "continuity of the ray properties").
 *     On one GPU the subdomains become per-subdomain ray queues in HBM.
 *
 * Conventions for every entry point:
 *   - status codes only; nothing throws across the ABI and nothing aborts;
 *   - on failure, sdd_last_error(ctx) describes the cause (ctx-owned string,
 *     valid until the next call on that context);
 *   - a context is not thread-safe; separate contexts are independent;
 *   - all input pointers are host pointers unless stated otherwise; inputs
 *     are deep-copied and stay owned by the caller;
 *   - the context owns all device memory it allocates (scene, BVHs, queues,
 *     path state, accumulators); sdd_destroy releases it.
 * Call order: sdd_create -> sdd_load_scene -> sdd_build_bvh ->
 *   sdd_trace_spectral* -> sdd_resolve_image.  Out of order: SDD_ERR_STATE.
 */
#ifndef SDD_H
#define SDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SDD_OK = 0,
    SDD_ERR_INVALID_ARG = -1,
    SDD_ERR_STATE = -2,
    SDD_ERR_OOM = -3,
    SDD_ERR_HIP = -4,
    SDD_ERR_OVERFLOW = -5,
    SDD_ERR_UNSUPPORTED = -6
} sdd_status;

enum { SDD_MAT_DIFFUSE = 0, SDD_MAT_GLASS_SLAB = 1, SDD_MAT_EMITTER = 2 };
enum { SDD_LIGHT_NONE = 0, SDD_LIGHT_PARALLELOGRAM = 1, SDD_LIGHT_POINT = 2 };

/* Limits (checked; exceeding one returns SDD_ERR_INVALID_ARG). */
#define SDD_MAX_LAMBDA 128
#define SDD_MAX_CELLS 512
#define SDD_MAX_DEPTH 64
#define SDD_MAX_LAYERS 8
#define SDD_MAX_RENDERS 256

typedef struct sdd_ctx sdd_ctx;

/*
 * Scene (sdd_load_scene).  Host arrays, row-major:
 *   verts     float  [n_verts][3]  metres
 *   tris      int32  [n_tris][3]   vertex indices in [0, n_verts)
 *   tri_mat   int32  [n_tris]      material index in [0, n_mats)
 *   lambda_nm float  [n_lambda]    wavelengths (nm), > 0
 *   lambda_w  double [n_lambda]    integration weights for the XYZ reduction
 *   cmf       double [n_lambda][3] colour matching functions
 *   mat_type  int32  [n_mats]      SDD_MAT_*
 *   mat_rho   float  [n_mats][n_lambda] diffuse reflectance in [0, 1]
 *   mat_n     float  [n_mats][n_lambda] real index n > 0        (Eq. 1)
 *   mat_k     float  [n_mats][n_lambda] absorption index k >= 0 (Eq. 1, k = n kappa)
 *   mat_thick float  [n_mats]      slab thickness (m) of GLASS_SLAB panes, >= 0
 *   mat_le    float  [n_mats][n_lambda] emitted radiance >= 0 (EMITTER: one-sided,
 *                                  counted per the NEE rule; DIFFUSE: two-sided,
 *                                  always counted; GLASS: must be 0)
 * Light (one at most): PARALLELOGRAM {p0, e1, e2} emits mat_le[light_mat] on
 *   the side of e1 x e2 (its triangles must also be in tris with an EMITTER
 *   material); POINT {p0} with intensity mat_le[light_mat] (Eq. 3).
 * Optional coatings (electrochromic windows; all NULL and max_layers = 0 for
 * none): a GLASS_SLAB material m may carry mat_n_layers[m] coherent thin
 * films on the face its triangles' geometric normal (v1 - v0) x (v2 - v0)
 * points out of, listed from the air side:
 *   max_layers   Lm in [0, SDD_MAX_LAYERS]
 *   mat_n_layers int32 [n_mats]          in [0, Lm] (0 for non-glass)
 *   mat_layer_d  float [n_mats][Lm]      thickness (m), >= 0
 *   mat_layer_n  float [n_mats][Lm][n_lambda]  n > 0
 *   mat_layer_k  float [n_mats][Lm][n_lambda]  k >= 0
 * The pane's R and T then come from the layers' characteristic (transfer)
 * matrices combined incoherently with the substrate (see sdd_debug_glass).
 */
typedef struct sdd_scene_desc {
    int32_t n_verts;
    const float *verts;
    int32_t n_tris;
    const int32_t *tris;
    const int32_t *tri_mat;
    int32_t n_lambda;
    const float *lambda_nm;
    const double *lambda_w;
    const double *cmf;
    int32_t n_mats;
    const int32_t *mat_type;
    const float *mat_rho;
    const float *mat_n;
    const float *mat_k;
    const float *mat_thick;
    const float *mat_le;
    int32_t light_type;
    float light_p0[3], light_e1[3], light_e2[3];
    int32_t light_mat;
    int32_t max_layers;
    const int32_t *mat_n_layers;
    const float *mat_layer_d;
    const float *mat_layer_n;
    const float *mat_layer_k;
} sdd_scene_desc;

/*
 * Subdomain grid and BVHs (sdd_build_bvh).  The scene's bounding box (light
 * included, slightly enlarged) is split into nx * ny * nz equal cells (the
 * paper's sub-domains, Sec. 5); every triangle is referenced in each cell
 * its padded bounding box overlaps, and each cell gets its own binned-SAH
 * BVH over its references.  nx = ny = nz = 1 is the undecomposed special case.
 *   leaf_max  triangles per leaf (1..8, 0 = default 3)
 *   sah_bins  SAH bins (2..64, 0 = default 16)
 */
typedef struct sdd_bvh_desc {
    int32_t nx, ny, nz;
    int32_t leaf_max;
    int32_t sah_bins;
    int32_t device_build;  /* nonzero: build the references and BVHs on the GPU
                              (linear BVH per cell from Morton-sorted reference
                              centroids, Karras 2012; sah_bins unused) */
} sdd_bvh_desc;

/* sdd_trace_desc.flags */
#define SDD_TRACE_ORTHO 1u        /* rays orthogonal to the image plane (Sec. 4) */
#define SDD_TRACE_TIME_KERNELS 2u /* time every launch with HIP events (stats) */
#define SDD_TRACE_COUNT_WORK 4u   /* count node visits / triangle tests (stats) */
#define SDD_TRACE_NRC 8u          /* radiance-cache estimator (see sdd_nrc_desc); one render per call */
#define SDD_TRACE_GRAPH 16u       /* capture the call's launches in a HIP graph; later calls with the
                                     same descs except sample_offset replay it (any reallocation, new
                                     render, reset or new scene/BVH recaptures).  Needs a context
                                     stream other than NULL; excludes NRC and TIME_KERNELS
                                     (SDD_ERR_UNSUPPORTED).  Same result as without it. */

/*
 * One call traces spp samples of every pixel of render render_id and adds
 * them to that render's FP32 spectral accumulator (created on first use
 * with this W, H; later calls must use the same W, H).  Sample s of pixel
 * p = py * W + px (py = 0 is the top row) draws its random numbers from
 * Philox4x32-10 with key (seed, render_id) and counter (p, s, depth, block),
 * s in [sample_offset, sample_offset + spp), so calls split or resumed over
 * sample ranges give the same result.  The call is stream-ordered and
 * asynchronous with respect to the host.
 *   eye, target, fov_deg: pinhole camera (up = +z); with SDD_TRACE_ORTHO the
 *     image plane is 2 ortho_half_h tall and rays are parallel.
 *   max_depth: surface vertices per path (1..SDD_MAX_DEPTH).
 *   hit_log / shadow_log: optional DEVICE int32 buffers [W*H][spp][max_depth]
 *     (this call's samples).  hit_log gets the hit triangle id of each vertex,
 *     -1 for a miss, -2 where the path had ended; shadow_log gets 1 (visible),
 *     0 (blocked) or -2 (no shadow ray) per vertex.  NULL to skip.
 *   glass_from, glass_to: material substitution for this render (photochromic
 *     states): pane triangles of GLASS_SLAB material glass_from are traced as
 *     GLASS_SLAB material glass_to.  Inactive when equal (e.g. both 0).
 *   crop_x0, crop_y0, crop_w, crop_h: a window of the W x H frame (all 0: the
 *     whole frame).  Only its pixels are traced; each keeps the camera ray and
 *     the random numbers of its place p in the frame, so a window's pixels
 *     equal the same pixels of a whole-frame render.  The render's
 *     accumulator, the logs and sdd_resolve_image then cover the window
 *     ([crop_h][crop_w] pixels, row-major), and the render's paths (and the
 *     radiance cache's training paths, SDD_TRACE_NRC) are numbered over the
 *     window's pixels: sample s of window pixel i is path s * crop_w * crop_h + i.
 *     SDD_ERR_INVALID_ARG unless 0 <= crop_x0, crop_x0 + crop_w <= W, and
 *     likewise for y, with crop_w, crop_h both 0 or both > 0.
 * (window pixels) * spp must be below 2^31.
 */
typedef struct sdd_trace_desc {
    double eye[3], target[3];
    double fov_deg;
    double ortho_half_h;
    int32_t W, H;
    int32_t spp;
    int32_t sample_offset;
    int32_t max_depth;
    uint32_t seed;
    int32_t render_id;
    uint32_t flags;
    int32_t *hit_log;
    int32_t *shadow_log;
    int32_t glass_from, glass_to;
    int32_t crop_x0, crop_y0, crop_w, crop_h;
} sdd_trace_desc;

/* Counters (sdd_get_stats); synchronises the context stream. */
typedef struct sdd_stats {
    int64_t ext_rays;          /* closest-hit rays generated */
    int64_t shadow_rays;       /* shadow rays generated */
    int64_t ext_cell_visits;   /* (ray, subdomain) traversals, closest-hit */
    int64_t shadow_cell_visits;/* (ray, subdomain) traversals, shadow */
    int64_t node_visits;       /* BVH inner nodes visited (SDD_TRACE_COUNT_WORK) */
    int64_t tri_tests;         /* ray / triangle tests (SDD_TRACE_COUNT_WORK) */
    int64_t batches;           /* path batches launched */
    int64_t launches_trace;    /* subdomain traversal launches */
    double ms_trace_ext;       /* summed launch durations (SDD_TRACE_TIME_KERNELS) */
    double ms_trace_shadow;
    double ms_shade;
    double ms_other;
    int64_t n_refs;            /* triangle references over all cells */
    int64_t n_nodes;           /* 4-wide BVH nodes over all cells */
    int32_t max_bvh_depth;     /* depth of the binary hierarchy the builder made (before widening) */
    int32_t n_cells;
    int64_t device_bytes;      /* device memory owned by the context */
    int64_t paths_per_batch;   /* paths per pipeline pass of the last trace call */
    int32_t overflow;          /* bits raised since sdd_reset_stats: 1 a shadow segment crossed
                                  more glass panes than are tracked (4), 2 a subdomain queue count
                                  exceeded its capacity (not expected: counts are bounded) */
    int32_t pad_;
    double ms_nrc_query;       /* cache-network launches of SDD_TRACE_NRC renders (SDD_TRACE_TIME_KERNELS;
                                  with BF16 queries the matrix-core kernel alone, its operand gathers
                                  count in ms_other) */
    double ms_nrc_train;       /* cache training after those renders (SDD_TRACE_TIME_KERNELS) */
    int64_t nrc_query_rows;    /* (path, wavelength) cache queries */
    int64_t nrc_query_launches;
    int64_t nrc_train_rows;    /* rows of the Adam steps */
    int64_t wave_node_steps;   /* node steps of traversal waves, counted once per wave however many
                                  of its lanes took one (SDD_TRACE_COUNT_WORK): node_visits /
                                  (64 wave_node_steps) is the node loop's lane utilisation */
    int64_t wave_tri_steps;    /* triangle-test steps of traversal waves, likewise (SDD_TRACE_COUNT_WORK) */
} sdd_stats;

/* Create a context on HIP device hip_device.  hip_stream is the hipStream_t
 * every launch and copy of the context goes to (NULL = the device's default
 * null stream); the caller keeps ownership of a stream it passes.  *out is
 * set on success. */
sdd_status sdd_create(int hip_device, void *hip_stream, sdd_ctx **out);

/* Release every device allocation of ctx.  NULL-safe. */
void sdd_destroy(sdd_ctx *ctx);

/* Description of the last failure on ctx ("" if none; "null context" for NULL). */
const char *sdd_last_error(const sdd_ctx *ctx);

/* Validate and deep-copy a scene to the device (Eq. 1 tables per material).
 * Invalidates any previous BVH and renders.  SDD_ERR_INVALID_ARG on: no
 * triangles, an index out of range, a non-finite vertex, n_lambda out of
 * [1, SDD_MAX_LAMBDA], rho outside [0, 1], n <= 0, k < 0, thickness < 0,
 * negative emission, emission on glass, a light without a valid emitter
 * material, or a degenerate parallelogram light. */
sdd_status sdd_load_scene(sdd_ctx *ctx, const sdd_scene_desc *scene);

/* Host-only argument check of a scene (no device needed); same rules as
 * sdd_load_scene.  msg (may be NULL) receives a NUL-terminated reason. */
sdd_status sdd_validate_scene(const sdd_scene_desc *scene, char *msg, int msg_len);

/* Build the subdomain grid and the per-subdomain BVHs (host), upload them.
 * SDD_ERR_STATE without a scene; SDD_ERR_INVALID_ARG for grid dims <= 0, more
 * than SDD_MAX_CELLS cells, or leaf_max / sah_bins out of range. */
sdd_status sdd_build_bvh(sdd_ctx *ctx, const sdd_bvh_desc *desc);

/* Trace (asynchronously) and accumulate; see sdd_trace_desc.  This is the
 * paper's rendering step: inverse ray tracing with a primary ray per pixel, a
 * shadow ray toward the light at every diffuse vertex and a reflected or
 * transmitted secondary ray, up to a bounce cap (Sec. 4; Eq. 2 estimated by
 * Monte-Carlo paths, Eq. 3 for the light sample), glass panes through their
 * Fresnel terms of n + i k (Eq. 1, Sec. 6), and every ray traced subdomain by
 * subdomain with its state handed across the interfaces (Sec. 5).
 * SDD_ERR_STATE without a BVH; SDD_ERR_INVALID_ARG for W, H, spp, max_depth
 * out of range, a render_id < 0, a changed W/H for an existing render, or a
 * degenerate camera (forward direction parallel to +z or eye == target). */
sdd_status sdd_trace_spectral(sdd_ctx *ctx, const sdd_trace_desc *desc);

/* Several renders in one pass of the pipeline (n in 1..SDD_MAX_RENDERS, all
 * with the same max_depth and distinct render_ids): their paths share the
 * per-subdomain queues and every traversal sweep, so many small or uneven
 * renders fill the GPU together.  Each render is traced exactly as
 * sdd_trace_spectral would trace it alone (same random numbers, same
 * result); TIME_KERNELS / COUNT_WORK apply if any desc sets them. */
sdd_status sdd_trace_batch(sdd_ctx *ctx, int32_t n, const sdd_trace_desc *descs);

/* Launch settings of the pipeline.  They change speed only: every setting
 * traces the same paths with the same random numbers, so images are
 * bit-identical under any of them.  0 in a field selects the library's
 * own choice.
 *   batch_paths  paths per pipeline pass, which is also the capacity of each
 *                subdomain queue; 0 = as many as the memory budget holds
 *                (SDD_MEM_BUDGET_GB if set, else half the device's memory,
 *                at most 3/4 of what is free plus what the context's batch
 *                holds, at least 4 GiB), else a multiple of 512 in
 *                [512, 2^24]; a call with more paths runs several passes
 *   trace_grid   traversal workgroups per sweep launch; 0 = all that stay
 *                resident on the device, else a multiple of 8 (one share per
 *                XCD) up to that resident maximum
 *   dir_bins     direction bins per subdomain when closest-hit rays are
 *                queued: 0 = 4 (signs of the direction's x and y) whenever
 *                4 x cells <= SDD_MAX_CELLS, 1 = cell only, 4 = as 0 */
typedef struct sdd_tuning {
    int64_t batch_paths;
    int32_t trace_grid;
    int32_t dir_bins;
} sdd_tuning;

/* Host-only check of the field ranges above (no device needed); msg (may be
 * NULL) receives a NUL-terminated reason.  SDD_ERR_INVALID_ARG if malformed. */
sdd_status sdd_validate_tuning(const sdd_tuning *t, char *msg, int msg_len);

/* Apply t to later calls (waits for the context's stream first).
 * SDD_ERR_INVALID_ARG for a malformed t or a trace_grid above the resident
 * maximum.  A captured SDD_TRACE_GRAPH sequence is recaptured. */
sdd_status sdd_set_tuning(sdd_ctx *ctx, const sdd_tuning *t);

/* Deferral of small subdomain queues, after the load-balancing rule of
 * Sec. 5 (a processor leaves a subdomain with few rays left while other
 * subdomains hold many, and comes back to it later).  On one device every
 * subdomain stays resident, so the rule becomes: in a sweep, the queue of a
 * subdomain holding fewer than below_rays rays of one kind waits for the
 * next sweep (its rays are carried over unchanged) as long as even its
 * worst-placed ray still drains within the depth's sweeps; extra_sweeps
 * (0..4) sweeps per depth are added to the S = nx + ny + nz - 2 that drain
 * every queue without deferral.  below_rays = 0 (the default) turns it off.
 * Images, logs and counters are unchanged by it (a ray's traversal does not
 * depend on when it runs).  Waits for the context's stream; a captured
 * SDD_TRACE_GRAPH sequence is recaptured.  SDD_ERR_INVALID_ARG for
 * below_rays < 0 or extra_sweeps outside 0..4. */
sdd_status sdd_set_deferral(sdd_ctx *ctx, int32_t below_rays, int32_t extra_sweeps);

/* Settings in force: batch_paths as requested (0 = from the budget; the
 * paths per pass of the last call are in sdd_stats.paths_per_batch), trace_grid and
 * dir_bins as launched (0 before sdd_build_bvh). */
sdd_status sdd_get_tuning(sdd_ctx *ctx, sdd_tuning *out);

/* Search launch settings for a call shaped like descs (as sdd_trace_batch
 * takes them) by timing that call on the device: direction bins, then the
 * traversal grid (all, 3/4, 1/2 of the resident workgroups), then the paths
 * per pass (the budget's, 1/2, 1/4), each candidate as one untimed and reps
 * (1..100) timed calls, keeping a candidate only if it is more than 1% faster.
 * The winner is applied as by sdd_set_tuning; *out receives it, *ms_out (may
 * be NULL) the time of one call under it.
 * With SDD_TUNE_VERBOSE set in the environment each candidate's time is
 * printed to stderr.
 * cache_path (may be NULL or ""): a text file of earlier results, one line per
 * key of sdd_tune_key; a result found there is applied without any timing
 * (*from_cache = 1), and a new result is stored there.
 * The search's calls are discarded: the render ids of descs must not hold
 * samples (SDD_ERR_STATE otherwise) and hold none afterwards.
 * SDD_ERR_UNSUPPORTED for SDD_TRACE_NRC (the calls would train the cache);
 * SDD_ERR_INVALID_ARG for hit or shadow logs; SDD_ERR_STATE if the file
 * cannot be written (the result is still applied). */
sdd_status sdd_autotune(sdd_ctx *ctx, int32_t n, const sdd_trace_desc *descs, int32_t reps, const char *cache_path,
                        sdd_tuning *out, double *ms_out, int32_t *from_cache);

/* The results-file key of a call shaped like descs: device name and compute
 * units, library build, scene size, subdomain grid, render count, total paths,
 * max_depth and the COUNT_WORK / GRAPH flags.  out: host buffer of out_len
 * bytes (SDD_ERR_INVALID_ARG if too small).  SDD_ERR_STATE before a BVH. */
sdd_status sdd_tune_key(sdd_ctx *ctx, int32_t n, const sdd_trace_desc *descs, char *out, int32_t out_len);

/* Host-only access to a results file.  lookup: *found = 1 and *out (and *ms,
 * may be NULL) from the last well-formed line of key, else *found = 0 (also
 * for a missing file).  store: replaces the key's lines by one new line,
 * through a temporary file renamed over path; SDD_ERR_INVALID_ARG for a key
 * with a tab or newline, a malformed t or ms < 0, SDD_ERR_STATE if the file
 * cannot be written. */
sdd_status sdd_tune_cache_lookup(const char *path, const char *key, sdd_tuning *out, double *ms, int32_t *found);
sdd_status sdd_tune_cache_store(const char *path, const char *key, const sdd_tuning *t, double ms);

/* Gathering of the results (Sec. 5): per-pixel mean radiance of render_id
 * over all samples traced so far, in FP64: spectral_out [H][W][n_lambda] and
 * xyz_out [H][W][3] (XYZ = sum_l lambda_w[l] cmf[l][:] L[l]).  Either may be
 * NULL.  Pointers are device pointers if out_is_device, else host pointers;
 * the caller owns them.  Synchronises the stream.  SDD_ERR_STATE for an
 * unknown render or one with no samples; SDD_ERR_OVERFLOW (the outputs are
 * written but not trustworthy) if a call that traced this render saw a shadow
 * segment cross more glass panes than the library tracks, or a queue count
 * above its capacity; sdd_last_error names which.  Other renders of the
 * context are not affected. */
sdd_status sdd_resolve_image(sdd_ctx *ctx, int32_t render_id, double *spectral_out, double *xyz_out,
                             int32_t out_is_device);

/* Forget render_id's accumulator (frees its device memory). */
sdd_status sdd_reset_render(sdd_ctx *ctx, int32_t render_id);

/* Copy the context counters (synchronises the stream). */
sdd_status sdd_get_stats(sdd_ctx *ctx, sdd_stats *out);

/* Zero the counters of sdd_get_stats (not the scene / BVH statistics). */
sdd_status sdd_reset_stats(sdd_ctx *ctx);

/* Diagnostics: evaluate the library's own device Philox4x32-10 on n counters.
 * ctr: host uint32 [n][4]; key: host uint32 [2]; out: host uint32 [n][4]. */
sdd_status sdd_debug_philox(sdd_ctx *ctx, int32_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out);

/* Diagnostics: the library's own polarisation-averaged pane reflectance R
 * and transmittance T (Fresnel terms of n + i k, Eq. 1; incoherent slab with
 * Beer-Lambert absorption) for n parameter rows params [n][5] =
 * (n, k, thickness m, wavelength nm, incidence cosine).  Host arrays. */
sdd_status sdd_debug_pane(sdd_ctx *ctx, int32_t n, const float *params, float *R_out, float *T_out);

/* Diagnostics: closest hits of n rays through the subdomain queues (the same
 * kernels as sdd_trace_spectral's extension phase).  o, d: host float [n][3];
 * t_out: host float [n] (+inf on a miss); prim_out: host int32 [n] (-1). */
sdd_status sdd_debug_trace_rays(sdd_ctx *ctx, int32_t n, const float *o, const float *d, float *t_out,
                                int32_t *prim_out);

/* Device evaluation of the loaded scene's glass terms, exactly as the path
 * uses them (Eq. 1; Sec. 6 slab; coated panes by characteristic matrices
 * combined incoherently with the substrate, polarisation-averaged).  For
 * i < n: material mat[i] (must be GLASS_SLAB), wavelength index lam[i],
 * signed incidence cosine cs[i] (|cs| = cos theta; cs > 0: the light
 * arrives on the face the geometric normal points out of, the coated face).
 * Host arrays; R_out, T_out: host float [n]. */
sdd_status sdd_debug_glass(sdd_ctx *ctx, int32_t n, const int32_t *mat, const int32_t *lam, const float *cs,
                           float *R_out, float *T_out);

/*
 * Learned radiance cache: a small network L(x, w, lambda) trained online on
 * radiance estimates the tracer produces (neural radiance caching, Mueller,
 * Rousselle, Novak, Keller 2021; multiresolution hash encoding, Mueller,
 * Evans, Schied, Keller 2022).  One cache per context.
 *   input   hash encoding of the position normalised to the box
 *           [aabb_lo, aabb_hi] (16 levels, resolutions floor(16 b^l) with
 *           b = exp(ln(2048 / 16) / 15), 2^table_log2 entries of 2 features
 *           per level, direct indexing where (N + 1)^3 fits the table, else
 *           the spatial hash with primes 1, 2654435761, 805459861), real
 *           spherical harmonics of the unit direction (bands 0..3, 16 values)
 *           and a one-blob encoding of the wavelength over
 *           [lambda_lo, lambda_hi] (16 Gaussian bins);
 *   network 5 hidden ReLU layers of 64, one linear output;
 *   loss    relative L2, mean of (y - t)^2 / (y^2 + 0.01), y^2 held constant;
 *   update  Adam (lr, beta1, beta2, eps).
 * Parameters: one flat FP32 array of sdd_nrc_param_count(table_log2) values,
 *   tables [16][T][2] | W [5][64][64] (out, in) | b [5][64] | wo [64] | bo [1].
 */
typedef struct sdd_nrc_desc {
    int32_t table_log2;            /* T = 2^table_log2, 10..24 */
    float aabb_lo[3], aabb_hi[3];  /* position box, hi > lo per axis */
    float lambda_lo, lambda_hi;    /* nm, hi > lo */
    float lr, beta1, beta2, eps;   /* lr > 0, 0 <= beta < 1, eps > 0 */
    const float *params;           /* host; initial parameters (copied) */
    /* renders with SDD_TRACE_NRC */
    int32_t train_paths;           /* training paths per call (>= 1) */
    int32_t train_steps;           /* Adam steps after each call (>= 0) */
    int32_t train_batch;           /* rows per step, 1..2^22 */
    int32_t precision;             /* cache queries: 0 FP32, 1 BF16 matrix cores */
    int32_t table_fp16;            /* 1: BF16 queries and BF16 rows gather the hash features from an FP16
                                      copy of the tables (round to nearest, refreshed after every Adam
                                      step); the FP32 tables stay the training copy.  0: FP32 tables */
} sdd_nrc_desc;

/* Parameter count for a table size; -1 if table_log2 is out of range. */
int64_t sdd_nrc_param_count(int32_t table_log2);

/* (Re)create the cache with the given parameters; Adam moments start at
 * zero.  SDD_ERR_INVALID_ARG for a bad desc or non-finite parameters. */
sdd_status sdd_nrc_init(sdd_ctx *ctx, const sdd_nrc_desc *desc);

/* Network output of n rows, stream-ordered.  x, w: DEVICE float [n][3]
 * (positions, unit directions); lambda_nm: DEVICE float [n]; y: DEVICE
 * float [n].  precision 0: FP32 throughout; 1: BF16 matrix-core products
 * with FP32 accumulation (inputs and hidden activations rounded to BF16
 * where they enter a product; output layer in FP32).  SDD_ERR_STATE
 * without sdd_nrc_init. */
sdd_status sdd_nrc_infer(sdd_ctx *ctx, int32_t n, const float *x, const float *w, const float *lambda_nm, float *y,
                         int32_t precision);

/* One optimisation step on n rows (1 <= n <= 2^22) with targets t: the
 * loss's gradient over all parameters (FP32), then, if apply, one Adam step.
 * x, w, lambda_nm, t: DEVICE arrays as in sdd_nrc_infer.  loss: host float
 * (the batch loss before the update; the call then synchronises) or NULL
 * (asynchronous).  The gradient stays readable (sdd_nrc_get_params) until
 * the next step. */
sdd_status sdd_nrc_train_step(sdd_ctx *ctx, int32_t n, const float *x, const float *w, const float *lambda_nm,
                              const float *t, int32_t apply, float *loss);

/*
 * Rendering with the cache (sdd_trace_desc.flags |= SDD_TRACE_NRC).  Path
 * (p, s) is a training path when (s * W * H + p) % stride == 0, stride =
 * ceil(W * H * spp / train_paths); training paths are traced exactly as
 * without the cache.  Every other path ends at its first diffuse vertex x of
 * depth >= 2: emission and the light sample there are added as usual, then
 * beta(lambda) * L(x, n, lambda), beta the path throughput after the vertex's
 * Lambert factor, L the cache at the hit point with the geometric normal n
 * on the side the ray arrived from as its direction input.  Each diffuse
 * vertex of depth >= 2 of a training path that continues gives one training
 * row at one wavelength l drawn from Philox counter (p, s, depth, 3) (l =
 * word 0 mod n_lambda): target the radiance the path carries back into the
 * vertex along its continuation, at l, the same terms the estimator adds.
 * After the call, S = train_steps Adam steps run on the call's rows: step k
 * on rows (k + i S) m, i < train_batch, m = max(1, rows / (S train_batch)).
 * The rows are compacted and counted on the context's stream before the call
 * returns; the steps then run on a stream of the context's own (default
 * priority), ordered after the rows by an event, so they overlap the next
 * call's tracing.  The next cache render waits for them on the device before
 * its cache query; every sdd_nrc_* call, sdd_get_stats and sdd_reset_stats
 * wait for them on the host first.  Gradient sums use atomics, so trained
 * caches differ between runs by rounding.
 */

/* Cache values of n surface points at every wavelength of the loaded scene,
 * as a cache render queries them: x4, n4 DEVICE float [n][4] (position;
 * normal as the direction input; w ignored); out DEVICE float [n][nlp], nlp
 * = n_lambda rounded up to a multiple of 4 (entries past n_lambda are not
 * written).  precision as in sdd_nrc_infer.  SDD_ERR_STATE without a scene
 * or cache. */
sdd_status sdd_nrc_query(sdd_ctx *ctx, int32_t n, const float *x4, const float *n4, float *out, int32_t precision);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the BF16
 * query of sdd_nrc_query (precision 1), same arguments and the same result,
 * bit for bit, with no allocation of any kind.  Its scratch (operand staging,
 * the sort of the points by the Morton code of their position, the sort's
 * temporary storage) is one static device array of 12 MiB per GPU, kept
 * until the process ends.  Every call on a GPU shares that array, so calls
 * that overlap on one GPU (two streams, two contexts, two threads) race; the
 * caller orders them.  Nothing in it needs clearing between calls.
 * SDD_ERR_INVALID_ARG for n above SDD_NRC_NOALLOC_MAX_PATHS; otherwise as
 * sdd_nrc_query. */
#define SDD_NRC_NOALLOC_MAX_PATHS 65536
sdd_status sdd_nrc_query_noalloc(sdd_ctx *ctx, int32_t n, const float *x4, const float *n4, float *out);

/* The last cache render's training rows (compacted, in path order): rows
 * host float [max_rows][8] = (x, y, z, lambda_nm, n_x, n_y, n_z, target);
 * n_rows gets the row count, n_steps the Adam steps taken, loss the last
 * step's loss.  Any output pointer may be NULL.  Synchronises. */
sdd_status sdd_nrc_last_rows(sdd_ctx *ctx, int32_t max_rows, float *rows, int32_t *n_rows, int32_t *n_steps,
                             float *loss);

/* Copy a parameter-sized array to the host: which 0 parameters, 1 last
 * gradient of sdd_nrc_train_step (the Adam steps after a cache render leave
 * the gradients at zero), 2 Adam first moments, 3 second moments.
 * Synchronises. */
sdd_status sdd_nrc_get_params(sdd_ctx *ctx, int32_t which, float *out);

#ifdef __cplusplus
}
#endif
#endif
