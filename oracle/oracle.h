/*
 * FP64 CPU oracle for spectral ray tracing of a lit room -- TEST INFRASTRUCTURE.
 *
 * This library exists only to check the HIP path against.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant with the GPU library; both read the same
 * seeded scene arrays (scenegen/), which carry no rendering arithmetic.
 *
 * What it computes (plain definitions, in FP64, no decomposition):
 *  - complex refractive index n + i k (Eq. 1) and the Fresnel reflectance of
 *    an air / absorbing-dielectric interface for s and p polarisation;
 *  - the incoherent thick-slab reflectance / transmittance of a pane with
 *    Beer-Lambert absorption ("direct use of the Fresnel definition", Sec. 6);
 *  - for electrochromic windows (the paper's subject, Sec. 1), a coherent
 *    thin-film coating on one face by characteristic (transfer) matrices,
 *    combined incoherently with the substrate;
 *  - the global closest hit of a ray (Sec. 4, inverse ray tracing): with the
 *    spatial decomposition of Sec. 5 the ray is handed from subdomain to
 *    subdomain unchanged, so the closest hit over all visited subdomains is
 *    the global closest hit -- the oracle computes it directly, either by
 *    brute force over all triangles or with its own median-split BVH;
 *  - a Monte-Carlo spectral path tracer estimating the rendering equation
 *    (Eq. 2) with one shadow ray per vertex toward the light (Eq. 3 for a
 *    point light; uniform area sampling for the parallelogram emitter),
 *    cosine-weighted diffuse bounces, a glass reflect/transmit choice, and a
 *    fixed bounce cap (Sec. 4).
 *
 * Randomness: Philox4x32-10 (Salmon et al., SC'11) keyed by (seed, render_id)
 * with counter (pixel, sample, depth, block); every 32-bit output x maps to
 * (x >> 8) * 2^-24.
 */
#ifndef ORA_ORACLE_H
#define ORA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_DIFFUSE = 0, ORA_GLASS = 1, ORA_EMITTER = 2 };
enum { ORA_LIGHT_NONE = 0, ORA_LIGHT_PARALLELOGRAM = 1, ORA_LIGHT_POINT = 2 };

typedef struct ora_scene {
    int n_verts;
    const float *verts;      /* [V][3] metres */
    int n_tris;
    const int32_t *tris;     /* [T][3] vertex indices */
    const int32_t *tri_mat;  /* [T] material index */
    int n_lambda;
    const float *lambda_nm;  /* [nl] */
    const double *lambda_w;  /* [nl] integration weights (nm) */
    const double *cmf;       /* [nl][3] */
    int n_mats;
    const int32_t *mat_type; /* [M] ORA_DIFFUSE / ORA_GLASS / ORA_EMITTER */
    const float *mat_rho;    /* [M][nl] */
    const float *mat_n;      /* [M][nl] */
    const float *mat_k;      /* [M][nl] */
    const float *mat_thick;  /* [M] metres */
    const float *mat_le;     /* [M][nl] */
    int light_type;
    const float *light_p0, *light_e1, *light_e2; /* [3] each */
    int light_mat;
    /* optional coherent coatings of glass materials (NULL: none) */
    int max_layers;              /* Lm, at most 8 */
    const int32_t *mat_n_layers; /* [M] layers on the normal-side face */
    const float *mat_layer_d;    /* [M][Lm] thickness (m), outermost first */
    const float *mat_layer_n;    /* [M][Lm][nl] */
    const float *mat_layer_k;    /* [M][Lm][nl] */
} ora_scene;

typedef struct ora_args {
    double eye[3], target[3];
    double fov_deg;
    int ortho;               /* 1: rays orthogonal to the image plane */
    double ortho_half_h;
    int W, H, spp, sample_offset, max_depth;
    uint32_t seed, render_id;
    int use_bvh;             /* 1: median-split BVH, 0: brute force */
    int n_threads;           /* <= 0: OpenMP default */
    int n_pix;               /* > 0: render only the listed pixels */
    const int32_t *pix;      /* [n_pix] pixel indices p = py*W + px */
    int window;              /* 1: pix lists a window of the frame in row-major order and the render's
                                paths are numbered over it (sample s of listed pixel i is path
                                s * n_pix + i); 0: paths are numbered over the frame, s * W * H + p */
    /* radiance-cache estimator (nrc != 0) with a closed-form cache
     * L(x, n) = c[0] + c[1..3] . xn + c[4..6] . n, xn = clip((x - lo) / (hi - lo), 0, 1):
     * training paths (path number % nrc_stride == 0, the path numbered as
     * `window` says) are traced as without it; any other path ends at its first
     * diffuse vertex of depth >= 2 after that vertex's light sample, adding
     * beta * L(x, n). */
    int nrc;
    uint32_t nrc_stride;
    double nrc_c[7];
    double nrc_lo[3], nrc_hi[3];
} ora_args;

typedef struct ora_out {
    double *spectral;        /* [n_out][nl] mean over spp, or NULL */
    double *xyz;             /* [n_out][3] or NULL */
    int32_t *hit_log;        /* [n_out][spp][D]: prim, -1 miss, -2 no ray; or NULL */
    int32_t *shadow_log;     /* [n_out][spp][D]: 1 visible, 0 blocked, -2 none; or NULL */
    double *path_L;          /* [n_out][spp][nl] per-sample radiance, or NULL */
    double *first_hit;       /* [n_out][spp][3] first vertex position (NaN if none), or NULL */
    double *nrc_rows;        /* [n_out][spp][D-1][9] training rows of training paths, or NULL:
                                (valid, x, y, z, lambda_nm, n_x, n_y, n_z, target) for the
                                diffuse vertex of depth 2 + index that continued the path */
    int64_t n_ext_rays;      /* closest-hit queries traced */
    int64_t n_shadow_rays;   /* shadow queries traced */
} ora_out;

typedef struct ora_accel ora_accel;

ora_accel *ora_build(const ora_scene *sc);
void ora_free(ora_accel *acc);
int ora_accel_nodes(const ora_accel *acc);

/* Render; acc == NULL or args->use_bvh == 0 selects brute force. 0 on success. */
int ora_render(const ora_scene *sc, const ora_accel *acc, const ora_args *args, ora_out *out);

/* Closest hits of n rays (FP64).  exclude[i] = prim to skip (-1 none). */
int ora_trace_rays(const ora_scene *sc, const ora_accel *acc, int n, const double *o,
                   const double *d, const int32_t *exclude, double *t_out, int32_t *prim_out);

/* Shadow transmittance of n segments (0 < t < r): out[i][nl]. */
int ora_shadow_rays(const ora_scene *sc, const ora_accel *acc, int n, const double *o,
                    const double *d, const double *r, const int32_t *exclude, double *out);

/* Replay of n path samples (pixel pix[i], sample index samp[i]; args->spp
 * and sample_offset unused) exposing, per depth d = 1..D, ORA_PROBE_STRIDE
 * doubles at out[(i * D + d - 1) * stride]: [0..2] origin and [3..5] unit
 * direction of the ray that finds vertex d, [6] its excluded prim; [7] the
 * glass-branch draw u and [8] P_R if vertex d is a pane that draws one; for a
 * diffuse vertex d with a light: [9..11] shadow-ray origin, [12..14] its unit
 * direction, [15] its length, [16] cos at the vertex, [17] cos at the light.
 * NaN where a quantity does not arise.  Test infrastructure: the parity tests
 * take the margins of the decisions where a GPU path left the oracle's. */
#define ORA_PROBE_STRIDE 18
int ora_probe_paths(const ora_scene *sc, const ora_accel *acc, const ora_args *args, int n, const int32_t *pix,
                    const int32_t *samp, double *out);

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double ora_u01(uint32_t x);

void ora_fresnel_sp(double n, double k, double c, double *Rs, double *Rp);
void ora_slab_sp(double n, double k, double thick_m, double lambda_nm, double c,
                 double *Rslab_s, double *Rslab_p, double *T_s, double *T_p);
void ora_slab(double n, double k, double thick_m, double lambda_nm, double c, double *R, double *T);
void ora_tmm_sp(int L, const double *d_m, const double *n, const double *k, double n_in, double k_in,
                double n_out, double k_out, double lambda_nm, double beta,
                double *Rs, double *Rp, double *Ts, double *Tp);
void ora_coated_pane(double n_s, double k_s, double thick_m, int L, const double *d_m, const double *n,
                     const double *k, double lambda_nm, double c, int coated_side, double *R, double *T);

void ora_cosine_hemisphere(const double n[3], double u0, double u1, double out[3]);
void ora_camera_ray(const ora_args *args, double x, double y, double o[3], double d[3]);

#ifdef __cplusplus
}
#endif
#endif
