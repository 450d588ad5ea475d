/* The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
 * plain renders (BVH and brute force, logs, per-sample radiance), a coated
 * scene, a radiance-cache render with training rows, a window render and the
 * path probe, on the scene directory given as argv[1].  Prints one checksum
 * line per render; any sanitizer report fails the calling test. */
#include <math.h>
#include <stdint.h>

#include "../../oracle/oracle.h"
#include "scene_io.h"

static double checksum(const double *a, long n) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * (double)(1 + i % 7);
    return s;
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const char *dir = argv[1];
    ora_scene sc;
    memset(&sc, 0, sizeof sc);
    const int V = (int)meta_get(dir, "n_verts"), T = (int)meta_get(dir, "n_tris");
    const int nl = (int)meta_get(dir, "n_lambda"), M = (int)meta_get(dir, "n_mats");
    sc.n_verts = V;
    sc.verts = read_bin(dir, "verts", 12L * V);
    sc.n_tris = T;
    sc.tris = read_bin(dir, "tris", 12L * T);
    sc.tri_mat = read_bin(dir, "tri_mat", 4L * T);
    sc.n_lambda = nl;
    sc.lambda_nm = read_bin(dir, "lambda_nm", 4L * nl);
    sc.lambda_w = read_bin(dir, "lambda_w", 8L * nl);
    sc.cmf = read_bin(dir, "cmf", 24L * nl);
    sc.n_mats = M;
    sc.mat_type = read_bin(dir, "mat_type", 4L * M);
    sc.mat_rho = read_bin(dir, "mat_rho", 4L * M * nl);
    sc.mat_n = read_bin(dir, "mat_n", 4L * M * nl);
    sc.mat_k = read_bin(dir, "mat_k", 4L * M * nl);
    sc.mat_thick = read_bin(dir, "mat_thick", 4L * M);
    sc.mat_le = read_bin(dir, "mat_le", 4L * M * nl);
    sc.light_type = (int)meta_get(dir, "light_type");
    sc.light_mat = (int)meta_get(dir, "light_mat");
    sc.light_p0 = read_bin(dir, "light_p0", 12);
    sc.light_e1 = read_bin(dir, "light_e1", 12);
    sc.light_e2 = read_bin(dir, "light_e2", 12);
    const int Lm = (int)meta_get(dir, "max_layers");
    if (Lm > 0) {
        sc.max_layers = Lm;
        sc.mat_n_layers = read_bin(dir, "mat_n_layers", 4L * M);
        sc.mat_layer_d = read_bin(dir, "mat_layer_d", 4L * M * Lm);
        sc.mat_layer_n = read_bin(dir, "mat_layer_n", 4L * M * Lm * nl);
        sc.mat_layer_k = read_bin(dir, "mat_layer_k", 4L * M * Lm * nl);
    }
    const double *cam = read_bin(dir, "camera", 8L * 9);  /* eye, target, fov, ortho, ortho_half_h */
    ora_accel *acc = ora_build(&sc);

    const int W = 12, H = 9, spp = 2, D = 5;
    ora_args a;
    memset(&a, 0, sizeof a);
    for (int k = 0; k < 3; ++k) { a.eye[k] = cam[k]; a.target[k] = cam[3 + k]; }
    a.fov_deg = cam[6];
    a.ortho = cam[7] != 0.0;
    a.ortho_half_h = cam[8];
    a.W = W; a.H = H; a.spp = spp; a.max_depth = D; a.n_threads = 2;
    const long n = (long)W * H;
    double *spec = calloc((size_t)n * nl, sizeof(double)), *xyz = calloc((size_t)n * 3, sizeof(double));
    double *pathL = calloc((size_t)n * spp * nl, sizeof(double));
    int32_t *hl = calloc((size_t)n * spp * D, sizeof(int32_t)), *sl = calloc((size_t)n * spp * D, sizeof(int32_t));
    double *rows = calloc((size_t)n * spp * (D - 1) * 9, sizeof(double));
    ora_out o;
    for (int bvh = 0; bvh < 2; ++bvh) {
        a.use_bvh = bvh;
        memset(&o, 0, sizeof o);
        o.spectral = spec; o.xyz = xyz; o.hit_log = hl; o.shadow_log = sl; o.path_L = pathL;
        if (ora_render(&sc, acc, &a, &o) != 0) return 3;
        printf("plain bvh=%d %.17g rays %lld\n", bvh, checksum(spec, n * nl), (long long)(o.n_ext_rays + o.n_shadow_rays));
    }
    /* radiance cache with a closed-form cache, every fifth path training */
    a.use_bvh = 1;
    a.nrc = 1; a.nrc_stride = 5;
    a.nrc_c[0] = 0.1; a.nrc_c[1] = 0.05; a.nrc_c[5] = 0.02;
    a.nrc_hi[0] = 4.0; a.nrc_hi[1] = 3.0; a.nrc_hi[2] = 2.5;
    memset(&o, 0, sizeof o);
    o.spectral = spec; o.hit_log = hl; o.shadow_log = sl; o.nrc_rows = rows;
    if (ora_render(&sc, acc, &a, &o) != 0) return 4;
    printf("cache %.17g rows %.17g\n", checksum(spec, n * nl), checksum(rows, n * spp * (D - 1) * 9));
    /* a window of the frame, its paths numbered over it */
    int32_t pix[12];
    for (int i = 0; i < 12; ++i) pix[i] = (3 + i / 4) * W + 5 + i % 4;
    a.n_pix = 12; a.pix = pix; a.window = 1;
    memset(&o, 0, sizeof o);
    o.spectral = spec;
    if (ora_render(&sc, acc, &a, &o) != 0) return 5;
    printf("window %.17g\n", checksum(spec, 12L * nl));
    /* path probe */
    int32_t samp[12];
    for (int i = 0; i < 12; ++i) samp[i] = i % spp;
    a.nrc = 0; a.n_pix = 0; a.pix = NULL; a.window = 0;
    double *probe = calloc((size_t)12 * D * ORA_PROBE_STRIDE, sizeof(double));
    if (ora_probe_paths(&sc, acc, &a, 12, pix, samp, probe) != 0) return 6;
    long finite = 0;
    for (long i = 0; i < 12L * D * ORA_PROBE_STRIDE; ++i) finite += isfinite(probe[i]);
    printf("probe finite %ld\n", finite);
    ora_free(acc);
    free(spec); free(xyz); free(pathL); free(hl); free(sl); free(rows); free(probe);
    free((void *)sc.verts); free((void *)sc.tris); free((void *)sc.tri_mat); free((void *)sc.lambda_nm);
    free((void *)sc.lambda_w); free((void *)sc.cmf); free((void *)sc.mat_type); free((void *)sc.mat_rho);
    free((void *)sc.mat_n); free((void *)sc.mat_k); free((void *)sc.mat_thick); free((void *)sc.mat_le);
    free((void *)sc.light_p0); free((void *)sc.light_e1); free((void *)sc.light_e2); free((void *)cam);
    if (Lm > 0) {
        free((void *)sc.mat_n_layers); free((void *)sc.mat_layer_d); free((void *)sc.mat_layer_n);
        free((void *)sc.mat_layer_k);
    }
    return 0;
}
