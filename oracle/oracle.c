/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain, slow and direct: every function is the textbook definition or the
 * paper's step written out, in double precision, with no blocking, fusion
 * or reordering beyond what the definition states.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PI 3.14159265358979323846
#define ORA_OFFSET 1e-4 /* origin offset (m) along the side the new ray leaves */
#define ORA_LEAF 4

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static v3 unit(v3 a) { return scl(a, 1.0 / sqrt(dot(a, a))); }
static double comp(v3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

static v3 vert(const ora_scene *sc, int i) {
    const float *p = sc->verts + 3 * (size_t)i;
    return mk((double)p[0], (double)p[1], (double)p[2]); /* exact widening */
}
static v3 fvec(const float *p) { return mk((double)p[0], (double)p[1], (double)p[2]); }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                        */
/* ------------------------------------------------------------------------ */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    /* round multipliers and Weyl key increments of the published generator */
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = M0 * (uint64_t)c0; /* (hi0, lo0) = mulhilo(M0, c0) */
        uint64_t p1 = M1 * (uint64_t)c2; /* (hi1, lo1) = mulhilo(M1, c2) */
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* top 24 bits -> [0, 1), exact in both FP32 and FP64 */
double ora_u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

static void rng_u(uint32_t seed, uint32_t render_id, uint32_t p, uint32_t s, uint32_t d,
                  uint32_t b, double u[4]) {
    uint32_t ctr[4] = {p, s, d, b}, key[2] = {seed, render_id}, o[4];
    ora_philox4x32_10(ctr, key, o);
    for (int i = 0; i < 4; ++i) u[i] = ora_u01(o[i]);
}

/* ------------------------------------------------------------------------ */
/* Fresnel terms from the complex index n + i k (Eq. 1)                      */
/* ------------------------------------------------------------------------ */
/* Reflectance of a plane interface air -> (n + i k) at incidence cosine c,
 * for s and p polarisation.  cos(theta_t) takes the principal square root. */
void ora_fresnel_sp(double n, double k, double c, double *Rs, double *Rp) {
    double complex nt = n + I * k;
    double complex sin2t = (1.0 - c * c) / (nt * nt);        /* Snell, complex */
    double complex cost = csqrt(1.0 - sin2t);
    double complex rs = (c - nt * cost) / (c + nt * cost);
    double complex rp = (nt * c - cost) / (nt * c + cost);
    *Rs = creal(rs) * creal(rs) + cimag(rs) * cimag(rs);
    *Rp = creal(rp) * creal(rp) + cimag(rp) * cimag(rp);
}

/* Incoherent slab of thickness d with identical faces: the sum over all
 * internal reflections of a ray that bounces between the two faces, each
 * crossing attenuated by tau = exp(-alpha d / cos theta_r), alpha = 4 pi k/lambda
 * (Beer-Lambert), cos theta_r from real Snell with n. */
void ora_slab_sp(double n, double k, double thick_m, double lambda_nm, double c,
                 double *Rslab_s, double *Rslab_p, double *T_s, double *T_p) {
    double Rs, Rp;
    ora_fresnel_sp(n, k, c, &Rs, &Rp);
    double sin2r = (1.0 - c * c) / (n * n);
    double cosr2 = 1.0 - sin2r;
    double tau = 0.0;
    if (cosr2 > 0.0) {
        double alpha = 4.0 * ORA_PI * k / (lambda_nm * 1e-9);
        tau = exp(-alpha * thick_m / sqrt(cosr2));
    }
    double R[2] = {Rs, Rp}, Rsl[2], Tsl[2];
    for (int i = 0; i < 2; ++i) {
        double denom = 1.0 - R[i] * R[i] * tau * tau;
        if (denom <= 0.0) { Rsl[i] = 1.0; Tsl[i] = 0.0; continue; }
        Tsl[i] = (1.0 - R[i]) * (1.0 - R[i]) * tau / denom;
        Rsl[i] = R[i] + (1.0 - R[i]) * (1.0 - R[i]) * R[i] * tau * tau / denom;
    }
    *Rslab_s = Rsl[0]; *Rslab_p = Rsl[1]; *T_s = Tsl[0]; *T_p = Tsl[1];
}

/* Polarisation is not tracked: the pane's R and T are (s + p) / 2. */
void ora_slab(double n, double k, double thick_m, double lambda_nm, double c, double *R, double *T) {
    double rs, rp, ts, tp;
    ora_slab_sp(n, k, thick_m, lambda_nm, c, &rs, &rp, &ts, &tp);
    *R = 0.5 * (rs + rp);
    *T = 0.5 * (ts + tp);
}

/* ------------------------------------------------------------------------ */
/* coherent thin-film stack (electrochromic coating): characteristic matrices */
/* ------------------------------------------------------------------------ */
/* Medium of complex index N crossed with Snell invariant beta = N sin(theta)
 * (the same in every layer): N cos(theta) is the principal root of
 * N^2 - beta^2, and the tilted optical admittance is N cos(theta) for s and
 * N / cos(theta) = N^2 / (N cos(theta)) for p polarisation. */
static double complex admittance(double complex N, double beta, int p_pol) {
    double complex Nc = csqrt(N * N - beta * beta);
    return p_pol ? N * N / Nc : Nc;
}

/* Stack of L layers (thickness d[j] m, index n[j] + i k[j]) between an
 * incidence medium N_in and an exit medium N_out, layers listed in the order
 * the light meets them.  With the index written n + i k (fields varying as
 * exp(i (N k0 z - omega t)), so k > 0 attenuates), each layer's
 * characteristic matrix is
 *   [[cos delta, -i sin delta / eta], [-i eta sin delta, cos delta]],
 * delta = 2 pi N cos(theta) d / lambda; with [B, C] = M_1 ... M_L [1, eta_out],
 * the amplitude reflectance is r = (eta_in B - C) / (eta_in B + C), the
 * reflectance R = |r|^2 and the transmittance into the exit medium
 * T = 4 Re(eta_in) Re(eta_out) / |eta_in B + C|^2. */
void ora_tmm_sp(int L, const double *d_m, const double *n, const double *k, double n_in, double k_in,
                double n_out, double k_out, double lambda_nm, double beta,
                double *Rs, double *Rp, double *Ts, double *Tp) {
    double lam = lambda_nm * 1e-9;
    for (int pol = 0; pol < 2; ++pol) {
        double complex m11 = 1.0, m12 = 0.0, m21 = 0.0, m22 = 1.0;
        for (int j = 0; j < L; ++j) {
            double complex N = n[j] + I * k[j];
            double complex Nc = csqrt(N * N - beta * beta);
            double complex eta = pol ? N * N / Nc : Nc;
            double complex delta = 2.0 * ORA_PI * Nc * d_m[j] / lam;
            double complex a11 = ccos(delta), a12 = -I * csin(delta) / eta;
            double complex a21 = -I * eta * csin(delta), a22 = ccos(delta);
            double complex t11 = m11 * a11 + m12 * a21, t12 = m11 * a12 + m12 * a22;
            double complex t21 = m21 * a11 + m22 * a21, t22 = m21 * a12 + m22 * a22;
            m11 = t11; m12 = t12; m21 = t21; m22 = t22;
        }
        double complex e_in = admittance(n_in + I * k_in, beta, pol);
        double complex e_out = admittance(n_out + I * k_out, beta, pol);
        double complex B = m11 + m12 * e_out, Cc = m21 + m22 * e_out;
        double complex r = (e_in * B - Cc) / (e_in * B + Cc);
        double complex den = e_in * B + Cc;
        double R = creal(r) * creal(r) + cimag(r) * cimag(r);
        double T = 4.0 * creal(e_in) * creal(e_out) / (creal(den) * creal(den) + cimag(den) * cimag(den));
        if (pol) { *Rp = R; *Tp = T; } else { *Rs = R; *Ts = T; }
    }
}

/* Pane with a coherent coating of L layers on one face of the incoherent
 * substrate (index n_s + i k_s, thickness thick_m).  Per polarisation:
 *  - coated face: R_c, T_c from air onto the stack into the substrate, R_c'
 *    from the substrate onto the reversed stack into air;
 *  - bare face: R_b = Fresnel of the substrate, T_b = 1 - R_b;
 *  - the substrate attenuates each crossing by tau (Beer-Lambert as for the
 *    uncoated slab) and the internal reflections sum incoherently:
 *      from the coated side: T = T_c tau T_b / (1 - R_c' R_b tau^2),
 *                            R = R_c + T_c T_c' R_b tau^2 / (1 - R_c' R_b tau^2)
 *      from the bare side:   T = T_b tau T_c' / (1 - R_b R_c' tau^2),
 *                            R = R_b + T_b^2 R_c' tau^2 / (1 - R_b R_c' tau^2)
 *  then (s + p) / 2.  c: incidence cosine in air; coated_side: 1 if the light
 *  arrives on the coated face. */
void ora_coated_pane(double n_s, double k_s, double thick_m, int L, const double *d_m, const double *n,
                     const double *k, double lambda_nm, double c, int coated_side, double *R, double *T) {
    double beta = sqrt(fmax(0.0, 1.0 - c * c));
    double Rc[2], Tc[2], Rc2[2], Tc2[2], Rb[2];
    ora_tmm_sp(L, d_m, n, k, 1.0, 0.0, n_s, k_s, lambda_nm, beta, &Rc[0], &Rc[1], &Tc[0], &Tc[1]);
    double dr[8], nr[8], kr[8];
    for (int j = 0; j < L; ++j) { dr[j] = d_m[L - 1 - j]; nr[j] = n[L - 1 - j]; kr[j] = k[L - 1 - j]; }
    ora_tmm_sp(L, dr, nr, kr, n_s, k_s, 1.0, 0.0, lambda_nm, beta, &Rc2[0], &Rc2[1], &Tc2[0], &Tc2[1]);
    ora_fresnel_sp(n_s, k_s, c, &Rb[0], &Rb[1]);
    double cosr2 = 1.0 - (1.0 - c * c) / (n_s * n_s);
    double tau = 0.0;
    if (cosr2 > 0.0) tau = exp(-4.0 * ORA_PI * k_s / (lambda_nm * 1e-9) * thick_m / sqrt(cosr2));
    double Rsum = 0.0, Tsum = 0.0;
    for (int i = 0; i < 2; ++i) {
        double Tb = 1.0 - Rb[i];
        double den = 1.0 - Rc2[i] * Rb[i] * tau * tau;
        if (den <= 0.0) { Rsum += 1.0; continue; }
        if (coated_side) {
            Tsum += Tc[i] * tau * Tb / den;
            Rsum += Rc[i] + Tc[i] * Tc2[i] * Rb[i] * tau * tau / den;
        } else {
            Tsum += Tb * tau * Tc2[i] / den;
            Rsum += Rb[i] + Tb * Tb * Rc2[i] * tau * tau / den;
        }
    }
    *R = 0.5 * Rsum;
    *T = 0.5 * Tsum;
}

/* R and T of glass material m at wavelength l for incidence cosine c; the
 * coating (if any) lies on the face the triangle's geometric normal points
 * out of, so a ray with dir . n_g < 0 meets it first. */
static void pane_RT(const ora_scene *sc, int m, int l, double c, int coated_side, double *R, double *T) {
    const int nl = sc->n_lambda;
    const int L = sc->mat_n_layers ? sc->mat_n_layers[m] : 0;
    const double n_s = sc->mat_n[(size_t)m * nl + l], k_s = sc->mat_k[(size_t)m * nl + l];
    if (L <= 0) {
        ora_slab(n_s, k_s, sc->mat_thick[m], sc->lambda_nm[l], c, R, T);
        return;
    }
    const int Lm = sc->max_layers;
    double d[8], n[8], k[8];
    for (int j = 0; j < L && j < 8; ++j) {
        d[j] = sc->mat_layer_d[(size_t)m * Lm + j];
        n[j] = sc->mat_layer_n[((size_t)m * Lm + j) * nl + l];
        k[j] = sc->mat_layer_k[((size_t)m * Lm + j) * nl + l];
    }
    ora_coated_pane(n_s, k_s, sc->mat_thick[m], L < 8 ? L : 8, d, n, k, sc->lambda_nm[l], c, coated_side, R, T);
}

/* ------------------------------------------------------------------------ */
/* sampling and camera                                                       */
/* ------------------------------------------------------------------------ */
/* cosine-weighted direction about n; orthonormal basis of Duff et al.
 * (JCGT 2017), with the branch sign taken as +1 for both signed zeros of n_z
 * so the basis never depends on how a zero component was rounded */
void ora_cosine_hemisphere(const double nn[3], double u0, double u1, double out[3]) {
    double nx = nn[0], ny = nn[1], nz = nn[2];
    double s = nz >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (s + nz);
    double b = nx * ny * a;
    v3 b1 = mk(1.0 + s * nx * nx * a, s * b, -s * nx);
    v3 b2 = mk(b, s + ny * ny * a, -ny);
    double r = sqrt(u0), phi = 2.0 * ORA_PI * u1;
    double lx = r * cos(phi), ly = r * sin(phi), lz = sqrt(1.0 - u0);
    v3 w = add(add(scl(b1, lx), scl(b2, ly)), scl(mk(nx, ny, nz), lz));
    out[0] = w.x; out[1] = w.y; out[2] = w.z;
}

/* Image-plane point (x, y) in pixel units, y = 0 at the top row.  Pinhole by
 * default; with ortho set, rays leave the image plane orthogonally (Sec. 4). */
void ora_camera_ray(const ora_args *a, double x, double y, double o[3], double d[3]) {
    v3 eye = mk(a->eye[0], a->eye[1], a->eye[2]);
    v3 f = unit(sub(mk(a->target[0], a->target[1], a->target[2]), eye));
    v3 r = unit(cross(f, mk(0, 0, 1)));
    v3 u = cross(r, f);
    double aspect = (double)a->W / (double)a->H;
    double sx = 2.0 * x / a->W - 1.0, sy = 1.0 - 2.0 * y / a->H;
    if (a->ortho) {
        v3 oo = add(eye, add(scl(r, sx * a->ortho_half_h * aspect), scl(u, sy * a->ortho_half_h)));
        o[0] = oo.x; o[1] = oo.y; o[2] = oo.z;
        d[0] = f.x; d[1] = f.y; d[2] = f.z;
    } else {
        double th = tan(0.5 * a->fov_deg * ORA_PI / 180.0);
        v3 dd = unit(add(f, add(scl(r, sx * th * aspect), scl(u, sy * th))));
        o[0] = eye.x; o[1] = eye.y; o[2] = eye.z;
        d[0] = dd.x; d[1] = dd.y; d[2] = dd.z;
    }
}

/* ------------------------------------------------------------------------ */
/* ray / triangle (Moller-Trumbore, inclusive barycentrics)                  */
/* ------------------------------------------------------------------------ */
static int tri_hit(const ora_scene *sc, int prim, v3 o, v3 d, double *t_out) {
    const int32_t *ix = sc->tris + 3 * (size_t)prim;
    v3 v0 = vert(sc, ix[0]), v1 = vert(sc, ix[1]), v2 = vert(sc, ix[2]);
    v3 e1 = sub(v1, v0), e2 = sub(v2, v0);
    v3 p = cross(d, e2);
    double det = dot(e1, p);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    v3 s = sub(o, v0);
    double u = dot(s, p) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    v3 q = cross(s, e1);
    double v = dot(d, q) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    *t_out = dot(e2, q) * inv;
    return 1;
}

static v3 tri_normal(const ora_scene *sc, int prim) {
    const int32_t *ix = sc->tris + 3 * (size_t)prim;
    v3 v0 = vert(sc, ix[0]), v1 = vert(sc, ix[1]), v2 = vert(sc, ix[2]);
    return unit(cross(sub(v1, v0), sub(v2, v0)));
}

/* ------------------------------------------------------------------------ */
/* median-split BVH (FP64 boxes), the oracle's own                           */
/* ------------------------------------------------------------------------ */
typedef struct { double lo[3], hi[3]; int left, right, first, count; } onode;

struct ora_accel {
    onode *nodes;
    int n_nodes, cap;
    int *prims;
    double *cen;     /* [T][3] centroids */
    double *blo, *bhi; /* [T][3] triangle boxes */
};

static int new_node(ora_accel *a) {
    if (a->n_nodes == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 1024;
        a->nodes = (onode *)realloc(a->nodes, sizeof(onode) * (size_t)a->cap);
    }
    return a->n_nodes++;
}

/* quickselect: order prims[lo..hi) so that the element of rank k is in place */
static void select_k(ora_accel *a, int lo, int hi, int k, int axis) {
    int *p = a->prims;
    while (hi - lo > 1) {
        double pivot = a->cen[3 * (size_t)p[(lo + hi) / 2] + axis];
        int i = lo, j = hi - 1;
        while (i <= j) {
            while (a->cen[3 * (size_t)p[i] + axis] < pivot) ++i;
            while (a->cen[3 * (size_t)p[j] + axis] > pivot) --j;
            if (i <= j) { int t = p[i]; p[i] = p[j]; p[j] = t; ++i; --j; }
        }
        if (k <= j) hi = j + 1;
        else if (k >= i) lo = i;
        else return;
    }
}

static int build_rec(ora_accel *a, int first, int count) {
    int id = new_node(a);
    onode nd;
    for (int k = 0; k < 3; ++k) { nd.lo[k] = INFINITY; nd.hi[k] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = first; i < first + count; ++i) {
        int pr = a->prims[i];
        for (int k = 0; k < 3; ++k) {
            nd.lo[k] = fmin(nd.lo[k], a->blo[3 * (size_t)pr + k]);
            nd.hi[k] = fmax(nd.hi[k], a->bhi[3 * (size_t)pr + k]);
            clo[k] = fmin(clo[k], a->cen[3 * (size_t)pr + k]);
            chi[k] = fmax(chi[k], a->cen[3 * (size_t)pr + k]);
        }
    }
    /* conservative: grow each box by a tiny margin so rounding in the slab
     * test can never reject a box that holds a hit */
    for (int k = 0; k < 3; ++k) {
        double m = 1e-9 * (1.0 + fmax(fabs(nd.lo[k]), fabs(nd.hi[k])));
        nd.lo[k] -= m; nd.hi[k] += m;
    }
    nd.left = nd.right = -1; nd.first = first; nd.count = count;
    if (count > ORA_LEAF) {
        int axis = 0;
        double ext = chi[0] - clo[0];
        for (int k = 1; k < 3; ++k) if (chi[k] - clo[k] > ext) { ext = chi[k] - clo[k]; axis = k; }
        int half = count / 2;
        select_k(a, first, first + count, first + half, axis);
        nd.count = 0;
        a->nodes[id] = nd;
        int l = build_rec(a, first, half);
        int r = build_rec(a, first + half, count - half);
        a->nodes[id].left = l;
        a->nodes[id].right = r;
        return id;
    }
    a->nodes[id] = nd;
    return id;
}

ora_accel *ora_build(const ora_scene *sc) {
    ora_accel *a = (ora_accel *)calloc(1, sizeof(ora_accel));
    int T = sc->n_tris;
    a->prims = (int *)malloc(sizeof(int) * (size_t)(T > 0 ? T : 1));
    a->cen = (double *)malloc(sizeof(double) * 3 * (size_t)(T > 0 ? T : 1));
    a->blo = (double *)malloc(sizeof(double) * 3 * (size_t)(T > 0 ? T : 1));
    a->bhi = (double *)malloc(sizeof(double) * 3 * (size_t)(T > 0 ? T : 1));
    for (int i = 0; i < T; ++i) {
        const int32_t *ix = sc->tris + 3 * (size_t)i;
        v3 v[3] = {vert(sc, ix[0]), vert(sc, ix[1]), vert(sc, ix[2])};
        for (int k = 0; k < 3; ++k) {
            double lo = fmin(fmin(comp(v[0], k), comp(v[1], k)), comp(v[2], k));
            double hi = fmax(fmax(comp(v[0], k), comp(v[1], k)), comp(v[2], k));
            a->blo[3 * (size_t)i + k] = lo;
            a->bhi[3 * (size_t)i + k] = hi;
            a->cen[3 * (size_t)i + k] = 0.5 * (lo + hi);
        }
        a->prims[i] = i;
    }
    if (T > 0) build_rec(a, 0, T);
    return a;
}

void ora_free(ora_accel *a) {
    if (!a) return;
    free(a->nodes); free(a->prims); free(a->cen); free(a->blo); free(a->bhi);
    free(a);
}

int ora_accel_nodes(const ora_accel *a) { return a ? a->n_nodes : 0; }

/* does the ray meet the box for some t in [tmin, tmax] ? */
static int box_hit(const onode *nd, v3 o, v3 d, double tmin, double tmax) {
    for (int k = 0; k < 3; ++k) {
        double ok = comp(o, k), dk = comp(d, k);
        if (dk == 0.0) {
            if (ok < nd->lo[k] || ok > nd->hi[k]) return 0;
            continue;
        }
        double t0 = (nd->lo[k] - ok) / dk, t1 = (nd->hi[k] - ok) / dk;
        if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
        if (t0 > tmin) tmin = t0;
        if (t1 < tmax) tmax = t1;
        if (tmin > tmax) return 0;
    }
    return 1;
}

/* closest hit: smallest t > 0, ties to the smaller prim id */
static void consider(const ora_scene *sc, int prim, v3 o, v3 d, int exclude, double *tb, int *pb) {
    if (prim == exclude) return;
    double t;
    if (!tri_hit(sc, prim, o, d, &t)) return;
    if (!(t > 0.0)) return;
    if (t < *tb || (t == *tb && (*pb < 0 || prim < *pb))) { *tb = t; *pb = prim; }
}

static int closest_hit(const ora_scene *sc, const ora_accel *a, v3 o, v3 d, int exclude, double *t_out) {
    double tb = INFINITY;
    int pb = -1;
    if (!a) {
        for (int i = 0; i < sc->n_tris; ++i) consider(sc, i, o, d, exclude, &tb, &pb);
    } else if (a->n_nodes > 0) {
        int stack[128], sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const onode *nd = &a->nodes[stack[--sp]];
            if (!box_hit(nd, o, d, 0.0, tb)) continue;
            if (nd->left < 0) {
                for (int i = nd->first; i < nd->first + nd->count; ++i)
                    consider(sc, a->prims[i], o, d, exclude, &tb, &pb);
            } else {
                stack[sp++] = nd->left;
                stack[sp++] = nd->right;
            }
        }
    }
    *t_out = tb;
    return pb;
}

/* One triangle on a shadow segment 0 < t < r.  Returns 0 when the segment
 * is blocked by an opaque (diffuse) triangle; multiplies T by the pane's
 * transmittance for a glass triangle; emitters are ignored. */
static int shadow_prim(const ora_scene *sc, int prim, v3 o, v3 w, double r, int exclude, double *T) {
    if (prim == exclude) return 1;
    int nl = sc->n_lambda;
    int m = sc->tri_mat[prim];
    int typ = sc->mat_type[m];
    if (typ == ORA_EMITTER) return 1;
    double t;
    if (!tri_hit(sc, prim, o, w, &t)) return 1;
    if (!(t > 0.0 && t < r)) return 1;
    if (typ == ORA_DIFFUSE) return 0;
    v3 ngs = tri_normal(sc, prim);
    double c = fabs(dot(w, ngs));
    for (int l = 0; l < nl; ++l) {
        double Rl, Tl;
        pane_RT(sc, m, l, c, dot(w, ngs) < 0.0, &Rl, &Tl);
        T[l] *= Tl;
    }
    return 1;
}

/* Shadow segment 0 < t < r: product of the transmittances of every pane it
 * crosses (order does not matter).  Returns 1 if unoccluded (T may still be
 * small), 0 if an opaque triangle blocks it (T is then all zero). */
static int shadow_T(const ora_scene *sc, const ora_accel *a, v3 o, v3 w, double r, int exclude, double *T) {
    int nl = sc->n_lambda;
    int visible = 1;
    for (int l = 0; l < nl; ++l) T[l] = 1.0;
    if (!a) {
        for (int i = 0; i < sc->n_tris && visible; ++i) visible = shadow_prim(sc, i, o, w, r, exclude, T);
    } else if (a->n_nodes > 0) {
        int stack[128], sp = 0;
        stack[sp++] = 0;
        while (sp > 0 && visible) {
            const onode *nd = &a->nodes[stack[--sp]];
            if (!box_hit(nd, o, w, 0.0, r)) continue;
            if (nd->left >= 0) { stack[sp++] = nd->left; stack[sp++] = nd->right; continue; }
            for (int i = nd->first; i < nd->first + nd->count && visible; ++i)
                visible = shadow_prim(sc, a->prims[i], o, w, r, exclude, T);
        }
    }
    if (!visible) for (int l = 0; l < nl; ++l) T[l] = 0.0;
    return visible;
}

int ora_trace_rays(const ora_scene *sc, const ora_accel *acc, int n, const double *o, const double *d,
                   const int32_t *exclude, double *t_out, int32_t *prim_out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        v3 oo = mk(o[3 * i], o[3 * i + 1], o[3 * i + 2]);
        v3 dd = mk(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
        double t;
        prim_out[i] = closest_hit(sc, acc, oo, dd, exclude ? exclude[i] : -1, &t);
        t_out[i] = t;
    }
    return 0;
}

int ora_shadow_rays(const ora_scene *sc, const ora_accel *acc, int n, const double *o, const double *d,
                    const double *r, const int32_t *exclude, double *out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        v3 oo = mk(o[3 * i], o[3 * i + 1], o[3 * i + 2]);
        v3 dd = mk(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
        shadow_T(sc, acc, oo, dd, r[i], exclude ? exclude[i] : -1, out + (size_t)i * sc->n_lambda);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* the spectral path tracer                                                  */
/* ------------------------------------------------------------------------ */
static int any_nonzero(const float *v, int n) {
    for (int i = 0; i < n; ++i) if (v[i] != 0.0f) return 1;
    return 0;
}

/* One path sample (pixel p = (px, py), sample index s).  Estimates Eq. 2 by
 * inverse ray tracing (Sec. 4): at every diffuse vertex a shadow ray is shot
 * toward the light (Eq. 3 for a point light, one uniform area sample for the
 * parallelogram emitter) and a secondary ray continues the path; a glass
 * vertex reflects or transmits with probability from the pane's R and T; the
 * path stops after max_depth surface vertices. */
/* Radiance-cache reading of the estimator (used when ar->nrc): a training
 * row at a diffuse vertex of depth d >= 2 that continues the path records
 * the wavelength index l = (Philox word 0 of counter (p, s, d, 3)) mod nl and
 * the radiance the path then carries back into the vertex along its
 * continuation, (L_end[l] - L_d[l]) / beta_d[l], with L_d and beta_d the
 * estimate and throughput right after the vertex's light sample. */
/* probe (NULL: none): per depth d, ORA_PROBE_STRIDE doubles at (d - 1) * stride:
 * the ray that finds vertex d (origin, direction, excluded prim), the glass
 * branch draw and P_R if vertex d is a pane that draws one, and the light
 * sample of a diffuse vertex d (shadow origin, unit direction, length, cos at
 * the vertex, cos at the light); NaN where a quantity does not arise. */
static void trace_path(const ora_scene *sc, const ora_accel *acc, const ora_args *ar, int px, int py,
                       uint32_t s, uint64_t q, double *L, int32_t *hlog, int32_t *slog, double *fhit,
                       double *beta, double *tmp_T, int64_t *n_ext, int64_t *n_sh, double *rows, double *probe) {
    const int nl = sc->n_lambda, D = ar->max_depth;
    const uint32_t p = (uint32_t)(py * ar->W + px);
    /* q: the path's number in the render (frame or window numbering) */
    const int train = ar->nrc && q % ar->nrc_stride == 0;
    /* per training row: estimate and throughput at its wavelength when recorded */
    double row_L[64], row_b[64];
    int row_l[64];
    if (rows) for (int k = 0; k < (D - 1) * 9; ++k) rows[k] = 0.0;
    double u[4], ub[4], uc[4];
    rng_u(ar->seed, ar->render_id, p, s, 0, 0, u);
    double oa[3], da[3];
    ora_camera_ray(ar, px + u[0], py + u[1], oa, da);
    v3 o = mk(oa[0], oa[1], oa[2]), dir = mk(da[0], da[1], da[2]);
    for (int l = 0; l < nl; ++l) { beta[l] = 1.0; L[l] = 0.0; }
    int countE = 1, exclude = -1;
    if (fhit) fhit[0] = fhit[1] = fhit[2] = NAN;

    int lt = sc->light_type;
    v3 lp0 = mk(0, 0, 0), le1 = mk(0, 0, 0), le2 = mk(0, 0, 0), nL = mk(0, 0, 0);
    double AL = 0.0;
    const float *LeL = NULL;
    if (lt != ORA_LIGHT_NONE) {
        lp0 = fvec(sc->light_p0);
        LeL = sc->mat_le + (size_t)sc->light_mat * nl;
        if (lt == ORA_LIGHT_PARALLELOGRAM) {
            le1 = fvec(sc->light_e1); le2 = fvec(sc->light_e2);
            v3 cr = cross(le1, le2);
            AL = sqrt(dot(cr, cr));
            nL = scl(cr, 1.0 / AL);
        }
    }

    if (probe) for (int k = 0; k < D * ORA_PROBE_STRIDE; ++k) probe[k] = NAN;
    for (int d = 1; d <= D; ++d) {
        double t;
        double *pr = probe ? probe + (size_t)(d - 1) * ORA_PROBE_STRIDE : NULL;
        if (pr) {
            pr[0] = o.x; pr[1] = o.y; pr[2] = o.z;
            pr[3] = dir.x; pr[4] = dir.y; pr[5] = dir.z;
            pr[6] = (double)exclude;
        }
        int prim = closest_hit(sc, acc, o, dir, exclude, &t);
        ++*n_ext;
        if (hlog) hlog[d - 1] = prim;
        if (prim < 0) break;                       /* no sky dome: a miss carries nothing */
        v3 x = add(o, scl(dir, t));
        if (d == 1 && fhit) { fhit[0] = x.x; fhit[1] = x.y; fhit[2] = x.z; }
        v3 ng = tri_normal(sc, prim);
        double cos_o = -dot(ng, dir);
        v3 n = cos_o > 0.0 ? ng : scl(ng, -1.0);
        int m = sc->tri_mat[prim];
        int typ = sc->mat_type[m];
        const float *le = sc->mat_le + (size_t)m * nl;

        if (typ == ORA_EMITTER) {                  /* one-sided, absorbing */
            if (countE && cos_o > 0.0)
                for (int l = 0; l < nl; ++l) L[l] += beta[l] * le[l];
            break;
        }
        if (typ == ORA_DIFFUSE) {
            const float *rho = sc->mat_rho + (size_t)m * nl;
            if (any_nonzero(le, nl))               /* diffuse emission, two-sided */
                for (int l = 0; l < nl; ++l) L[l] += beta[l] * le[l];
            rng_u(ar->seed, ar->render_id, p, s, (uint32_t)d, 0, ub);
            rng_u(ar->seed, ar->render_id, p, s, (uint32_t)d, 1, uc);
            v3 xo = add(x, scl(n, ORA_OFFSET));
            /* beta after the Lambert factor rho; the BRDF is rho / pi */
            for (int l = 0; l < nl; ++l) beta[l] *= (double)rho[l];
            if (lt != ORA_LIGHT_NONE) {
                v3 y = lp0;
                if (lt == ORA_LIGHT_PARALLELOGRAM) y = add(lp0, add(scl(le1, ub[0]), scl(le2, ub[1])));
                v3 w = sub(y, xo);
                double r2 = dot(w, w), r = sqrt(r2);
                v3 om = scl(w, 1.0 / r);
                double cx = dot(n, om);
                double cy = lt == ORA_LIGHT_PARALLELOGRAM ? -dot(nL, om) : 1.0;
                if (pr) {
                    pr[9] = xo.x; pr[10] = xo.y; pr[11] = xo.z;
                    pr[12] = om.x; pr[13] = om.y; pr[14] = om.z;
                    pr[15] = r; pr[16] = cx; pr[17] = cy;
                }
                if (cx > 0.0 && cy > 0.0) {
                    int vis = shadow_T(sc, acc, xo, om, r, prim, tmp_T);
                    ++*n_sh;
                    if (slog) slog[d - 1] = vis;
                    /* (rho / pi) Le cos_x cos_y / r^2 * A_L  (area light, pdf 1/A_L)
                     * (rho / pi) I cos_x / r^2              (point light, Eq. 3) */
                    double g = (lt == ORA_LIGHT_PARALLELOGRAM ? cx * cy / r2 * AL : cx / r2) / ORA_PI;
                    if (vis)
                        for (int l = 0; l < nl; ++l) L[l] += beta[l] * (double)LeL[l] * g * tmp_T[l];
                }
            }
            countE = 0;
            if (ar->nrc && d >= 2 && !train) {     /* the cache takes the rest of the path */
                double c = ar->nrc_c[0];
                const double xv[3] = {x.x, x.y, x.z}, nv[3] = {n.x, n.y, n.z};
                for (int k = 0; k < 3; ++k) {
                    double u = (xv[k] - ar->nrc_lo[k]) / (ar->nrc_hi[k] - ar->nrc_lo[k]);
                    u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
                    c += ar->nrc_c[1 + k] * u + ar->nrc_c[4 + k] * nv[k];
                }
                for (int l = 0; l < nl; ++l) L[l] += beta[l] * c;
                break;
            }
            if (d == D) break;
            if (ar->nrc && train && d >= 2 && rows && d - 2 < 64) {
                uint32_t ctr[4] = {p, s, (uint32_t)d, 3u}, key[2] = {ar->seed, ar->render_id}, o[4];
                ora_philox4x32_10(ctr, key, o);
                const int l = (int)(o[0] % (uint32_t)nl);
                double *r = rows + (size_t)(d - 2) * 9;
                r[0] = 1.0; r[1] = x.x; r[2] = x.y; r[3] = x.z; r[4] = (double)sc->lambda_nm[l];
                r[5] = n.x; r[6] = n.y; r[7] = n.z;
                row_l[d - 2] = l; row_L[d - 2] = L[l]; row_b[d - 2] = beta[l];
            }
            double nn[3] = {n.x, n.y, n.z}, wd[3];
            ora_cosine_hemisphere(nn, uc[0], uc[1], wd);
            dir = mk(wd[0], wd[1], wd[2]);
            o = xo;
            exclude = prim;
            continue;
        }
        /* glass pane: zero-thickness geometry carrying a slab of thickness d */
        {
            double c = fabs(dot(dir, ng));
            int coated_side = dot(dir, ng) < 0.0;
            double sumR = 0.0, sumT = 0.0;
            for (int l = 0; l < nl; ++l) {
                double Rl, Tl;
                pane_RT(sc, m, l, c, coated_side, &Rl, &Tl);
                sumR += Rl; sumT += Tl;
                tmp_T[l] = Rl;          /* keep R; T is recomputed if the ray transmits */
            }
            if (!(sumR + sumT > 0.0)) break;
            double PR = sumR / (sumR + sumT);
            if (d == D) break;
            rng_u(ar->seed, ar->render_id, p, s, (uint32_t)d, 0, ub);
            if (pr) { pr[7] = ub[2]; pr[8] = PR; }
            if (ub[2] < PR) {
                for (int l = 0; l < nl; ++l) beta[l] *= tmp_T[l] / PR;
                dir = sub(dir, scl(ng, 2.0 * dot(dir, ng)));
                countE = 1;
                o = add(x, scl(n, ORA_OFFSET));
            } else {
                for (int l = 0; l < nl; ++l) {
                    double Rl, Tl;
                    pane_RT(sc, m, l, c, coated_side, &Rl, &Tl);
                    beta[l] *= Tl / (1.0 - PR);
                }
                o = sub(x, scl(n, ORA_OFFSET));
            }
            exclude = prim;
        }
    }
    if (rows)
        for (int k = 0; k < D - 1 && k < 64; ++k)
            if (rows[(size_t)k * 9] != 0.0)
                rows[(size_t)k * 9 + 8] = row_b[k] != 0.0 ? (L[row_l[k]] - row_L[k]) / row_b[k] : NAN;
}

int ora_render(const ora_scene *sc, const ora_accel *acc, const ora_args *ar, ora_out *out) {
    if (!sc || !ar || !out || ar->W <= 0 || ar->H <= 0 || ar->spp <= 0 || ar->max_depth <= 0) return -1;
    if (sc->n_lambda <= 0) return -1;
    const ora_accel *a = ar->use_bvh ? acc : NULL;
    const int nl = sc->n_lambda, D = ar->max_depth, spp = ar->spp;
    const int n_out = ar->n_pix > 0 ? ar->n_pix : ar->W * ar->H;
    int64_t n_ext = 0, n_sh = 0;
    if (ar->n_threads > 0) {
#ifdef _OPENMP
        omp_set_num_threads(ar->n_threads);
#endif
    }
#pragma omp parallel reduction(+ : n_ext, n_sh)
    {
        double *L = (double *)malloc(sizeof(double) * (size_t)nl);
        double *acc_l = (double *)malloc(sizeof(double) * (size_t)nl);
        double *beta = (double *)malloc(sizeof(double) * (size_t)nl);
        double *tmpT = (double *)malloc(sizeof(double) * (size_t)nl);
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < n_out; ++i) {
            int p = ar->n_pix > 0 ? ar->pix[i] : i;
            int px = p % ar->W, py = p / ar->W;
            for (int l = 0; l < nl; ++l) acc_l[l] = 0.0;
            for (int j = 0; j < spp; ++j) {
                size_t slot = (size_t)i * spp + j;
                int32_t *hl = out->hit_log ? out->hit_log + slot * D : NULL;
                int32_t *sl = out->shadow_log ? out->shadow_log + slot * D : NULL;
                if (hl) for (int d = 0; d < D; ++d) hl[d] = -2;
                if (sl) for (int d = 0; d < D; ++d) sl[d] = -2;
                double *fh = out->first_hit ? out->first_hit + slot * 3 : NULL;
                double *rw = out->nrc_rows ? out->nrc_rows + slot * (size_t)(D - 1) * 9 : NULL;
                const uint32_t s = (uint32_t)(ar->sample_offset + j);
                const uint64_t q = ar->window ? (uint64_t)s * (uint64_t)n_out + (uint64_t)i
                                              : (uint64_t)s * (uint64_t)ar->W * (uint64_t)ar->H + (uint64_t)p;
                trace_path(sc, a, ar, px, py, s, q, L, hl, sl, fh, beta, tmpT, &n_ext, &n_sh, rw, NULL);
                if (out->path_L) memcpy(out->path_L + slot * nl, L, sizeof(double) * (size_t)nl);
                for (int l = 0; l < nl; ++l) acc_l[l] += L[l];
            }
            if (out->spectral)
                for (int l = 0; l < nl; ++l) out->spectral[(size_t)i * nl + l] = acc_l[l] / spp;
            if (out->xyz) {
                for (int c = 0; c < 3; ++c) {
                    double v = 0.0;
                    for (int l = 0; l < nl; ++l) v += sc->lambda_w[l] * sc->cmf[3 * l + c] * (acc_l[l] / spp);
                    out->xyz[(size_t)i * 3 + c] = v;
                }
            }
        }
        free(L); free(acc_l); free(beta); free(tmpT);
    }
    out->n_ext_rays = n_ext;
    out->n_shadow_rays = n_sh;
    return 0;
}

int ora_probe_paths(const ora_scene *sc, const ora_accel *acc, const ora_args *ar, int n, const int32_t *pix,
                    const int32_t *samp, double *out) {
    if (!sc || !ar || !out || n < 0 || ar->max_depth <= 0 || sc->n_lambda <= 0) return -1;
    const ora_accel *a = ar->use_bvh ? acc : NULL;
    const int nl = sc->n_lambda, D = ar->max_depth;
    int rc = 0;
#pragma omp parallel
    {
        double *L = (double *)malloc(sizeof(double) * (size_t)nl);
        double *beta = (double *)malloc(sizeof(double) * (size_t)nl);
        double *tmpT = (double *)malloc(sizeof(double) * (size_t)nl);
        int64_t ne = 0, ns = 0;
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < n; ++i) {
            const int p = pix[i];
            if (p < 0 || p >= ar->W * ar->H) { rc = -1; continue; }
            const uint64_t q = (uint64_t)(uint32_t)samp[i] * (uint64_t)ar->W * (uint64_t)ar->H + (uint64_t)p;
            trace_path(sc, a, ar, p % ar->W, p / ar->W, (uint32_t)samp[i], q, L, NULL, NULL, NULL, beta, tmpT, &ne,
                       &ns, NULL, out + (size_t)i * D * ORA_PROBE_STRIDE);
        }
        free(L); free(beta); free(tmpT);
    }
    return rc;
}
