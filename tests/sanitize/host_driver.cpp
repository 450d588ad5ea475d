// The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
// (device code is linked uninstrumented and never launched): scene validation
// on the scene of argv[1] and on damaged copies of it, the subdomain grid and
// binned-SAH BVH builder over several grids and leaf sizes, the launch-setting
// checks and the tuning results file (argv[2], a scratch path).  Any sanitizer
// report fails the calling test.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bvh_build.h"
#include "sdd.h"
extern "C" {
#include "scene_io.h"
}

int main(int argc, char** argv) {
    if (argc < 3) return 2;
    const char* dir = argv[1];
    const int V = (int)meta_get(dir, "n_verts"), T = (int)meta_get(dir, "n_tris");
    const int nl = (int)meta_get(dir, "n_lambda"), M = (int)meta_get(dir, "n_mats");
    sdd_scene_desc d{};
    d.n_verts = V;
    d.verts = (const float*)read_bin(dir, "verts", 12L * V);
    d.n_tris = T;
    d.tris = (const int32_t*)read_bin(dir, "tris", 12L * T);
    d.tri_mat = (const int32_t*)read_bin(dir, "tri_mat", 4L * T);
    d.n_lambda = nl;
    d.lambda_nm = (const float*)read_bin(dir, "lambda_nm", 4L * nl);
    d.lambda_w = (const double*)read_bin(dir, "lambda_w", 8L * nl);
    d.cmf = (const double*)read_bin(dir, "cmf", 24L * nl);
    d.n_mats = M;
    d.mat_type = (const int32_t*)read_bin(dir, "mat_type", 4L * M);
    d.mat_rho = (const float*)read_bin(dir, "mat_rho", 4L * M * nl);
    d.mat_n = (const float*)read_bin(dir, "mat_n", 4L * M * nl);
    d.mat_k = (const float*)read_bin(dir, "mat_k", 4L * M * nl);
    d.mat_thick = (const float*)read_bin(dir, "mat_thick", 4L * M);
    d.mat_le = (const float*)read_bin(dir, "mat_le", 4L * M * nl);
    d.light_type = (int)meta_get(dir, "light_type");
    d.light_mat = (int)meta_get(dir, "light_mat");
    float* lp[3] = {(float*)read_bin(dir, "light_p0", 12), (float*)read_bin(dir, "light_e1", 12),
                    (float*)read_bin(dir, "light_e2", 12)};
    std::memcpy(d.light_p0, lp[0], 12);
    std::memcpy(d.light_e1, lp[1], 12);
    std::memcpy(d.light_e2, lp[2], 12);
    const int Lm = (int)meta_get(dir, "max_layers");
    if (Lm > 0) {
        d.max_layers = Lm;
        d.mat_n_layers = (const int32_t*)read_bin(dir, "mat_n_layers", 4L * M);
        d.mat_layer_d = (const float*)read_bin(dir, "mat_layer_d", 4L * M * Lm);
        d.mat_layer_n = (const float*)read_bin(dir, "mat_layer_n", 4L * M * Lm * nl);
        d.mat_layer_k = (const float*)read_bin(dir, "mat_layer_k", 4L * M * Lm * nl);
    }
    char msg[256];
    int bad = 0;
    if (sdd_validate_scene(&d, msg, sizeof msg) != SDD_OK) {
        std::printf("valid scene rejected: %s\n", msg);
        bad = 1;
    }
    // damaged copies: an index out of range, a non-finite vertex, rho above 1, no triangles
    std::vector<int32_t> tris(d.tris, d.tris + 3L * T);
    std::vector<float> verts(d.verts, d.verts + 3L * V), rho(d.mat_rho, d.mat_rho + (long)M * nl);
    sdd_scene_desc e = d;
    tris[4] = V;
    e.tris = tris.data();
    bad |= sdd_validate_scene(&e, msg, sizeof msg) != SDD_ERR_INVALID_ARG;
    e = d;
    verts[7] = 1.0f / 0.0f;
    e.verts = verts.data();
    bad |= sdd_validate_scene(&e, msg, sizeof msg) != SDD_ERR_INVALID_ARG;
    e = d;
    rho[0] = 1.5f;
    e.mat_rho = rho.data();
    bad |= sdd_validate_scene(&e, msg, sizeof msg) != SDD_ERR_INVALID_ARG;
    e = d;
    e.n_tris = 0;
    bad |= sdd_validate_scene(&e, msg, sizeof msg) != SDD_ERR_INVALID_ARG;

    // the host grid and BVH builder
    std::vector<int32_t> glass_of(M, -1), emits(M, 0);
    int ng = 0;
    for (int m = 0; m < M; ++m) {
        if (d.mat_type[m] == SDD_MAT_GLASS_SLAB) glass_of[m] = ng++;
        for (int l = 0; l < nl; ++l) emits[m] |= d.mat_le[(long)m * nl + l] > 0.0f;
    }
    const int grids[4][3] = {{1, 1, 1}, {2, 2, 1}, {4, 4, 2}, {3, 5, 2}};
    for (const auto& g : grids)
        for (int leaf : {1, 3, 8}) {
            sdd::BuildInput in{d.verts, V, d.tris, T, d.tri_mat, d.mat_type, glass_of.data(), emits.data(),
                               g[0], g[1], g[2], leaf, 16};
            sdd::GridBvh out;
            std::string err;
            if (!sdd::build_grid_bvh(in, out, err) || out.n_refs < T || out.nodes.empty()) {
                std::printf("build %dx%dx%d leaf %d failed: %s\n", g[0], g[1], g[2], leaf, err.c_str());
                bad = 1;
            } else {
                std::printf("build %dx%dx%d leaf %d: refs %lld nodes %zu depth %d\n", g[0], g[1], g[2], leaf,
                            (long long)out.n_refs, out.nodes.size() / 8, out.max_depth);
            }
        }
    std::vector<sdd::HostF4> info;
    sdd::BuildInput in{d.verts, V, d.tris, T, d.tri_mat, d.mat_type, glass_of.data(), emits.data(), 1, 1, 1, 3, 16};
    sdd::triangle_info(in, info);
    bad |= (long)info.size() != T;

    // launch settings and the tuning results file
    sdd_tuning t{};
    bad |= sdd_validate_tuning(&t, msg, sizeof msg) != SDD_OK;
    t.batch_paths = 511;
    bad |= sdd_validate_tuning(&t, msg, sizeof msg) != SDD_ERR_INVALID_ARG;
    t = sdd_tuning{1 << 20, 64, 4};
    bad |= sdd_tune_cache_store(argv[2], "key one", &t, 12.5) != SDD_OK;
    bad |= sdd_tune_cache_store(argv[2], "key\ttwo", &t, 1.0) != SDD_ERR_INVALID_ARG;
    FILE* f = std::fopen(argv[2], "a");
    std::fputs("key one\tgarbage line\nkey one\t12\n", f);
    std::fclose(f);
    sdd_tuning r{};
    double ms = 0.0;
    int32_t found = 0;
    bad |= sdd_tune_cache_lookup(argv[2], "key one", &r, &ms, &found) != SDD_OK;
    bad |= !(found == 1 && r.batch_paths == (1 << 20) && r.trace_grid == 64 && r.dir_bins == 4 && ms == 12.5);
    bad |= sdd_tune_cache_lookup(argv[2], "absent", &r, &ms, &found) != SDD_OK || found != 0;
    std::printf("host checks %s\n", bad ? "FAILED" : "ok");

    for (const void* p : {(const void*)d.verts, (const void*)d.tris, (const void*)d.tri_mat, (const void*)d.lambda_nm,
                          (const void*)d.lambda_w, (const void*)d.cmf, (const void*)d.mat_type, (const void*)d.mat_rho,
                          (const void*)d.mat_n, (const void*)d.mat_k, (const void*)d.mat_thick, (const void*)d.mat_le})
        std::free(const_cast<void*>(p));
    for (float* p : lp) std::free(p);
    if (Lm > 0)
        for (const void* p : {(const void*)d.mat_n_layers, (const void*)d.mat_layer_d, (const void*)d.mat_layer_n,
                              (const void*)d.mat_layer_k})
            std::free(const_cast<void*>(p));
    return bad;
}
