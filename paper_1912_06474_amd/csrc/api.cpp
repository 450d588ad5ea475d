// C ABI of libsdd (include/sdd.h): context, validation, device memory, and
// the host scheduler that drives the per-subdomain queue sweeps.
//
// Sweep schedule of one batch of paths (Sec. 4 inverse ray tracing organised
// as the Sec. 5 domain decomposition):
//   camgen -> for depth d = 1..D:
//       S sweeps of k_trace<closest>  over the subdomain queues
//       k_shade(d)                     (resolves the shadow rays of d-1)
//       S sweeps of k_trace<shadow>
//   k_shade(final) -> k_flush
// S = nx + ny + nz - 2 bounds the number of cells a straight ray can visit,
// so a fixed number of sweeps drains every queue with no host round trip; a
// sweep over empty queues exits after reading the per-cell counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <sstream>
#include <unistd.h>
#include <new>
#include <string>
#include <vector>

#include "bvh_build.h"
#include "bvh_device.h"
#include "bvh_wide.h"
#include "kernels.h"
#include "layout.h"
#include "nrc.h"
#include "sdd.h"

using namespace sdd;

namespace {

struct Render {
    int W = 0, H = 0;      // accumulator size: the render's window
    int fW = 0, fH = 0, x0 = 0, y0 = 0;  // its frame and the window's place in it
    float* acc = nullptr;  // [nl][W*H] FP32
    int* ovf = nullptr;    // overflow bits (kOverflow*) of every call that traced this render
    long long spp_done = 0;
};

struct TimedLaunch {
    int cls;  // 0 ext trace, 1 shadow trace, 2 shade, 3 other, 4 cache query, 5 cache training
    hipEvent_t a, b;
};

}  // namespace

struct sdd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int n_cu = 256;
    int trace_grid = 0, trace_grid_max = 0;
    int ext_bins = 1;  // direction bins per cell of the closest-hit routing
    // launch settings requested through sdd_set_tuning (0: the library's choice)
    long long tune_batch = 0;
    int tune_grid = 0, tune_bins = 0;
    long long last_nb = 0;  // paths per pass of the last trace call

    // scene (host copies used by the builder)
    bool has_scene = false, has_bvh = false;
    int V = 0, T = 0, M = 0, nl = 0, nlp = 0;
    std::vector<float> verts;
    std::vector<int32_t> tris, tri_mat, mat_type, glass_of, mat_emits;
    int n_glass = 0;
    int light_type = 0, light_mat = -1;
    // light geometry in double (FP32 scene values widened exactly; normal and area in double)
    double lp0[3] = {0, 0, 0}, le1[3] = {0, 0, 0}, le2[3] = {0, 0, 0}, nL[3] = {0, 0, 0};
    double light_area = 0.0;

    // device scene
    float4* d_prim_info = nullptr;
    float4* d_prim_v = nullptr;  // [T][3] triangle vertices (w unused), for FP64 shading geometry
    float4* d_pane = nullptr;  // [n_glass][nlp] pane constants
    float4* d_coat = nullptr;  // [n_glass][coat_layers][nlp] coating layer constants (if any)
    int* d_coat_n = nullptr;   // [n_glass] coating layers (if any)
    int max_layers = 0, coat_layers = 0;
    float* d_rho = nullptr;
    float* d_le = nullptr;
    double* d_w = nullptr;
    double* d_cmf = nullptr;

    // device accel
    GridBvh gb;
    uint4* d_nodes = nullptr;
    float4* d_cell_q = nullptr;
    int* d_cell_nodes = nullptr;
    float4* d_tris = nullptr;
    int* d_cell_root = nullptr;
    float* d_planes = nullptr;
    GridParams grid{};
    int G = 0, S = 0;

    // batch buffers
    long long ncap = 0;
    int dcap = 0;  // depth capacity of the counter arrays
    D4* ray_o = nullptr;  // FP64 path state
    D4* ray_d = nullptr;
    float2* hit = nullptr;
    uint32_t* flags = nullptr;
    // path history [depth][path]
    int4* vrec = nullptr;
    int* sh_state = nullptr;
    float2* sh_glass = nullptr;
    // queue buffers: 0/1 closest-hit ping-pong, 2/3 shadow ping-pong
    float4* qa[4] = {nullptr, nullptr, nullptr, nullptr};
    float4* qb[4] = {nullptr, nullptr, nullptr, nullptr};
    int2* qc[4] = {nullptr, nullptr, nullptr, nullptr};
    // rays staged in path order before routing: [0] closest-hit, [1] shadow
    Stage stage[2] = {};
    int n_blocks = 0;
    int* d_counts = nullptr;
    int defer_rays = 0, defer_extra = 0;  // sdd_set_deferral
    long long counts_len = 0;
    long long batch_bytes = 0;  // device bytes of the path batch (ensure_batch)
    long long call_budget = 0;  // memory budget of the current call (set before any capture)
    void* noalloc_scratch = nullptr;  // device address of this device's allocation-free query scratch
    int* d_overflow = nullptr;   // overflow bits of the current trace call (cleared at its start)
    int* d_ovf_stats = nullptr;  // overflow bits since sdd_reset_stats
    int* d_ktot = nullptr;  // routing key totals [2][kMaxCells * kExtBins]
    int* d_gstack = nullptr;  // traversal stack spill: (kStack - kLdsStack) ints per trace thread
    unsigned long long* d_stats = nullptr;

    std::map<int, Render> renders;
    std::map<void*, size_t> allocs;
    long long device_bytes = 0;

    // learned radiance cache
    bool has_nrc = false;
    NrcNet nrc{};
    float nrc_lr = 0.0f, nrc_b1 = 0.0f, nrc_b2 = 0.0f, nrc_eps = 0.0f;
    int nrc_t = 0;  // Adam steps taken
    long long nrc_cap = 0;
    float* nrc_acts = nullptr;
    float* nrc_dz = nullptr;
    float* nrc_y = nullptr;
    float* nrc_dy = nullptr;
    float* nrc_loss = nullptr;
    // cache settings for renders
    int nrc_train_paths = 0, nrc_train_steps = 0, nrc_train_batch = 0, nrc_precision = 1;
    // render buffers of the cache: per batch path, per training slot, training rows
    long long nrc_pcap = 0, nrc_scap = 0;
    int nrc_dcap = 0;
    float4* nrc_cx = nullptr;
    float4* nrc_cn = nullptr;
    float* nrc_lhat = nullptr;
    float4* nrc_tx = nullptr;
    float4* nrc_tn = nullptr;
    float4* nrc_rows = nullptr;
    int* nrc_ok = nullptr;
    float4* nrc_crows = nullptr;
    int* nrc_count = nullptr;
    void* nrc_tmp = nullptr;
    size_t nrc_tmp_bytes = 0;
    float* nrc_bx = nullptr;  // training batch, SoA
    float* nrc_bw = nullptr;
    float* nrc_blam = nullptr;
    float* nrc_bt = nullptr;
    long long nrc_bcap = 0;
    long long nrc_last_rows = 0;
    int nrc_last_steps = 0;
    float nrc_last_loss = 0.0f;
    // the Adam steps after a cache render run on a stream of their own and
    // overlap the next call's tracing: nrc_pending until ev_trained is waited for
    hipStream_t nrc_stream = nullptr;
    hipEvent_t nrc_ev_rows = nullptr, nrc_ev_trained = nullptr;
    bool nrc_pending = false;
    float* nrc_h_loss = nullptr;  // pinned: the last step's loss
    uint32_t* nrc_t16 = nullptr;  // FP16 copy of the tables for BF16 queries (sdd_nrc_desc.table_fp16)
    bool nrc_g_dirty = false;     // gradients hold a step's sums (sdd_nrc_train_step leaves them readable)
    float* d_lam = nullptr;  // scene wavelengths (nm), FP32
    uint4* nrc_hop = nullptr;  // staged matrix operands of cache queries
    uint2* nrc_sop = nullptr;
    uint32_t* nrc_okeys = nullptr;  // gather order of the cache queries: sort keys [2][paths],
    int* nrc_ovals = nullptr;       // path indices [2][paths], and the sort's scratch
    char* nrc_otemp = nullptr;
    size_t nrc_otemp_bytes = 0;
    int* nrc_flags = nullptr;  // a render query's paths with a cache vertex: flags, rows (paths + 1 each),
    int* nrc_rank = nullptr;   // and the path of each row
    int* nrc_cp = nullptr;
    long long nrc_ocap = 0;

    // graph replay of repeated trace calls (SDD_TRACE_GRAPH)
    long long gen = 0;            // bumped whenever a buffer a captured graph may use is (re)allocated or freed
    int* d_s0 = nullptr;          // per-render first sample index, read by the kernels of a graph
    int s0_cap = 0;
    std::vector<int> h_s0;
    std::string graph_key;
    hipGraphExec_t graph_exec = nullptr;
    long long graph_cam_rays = 0, graph_launches = 0, graph_batches = 0;

    // host stats
    long long batches = 0, launches_trace = 0, cam_rays = 0;
    double ms[6] = {0, 0, 0, 0, 0, 0};
    long long nrc_query_rows = 0, nrc_query_launches = 0, nrc_train_rows = 0;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    int leftover = 0;
};

namespace {

sdd_status fail(sdd_ctx* c, sdd_status st, const std::string& msg) {
    if (c) c->err = msg;
    return st;
}

// trace workgroups: as many as stay resident on every CU, a multiple of the XCD count
int trace_grid_for(const sdd_ctx* c, int n_cells) {
    return std::max(kXcd, (c->n_cu * trace_blocks_per_cu(n_cells) / kXcd) * kXcd);
}

// traversal grid and direction bins from the requested settings and the grid of cells
void apply_tuning(sdd_ctx* c) {
    const int g_auto = std::min(c->trace_grid_max, trace_grid_for(c, c->G));
    c->trace_grid = c->tune_grid > 0 ? std::min(c->tune_grid, c->trace_grid_max) : g_auto;
    c->ext_bins = (c->tune_bins == 1 || c->G * kExtBins > kMaxCells) ? 1 : kExtBins;
}

// reason a tuning is malformed, or nullptr (host-only checks)
const char* tuning_problem(const sdd_tuning* t) {
    if (!t) return "null tuning";
    if (t->batch_paths != 0 &&
        (t->batch_paths < kShadeBlock || t->batch_paths > kMaxBatch || t->batch_paths % kShadeBlock != 0))
        return "batch_paths must be 0 or a multiple of 512 in [512, 2^24]";
    if (t->trace_grid < 0 || t->trace_grid % kXcd != 0) return "trace_grid must be 0 or a positive multiple of 8";
    if (t->dir_bins != 0 && t->dir_bins != 1 && t->dir_bins != kExtBins) return "dir_bins must be 0, 1 or 4";
    return nullptr;
}

sdd_status hip_fail(sdd_ctx* c, hipError_t e, const char* what) {
    return fail(c, SDD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                          \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return hip_fail((c), e_, #expr);    \
    } while (0)

template <class T>
sdd_status dalloc(sdd_ctx* c, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, SDD_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    c->allocs[q] = bytes;
    c->device_bytes += (long long)bytes;
    *p = static_cast<T*>(q);
    return SDD_OK;
}

template <class T>
void dfree(sdd_ctx* c, T*& p) {
    if (!p) return;
    auto it = c->allocs.find((void*)p);
    if (it != c->allocs.end()) {
        c->device_bytes -= (long long)it->second;
        c->allocs.erase(it);
    }
    (void)hipFree((void*)p);
    p = nullptr;
}

template <class T>
sdd_status upload(sdd_ctx* c, T** p, const T* src, size_t count) {
    sdd_status st = dalloc(c, p, count);
    if (st != SDD_OK) return st;
    if (count) HIP_TRY(c, hipMemcpyAsync(*p, src, count * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return SDD_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void free_scene(sdd_ctx* c) {
    ++c->gen;
    dfree(c, c->d_prim_info);
    dfree(c, c->d_prim_v);
    dfree(c, c->d_pane);
    dfree(c, c->d_coat);
    dfree(c, c->d_coat_n);
    c->coat_layers = 0;
    dfree(c, c->d_rho);
    dfree(c, c->d_le);
    dfree(c, c->d_w);
    dfree(c, c->d_cmf);
    dfree(c, c->d_lam);
    c->has_scene = false;
}

void free_accel(sdd_ctx* c) {
    ++c->gen;
    dfree(c, c->d_nodes);
    dfree(c, c->d_cell_q);
    dfree(c, c->d_cell_nodes);
    dfree(c, c->d_tris);
    dfree(c, c->d_cell_root);
    dfree(c, c->d_planes);
    c->has_bvh = false;
}

void free_batch(sdd_ctx* c) {
    ++c->gen;
    dfree(c, c->ray_o);
    dfree(c, c->ray_d);
    dfree(c, c->hit);
    dfree(c, c->flags);
    dfree(c, c->vrec);
    dfree(c, c->sh_state);
    dfree(c, c->sh_glass);
    for (int i = 0; i < 4; ++i) {
        dfree(c, c->qa[i]);
        dfree(c, c->qb[i]);
        dfree(c, c->qc[i]);
    }
    for (int k = 0; k < 2; ++k) {
        dfree(c, c->stage[k].qa);
        dfree(c, c->stage[k].qb);
        dfree(c, c->stage[k].qc);
        dfree(c, c->stage[k].tag);
        dfree(c, c->stage[k].hist);
    }
    dfree(c, c->d_counts);
    c->ncap = 0;
    c->dcap = 0;
    c->batch_bytes = 0;
}

hipError_t nrc_wait_host(sdd_ctx* c);

void free_nrc_batch(sdd_ctx* c) {
    dfree(c, c->nrc_acts);
    dfree(c, c->nrc_dz);
    dfree(c, c->nrc_y);
    dfree(c, c->nrc_dy);
    c->nrc_cap = 0;
}

void free_nrc_render(sdd_ctx* c) {
    dfree(c, c->nrc_cx);
    dfree(c, c->nrc_cn);
    dfree(c, c->nrc_lhat);
    dfree(c, c->nrc_tx);
    dfree(c, c->nrc_tn);
    dfree(c, c->nrc_rows);
    dfree(c, c->nrc_ok);
    dfree(c, c->nrc_crows);
    dfree(c, c->nrc_count);
    dfree(c, c->nrc_tmp);
    dfree(c, c->nrc_bx);
    dfree(c, c->nrc_bw);
    dfree(c, c->nrc_blam);
    dfree(c, c->nrc_bt);
    c->nrc_pcap = c->nrc_scap = c->nrc_bcap = 0;
    c->nrc_dcap = 0;
    c->nrc_tmp_bytes = 0;
}

void free_nrc(sdd_ctx* c) {
    (void)nrc_wait_host(c);
    if (c->nrc_stream) (void)hipStreamDestroy(c->nrc_stream);
    if (c->nrc_ev_rows) (void)hipEventDestroy(c->nrc_ev_rows);
    if (c->nrc_ev_trained) (void)hipEventDestroy(c->nrc_ev_trained);
    if (c->nrc_h_loss) (void)hipHostFree(c->nrc_h_loss);
    c->nrc_stream = nullptr;
    c->nrc_ev_rows = c->nrc_ev_trained = nullptr;
    c->nrc_h_loss = nullptr;
    dfree(c, c->nrc_t16);
    free_nrc_render(c);
    dfree(c, c->nrc_hop);
    dfree(c, c->nrc_sop);
    dfree(c, c->nrc_okeys);
    dfree(c, c->nrc_flags);
    dfree(c, c->nrc_rank);
    dfree(c, c->nrc_cp);
    dfree(c, c->nrc_ovals);
    dfree(c, c->nrc_otemp);
    c->nrc_ocap = 0;
    c->nrc_otemp_bytes = 0;
    free_nrc_batch(c);
    dfree(c, c->nrc_loss);
    dfree(c, c->nrc.p);
    dfree(c, c->nrc.g);
    dfree(c, c->nrc.m);
    dfree(c, c->nrc.v);
    dfree(c, c->nrc.wq);
    dfree(c, c->nrc.wf);
    c->has_nrc = false;
}

void free_renders(sdd_ctx* c) {
    ++c->gen;
    for (auto& kv : c->renders) {
        dfree(c, kv.second.acc);
        dfree(c, kv.second.ovf);
    }
    c->renders.clear();
}

std::string validate(const sdd_scene_desc* s) {
    if (!s) return "null scene";
    if (s->n_tris <= 0) return "scene has no triangles";
    if (s->n_verts <= 0 || !s->verts) return "scene has no vertices";
    if (!s->tris || !s->tri_mat) return "null triangle arrays";
    if (s->n_lambda < 1 || s->n_lambda > SDD_MAX_LAMBDA) return "n_lambda out of range";
    if (!s->lambda_nm || !s->lambda_w || !s->cmf) return "null wavelength arrays";
    if (s->n_mats <= 0 || !s->mat_type || !s->mat_rho || !s->mat_n || !s->mat_k || !s->mat_thick || !s->mat_le)
        return "null material arrays";
    for (long long i = 0; i < 3LL * s->n_verts; ++i)
        if (!std::isfinite(s->verts[i])) return "non-finite vertex coordinate at " + std::to_string(i / 3);
    for (long long i = 0; i < 3LL * s->n_tris; ++i)
        if (s->tris[i] < 0 || s->tris[i] >= s->n_verts) return "vertex index out of range in triangle " + std::to_string(i / 3);
    for (int i = 0; i < s->n_tris; ++i)
        if (s->tri_mat[i] < 0 || s->tri_mat[i] >= s->n_mats) return "material index out of range in triangle " + std::to_string(i);
    for (int l = 0; l < s->n_lambda; ++l) {
        if (!(s->lambda_nm[l] > 0.0f) || !std::isfinite(s->lambda_nm[l])) return "wavelength must be positive";
        if (!std::isfinite(s->lambda_w[l])) return "non-finite wavelength weight";
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(s->cmf[3 * l + k])) return "non-finite colour matching value";
    }
    const int nl = s->n_lambda;
    for (int m = 0; m < s->n_mats; ++m) {
        const int t = s->mat_type[m];
        if (t != SDD_MAT_DIFFUSE && t != SDD_MAT_GLASS_SLAB && t != SDD_MAT_EMITTER) return "unknown material type";
        if (!(s->mat_thick[m] >= 0.0f) || !std::isfinite(s->mat_thick[m])) return "slab thickness must be >= 0";
        for (int l = 0; l < nl; ++l) {
            const size_t i = (size_t)m * nl + l;
            if (!(s->mat_rho[i] >= 0.0f && s->mat_rho[i] <= 1.0f)) return "reflectance outside [0, 1]";
            if (!(s->mat_n[i] > 0.0f) || !std::isfinite(s->mat_n[i])) return "refractive index n must be > 0";
            if (!(s->mat_k[i] >= 0.0f) || !std::isfinite(s->mat_k[i])) return "absorption index k must be >= 0";
            if (!(s->mat_le[i] >= 0.0f) || !std::isfinite(s->mat_le[i])) return "emission must be >= 0";
            if (t == SDD_MAT_GLASS_SLAB && s->mat_le[i] != 0.0f) return "glass material cannot emit";
        }
    }
    if (s->max_layers < 0 || s->max_layers > SDD_MAX_LAYERS) return "max_layers out of range";
    if (s->max_layers > 0) {
        if (!s->mat_n_layers || !s->mat_layer_d || !s->mat_layer_n || !s->mat_layer_k) return "null coating arrays";
        const int Lm = s->max_layers;
        for (int m = 0; m < s->n_mats; ++m) {
            const int L = s->mat_n_layers[m];
            if (L < 0 || L > Lm) return "coating layer count out of range";
            if (L > 0 && s->mat_type[m] != SDD_MAT_GLASS_SLAB) return "only glass materials carry coatings";
            for (int j = 0; j < L; ++j) {
                const float d = s->mat_layer_d[(size_t)m * Lm + j];
                if (!(d >= 0.0f) || !std::isfinite(d)) return "coating layer thickness must be >= 0";
                for (int l = 0; l < nl; ++l) {
                    const size_t i = ((size_t)m * Lm + j) * nl + l;
                    if (!(s->mat_layer_n[i] > 0.0f) || !std::isfinite(s->mat_layer_n[i])) return "coating n must be > 0";
                    if (!(s->mat_layer_k[i] >= 0.0f) || !std::isfinite(s->mat_layer_k[i])) return "coating k must be >= 0";
                }
            }
        }
    }
    if (s->light_type != SDD_LIGHT_NONE && s->light_type != SDD_LIGHT_PARALLELOGRAM && s->light_type != SDD_LIGHT_POINT)
        return "unknown light type";
    if (s->light_type != SDD_LIGHT_NONE) {
        if (s->light_mat < 0 || s->light_mat >= s->n_mats) return "light material out of range";
        if (s->mat_type[s->light_mat] != SDD_MAT_EMITTER) return "light material must be an emitter";
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(s->light_p0[k]) || !std::isfinite(s->light_e1[k]) || !std::isfinite(s->light_e2[k]))
                return "non-finite light geometry";
        if (s->light_type == SDD_LIGHT_PARALLELOGRAM) {
            const double e1[3] = {s->light_e1[0], s->light_e1[1], s->light_e1[2]};
            const double e2[3] = {s->light_e2[0], s->light_e2[1], s->light_e2[2]};
            const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                         cz = e1[0] * e2[1] - e1[1] * e2[0];
            if (!(cx * cx + cy * cy + cz * cz > 0.0)) return "degenerate parallelogram light";
        }
    }
    return "";
}

hipEvent_t take_event(sdd_ctx* c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// collect the durations of finished timed launches (stream must be synchronised)
void harvest_events(sdd_ctx* c) {
    for (auto& t : c->timed) {
        float ms = 0.0f;
        if (t.a && t.b && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) c->ms[t.cls] += ms;
        if (t.a) c->event_pool.push_back(t.a);
        if (t.b) c->event_pool.push_back(t.b);
    }
    c->timed.clear();
}

struct Timer {
    sdd_ctx* c;
    bool on;
    hipStream_t st;
    TimedLaunch t{};
    Timer(sdd_ctx* ctx, bool enabled, int cls, hipStream_t stream = nullptr)
        : c(ctx), on(enabled), st(stream ? stream : ctx->stream) {
        if (!on) return;
        t.cls = cls;
        t.a = take_event(c);
        t.b = take_event(c);
        if (t.a) (void)hipEventRecord(t.a, st);
    }
    ~Timer() {
        if (!on) return;
        if (t.b) (void)hipEventRecord(t.b, st);
        c->timed.push_back(t);
    }
};

// The cache's Adam steps after a render (nrc_train_after_call) may still run
// on c->nrc_stream.  nrc_wait_gpu orders the context stream after them (the
// next render's cache query); nrc_wait_host waits for them on the host (every
// API call that reads, changes or frees the cache, and statistics).
void nrc_wait_gpu(sdd_ctx* c) {
    if (c->nrc_pending) (void)hipStreamWaitEvent(c->stream, c->nrc_ev_trained, 0);
}

// the network as BF16 queries and BF16 rows evaluate it: with the FP16 copy
// of the tables when the cache keeps one (training reads c->nrc, FP32 tables)
NrcNet qnet(const sdd_ctx* c) {
    NrcNet n = c->nrc;
    n.t16 = c->nrc_t16;
    return n;
}

hipError_t nrc_wait_host(sdd_ctx* c) {
    if (!c->nrc_pending) return hipSuccess;
    const hipError_t e = hipEventSynchronize(c->nrc_ev_trained);
    c->nrc_pending = false;
    if (c->nrc_h_loss) c->nrc_last_loss = *c->nrc_h_loss;
    return e;
}

// Device memory the path batch (queues, path state, history) may take:
// SDD_MEM_BUDGET_GB if set, else half the device's memory, at most three
// quarters of what is free plus what this context's batch already holds (it
// is freed before a larger one is allocated), and at least 4 GiB.  Queues
// take O(cells x batch) memory, so many-cell grids run larger batches, and
// fewer of them, when the budget is larger.
long long mem_budget_bytes(const sdd_ctx* c) {
    constexpr double kGiB = 1024.0 * 1024.0 * 1024.0;
    if (const char* s = std::getenv("SDD_MEM_BUDGET_GB")) {
        const double gb = std::atof(s);
        if (gb > 0.0) return (long long)(gb * kGiB);
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || total_b == 0) return (long long)(48.0 * kGiB);
    const double avail = (double)free_b + (double)c->batch_bytes;
    const double budget = std::min(0.5 * (double)total_b, 0.75 * avail);
    return (long long)std::max(budget, 4.0 * kGiB);
}

long long bytes_per_path(const sdd_ctx* c, int max_depth) {
    return 4LL * c->G * (16 + 16 + 8) + 2 * (16 + 16 + 8 + 4) + 2 * (long long)sizeof(D4) + 8 + 4 +
           (long long)max_depth * (16 + 4 + 8 * kMaxGlass);
}

sdd_status ensure_batch(sdd_ctx* c, long long n, int max_depth) {
    const long long cnt_len = (long long)(2 * max_depth + 1) * (c->S + kMaxDeferExtra + 1) * c->G * kCntStride;
    if (n <= c->ncap && max_depth <= c->dcap) return SDD_OK;
    free_batch(c);
    const long long bytes0 = c->device_bytes;
    sdd_status st;
    const long long qn = (long long)c->G * n;
#define ALLOC(ptr, cnt)                            \
    if ((st = dalloc(c, &(ptr), (size_t)(cnt))) != SDD_OK) { \
        free_batch(c);                             \
        return st;                                 \
    }
    ALLOC(c->ray_o, n);
    ALLOC(c->ray_d, n);
    ALLOC(c->hit, n);
    ALLOC(c->flags, n);
    ALLOC(c->vrec, n * max_depth);
    ALLOC(c->sh_state, n * max_depth);
    ALLOC(c->sh_glass, n * max_depth * kMaxGlass);
    for (int i = 0; i < 4; ++i) {
        ALLOC(c->qa[i], qn);
        ALLOC(c->qb[i], qn);
        ALLOC(c->qc[i], qn);
    }
    const long long nblk = (n + kShadeBlock - 1) / kShadeBlock;
    for (int k = 0; k < 2; ++k) {
        ALLOC(c->stage[k].qa, n);
        ALLOC(c->stage[k].qb, n);
        ALLOC(c->stage[k].qc, n);
        ALLOC(c->stage[k].tag, n);
        ALLOC(c->stage[k].hist, nblk * c->G * kExtBins);
    }
    ALLOC(c->d_counts, cnt_len);
#undef ALLOC
    // the path history is replayed up to each path's end; zero it once so
    // that no record is ever uninitialised memory
    HIP_TRY(c, hipMemsetAsync(c->vrec, 0, sizeof(int4) * (size_t)(n * max_depth), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->sh_state, 0, sizeof(int) * (size_t)(n * max_depth), c->stream));
    c->counts_len = cnt_len;
    c->ncap = n;
    c->dcap = max_depth;
    c->batch_bytes = c->device_bytes - bytes0;
    return SDD_OK;
}

// counters of (phase, sweep); phase 2(d-1) holds the closest-hit rays of
// depth d, phase 2(d-1)+1 the shadow rays of depth d
// sweeps per depth: the S that drain every queue, plus a deferral schedule's extra sweeps
inline int n_sweeps(const sdd_ctx* c) { return c->S + (c->defer_rays > 0 ? c->defer_extra : 0); }

inline int* counts_at(sdd_ctx* c, int phase, int k) {
    return c->d_counts + ((long long)phase * (c->S + kMaxDeferExtra + 1) + k) * c->G * kCntStride;
}
inline int ph_ext(int d) { return 2 * (d - 1); }
inline int ph_sh(int d) { return 2 * (d - 1) + 1; }

QueueSet queue_set(sdd_ctx* c, int in_buf, int out_buf, int phase, int k) {
    QueueSet q{};
    q.qa_in = c->qa[in_buf];
    q.qb_in = c->qb[in_buf];
    q.qc_in = c->qc[in_buf];
    q.cnt_in = counts_at(c, phase, k);
    q.qa_out = c->qa[out_buf];
    q.qb_out = c->qb[out_buf];
    q.qc_out = c->qc[out_buf];
    q.cnt_out = counts_at(c, phase, k + 1);
    return q;
}

// S sweeps over the subdomain queues.  ext_phase / sh_phase < 0: that kind is
// idle.  Closest-hit rays start in buffer 0 (partner 1), shadow rays in
// buffer 2 (partner 3); their results go to the history arrays of depth
// sh_depth (path stride n_paths).
sdd_status run_sweeps(sdd_ctx* c, int ext_phase, int sh_phase, long long cap, bool count, bool timing,
                      int sh_depth = 0, long long n_paths = 0) {
    const int S = n_sweeps(c);
    for (int k = 0; k < S; ++k) {
        TraceParams p{};
        p.defer_below = c->defer_rays;
        p.sweep = k;
        p.n_sweeps = S;
        const bool even = k % 2 == 0;
        if (ext_phase >= 0) p.q[0] = queue_set(c, even ? 0 : 1, even ? 1 : 0, ext_phase, k);
        if (sh_phase >= 0) p.q[1] = queue_set(c, even ? 2 : 3, even ? 3 : 2, sh_phase, k);
        p.active[0] = ext_phase >= 0;
        p.active[1] = sh_phase >= 0;
        p.cap = cap;
        p.n_cells = c->G;
        p.grid = c->grid;
        p.nodes = c->d_nodes;
        p.cell_q = c->d_cell_q;
        p.cell_nodes = c->d_cell_nodes;
        p.tris = c->d_tris;
        p.cell_root = c->d_cell_root;
        p.prim_info = c->d_prim_info;
        p.hit = c->hit;
        if (sh_depth > 0) {
            const long long off = (long long)(sh_depth - 1) * n_paths;
            p.sh_state = c->sh_state + off;
            p.sh_glass = c->sh_glass + off * kMaxGlass;
        }
        p.overflow = c->d_overflow;
        p.gstack = c->d_gstack;
        p.stats = c->d_stats;
        Timer tm(c, timing, sh_phase >= 0 && ext_phase < 0 ? 1 : 0);
        HIP_TRY(c, launch_trace(p, count, c->trace_grid, c->stream));
        ++c->launches_trace;
    }
    return SDD_OK;
}

// scatter the staged rays of a batch into the per-cell queues: closest-hit
// rays to buffer 0 (counters of ext_phase), shadow rays to buffer 2
sdd_status route(sdd_ctx* c, int N, long long cap, int ext_phase, int sh_phase, bool count_ext, bool timing) {
    RouteParams r{};
    r.N = N;
    r.n_blocks = (N + kShadeBlock - 1) / kShadeBlock;
    r.n_cells = c->G;
    r.cap = cap;
    r.active[0] = ext_phase >= 0;
    r.active[1] = sh_phase >= 0;
    r.nbin[0] = c->ext_bins;
    r.nbin[1] = 1;
    r.ktot[0] = c->d_ktot;
    r.ktot[1] = c->d_ktot + kMaxCells * kExtBins;
    for (int k = 0; k < 2; ++k) r.st[k] = c->stage[k];
    r.qa[0] = c->qa[0];
    r.qb[0] = c->qb[0];
    r.qc[0] = c->qc[0];
    r.qa[1] = c->qa[2];
    r.qb[1] = c->qb[2];
    r.qc[1] = c->qc[2];
    r.cnt[0] = ext_phase >= 0 ? counts_at(c, ext_phase, 0) : nullptr;
    r.cnt[1] = sh_phase >= 0 ? counts_at(c, sh_phase, 0) : nullptr;
    // camera rays are counted on the host (every one is cast, also one that misses the grid)
    r.count[0] = count_ext ? 1 : 0;
    r.count[1] = 1;
    r.stats = c->d_stats;
    Timer tm(c, timing, 3);
    HIP_TRY(c, launch_route(r, c->stream));
    return SDD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

sdd_status sdd_create(int hip_device, void* hip_stream, sdd_ctx** out) {
    if (!out) return SDD_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return SDD_ERR_HIP;
    if (hip_device < 0 || hip_device >= ndev) return SDD_ERR_INVALID_ARG;
    sdd_ctx* c = new (std::nothrow) sdd_ctx();
    if (!c) return SDD_ERR_OOM;
    c->device = hip_device;
    DeviceGuard g(hip_device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    c->stream = (hipStream_t)hip_stream;  // NULL: the null stream, ordered with other default-stream work
    // the spill stack is sized for the largest trace grid (one subdomain); build_bvh
    // sets the grid for its subdomain count, never above this
    c->trace_grid_max = trace_grid_for(c, 1);
    c->trace_grid = c->trace_grid_max;
    // the allocation-free query's scratch: its device address, resolved once per device
    if (nrc_noalloc_scratch(hip_device, &c->noalloc_scratch) != hipSuccess) {
        delete c;
        return SDD_ERR_HIP;
    }
    if (dalloc(c, &c->d_overflow, 1) != SDD_OK || dalloc(c, &c->d_ovf_stats, 1) != SDD_OK ||
        dalloc(c, &c->d_stats, kStatCount) != SDD_OK ||
        dalloc(c, &c->d_ktot, 2 * (size_t)kMaxCells * kExtBins) != SDD_OK ||
        dalloc(c, &c->d_gstack, (size_t)c->trace_grid_max * kTraceBlock * (kStack - kLdsStack)) != SDD_OK) {
        sdd_destroy(c);
        return SDD_ERR_OOM;
    }
    if (hipMemsetAsync(c->d_overflow, 0, sizeof(int), c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_ovf_stats, 0, sizeof(int), c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_stats, 0, sizeof(unsigned long long) * kStatCount, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        sdd_destroy(c);
        return SDD_ERR_HIP;
    }
    *out = c;
    return SDD_OK;
}

void sdd_destroy(sdd_ctx* c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    dfree(c, c->d_s0);
    harvest_events(c);
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    c->event_pool.clear();
    free_renders(c);
    free_batch(c);
    free_accel(c);
    free_scene(c);
    free_nrc(c);
    dfree(c, c->d_overflow);
    dfree(c, c->d_ovf_stats);
    dfree(c, c->d_ktot);
    dfree(c, c->d_gstack);
    dfree(c, c->d_stats);
    for (auto& kv : c->allocs) (void)hipFree(kv.first);
    c->allocs.clear();
    delete c;
}

const char* sdd_last_error(const sdd_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

sdd_status sdd_validate_scene(const sdd_scene_desc* scene, char* msg, int msg_len) {
    const std::string e = validate(scene);
    if (msg && msg_len > 0) {
        std::snprintf(msg, (size_t)msg_len, "%s", e.c_str());
    }
    return e.empty() ? SDD_OK : SDD_ERR_INVALID_ARG;
}

sdd_status sdd_load_scene(sdd_ctx* c, const sdd_scene_desc* s) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    const std::string e = validate(s);
    if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_renders(c);
    free_batch(c);
    free_accel(c);
    free_scene(c);
    c->V = s->n_verts;
    c->T = s->n_tris;
    c->M = s->n_mats;
    c->nl = s->n_lambda;
    c->nlp = (c->nl + 3) / 4 * 4;
    c->verts.assign(s->verts, s->verts + 3 * (size_t)c->V);
    c->tris.assign(s->tris, s->tris + 3 * (size_t)c->T);
    c->tri_mat.assign(s->tri_mat, s->tri_mat + c->T);
    c->mat_type.assign(s->mat_type, s->mat_type + c->M);
    c->light_type = s->light_type;
    c->light_mat = s->light_mat;
    for (int k = 0; k < 3; ++k) {
        c->lp0[k] = s->light_p0[k];
        c->le1[k] = s->light_e1[k];
        c->le2[k] = s->light_e2[k];
    }
    if (c->light_type == SDD_LIGHT_PARALLELOGRAM) {
        const double e1[3] = {s->light_e1[0], s->light_e1[1], s->light_e1[2]};
        const double e2[3] = {s->light_e2[0], s->light_e2[1], s->light_e2[2]};
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double a = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; ++k) c->nL[k] = n[k] / a;
        c->light_area = a;
    } else {
        c->nL[0] = c->nL[1] = c->nL[2] = 0.0;
        c->light_area = 0.0;
    }
    // per-material tables padded to nlp wavelengths; glass materials get a
    // compact index and their pane constants (double, rounded once)
    const int nl = c->nl, nlp = c->nlp, M = c->M;
    std::vector<float> rho((size_t)M * nlp, 0.0f), le((size_t)M * nlp, 0.0f);
    c->glass_of.assign(M, -1);
    c->mat_emits.assign(M, 0);
    c->n_glass = 0;
    for (int m = 0; m < M; ++m)
        if (s->mat_type[m] == SDD_MAT_GLASS_SLAB) c->glass_of[m] = c->n_glass++;
    std::vector<float4> pane((size_t)std::max(1, c->n_glass) * nlp, make_float4(0.0f, 0.0f, 1.0f, 0.0f));
    for (int m = 0; m < M; ++m)
        for (int l = 0; l < nl; ++l) {
            const size_t i = (size_t)m * nl + l, j = (size_t)m * nlp + l;
            rho[j] = s->mat_rho[i];
            le[j] = s->mat_le[i];
            if (s->mat_le[i] != 0.0f) c->mat_emits[m] = 1;
            if (c->glass_of[m] >= 0) {
                const double n = s->mat_n[i], k = s->mat_k[i];
                const double at = 4.0 * M_PI * k * (double)s->mat_thick[m] / ((double)s->lambda_nm[l] * 1e-9);
                pane[(size_t)c->glass_of[m] * nlp + l] =
                    make_float4((float)(n * n - k * k), (float)(2.0 * n * k), (float)(1.0 / (n * n)), (float)at);
            }
        }
    // coherent coatings: per (glass, layer, wavelength) (Re N^2, Im N^2, 2 pi d / lambda)
    c->max_layers = s->max_layers > 0 ? s->max_layers : 0;
    std::vector<int> coat_n((size_t)std::max(1, c->n_glass), 0);
    bool any_coat = false;
    if (c->max_layers > 0)
        for (int m = 0; m < M; ++m)
            if (c->glass_of[m] >= 0) {
                coat_n[c->glass_of[m]] = s->mat_n_layers[m];
                any_coat = any_coat || s->mat_n_layers[m] > 0;
            }
    const int Lm = std::max(1, c->max_layers);
    std::vector<float4> coat((size_t)std::max(1, c->n_glass) * Lm * nlp, make_float4(1.0f, 0.0f, 0.0f, 0.0f));
    if (any_coat)
        for (int m = 0; m < M; ++m) {
            const int g = c->glass_of[m];
            if (g < 0) continue;
            for (int j = 0; j < s->mat_n_layers[m]; ++j) {
                const double d = s->mat_layer_d[(size_t)m * c->max_layers + j];
                for (int l = 0; l < nl; ++l) {
                    const size_t i = ((size_t)m * c->max_layers + j) * nl + l;
                    const double n = s->mat_layer_n[i], k = s->mat_layer_k[i];
                    coat[((size_t)g * Lm + j) * nlp + l] = make_float4(
                        (float)(n * n - k * k), (float)(2.0 * n * k),
                        (float)(2.0 * M_PI * d / ((double)s->lambda_nm[l] * 1e-9)), 0.0f);
                }
            }
        }
    c->coat_layers = any_coat ? Lm : 0;
    BuildInput bi{c->verts.data(), c->V, c->tris.data(), c->T, c->tri_mat.data(), c->mat_type.data(),
                  c->glass_of.data(), c->mat_emits.data(), 1, 1, 1, 4, 16};
    std::vector<HostF4> info;
    triangle_info(bi, info);
    std::vector<float4> prim_v(3 * (size_t)c->T);
    for (int i = 0; i < c->T; ++i)
        for (int j = 0; j < 3; ++j) {
            const float* v = c->verts.data() + 3 * (size_t)c->tris[3 * (size_t)i + j];
            prim_v[3 * (size_t)i + j] = make_float4(v[0], v[1], v[2], 0.0f);
        }
    sdd_status st;
    if ((st = upload(c, &c->d_prim_info, reinterpret_cast<const float4*>(info.data()), info.size())) != SDD_OK ||
        (st = upload(c, &c->d_prim_v, prim_v.data(), prim_v.size())) != SDD_OK ||
        (st = upload(c, &c->d_pane, pane.data(), pane.size())) != SDD_OK ||
        (any_coat && (st = upload(c, &c->d_coat, coat.data(), coat.size())) != SDD_OK) ||
        (any_coat && (st = upload(c, &c->d_coat_n, coat_n.data(), coat_n.size())) != SDD_OK) ||
        (st = upload(c, &c->d_rho, rho.data(), rho.size())) != SDD_OK ||
        (st = upload(c, &c->d_le, le.data(), le.size())) != SDD_OK ||
        (st = upload(c, &c->d_w, s->lambda_w, (size_t)nl)) != SDD_OK ||
        (st = upload(c, &c->d_cmf, s->cmf, (size_t)nl * 3)) != SDD_OK ||
        (st = upload(c, &c->d_lam, s->lambda_nm, (size_t)nl)) != SDD_OK) {
        free_scene(c);
        return st;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->has_scene = true;
    return SDD_OK;
}

}  // extern "C"

namespace {

// Grid planes on the host, references and BVHs on the device (bvh_device.hip);
// fills the context's device arrays and gb's host-side counts.
sdd_status device_bvh(sdd_ctx* c, const BuildInput& bi, GridBvh& gb) {
    std::string err;
    double ext = 0.0;
    if (!grid_planes(bi, gb, ext, err)) return fail(c, SDD_ERR_INVALID_ARG, err);
    sdd_status st = upload(c, &c->d_planes, gb.planes.data(), gb.planes.size());
    if (st != SDD_OK) return st;
    const int G = bi.nx * bi.ny * bi.nz;
    DevBuildArgs a{};
    a.T = bi.n_tris;
    a.prim_v = c->d_prim_v;
    a.prim_info = c->d_prim_info;
    a.planes = c->d_planes;
    a.n[0] = bi.nx;
    a.n[1] = bi.ny;
    a.n[2] = bi.nz;
    a.G = G;
    a.cpad = 1e-4 * ext;
    a.npad = 2e-6 * ext;
    a.leaf_max = bi.leaf_max;
    DevBuildBufs b{};
    std::vector<void*> temps;
    auto tmp_alloc = [&](auto** p, size_t n) -> sdd_status {
        sdd_status s2 = dalloc(c, p, n);
        if (s2 == SDD_OK) temps.push_back((void*)*p);
        return s2;
    };
    auto release = [&]() {
        for (void* p : temps) dfree(c, p);
        temps.clear();
    };
    // references per triangle and their prefix
    size_t scan_bytes = 0;
    if ((st = tmp_alloc(&b.count, (size_t)a.T)) != SDD_OK || (st = tmp_alloc(&b.offset, (size_t)a.T)) != SDD_OK) {
        release();
        return st;
    }
    hipError_t e = dev_count_refs(a, b.count, b.offset, nullptr, scan_bytes, c->stream);
    char* scan_tmp = nullptr;
    if (e == hipSuccess && (st = tmp_alloc(&scan_tmp, std::max<size_t>(1, scan_bytes))) != SDD_OK) {
        release();
        return st;
    }
    if (e == hipSuccess) e = dev_count_refs(a, b.count, b.offset, scan_tmp, scan_bytes, c->stream);
    int last[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(&last[0], b.offset + a.T - 1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&last[1], b.count + a.T - 1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        release();
        return hip_fail(c, e, "device BVH: reference count");
    }
    const long long total = (long long)last[0] + last[1];
    if (total <= 0 || total >= (1LL << 31) / 3) {
        release();
        return fail(c, SDD_ERR_UNSUPPORTED, "device BVH: reference count out of range");
    }
    b.total = total;
    size_t sort_bytes = 0;
    e = dev_sort_bytes(total, sort_bytes);
    if (e != hipSuccess) {
        release();
        return hip_fail(c, e, "device BVH: sort scratch");
    }
    b.tmp_bytes = std::max<size_t>(1, sort_bytes);
    char* sort_tmp = nullptr;
    const size_t T3 = (size_t)total;
    if ((st = tmp_alloc(&sort_tmp, b.tmp_bytes)) != SDD_OK || (st = tmp_alloc(&b.ref_lo, T3)) != SDD_OK ||
        (st = tmp_alloc(&b.ref_hi, T3)) != SDD_OK || (st = tmp_alloc(&b.key_in, T3)) != SDD_OK ||
        (st = tmp_alloc(&b.key, T3)) != SDD_OK || (st = tmp_alloc(&b.val_in, T3)) != SDD_OK ||
        (st = tmp_alloc(&b.val, T3)) != SDD_OK || (st = tmp_alloc(&b.cell_start, (size_t)G + 1)) != SDD_OK ||
        (st = tmp_alloc(&b.child, T3)) != SDD_OK || (st = tmp_alloc(&b.range, T3)) != SDD_OK ||
        (st = tmp_alloc(&b.parent, 2 * T3)) != SDD_OK || (st = tmp_alloc(&b.arrive, T3)) != SDD_OK ||
        (st = tmp_alloc(&b.box_lo, T3)) != SDD_OK || (st = tmp_alloc(&b.box_hi, T3)) != SDD_OK ||
        (st = tmp_alloc(&b.level_a, T3)) != SDD_OK || (st = tmp_alloc(&b.level_b, T3)) != SDD_OK ||
        (st = tmp_alloc(&b.last_flag, T3)) != SDD_OK || (st = tmp_alloc(&b.max_depth, 2)) != SDD_OK ||
        (st = dalloc(c, &c->d_nodes, 2 * (T3 + (size_t)G))) != SDD_OK ||
        (st = dalloc(c, &c->d_tris, 3 * T3)) != SDD_OK || (st = dalloc(c, &c->d_cell_q, 2 * (size_t)G)) != SDD_OK ||
        (st = dalloc(c, &c->d_cell_root, (size_t)G)) != SDD_OK ||
        (st = dalloc(c, &c->d_cell_nodes, (size_t)G)) != SDD_OK) {
        release();
        return st;
    }
    b.tmp = sort_tmp;
    b.error = b.max_depth + 1;
    b.nodes = c->d_nodes;
    b.tris = c->d_tris;
    b.cell_q = c->d_cell_q;
    b.cell_root = c->d_cell_root;
    b.cell_nodes = c->d_cell_nodes;
    int flags[2] = {0, 0};
    gb.cell_nodes.assign(G, 0);
    e = hipMemsetAsync(b.max_depth, 0, 2 * sizeof(int), c->stream);
    if (e == hipSuccess) e = dev_build(a, b, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(flags, b.max_depth, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(gb.cell_nodes.data(), c->d_cell_nodes, sizeof(int) * G, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    release();
    if (e != hipSuccess) return hip_fail(c, e, "device BVH build");
    if (flags[1] != 0) return fail(c, SDD_ERR_HIP, "device BVH build produced an inconsistent hierarchy");
    gb.n_refs = total;
    gb.max_depth = flags[0];
    gb.cell_root.assign(G, 0);
    gb.cell_refs.assign(G, 0);
    return SDD_OK;
}

// Replaces the binary nodes on the device (n2 slots; cell roots and node
// counts in c->d_cell_root / c->d_cell_nodes and gb.cell_nodes) by the 4-wide
// nodes the traversal reads, and updates gb.cell_root / gb.cell_nodes.
sdd_status widen_bvh(sdd_ctx* c, long long n2, GridBvh& gb) {
    const int G = (int)gb.cell_nodes.size();
    if (n2 <= 0 || n2 >= (1LL << 31) - 1) return fail(c, SDD_ERR_UNSUPPORTED, "BVH node count out of range");
    WidenBufs b{};
    b.n2 = (int)n2;
    b.nodes2 = c->d_nodes;
    b.cell_root = c->d_cell_root;
    b.cell_nodes = c->d_cell_nodes;
    b.G = G;
    b.max_cell_nodes = 0;
    for (int v : gb.cell_nodes) {
        // every builder gives each cell a root (a wrapper node for an empty cell)
        if (v <= 0) return fail(c, SDD_ERR_HIP, "widen: a cell without BVH nodes");
        b.max_cell_nodes = std::max(b.max_cell_nodes, v);
    }
    std::vector<void*> temps;
    auto tmp_alloc = [&](auto** p, size_t n) -> sdd_status {
        sdd_status s2 = dalloc(c, p, n);
        if (s2 == SDD_OK) temps.push_back((void*)*p);
        return s2;
    };
    auto release = [&]() {
        for (void* p : temps) dfree(c, p);
        temps.clear();
    };
    const size_t n1 = (size_t)n2 + 1;
    sdd_status st;
    hipError_t e = widen_mark(b, c->stream);  // scratch size only
    if (e != hipSuccess) return hip_fail(c, e, "widen: scan scratch");
    char* tmp = nullptr;
    if ((st = tmp_alloc(&b.anc[0], n1)) != SDD_OK || (st = tmp_alloc(&b.anc[1], n1)) != SDD_OK ||
        (st = tmp_alloc(&b.dist[0], n1)) != SDD_OK || (st = tmp_alloc(&b.dist[1], n1)) != SDD_OK ||
        (st = tmp_alloc(&b.flag, n1)) != SDD_OK || (st = tmp_alloc(&b.idx, n1)) != SDD_OK ||
        (st = tmp_alloc(&tmp, std::max<size_t>(1, b.tmp_bytes))) != SDD_OK) {
        release();
        return st;
    }
    b.tmp = tmp;
    int total = 0;
    e = widen_mark(b, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&total, b.idx + n2, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        release();
        return hip_fail(c, e, "widen: node depths");
    }
    uint4* nodes4 = nullptr;
    int *root4 = nullptr, *cnt4 = nullptr;
    if (total <= 0) {
        release();
        return fail(c, SDD_ERR_HIP, "widen: no nodes");
    }
    if ((st = dalloc(c, &nodes4, 4 * (size_t)total)) != SDD_OK || (st = dalloc(c, &root4, (size_t)G)) != SDD_OK ||
        (st = dalloc(c, &cnt4, (size_t)G)) != SDD_OK) {
        dfree(c, nodes4);
        dfree(c, root4);
        dfree(c, cnt4);
        release();
        return st;
    }
    e = widen_emit(b, nodes4, root4, cnt4, c->stream);
    gb.cell_root.assign(G, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(gb.cell_root.data(), root4, sizeof(int) * G, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(gb.cell_nodes.data(), cnt4, sizeof(int) * G, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    release();
    bool rooted = e == hipSuccess;
    for (int c2 = 0; rooted && c2 < G; ++c2) rooted = gb.cell_nodes[c2] >= 1 && gb.cell_root[c2] < total;
    if (!rooted) {
        dfree(c, nodes4);
        dfree(c, root4);
        dfree(c, cnt4);
        return e != hipSuccess ? hip_fail(c, e, "widen: 4-wide nodes")
                               : fail(c, SDD_ERR_HIP, "widen: a cell without a 4-wide root");
    }
    dfree(c, c->d_nodes);
    dfree(c, c->d_cell_root);
    dfree(c, c->d_cell_nodes);
    c->d_nodes = nodes4;
    c->d_cell_root = root4;
    c->d_cell_nodes = cnt4;
    return SDD_OK;
}

}  // namespace

extern "C" {

sdd_status sdd_build_bvh(sdd_ctx* c, const sdd_bvh_desc* d) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!d) return fail(c, SDD_ERR_INVALID_ARG, "null bvh desc");
    if (!c->has_scene) return fail(c, SDD_ERR_STATE, "sdd_build_bvh before sdd_load_scene");
    if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0) return fail(c, SDD_ERR_INVALID_ARG, "grid dims must be > 0");
    if ((long long)d->nx * d->ny * d->nz > SDD_MAX_CELLS) return fail(c, SDD_ERR_INVALID_ARG, "too many cells");
    const int leaf = d->leaf_max == 0 ? 3 : d->leaf_max;  // 3 measured fastest on the 4-wide tree
    const int bins = d->sah_bins == 0 ? 16 : d->sah_bins;
    if (leaf < 1 || leaf > 8) return fail(c, SDD_ERR_INVALID_ARG, "leaf_max out of range");
    if (bins < 2 || bins > 64) return fail(c, SDD_ERR_INVALID_ARG, "sah_bins out of range");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_renders(c);
    free_batch(c);
    free_accel(c);
    BuildInput bi{c->verts.data(), c->V, c->tris.data(), c->T, c->tri_mat.data(), c->mat_type.data(),
                  c->glass_of.data(), c->mat_emits.data(), d->nx, d->ny, d->nz, leaf, bins};
    std::string err;
    GridBvh gb;
    sdd_status st;
    if (d->device_build) {
        st = device_bvh(c, bi, gb);
        if (st != SDD_OK) {
            free_accel(c);
            return st;
        }
    } else if (!build_grid_bvh(bi, gb, err)) {
        return fail(c, SDD_ERR_INVALID_ARG, err);
    } else if ((st = upload(c, &c->d_nodes, reinterpret_cast<const uint4*>(gb.nodes.data()), gb.nodes.size() / 4)) != SDD_OK ||
        (st = upload(c, &c->d_cell_q, reinterpret_cast<const float4*>(gb.cell_q.data()), gb.cell_q.size())) != SDD_OK ||
        (st = upload(c, &c->d_cell_nodes, gb.cell_nodes.data(), gb.cell_nodes.size())) != SDD_OK ||
        (st = upload(c, &c->d_tris, reinterpret_cast<const float4*>(gb.tris.data()), gb.tris.size())) != SDD_OK ||
        (st = upload(c, &c->d_cell_root, gb.cell_root.data(), gb.cell_root.size())) != SDD_OK ||
        (st = upload(c, &c->d_planes, gb.planes.data(), gb.planes.size())) != SDD_OK) {
        free_accel(c);
        return st;
    }
    const long long n2 = d->device_build ? gb.n_refs + (long long)d->nx * d->ny * d->nz : (long long)gb.nodes.size() / 8;
    if ((st = widen_bvh(c, n2, gb)) != SDD_OK) {
        free_accel(c);
        return st;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->G = d->nx * d->ny * d->nz;
    c->S = d->nx + d->ny + d->nz - 2;
    apply_tuning(c);
    GridParams& gp = c->grid;
    gp.planes = c->d_planes;
    gp.nx = d->nx;
    gp.ny = d->ny;
    gp.nz = d->nz;
    gp.off_y = d->nx + 1;
    gp.off_z = d->nx + 1 + d->ny + 1;
    const int n[3] = {d->nx, d->ny, d->nz};
    const int off[3] = {0, gp.off_y, gp.off_z};
    for (int a = 0; a < 3; ++a) {
        gp.lo[a] = gb.planes[off[a]];
        gp.hi[a] = gb.planes[off[a] + n[a]];
        gp.inv_h[a] = (float)((double)n[a] / ((double)gp.hi[a] - (double)gp.lo[a]));
    }
    c->gb = std::move(gb);
    c->gb.nodes.clear();
    c->gb.nodes.shrink_to_fit();
    c->gb.tris.clear();
    c->gb.tris.shrink_to_fit();
    c->has_bvh = true;
    return SDD_OK;
}

}  // extern "C"

namespace {

sdd_status nrc_reserve(sdd_ctx* c, long long n);

// Operand staging of BF16 cache queries of n paths, and the sort's temporary
// storage for a sort of n or of n_other paths (0: none).  The sort's need is
// not monotonic in its size (a small sort takes another algorithm than a
// large one), so every size a caller will sort is asked for separately.
sdd_status nrc_ensure_ops(sdd_ctx* c, int n, int n_other = 0) {
    const long long need = nrc_query_ops_paths(std::max(n, n_other));
    size_t tb = 1;
    for (int m : {n, n_other})
        if (m > 0)
            tb = std::max({tb, nrc_order_temp_bytes(m), nrc_order_temp_bytes((int)nrc_query_ops_paths(m)),
                           nrc_scan_temp_bytes(m + 1)});
    sdd_status st;
    if (need > c->nrc_ocap) {
        dfree(c, c->nrc_hop);
        dfree(c, c->nrc_sop);
        dfree(c, c->nrc_okeys);
        dfree(c, c->nrc_ovals);
        dfree(c, c->nrc_flags);
        dfree(c, c->nrc_rank);
        dfree(c, c->nrc_cp);
        c->nrc_ocap = 0;
        if ((st = dalloc(c, &c->nrc_hop, (size_t)(4 * need))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_sop, (size_t)(4 * need))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_okeys, (size_t)(2 * need))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_ovals, (size_t)(2 * need))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_flags, (size_t)(need + 1))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_rank, (size_t)(need + 1))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_cp, (size_t)need)) != SDD_OK)
            return st;
        c->nrc_ocap = need;
    }
    if (tb > c->nrc_otemp_bytes) {
        dfree(c, c->nrc_otemp);
        c->nrc_otemp_bytes = 0;
        if ((st = dalloc(c, &c->nrc_otemp, tb)) != SDD_OK) return st;
        c->nrc_otemp_bytes = tb;
    }
    return SDD_OK;
}

// the gather order scratch of the cache queries (valid after nrc_ensure_ops)
NrcOrder nrc_order(sdd_ctx* c) { return NrcOrder{c->nrc_okeys, c->nrc_ovals, c->nrc_otemp, c->nrc_otemp_bytes}; }

// render buffers of the radiance cache: n batch paths (n_last in the call's
// last batch), slots training paths of depth D
sdd_status nrc_ensure_render(sdd_ctx* c, long long n, long long n_last, long long slots, int D) {
    sdd_status st;
    if (n > c->nrc_pcap || slots > c->nrc_scap || D > c->nrc_dcap || c->nrc_train_batch > c->nrc_bcap)
        HIP_TRY(c, nrc_wait_host(c));  // buffers the pending Adam steps may still read
    if (n > c->nrc_pcap) {
        dfree(c, c->nrc_cx);
        dfree(c, c->nrc_cn);
        dfree(c, c->nrc_lhat);
        c->nrc_pcap = 0;
        if ((st = dalloc(c, &c->nrc_cx, (size_t)n)) != SDD_OK || (st = dalloc(c, &c->nrc_cn, (size_t)n)) != SDD_OK ||
            (st = dalloc(c, &c->nrc_lhat, (size_t)n * c->nlp)) != SDD_OK)
            return st;
        c->nrc_pcap = n;
    }
    if (slots > c->nrc_scap || D > c->nrc_dcap) {
        dfree(c, c->nrc_tx);
        dfree(c, c->nrc_tn);
        dfree(c, c->nrc_rows);
        dfree(c, c->nrc_ok);
        dfree(c, c->nrc_crows);
        dfree(c, c->nrc_tmp);
        c->nrc_scap = 0;
        c->nrc_dcap = 0;
        const long long rows = slots * std::max(1, D - 1);
        if ((st = dalloc(c, &c->nrc_tx, (size_t)(slots * D))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_tn, (size_t)(slots * D))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_rows, (size_t)(2 * rows))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_ok, (size_t)rows)) != SDD_OK ||
            (st = dalloc(c, &c->nrc_crows, (size_t)(2 * rows))) != SDD_OK)
            return st;
        size_t tb = 0;
        HIP_TRY(c, nrc_select_rows(c->nrc_rows, c->nrc_ok, (int)rows, c->nrc_crows, c->nrc_count, nullptr, &tb,
                                   c->stream));
        c->nrc_tmp_bytes = std::max<size_t>(tb, 16);
        if ((st = dalloc(c, reinterpret_cast<char**>(&c->nrc_tmp), c->nrc_tmp_bytes)) != SDD_OK) return st;
        c->nrc_scap = slots;
        c->nrc_dcap = D;
    }
    if (!c->nrc_count && (st = dalloc(c, &c->nrc_count, 1)) != SDD_OK) return st;
    if ((st = nrc_ensure_ops(c, (int)n, (int)n_last)) != SDD_OK) return st;
    const long long bn = c->nrc_train_batch;
    if (bn > c->nrc_bcap) {
        dfree(c, c->nrc_bx);
        dfree(c, c->nrc_bw);
        dfree(c, c->nrc_blam);
        dfree(c, c->nrc_bt);
        c->nrc_bcap = 0;
        if ((st = dalloc(c, &c->nrc_bx, (size_t)(3 * bn))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_bw, (size_t)(3 * bn))) != SDD_OK ||
            (st = dalloc(c, &c->nrc_blam, (size_t)bn)) != SDD_OK || (st = dalloc(c, &c->nrc_bt, (size_t)bn)) != SDD_OK)
            return st;
        c->nrc_bcap = bn;
    }
    return SDD_OK;
}

// After a cache render: compact the training rows the call produced and take
// up to train_steps Adam steps (S), step k on rows (k + i S) m, i < train_batch,
// with m = max(1, rows / (S train_batch)): spread over the whole image.  The
// rows are compacted and counted on the context stream; the steps then run
// on c->nrc_stream, after an event on the context stream, so they overlap
// the next call's tracing (its cache query waits for them: nrc_wait_gpu).
sdd_status nrc_train_after_call(sdd_ctx* c, long long n_rows, bool timing) {
    HIP_TRY(c, nrc_wait_host(c));
    c->nrc_last_rows = 0;
    c->nrc_last_steps = 0;
    c->nrc_last_loss = 0.0f;
    if (n_rows <= 0) return SDD_OK;
    {
        Timer tm(c, timing, 5);
        size_t tb = c->nrc_tmp_bytes;
        HIP_TRY(c, nrc_select_rows(c->nrc_rows, c->nrc_ok, (int)n_rows, c->nrc_crows, c->nrc_count, c->nrc_tmp, &tb,
                                   c->stream));
    }
    int count = 0;
    HIP_TRY(c, hipMemcpyAsync(&count, c->nrc_count, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->nrc_last_rows = count;
    if (count <= 0) return SDD_OK;
    const int S = std::min(c->nrc_train_steps, count);
    if (S <= 0) return SDD_OK;
    sdd_status st = nrc_reserve(c, c->nrc_train_batch);
    if (st != SDD_OK) return st;
    if (!c->nrc_stream) {  // the training stream, at the default priority
        HIP_TRY(c, hipStreamCreateWithFlags(&c->nrc_stream, hipStreamNonBlocking));
        HIP_TRY(c, hipEventCreateWithFlags(&c->nrc_ev_rows, hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->nrc_ev_trained, hipEventDisableTiming));
        HIP_TRY(c, hipHostMalloc((void**)&c->nrc_h_loss, sizeof(float), hipHostMallocDefault));
        *c->nrc_h_loss = 0.0f;
    }
    hipStream_t ts = c->nrc_stream;
    HIP_TRY(c, hipEventRecord(c->nrc_ev_rows, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(ts, c->nrc_ev_rows, 0));
    // more rows than S steps take: every m-th row (spread over the whole image)
    const long long used = (long long)S * c->nrc_train_batch;
    const int m = count > used ? (int)(count / used) : 1;
    for (int k = 0; k < S; ++k) {
        const int nk = (int)std::min<long long>(c->nrc_train_batch, ((long long)count / m - k + S - 1) / S);
        c->nrc_train_rows += nk;
        Timer tm(c, timing, 5, ts);
        HIP_TRY(c, nrc_launch_unpack(c->nrc_crows, k, S, m, nk, c->nrc_bx, c->nrc_bw, c->nrc_blam, c->nrc_bt, ts));
        NrcBatch b{nk, c->nrc_bx, c->nrc_bw, c->nrc_blam, c->nrc_bt, c->nrc_acts, c->nrc_dz, c->nrc_y, c->nrc_dy,
                   c->nrc_loss};
        if (c->nrc_g_dirty) HIP_TRY(c, nrc_launch_zero(c->nrc.g, c->nrc.n_all, ts));
        HIP_TRY(c, nrc_launch_zero(c->nrc_loss, 1, ts));
        HIP_TRY(c, nrc_launch_grad(c->nrc, b, ts));
        // Adam leaves the gradients at zero for the next step (no zeroing pass over the tables)
        HIP_TRY(c, nrc_launch_adam(c->nrc, c->nrc_t + 1, c->nrc_lr, c->nrc_b1, c->nrc_b2, c->nrc_eps, ts, true));
        c->nrc_g_dirty = false;
        HIP_TRY(c, nrc_launch_pack(c->nrc, ts));
        ++c->nrc_t;
    }
    if (c->nrc_t16) HIP_TRY(c, nrc_launch_tables_f16(c->nrc, c->nrc_t16, ts));
    // the last step's loss, read when asked for (nrc_wait_host)
    HIP_TRY(c, hipMemcpyAsync(c->nrc_h_loss, c->nrc_loss, sizeof(float), hipMemcpyDeviceToHost, ts));
    HIP_TRY(c, hipEventRecord(c->nrc_ev_trained, ts));
    c->nrc_pending = true;
    c->nrc_last_steps = S;
    return SDD_OK;
}

// one render of a trace call
struct Job {
    const sdd_trace_desc* t = nullptr;
    Render* rd = nullptr;
    int WH = 0;            // pixels of the render's window
    PixWindow win{};
    long long total = 0;  // WH * spp paths
    long long start = 0;  // first index in the call's path space (multiple of kShadeBlock)
    double f[3], r[3], u[3];
    bool ortho = false;
    int glass_from = -1, glass_to = -1;  // compact glass indices of the substitution
};

// pixels a render traces: its window, or the whole frame
long long window_pixels(const sdd_trace_desc* t) {
    return t->crop_w != 0 ? (long long)t->crop_w * t->crop_h : (long long)t->W * t->H;
}

// argument checks and camera basis of one render (no device work)
sdd_status check_desc(sdd_ctx* c, const sdd_trace_desc* t, Job& j) {
    if (!t) return fail(c, SDD_ERR_INVALID_ARG, "null trace desc");
    if (t->W <= 0 || t->H <= 0 || t->spp <= 0) return fail(c, SDD_ERR_INVALID_ARG, "W, H and spp must be > 0");
    if ((long long)t->W * t->H > (1LL << 28)) return fail(c, SDD_ERR_INVALID_ARG, "image too large");
    const bool crop = t->crop_w != 0 || t->crop_h != 0;
    if (crop && (t->crop_w <= 0 || t->crop_h <= 0 || t->crop_x0 < 0 || t->crop_y0 < 0 ||
                 (long long)t->crop_x0 + t->crop_w > t->W || (long long)t->crop_y0 + t->crop_h > t->H))
        return fail(c, SDD_ERR_INVALID_ARG, "crop window outside the frame");
    if (!crop && (t->crop_x0 != 0 || t->crop_y0 != 0))
        return fail(c, SDD_ERR_INVALID_ARG, "crop origin without a crop size");
    if (window_pixels(t) * t->spp >= (1LL << 31))
        return fail(c, SDD_ERR_INVALID_ARG, "window pixels * spp must be < 2^31 per call");
    if (t->max_depth < 1 || t->max_depth > SDD_MAX_DEPTH) return fail(c, SDD_ERR_INVALID_ARG, "max_depth out of range");
    if (t->render_id < 0) return fail(c, SDD_ERR_INVALID_ARG, "render_id must be >= 0");
    if (t->sample_offset < 0) return fail(c, SDD_ERR_INVALID_ARG, "sample_offset must be >= 0");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(t->eye[k]) || !std::isfinite(t->target[k]))
            return fail(c, SDD_ERR_INVALID_ARG, "non-finite camera");
    const double f0[3] = {t->target[0] - t->eye[0], t->target[1] - t->eye[1], t->target[2] - t->eye[2]};
    const double fl = std::sqrt(f0[0] * f0[0] + f0[1] * f0[1] + f0[2] * f0[2]);
    if (!(fl > 0.0)) return fail(c, SDD_ERR_INVALID_ARG, "eye == target");
    for (int k = 0; k < 3; ++k) j.f[k] = f0[k] / fl;
    double r[3] = {j.f[1], -j.f[0], 0.0};  // f x z
    const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1]);
    if (!(rl > 1e-9)) return fail(c, SDD_ERR_INVALID_ARG, "view direction parallel to +z");
    for (int k = 0; k < 3; ++k) j.r[k] = r[k] / rl;
    j.u[0] = j.r[1] * j.f[2] - j.r[2] * j.f[1];
    j.u[1] = j.r[2] * j.f[0] - j.r[0] * j.f[2];
    j.u[2] = j.r[0] * j.f[1] - j.r[1] * j.f[0];
    j.ortho = (t->flags & SDD_TRACE_ORTHO) != 0;
    if (!j.ortho && !(t->fov_deg > 0.0 && t->fov_deg < 180.0)) return fail(c, SDD_ERR_INVALID_ARG, "fov out of range");
    if (j.ortho && !(t->ortho_half_h > 0.0)) return fail(c, SDD_ERR_INVALID_ARG, "ortho_half_h must be > 0");
    if (t->glass_from != t->glass_to) {
        const int a = t->glass_from, b = t->glass_to;
        if (a < 0 || a >= c->M || b < 0 || b >= c->M || c->glass_of[a] < 0 || c->glass_of[b] < 0)
            return fail(c, SDD_ERR_INVALID_ARG, "glass substitution needs two glass materials");
        j.glass_from = c->glass_of[a];
        j.glass_to = c->glass_of[b];
    }
    j.t = t;
    j.WH = (int)window_pixels(t);
    j.win = crop ? PixWindow{t->W, t->crop_x0, t->crop_y0, t->crop_w} : PixWindow{t->W, 0, 0, 0};
    j.total = (long long)j.WH * t->spp;
    return SDD_OK;
}

// The renders of one call share one path space: render j occupies
// [start_j, start_j + total_j), each start a multiple of kShadeBlock (the
// gaps hold no path).  The space is traced in batches; every batch runs the
// whole pipeline once, with the per-render kernels (camera rays, shading,
// spectral replay) launched per render segment and the routing and
// traversal sweeps over the whole batch.
// Path-space layout of a call's renders and the batch size (paths per pass).
long long plan_batches(sdd_ctx* c, std::vector<Job>& jobs, long long& total_pad) {
    const int D = jobs[0].t->max_depth;
    uint32_t any_flags = 0;
    for (const Job& j : jobs) any_flags |= j.t->flags;
    total_pad = 0;
    for (Job& j : jobs) {
        j.start = total_pad;
        total_pad += (j.total + kShadeBlock - 1) / kShadeBlock * kShadeBlock;
    }
    const bool nrc = (any_flags & SDD_TRACE_NRC) != 0;
    if (c->call_budget <= 0) c->call_budget = mem_budget_bytes(c);
    long long nb = c->tune_batch > 0 ? c->tune_batch
                                     : c->call_budget / (bytes_per_path(c, D) + (nrc ? 32 + 4LL * c->nlp : 0));
    nb = std::min<long long>(nb, kMaxBatch);
    nb = std::max<long long>(kShadeBlock, nb / kShadeBlock * kShadeBlock);
    return std::min(nb, total_pad);
}

// s0_dev: if set, the kernels read each render's first sample index from
// s0_dev[job] (a captured graph replays with new sample ranges)
sdd_status trace_jobs(sdd_ctx* c, std::vector<Job>& jobs, const int* s0_dev = nullptr) {
    const int D = jobs[0].t->max_depth;
    uint32_t any_flags = 0;
    for (const Job& j : jobs) any_flags |= j.t->flags;
    const bool timing = (any_flags & SDD_TRACE_TIME_KERNELS) != 0;
    const bool count = (any_flags & SDD_TRACE_COUNT_WORK) != 0;
    const bool nrc = (any_flags & SDD_TRACE_NRC) != 0;
    long long total_pad = 0;
    const long long nb = plan_batches(c, jobs, total_pad);
    sdd_status st = ensure_batch(c, nb, D);
    if (st != SDD_OK) return st;
    c->last_nb = nb;
    // radiance cache (one render per call): training paths are those with
    // (s * WH + p) % stride == 0; in the call's path numbering qc = (s - s0) WH + p
    // they are qc = r + j * stride, j the training slot
    NrcPaths np{};
    uint32_t stride = 1;
    long long r_nrc = 0, n_slots = 0;
    if (nrc) {
        const Job& j = jobs[0];
        stride = (uint32_t)std::max<long long>(1, (j.total + c->nrc_train_paths - 1) / c->nrc_train_paths);
        const unsigned long long sw = (unsigned long long)(uint32_t)j.t->sample_offset * (unsigned long long)j.WH;
        r_nrc = (long long)((stride - sw % stride) % stride);
        n_slots = j.total > r_nrc ? (j.total - 1 - r_nrc) / stride + 1 : 0;
        const long long n_last = total_pad - (total_pad - 1) / nb * nb;  // paths of the call's last batch
        if ((st = nrc_ensure_render(c, nb, n_last, std::max<long long>(1, n_slots), D)) != SDD_OK) return st;
        np = NrcPaths{1, stride, c->nrc_cx, c->nrc_cn, c->nrc_tx, c->nrc_tn};
    }
    {  // this call's overflow bits start clear; they are folded into its renders at the end
        Timer tm(c, timing, 3);
        HIP_TRY(c, launch_fill_i32(c->d_overflow, 1, 0, c->stream));
    }
    for (const Job& j : jobs) {
        if (j.t->hit_log) {
            Timer tm(c, timing, 3);
            HIP_TRY(c, launch_fill_i32(j.t->hit_log, j.total * D, -2, c->stream));
        }
        if (j.t->shadow_log) {
            Timer tm(c, timing, 3);
            HIP_TRY(c, launch_fill_i32(j.t->shadow_log, j.total * D, -2, c->stream));
        }
    }
    struct Seg {
        const Job* j;
        long long q0;  // first path of the render in this segment
        int n;         // paths
        int pid_off;   // position in the batch (multiple of kShadeBlock)
    };
    std::vector<Seg> segs;
    for (long long g0 = 0; g0 < total_pad; g0 += nb) {
        const int N = (int)std::min(nb, total_pad - g0);
        const long long cap = N;
        segs.clear();
        for (const Job& j : jobs) {
            const long long a = std::max(g0, j.start), b = std::min(g0 + N, j.start + j.total);
            if (a < b) segs.push_back(Seg{&j, a - j.start, (int)(b - a), (int)(a - g0)});
        }
        {
            Timer tm(c, timing, 3);
            HIP_TRY(c, launch_fill_i32(c->d_counts, c->counts_len, 0, c->stream));
        }
        const int n_blocks = N / kShadeBlock;
        for (const Seg& sg : segs) {
            const sdd_trace_desc* t = sg.j->t;
            CamParams cp{};
            cp.N = sg.n;
            cp.pid_off = sg.pid_off;
            cp.pb = (int)(sg.q0 % sg.j->WH);
            cp.sb = (int)(sg.q0 / sg.j->WH);
            cp.fwh = make_fastdiv((uint32_t)sg.j->WH);
            cp.W = t->W;
            cp.H = t->H;
            cp.WH = sg.j->WH;
            cp.win = sg.j->win;
            cp.s0 = t->sample_offset;
            cp.s0p = s0_dev ? s0_dev + (sg.j - jobs.data()) : nullptr;
            cp.key = make_uint2(t->seed, (uint32_t)t->render_id);
            cp.ortho = sg.j->ortho ? 1 : 0;
            for (int k = 0; k < 3; ++k) {
                cp.eye[k] = t->eye[k];
                cp.fwd[k] = sg.j->f[k];
                cp.right[k] = sg.j->r[k];
                cp.up[k] = sg.j->u[k];
            }
            cp.tan_half = std::tan(0.5 * t->fov_deg * M_PI / 180.0);
            cp.aspect = (double)t->W / (double)t->H;
            cp.ortho_half_h = t->ortho_half_h;
            cp.flags = c->flags;
            cp.ray_o = c->ray_o;
            cp.ray_d = c->ray_d;
            cp.hit = c->hit;
            cp.grid = c->grid;
            cp.n_cells = c->G;
            cp.se = c->stage[0];
            cp.ext_bins = c->ext_bins;
            cp.n_blocks = n_blocks;
            cp.stats = c->d_stats;
            cp.nrc = np;
            Timer tm(c, timing, 3);
            HIP_TRY(c, launch_camgen(cp, c->stream));
            c->cam_rays += sg.n;
        }
        st = route(c, N, cap, ph_ext(1), -1, false, timing);
        if (st != SDD_OK) return st;
        ShadeParams sp{};
        sp.max_depth = D;
        sp.flags = c->flags;
        sp.ray_o = c->ray_o;
        sp.ray_d = c->ray_d;
        sp.hit = c->hit;
        sp.prim_info = c->d_prim_info;
        sp.prim_v = c->d_prim_v;
        sp.pane = c->d_pane;
        sp.coat = c->d_coat;
        sp.coat_n = c->coat_layers ? c->d_coat_n : nullptr;
        sp.coat_layers = c->coat_layers;
        sp.n_glass = c->n_glass;
        sp.nl = c->nl;
        sp.nlp = c->nlp;
        sp.light_type = c->light_type;
        for (int k = 0; k < 3; ++k) {
            sp.lp0[k] = c->lp0[k];
            sp.le1[k] = c->le1[k];
            sp.le2[k] = c->le2[k];
            sp.nL[k] = c->nL[k];
        }
        sp.light_area = c->light_area;
        sp.grid = c->grid;
        sp.n_cells = c->G;
        sp.se = c->stage[0];
        sp.ss = c->stage[1];
        sp.ext_bins = c->ext_bins;
        sp.n_blocks = n_blocks;
        sp.stats = c->d_stats;
        sp.nrc = np;
        for (int d = 1; d <= D; ++d) {
            // closest-hit rays of depth d share the sweeps with the shadow rays of depth d - 1
            st = run_sweeps(c, ph_ext(d), d >= 2 ? ph_sh(d - 1) : -1, cap, count, timing, d - 1, N);
            if (st != SDD_OK) return st;
            sp.depth = d;
            sp.vrec = c->vrec + (long long)(d - 1) * N;
            sp.sh_state = c->sh_state + (long long)(d - 1) * N;
            for (const Seg& sg : segs) {
                const sdd_trace_desc* t = sg.j->t;
                sp.N = sg.n;
                sp.pid_off = sg.pid_off;
                sp.pb = (int)(sg.q0 % sg.j->WH);
                sp.sb = (int)(sg.q0 / sg.j->WH);
                sp.fwh = make_fastdiv((uint32_t)sg.j->WH);
                sp.W = t->W;
                sp.WH = sg.j->WH;
                sp.win = sg.j->win;
                sp.s0 = t->sample_offset;
                sp.s0p = s0_dev ? s0_dev + (sg.j - jobs.data()) : nullptr;
                sp.spp_call = t->spp;
                sp.key = make_uint2(t->seed, (uint32_t)t->render_id);
                sp.hit_log = t->hit_log;
                sp.glass_from = sg.j->glass_from;
                sp.glass_to = sg.j->glass_to;
                Timer tm(c, timing, 2);
                HIP_TRY(c, launch_shade(sp, c->stream));
            }
            st = route(c, N, cap, d < D ? ph_ext(d + 1) : -1, ph_sh(d), true, timing);
            if (st != SDD_OK) return st;
        }
        st = run_sweeps(c, -1, ph_sh(D), cap, count, timing, D, N);
        if (st != SDD_OK) return st;
        if (nrc) {  // cache values at the batch's cache vertices, every wavelength
            nrc_wait_gpu(c);  // the previous call's Adam steps (on the training stream)
            ++c->nrc_query_launches;
            if (c->nrc_precision == 0) {
                c->nrc_query_rows += (long long)N * c->nl;  // every path slot
                Timer tm(c, timing, 4);
                HIP_TRY(c, nrc_launch_query(c->nrc, N, c->nrc_cx, c->nrc_cn, c->d_lam, c->nl, c->nlp, c->nrc_lhat, 1,
                                            0, c->nrc_hop, c->nrc_sop, nullptr, c->stream));
            } else {
                // only the paths that own a cache vertex (the kernel counts their rows)
                {
                    Timer tm(c, timing, 3);
                    const NrcOrder ord = nrc_order(c);
                    HIP_TRY(c, nrc_launch_cache_operands(qnet(c), N, c->nrc_cx, c->nrc_cn, c->nrc_hop, c->nrc_sop,
                                                         &ord, c->nrc_flags, c->nrc_rank, c->nrc_cp, c->stream));
                }
                Timer tm(c, timing, 4);  // the matrix-core kernel alone
                HIP_TRY(c, nrc_launch_query_mfma(c->nrc, N, c->nrc_hop, c->nrc_sop, c->d_lam, c->nl, c->nlp,
                                                 c->nrc_lhat, 1, c->stream, c->nrc_rank + N, c->nrc_cp,
                                                 c->d_stats + kStatNrcRows));
            }
        }
        for (const Seg& sg : segs) {
            const sdd_trace_desc* t = sg.j->t;
            SpectralParams xp{};
            xp.N = sg.n;
            xp.pid_off = sg.pid_off;
            xp.N_all = N;
            xp.pb = (int)(sg.q0 % sg.j->WH);
            xp.sb = (int)(sg.q0 / sg.j->WH);
            xp.fwh = make_fastdiv((uint32_t)sg.j->WH);
            xp.ngrp = c->nlp / 4;
            xp.fgrp = make_fastdiv((uint32_t)xp.ngrp);
            xp.WH = sg.j->WH;
            xp.s0 = t->sample_offset;
            xp.s0p = s0_dev ? s0_dev + (sg.j - jobs.data()) : nullptr;
            xp.spp_call = t->spp;
            xp.max_depth = D;
            xp.vrec = c->vrec;
            xp.sh_state = c->sh_state;
            xp.sh_glass = c->sh_glass;
            xp.pane = c->d_pane;
            xp.n_glass = std::max(1, c->n_glass);
            xp.coat = c->d_coat;
            xp.coat_n = c->coat_layers ? c->d_coat_n : nullptr;
            xp.coat_layers = c->coat_layers;
            xp.glass_from = sg.j->glass_from;
            xp.glass_to = sg.j->glass_to;
            xp.n_mats = c->M;
            xp.rho = c->d_rho;
            xp.le = c->d_le;
            xp.nl = c->nl;
            xp.nlp = c->nlp;
            xp.light_mat = c->light_mat < 0 ? 0 : c->light_mat;
            xp.acc = sg.j->rd->acc;
            xp.shadow_log = t->shadow_log;
            xp.lhat = nrc ? c->nrc_lhat : nullptr;
            Timer tm(c, timing, 3);
            HIP_TRY(c, launch_spectral(xp, c->stream));
            if (nrc) {  // training rows of the segment's training paths
                const long long a = sg.q0, b = sg.q0 + sg.n;  // call path indices of the segment
                const long long jlo = a <= r_nrc ? 0 : (a - r_nrc + stride - 1) / stride;
                const long long jhi = b - 1 < r_nrc ? -1 : (b - 1 - r_nrc) / stride;
                if (jhi >= jlo) {
                    NrcRowParams rp{};
                    rp.n = (int)(jhi - jlo + 1);
                    rp.j0 = jlo;
                    rp.r = r_nrc;
                    rp.stride = stride;
                    rp.q0 = sg.q0;
                    rp.pid_off = sg.pid_off;
                    rp.N_all = N;
                    rp.WH = sg.j->WH;
                    rp.win = sg.j->win;
                    rp.s0 = t->sample_offset;
                    rp.key = make_uint2(t->seed, (uint32_t)t->render_id);
                    rp.max_depth = D;
                    rp.nl = c->nl;
                    rp.nlp = c->nlp;
                    rp.n_glass = c->n_glass;
                    rp.n_mats = c->M;
                    rp.glass_from = sg.j->glass_from;
                    rp.glass_to = sg.j->glass_to;
                    rp.vrec = c->vrec;
                    rp.sh_state = c->sh_state;
                    rp.sh_glass = c->sh_glass;
                    rp.pane = c->d_pane;
                    rp.coat = c->d_coat;
                    rp.coat_n = c->coat_layers ? c->d_coat_n : nullptr;
                    rp.coat_layers = c->coat_layers;
                    rp.rho = c->d_rho;
                    rp.le = c->d_le;
                    rp.light_mat = c->light_mat < 0 ? 0 : c->light_mat;
                    rp.lam_nm = c->d_lam;
                    rp.tx = c->nrc_tx;
                    rp.tn = c->nrc_tn;
                    rp.rows = c->nrc_rows;
                    rp.row_ok = c->nrc_ok;
                    HIP_TRY(c, launch_nrc_rows(rp, c->stream));
                }
            }
        }
        ++c->batches;
    }
    {
        std::vector<int*> dst;
        dst.reserve(jobs.size() + 1);
        dst.push_back(c->d_ovf_stats);
        for (const Job& j : jobs) dst.push_back(j.rd->ovf);
        Timer tm(c, timing, 3);
        HIP_TRY(c, launch_fold_flags(c->d_overflow, dst.data(), (int)dst.size(), c->stream));
    }
    for (Job& j : jobs) j.rd->spp_done += j.t->spp;
    if (nrc) return nrc_train_after_call(c, n_slots * (D - 1), timing);
    return SDD_OK;
}

// the accumulator of render_id (created on first use)
sdd_status render_for(sdd_ctx* c, const sdd_trace_desc* t, Render*& out) {
    auto it = c->renders.find(t->render_id);
    const bool crop = t->crop_w != 0;
    const int ww = crop ? t->crop_w : t->W, wh = crop ? t->crop_h : t->H;
    const int x0 = crop ? t->crop_x0 : 0, y0 = crop ? t->crop_y0 : 0;
    if (it != c->renders.end() && (it->second.fW != t->W || it->second.fH != t->H || it->second.W != ww ||
                                   it->second.H != wh || it->second.x0 != x0 || it->second.y0 != y0))
        return fail(c, SDD_ERR_INVALID_ARG, "render_id reused with a different W, H or window");
    if (it == c->renders.end()) {
        Render rd;
        rd.W = ww;
        rd.H = wh;
        rd.fW = t->W;
        rd.fH = t->H;
        rd.x0 = x0;
        rd.y0 = y0;
        const size_t n = (size_t)c->nlp * ww * wh;
        ++c->gen;
        sdd_status st = dalloc(c, &rd.acc, n);
        if (st != SDD_OK) return st;
        if ((st = dalloc(c, &rd.ovf, 1)) != SDD_OK) {
            dfree(c, rd.acc);
            return st;
        }
        HIP_TRY(c, hipMemsetAsync(rd.acc, 0, sizeof(float) * n, c->stream));
        HIP_TRY(c, launch_fill_i32(rd.ovf, 1, 0, c->stream));
        it = c->renders.emplace(t->render_id, rd).first;
    }
    out = &it->second;
    return SDD_OK;
}

// SDD_TRACE_GRAPH: the call's whole launch sequence is captured once into a
// HIP graph and replayed by later calls that differ only in sample_offset
// (the kernels read each render's first sample index from d_s0).  A graph is
// keyed by the descs without their sample offsets and by the buffer
// generation, so any reallocation or reset recaptures.
sdd_status trace_graph(sdd_ctx* c, int n, const sdd_trace_desc* descs, std::vector<Job>& jobs) {
    long long total_pad = 0;
    const long long nb = plan_batches(c, jobs, total_pad);
    sdd_status st = ensure_batch(c, nb, descs[0].max_depth);  // allocate before any capture
    if (st != SDD_OK) return st;
    c->last_nb = nb;
    if (n > c->s0_cap) {
        dfree(c, c->d_s0);
        c->s0_cap = 0;
        if ((st = dalloc(c, &c->d_s0, (size_t)SDD_MAX_RENDERS)) != SDD_OK) return st;
        c->s0_cap = SDD_MAX_RENDERS;
        ++c->gen;
    }
    std::string key(reinterpret_cast<const char*>(&c->gen), sizeof(c->gen));
    key.append(reinterpret_cast<const char*>(&nb), sizeof(nb));
    c->h_s0.assign((size_t)n, 0);
    for (int i = 0; i < n; ++i) {
        sdd_trace_desc d = descs[i];
        c->h_s0[(size_t)i] = d.sample_offset;
        d.sample_offset = 0;
        key.append(reinterpret_cast<const char*>(&d), sizeof(d));
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_s0, c->h_s0.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, c->stream));
    if (c->graph_exec && key == c->graph_key) {
        HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
        c->cam_rays += c->graph_cam_rays;
        c->launches_trace += c->graph_launches;
        c->batches += c->graph_batches;
        for (Job& j : jobs) j.rd->spp_done += j.t->spp;
        return SDD_OK;
    }
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    c->graph_key.clear();
    const long long cr0 = c->cam_rays, lt0 = c->launches_trace, b0 = c->batches;
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    st = trace_jobs(c, jobs, c->d_s0);
    hipGraph_t gr = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->stream, &gr);
    if (st != SDD_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
    }
    if (ee != hipSuccess) return hip_fail(c, ee, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ei != hipSuccess) return hip_fail(c, ei, "hipGraphInstantiate");
    c->graph_exec = ex;
    c->graph_key = key;
    c->graph_cam_rays = c->cam_rays - cr0;
    c->graph_launches = c->launches_trace - lt0;
    c->graph_batches = c->batches - b0;
    HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));  // the captured work has not run yet
    return SDD_OK;
}

sdd_status trace_call(sdd_ctx* c, int n, const sdd_trace_desc* descs) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->has_bvh) return fail(c, SDD_ERR_STATE, "trace before sdd_build_bvh");
    if (n < 1 || n > SDD_MAX_RENDERS || !descs) return fail(c, SDD_ERR_INVALID_ARG, "bad render count");
    std::vector<Job> jobs((size_t)n);
    for (int i = 0; i < n; ++i) {
        sdd_status st = check_desc(c, &descs[i], jobs[i]);
        if (st != SDD_OK) return st;
        if (descs[i].max_depth != descs[0].max_depth)
            return fail(c, SDD_ERR_INVALID_ARG, "renders of one call must share max_depth");
        for (int k = 0; k < i; ++k)
            if (descs[k].render_id == descs[i].render_id)
                return fail(c, SDD_ERR_INVALID_ARG, "render_id repeated within one call");
    }
    for (int i = 0; i < n; ++i)
        if (descs[i].flags & SDD_TRACE_NRC) {
            if (n != 1) return fail(c, SDD_ERR_UNSUPPORTED, "radiance-cache rendering takes one render per call");
            if (!c->has_nrc) return fail(c, SDD_ERR_STATE, "SDD_TRACE_NRC before sdd_nrc_init");
        }
    bool graph = false;
    for (int i = 0; i < n; ++i) graph = graph || (descs[i].flags & SDD_TRACE_GRAPH);
    if (graph) {
        for (int i = 0; i < n; ++i)
            if (descs[i].flags & (SDD_TRACE_NRC | SDD_TRACE_TIME_KERNELS))
                return fail(c, SDD_ERR_UNSUPPORTED, "SDD_TRACE_GRAPH excludes SDD_TRACE_NRC and SDD_TRACE_TIME_KERNELS");
        if (!c->stream) return fail(c, SDD_ERR_UNSUPPORTED, "SDD_TRACE_GRAPH needs a context stream other than NULL");
    }
    DeviceGuard g(c->device);
    for (int i = 0; i < n; ++i) {
        sdd_status st = render_for(c, &descs[i], jobs[i].rd);
        if (st != SDD_OK) return st;
    }
    c->call_budget = mem_budget_bytes(c);  // once per call: plan_batches also runs under graph capture
    if (!graph) return trace_jobs(c, jobs);
    return trace_graph(c, n, descs, jobs);
}

// ---------------------------------------------------------------------------
// launch-setting search (sdd_autotune) and its results file
// ---------------------------------------------------------------------------
// One line per configuration: "<key>\t<batch_paths> <trace_grid> <dir_bins> <ms>".
bool tune_cache_read(const char* path, const std::string& key, sdd_tuning* t, double* ms) {
    std::ifstream f(path);
    if (!f) return false;
    bool found = false;
    std::string line;
    while (std::getline(f, line)) {
        const size_t tab = line.rfind('\t');
        if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != key.size()) continue;
        long long b = 0;
        int g = 0, d = 0;
        double m = 0.0;
        if (std::sscanf(line.c_str() + tab + 1, "%lld %d %d %lf", &b, &g, &d, &m) != 4) continue;
        sdd_tuning u{};
        u.batch_paths = b;
        u.trace_grid = g;
        u.dir_bins = d;
        if (tuning_problem(&u)) continue;  // a damaged line is skipped
        *t = u;
        if (ms) *ms = m;
        found = true;  // the last valid line of the key wins
    }
    return found;
}

// rewrites the file without the key's old lines, then appends the new one
// (written to a temporary file and renamed, so readers never see half a file)
bool tune_cache_write(const char* path, const std::string& key, const sdd_tuning& t, double ms) {
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            const size_t tab = line.rfind('\t');
            if (tab != std::string::npos && tab == key.size() && line.compare(0, tab, key) == 0) continue;
            if (!line.empty()) keep.push_back(line);
        }
    }
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o) return false;
        for (const std::string& l : keep) o << l << '\n';
        char buf[128];
        std::snprintf(buf, sizeof(buf), "\t%lld %d %d %.6f\n", (long long)t.batch_paths, t.trace_grid, t.dir_bins, ms);
        o << key << buf;
        if (!o.good()) {
            std::remove(tmp.c_str());
            return false;
        }
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

// what the best settings depend on: the device, the library build, the scene
// and its grid of cells, and the shape of the call (not its sample offsets or
// camera poses)
std::string tune_key(const sdd_ctx* c, int n, const sdd_trace_desc* d) {
    hipDeviceProp_t pr{};
    if (hipGetDeviceProperties(&pr, c->device) != hipSuccess) std::snprintf(pr.gcnArchName, sizeof(pr.gcnArchName), "?");
    long long paths = 0;
    uint32_t fl = 0;
    for (int i = 0; i < n; ++i) {
        paths += window_pixels(&d[i]) * d[i].spp;
        fl |= d[i].flags & (SDD_TRACE_COUNT_WORK | SDD_TRACE_GRAPH);
    }
    std::ostringstream k;
    k << "sdd-tune-1 dev=" << pr.gcnArchName << "/" << pr.multiProcessorCount << "cu build=" << __DATE__ << " "
      << __TIME__ << " tris=" << c->T << " lambda=" << c->nl << " glass=" << c->n_glass << " coats=" << c->coat_layers
      << " cells=" << c->grid.nx << "x" << c->grid.ny << "x" << c->grid.nz << " renders=" << n << " paths=" << paths
      << " depth=" << d[0].max_depth << " flags=" << fl;
    std::string s = k.str();
    for (char& ch : s)
        if (ch == '\t' || ch == '\n' || ch == '\r') ch = ' ';
    return s;
}

void set_tuning_fields(sdd_ctx* c, const sdd_tuning& t) {
    c->tune_batch = t.batch_paths;
    c->tune_grid = t.trace_grid;
    c->tune_bins = t.dir_bins;
    if (c->has_bvh) apply_tuning(c);
    ++c->gen;  // a captured graph holds the old launch shapes
}

// drops the accumulators of the call's renders (the search's samples)
void drop_renders(sdd_ctx* c, int n, const sdd_trace_desc* d) {
    (void)hipStreamSynchronize(c->stream);
    for (int i = 0; i < n; ++i) {
        auto it = c->renders.find(d[i].render_id);
        if (it == c->renders.end()) continue;
        dfree(c, it->second.acc);
        c->renders.erase(it);
    }
    ++c->gen;
}

// time of one call under tuning t: one untimed call (allocation, graph
// capture), then the fastest of reps timed calls
sdd_status time_call(sdd_ctx* c, int n, const sdd_trace_desc* descs, int reps, const sdd_tuning& t, hipEvent_t a,
                     hipEvent_t b, double& ms) {
    set_tuning_fields(c, t);
    sdd_status st = trace_call(c, n, descs);
    if (st != SDD_OK) return st;
    ms = std::numeric_limits<double>::infinity();
    for (int r = 0; r < reps; ++r) {
        HIP_TRY(c, hipEventRecord(a, c->stream));
        if ((st = trace_call(c, n, descs)) != SDD_OK) return st;
        HIP_TRY(c, hipEventRecord(b, c->stream));
        HIP_TRY(c, hipEventSynchronize(b));
        float e = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&e, a, b));
        ms = std::min(ms, (double)e);
    }
    return SDD_OK;
}

// coordinate search from the library's own choices: direction bins, then the
// traversal grid, then the paths per pass; a candidate must win by more than
// 1% to replace the incumbent, so timing noise keeps the defaults
sdd_status search_tuning(sdd_ctx* c, int n, const sdd_trace_desc* descs, int reps, sdd_tuning& best, double& best_ms) {
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(c, hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(c, SDD_ERR_HIP, "hipEventCreate");
    }
    const bool verbose = std::getenv("SDD_TUNE_VERBOSE") != nullptr;  // one stderr line per candidate
    auto report = [&](const sdd_tuning& t, double ms) {
        if (verbose)
            std::fprintf(stderr, "[sdd tune] batch_paths %lld trace_grid %d dir_bins %d: %.3f ms (launched grid %d, bins %d)\n",
                         (long long)t.batch_paths, t.trace_grid, t.dir_bins, ms, c->trace_grid, c->ext_bins);
    };
    best = sdd_tuning{};
    sdd_status st = time_call(c, n, descs, reps, best, a, b, best_ms);
    if (st == SDD_OK) report(best, best_ms);
    auto consider = [&](const sdd_tuning& t) {
        if (st != SDD_OK) return;
        double ms = 0.0;
        st = time_call(c, n, descs, reps, t, a, b, ms);
        if (st == SDD_OK) report(t, ms);
        if (st == SDD_OK && ms < 0.99 * best_ms) {
            best = t;
            best_ms = ms;
        }
    };
    if (c->G * kExtBins <= kMaxCells) {
        sdd_tuning t = best;
        t.dir_bins = 1;
        consider(t);
    }
    const int g_auto = std::min(c->trace_grid_max, trace_grid_for(c, c->G));
    for (int num : {3, 2}) {
        const int g = std::max(kXcd, g_auto * num / 4 / kXcd * kXcd);
        if (g >= g_auto) continue;
        sdd_tuning t = best;
        t.trace_grid = g;
        consider(t);
    }
    long long total_pad = 0;
    {
        std::vector<Job> jobs((size_t)n);
        for (int i = 0; i < n; ++i) jobs[i].t = &descs[i];
        for (int i = 0; i < n; ++i) jobs[i].total = window_pixels(&descs[i]) * descs[i].spp;
        const long long keep = c->tune_batch;
        c->tune_batch = 0;
        c->call_budget = mem_budget_bytes(c);
        const long long nb_auto = plan_batches(c, jobs, total_pad);
        c->tune_batch = keep;
        for (int div : {2, 4}) {
            const long long nb = (nb_auto / div + kShadeBlock - 1) / kShadeBlock * kShadeBlock;
            if (nb < (1LL << 16)) continue;  // small passes only add sweep overhead
            sdd_tuning t = best;
            t.batch_paths = nb;
            consider(t);
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

}  // namespace

extern "C" {

sdd_status sdd_trace_spectral(sdd_ctx* c, const sdd_trace_desc* t) {
    if (c && !t) {
        c->err = "null trace desc";
        return SDD_ERR_INVALID_ARG;
    }
    return trace_call(c, 1, t);
}

sdd_status sdd_trace_batch(sdd_ctx* c, int32_t n, const sdd_trace_desc* descs) { return trace_call(c, n, descs); }

sdd_status sdd_validate_tuning(const sdd_tuning* t, char* msg, int msg_len) {
    const char* e = tuning_problem(t);
    if (msg && msg_len > 0) std::snprintf(msg, (size_t)msg_len, "%s", e ? e : "");
    return e ? SDD_ERR_INVALID_ARG : SDD_OK;
}

sdd_status sdd_set_tuning(sdd_ctx* c, const sdd_tuning* t) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (const char* e = tuning_problem(t)) return fail(c, SDD_ERR_INVALID_ARG, e);
    if (t->trace_grid > c->trace_grid_max)
        return fail(c, SDD_ERR_INVALID_ARG, "trace_grid above the device's resident maximum of " +
                                                std::to_string(c->trace_grid_max));
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    set_tuning_fields(c, *t);
    return SDD_OK;
}

sdd_status sdd_set_deferral(sdd_ctx* c, int32_t below_rays, int32_t extra_sweeps) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (below_rays < 0 || extra_sweeps < 0 || extra_sweeps > kMaxDeferExtra)
        return fail(c, SDD_ERR_INVALID_ARG,
                    "below_rays must be >= 0 and extra_sweeps in 0.." + std::to_string(kMaxDeferExtra));
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->defer_rays = below_rays;
    c->defer_extra = extra_sweeps;
    ++c->gen;  // a captured launch sequence has another number of sweeps
    return SDD_OK;
}

sdd_status sdd_get_tuning(sdd_ctx* c, sdd_tuning* out) {
    if (!c || !out) return SDD_ERR_INVALID_ARG;
    out->batch_paths = c->tune_batch;
    out->trace_grid = c->has_bvh ? c->trace_grid : 0;
    out->dir_bins = c->has_bvh ? c->ext_bins : 0;
    return SDD_OK;
}

sdd_status sdd_tune_cache_lookup(const char* path, const char* key, sdd_tuning* out, double* ms, int32_t* found) {
    if (!path || !key || !out || !found) return SDD_ERR_INVALID_ARG;
    *found = tune_cache_read(path, key, out, ms) ? 1 : 0;
    return SDD_OK;
}

sdd_status sdd_tune_cache_store(const char* path, const char* key, const sdd_tuning* t, double ms) {
    if (!path || !*path || !key || !*key || tuning_problem(t) || !(ms >= 0.0)) return SDD_ERR_INVALID_ARG;
    for (const char* p = key; *p; ++p)
        if (*p == '\t' || *p == '\n' || *p == '\r') return SDD_ERR_INVALID_ARG;
    return tune_cache_write(path, key, *t, ms) ? SDD_OK : SDD_ERR_STATE;
}

sdd_status sdd_tune_key(sdd_ctx* c, int32_t n, const sdd_trace_desc* descs, char* out, int32_t out_len) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!descs || n < 1 || n > SDD_MAX_RENDERS || !out || out_len < 1)
        return fail(c, SDD_ERR_INVALID_ARG, "bad arguments to sdd_tune_key");
    if (!c->has_bvh) return fail(c, SDD_ERR_STATE, "sdd_tune_key before sdd_build_bvh");
    const std::string k = tune_key(c, n, descs);
    if ((int)k.size() >= out_len) return fail(c, SDD_ERR_INVALID_ARG, "key buffer too small");
    std::snprintf(out, (size_t)out_len, "%s", k.c_str());
    return SDD_OK;
}

sdd_status sdd_autotune(sdd_ctx* c, int32_t n, const sdd_trace_desc* descs, int32_t reps, const char* cache_path,
                        sdd_tuning* out, double* ms_out, int32_t* from_cache) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!descs || !out || n < 1 || n > SDD_MAX_RENDERS) return fail(c, SDD_ERR_INVALID_ARG, "bad arguments to sdd_autotune");
    if (reps < 1 || reps > 100) return fail(c, SDD_ERR_INVALID_ARG, "reps must be in 1..100");
    if (!c->has_bvh) return fail(c, SDD_ERR_STATE, "sdd_autotune before sdd_build_bvh");
    for (int i = 0; i < n; ++i) {
        if (descs[i].flags & SDD_TRACE_NRC)
            return fail(c, SDD_ERR_UNSUPPORTED, "autotune of radiance-cache renders (the calls would train the cache)");
        if (descs[i].hit_log || descs[i].shadow_log) return fail(c, SDD_ERR_INVALID_ARG, "autotune takes no logs");
        if (c->renders.count(descs[i].render_id))
            return fail(c, SDD_ERR_STATE, "autotune needs render ids that hold no samples (its calls are discarded)");
    }
    DeviceGuard g(c->device);
    if (from_cache) *from_cache = 0;
    const std::string key = tune_key(c, n, descs);
    sdd_tuning t{};
    double ms = 0.0;
    if (cache_path && *cache_path && tune_cache_read(cache_path, key, &t, &ms) && t.trace_grid <= c->trace_grid_max) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        set_tuning_fields(c, t);
        *out = t;
        if (ms_out) *ms_out = ms;
        if (from_cache) *from_cache = 1;
        return SDD_OK;
    }
    const sdd_tuning before{c->tune_batch, c->tune_grid, c->tune_bins};
    sdd_status st = search_tuning(c, n, descs, reps, t, ms);
    drop_renders(c, n, descs);
    if (st != SDD_OK) {
        const std::string e = c->err;
        set_tuning_fields(c, before);
        c->err = e;
        return st;
    }
    set_tuning_fields(c, t);
    *out = t;
    if (ms_out) *ms_out = ms;
    if (cache_path && *cache_path && !tune_cache_write(cache_path, key, t, ms))
        return fail(c, SDD_ERR_STATE, std::string("cannot write the tuning file ") + cache_path);
    return SDD_OK;
}

sdd_status sdd_resolve_image(sdd_ctx* c, int32_t render_id, double* spectral_out, double* xyz_out,
                             int32_t out_is_device) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    auto it = c->renders.find(render_id);
    if (it == c->renders.end()) return fail(c, SDD_ERR_STATE, "unknown render_id");
    Render& rd = it->second;
    if (rd.spp_done <= 0) return fail(c, SDD_ERR_STATE, "render has no samples");
    DeviceGuard g(c->device);
    const int WH = rd.W * rd.H;
    double* ds = spectral_out;
    double* dx = xyz_out;
    double* tmp_s = nullptr;
    double* tmp_x = nullptr;
    if (!out_is_device) {
        if (spectral_out && dalloc(c, &tmp_s, (size_t)WH * c->nl) != SDD_OK) return SDD_ERR_OOM;
        if (xyz_out && dalloc(c, &tmp_x, (size_t)WH * 3) != SDD_OK) {
            dfree(c, tmp_s);
            return SDD_ERR_OOM;
        }
        ds = tmp_s;
        dx = tmp_x;
    }
    hipError_t e =
        launch_resolve(WH, c->nl, c->nlp, 1.0 / (double)rd.spp_done, rd.acc, c->d_w, c->d_cmf, ds, dx, c->stream);
    if (e == hipSuccess && !out_is_device) {
        if (spectral_out)
            e = hipMemcpyAsync(spectral_out, tmp_s, sizeof(double) * (size_t)WH * c->nl, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && xyz_out)
            e = hipMemcpyAsync(xyz_out, tmp_x, sizeof(double) * (size_t)WH * 3, hipMemcpyDeviceToHost, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(c, tmp_s);
    dfree(c, tmp_x);
    if (e != hipSuccess) return hip_fail(c, e, "resolve");
    int ovf = 0;
    HIP_TRY(c, hipMemcpy(&ovf, rd.ovf, sizeof(int), hipMemcpyDeviceToHost));
    if (ovf & kOverflowPanes)
        return fail(c, SDD_ERR_OVERFLOW, "a shadow segment crossed more than " + std::to_string(kMaxGlass) +
                                              " glass panes (only the first are tracked)");
    if (ovf & kOverflowQueue) return fail(c, SDD_ERR_OVERFLOW, "a subdomain queue count exceeded its capacity");
    return SDD_OK;
}

sdd_status sdd_reset_render(sdd_ctx* c, int32_t render_id) {
    if (c) ++c->gen;
    if (!c) return SDD_ERR_INVALID_ARG;
    auto it = c->renders.find(render_id);
    if (it == c->renders.end()) return fail(c, SDD_ERR_STATE, "unknown render_id");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c, it->second.acc);
    dfree(c, it->second.ovf);
    c->renders.erase(it);
    return SDD_OK;
}

sdd_status sdd_get_stats(sdd_ctx* c, sdd_stats* out) {
    if (!c || !out) return SDD_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, nrc_wait_host(c));
    harvest_events(c);
    unsigned long long s[kStatCount];
    HIP_TRY(c, hipMemcpy(s, c->d_stats, sizeof(s), hipMemcpyDeviceToHost));
    int ovf = 0;
    HIP_TRY(c, hipMemcpy(&ovf, c->d_ovf_stats, sizeof(int), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->ext_rays = (int64_t)s[kStatExtRays] + c->cam_rays;
    out->shadow_rays = (int64_t)s[kStatShadowRays];
    out->ext_cell_visits = (int64_t)s[kStatExtVisits];
    out->shadow_cell_visits = (int64_t)s[kStatShadowVisits];
    out->node_visits = (int64_t)s[kStatNodes];
    out->tri_tests = (int64_t)s[kStatTris];
    out->wave_node_steps = (int64_t)s[kStatNodeSteps];
    out->wave_tri_steps = (int64_t)s[kStatTriSteps];
    out->batches = c->batches;
    out->launches_trace = c->launches_trace;
    out->ms_trace_ext = c->ms[0];
    out->ms_trace_shadow = c->ms[1];
    out->ms_shade = c->ms[2];
    out->ms_other = c->ms[3];
    out->ms_nrc_query = c->ms[4];
    out->ms_nrc_train = c->ms[5];
    out->nrc_query_rows = c->nrc_query_rows + (int64_t)s[kStatNrcRows];
    out->nrc_query_launches = c->nrc_query_launches;
    out->nrc_train_rows = c->nrc_train_rows;
    out->n_refs = c->has_bvh ? c->gb.n_refs : 0;
    long long nn = 0;
    for (int v : c->gb.cell_nodes) nn += v;
    out->n_nodes = c->has_bvh ? nn : 0;
    out->max_bvh_depth = c->has_bvh ? c->gb.max_depth : 0;
    out->n_cells = c->has_bvh ? c->G : 0;
    out->device_bytes = c->device_bytes;
    out->paths_per_batch = c->last_nb;
    out->overflow = ovf;
    return SDD_OK;
}

sdd_status sdd_reset_stats(sdd_ctx* c) {
    if (!c) return SDD_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, nrc_wait_host(c));
    harvest_events(c);
    HIP_TRY(c, hipMemsetAsync(c->d_stats, 0, sizeof(unsigned long long) * kStatCount, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_ovf_stats, 0, sizeof(int), c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->batches = 0;
    c->cam_rays = 0;
    c->launches_trace = 0;
    for (double& m : c->ms) m = 0.0;
    c->nrc_query_rows = c->nrc_query_launches = c->nrc_train_rows = 0;
    return SDD_OK;
}

sdd_status sdd_debug_philox(sdd_ctx* c, int32_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    if (!c) return SDD_ERR_INVALID_ARG;
    if (n < 0 || (n > 0 && (!ctr || !key || !out))) return fail(c, SDD_ERR_INVALID_ARG, "bad philox arguments");
    if (n == 0) return SDD_OK;
    DeviceGuard g(c->device);
    uint4* dc = nullptr;
    uint4* dout = nullptr;
    if (dalloc(c, &dc, (size_t)n) != SDD_OK || dalloc(c, &dout, (size_t)n) != SDD_OK) {
        dfree(c, dc);
        return SDD_ERR_OOM;
    }
    hipError_t e = hipMemcpyAsync(dc, ctr, sizeof(uint4) * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_philox(n, dc, make_uint2(key[0], key[1]), dout, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(uint4) * (size_t)n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(c, dc);
    dfree(c, dout);
    if (e != hipSuccess) return hip_fail(c, e, "debug philox");
    return SDD_OK;
}

sdd_status sdd_debug_pane(sdd_ctx* c, int32_t n, const float* params, float* R_out, float* T_out) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (n < 0 || (n > 0 && (!params || !R_out || !T_out))) return fail(c, SDD_ERR_INVALID_ARG, "bad pane arguments");
    if (n == 0) return SDD_OK;
    std::vector<float4> pc((size_t)n);
    std::vector<float> cc((size_t)n);
    for (int i = 0; i < n; ++i) {
        const float* q = params + 5 * (size_t)i;
        const double nn = q[0], k = q[1], th = q[2], lam = q[3];
        if (!(nn > 0.0) || !(k >= 0.0) || !(th >= 0.0) || !(lam > 0.0) || !(q[4] >= 0.0f && q[4] <= 1.0f))
            return fail(c, SDD_ERR_INVALID_ARG, "pane parameters out of range");
        pc[i] = make_float4((float)(nn * nn - k * k), (float)(2.0 * nn * k), (float)(1.0 / (nn * nn)),
                            (float)(4.0 * M_PI * k * th / (lam * 1e-9)));
        cc[i] = q[4];
    }
    DeviceGuard g(c->device);
    float4* dpc = nullptr;
    float* dc = nullptr;
    float2* dout = nullptr;
    if (dalloc(c, &dpc, (size_t)n) != SDD_OK || dalloc(c, &dc, (size_t)n) != SDD_OK ||
        dalloc(c, &dout, (size_t)n) != SDD_OK) {
        dfree(c, dpc);
        dfree(c, dc);
        return SDD_ERR_OOM;
    }
    std::vector<float2> h((size_t)n);
    hipError_t e = hipMemcpyAsync(dpc, pc.data(), sizeof(float4) * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dc, cc.data(), sizeof(float) * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_pane(n, dpc, dc, dout, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), dout, sizeof(float2) * (size_t)n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(c, dpc);
    dfree(c, dc);
    dfree(c, dout);
    if (e != hipSuccess) return hip_fail(c, e, "debug pane");
    for (int i = 0; i < n; ++i) {
        R_out[i] = h[i].x;
        T_out[i] = h[i].y;
    }
    return SDD_OK;
}

sdd_status sdd_debug_glass(sdd_ctx* c, int32_t n, const int32_t* mat, const int32_t* lam, const float* cs,
                           float* R_out, float* T_out) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->has_scene) return fail(c, SDD_ERR_STATE, "sdd_debug_glass before sdd_load_scene");
    if (n < 0 || (n > 0 && (!mat || !lam || !cs || !R_out || !T_out)))
        return fail(c, SDD_ERR_INVALID_ARG, "bad glass arguments");
    if (n == 0) return SDD_OK;
    std::vector<int4> q((size_t)n);
    for (int i = 0; i < n; ++i) {
        if (mat[i] < 0 || mat[i] >= c->M || c->glass_of[mat[i]] < 0)
            return fail(c, SDD_ERR_INVALID_ARG, "material is not a glass material");
        if (lam[i] < 0 || lam[i] >= c->nl) return fail(c, SDD_ERR_INVALID_ARG, "wavelength index out of range");
        if (!(std::fabs(cs[i]) <= 1.0f)) return fail(c, SDD_ERR_INVALID_ARG, "cosine outside [-1, 1]");
        float f = cs[i];
        int bits;
        std::memcpy(&bits, &f, 4);
        q[i] = make_int4(c->glass_of[mat[i]], lam[i], bits, 0);
    }
    DeviceGuard g(c->device);
    int4* dq = nullptr;
    float2* dout = nullptr;
    if (dalloc(c, &dq, (size_t)n) != SDD_OK || dalloc(c, &dout, (size_t)n) != SDD_OK) {
        dfree(c, dq);
        return SDD_ERR_OOM;
    }
    std::vector<float2> h((size_t)n);
    GlassTable tab{c->d_pane, c->d_coat, c->coat_layers ? c->d_coat_n : nullptr, c->coat_layers, c->nlp};
    hipError_t e = hipMemcpyAsync(dq, q.data(), sizeof(int4) * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_glass(n, tab, dq, dout, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), dout, sizeof(float2) * (size_t)n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(c, dq);
    dfree(c, dout);
    if (e != hipSuccess) return hip_fail(c, e, "debug glass");
    for (int i = 0; i < n; ++i) {
        R_out[i] = h[i].x;
        T_out[i] = h[i].y;
    }
    return SDD_OK;
}

sdd_status sdd_debug_trace_rays(sdd_ctx* c, int32_t n, const float* o, const float* d, float* t_out,
                                int32_t* prim_out) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->has_bvh) return fail(c, SDD_ERR_STATE, "sdd_debug_trace_rays before sdd_build_bvh");
    if (n < 0 || (n > 0 && (!o || !d || !t_out || !prim_out))) return fail(c, SDD_ERR_INVALID_ARG, "bad ray arguments");
    if (n == 0) return SDD_OK;
    for (long long i = 0; i < 3LL * n; ++i)
        if (!std::isfinite(o[i]) || !std::isfinite(d[i])) return fail(c, SDD_ERR_INVALID_ARG, "non-finite ray");
    DeviceGuard g(c->device);
    sdd_status st = ensure_batch(c, std::max<long long>(n, c->ncap), std::max(1, c->dcap));
    if (st != SDD_OK) return st;
    float* dor = nullptr;
    float* ddr = nullptr;
    if (dalloc(c, &dor, 3 * (size_t)n) != SDD_OK || dalloc(c, &ddr, 3 * (size_t)n) != SDD_OK) {
        dfree(c, dor);
        return SDD_ERR_OOM;
    }
    hipError_t e = hipMemcpyAsync(dor, o, sizeof(float) * 3 * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ddr, d, sizeof(float) * 3 * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_fill_i32(c->d_counts, c->counts_len, 0, c->stream);
    if (e == hipSuccess)
        e = launch_debug_rays(n, dor, ddr, c->grid, c->hit, c->qa[0], c->qb[0], c->qc[0], counts_at(c, 0, 0), n,
                              c->stream);
    if (e != hipSuccess) {
        dfree(c, dor);
        dfree(c, ddr);
        return hip_fail(c, e, "debug rays");
    }
    st = run_sweeps(c, ph_ext(1), -1, n, false, false);
    std::vector<float2> h((size_t)n);
    if (st == SDD_OK) {
        e = hipMemcpyAsync(h.data(), c->hit, sizeof(float2) * (size_t)n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    dfree(c, dor);
    dfree(c, ddr);
    if (st != SDD_OK) return st;
    if (e != hipSuccess) return hip_fail(c, e, "debug rays copy");
    for (int i = 0; i < n; ++i) {
        t_out[i] = h[i].x;
        int p;
        std::memcpy(&p, &h[i].y, 4);
        prim_out[i] = p;
    }
    return SDD_OK;
}

}  // extern "C"

// ===========================================================================
// Learned radiance cache
// ===========================================================================
namespace {

constexpr int kNrcMinLog2 = 10, kNrcMaxLog2 = 24;
constexpr int kNrcMaxRows = 1 << 22;

long long nrc_count(int log2) {
    const long long T = 1LL << log2;
    return (long long)kNrcLevels * T * kNrcFeat + kNrcW + kNrcLayers * kNrcHid + kNrcHid + 1;
}

// K_l^|m| = sqrt((2l + 1) / (4 pi) (l - |m|)! / (l + |m|)!) in (l, m) order
void sh_constants(float* K) {
    auto fact = [](int k) {
        double f = 1.0;
        for (int i = 2; i <= k; ++i) f *= i;
        return f;
    };
    int k = 0;
    for (int l = 0; l < 4; ++l)
        for (int m = -l; m <= l; ++m, ++k) {
            const int am = m < 0 ? -m : m;
            K[k] = (float)std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * fact(l - am) / fact(l + am));
        }
}

sdd_status nrc_reserve(sdd_ctx* c, long long n) {
    if (n <= c->nrc_cap) return SDD_OK;
    HIP_TRY(c, nrc_wait_host(c));
    free_nrc_batch(c);
    sdd_status st;
    if ((st = dalloc(c, &c->nrc_acts, (size_t)(kNrcLayers + 1) * kNrcHid * n)) != SDD_OK ||
        (st = dalloc(c, &c->nrc_dz, (size_t)kNrcLayers * kNrcHid * n)) != SDD_OK ||
        (st = dalloc(c, &c->nrc_y, (size_t)n)) != SDD_OK || (st = dalloc(c, &c->nrc_dy, (size_t)n)) != SDD_OK) {
        free_nrc_batch(c);
        return st;
    }
    c->nrc_cap = n;
    return SDD_OK;
}

}  // namespace

extern "C" {

int64_t sdd_nrc_param_count(int32_t table_log2) {
    if (table_log2 < kNrcMinLog2 || table_log2 > kNrcMaxLog2) return -1;
    return nrc_count(table_log2);
}

sdd_status sdd_nrc_init(sdd_ctx* c, const sdd_nrc_desc* d) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!d) return fail(c, SDD_ERR_INVALID_ARG, "null nrc desc");
    if (d->table_log2 < kNrcMinLog2 || d->table_log2 > kNrcMaxLog2)
        return fail(c, SDD_ERR_INVALID_ARG, "table_log2 out of range");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d->aabb_lo[a]) || !std::isfinite(d->aabb_hi[a]) || !(d->aabb_hi[a] > d->aabb_lo[a]))
            return fail(c, SDD_ERR_INVALID_ARG, "bad position box");
    if (!std::isfinite(d->lambda_lo) || !std::isfinite(d->lambda_hi) || !(d->lambda_hi > d->lambda_lo))
        return fail(c, SDD_ERR_INVALID_ARG, "bad wavelength range");
    if (!(d->lr > 0.0f) || !std::isfinite(d->lr) || !(d->beta1 >= 0.0f && d->beta1 < 1.0f) ||
        !(d->beta2 >= 0.0f && d->beta2 < 1.0f) || !(d->eps > 0.0f) || !std::isfinite(d->eps))
        return fail(c, SDD_ERR_INVALID_ARG, "bad Adam hyper-parameters");
    if (!d->params) return fail(c, SDD_ERR_INVALID_ARG, "null parameters");
    if (d->train_paths < 1 || d->train_steps < 0 || d->train_batch < 1 || d->train_batch > kNrcMaxRows ||
        (d->precision != 0 && d->precision != 1) || (d->table_fp16 != 0 && d->table_fp16 != 1))
        return fail(c, SDD_ERR_INVALID_ARG,
                    "bad render settings (train_paths, train_steps, train_batch, precision, table_fp16)");
    const long long n_all = nrc_count(d->table_log2);
    for (long long i = 0; i < n_all; ++i)
        if (!std::isfinite(d->params[i])) return fail(c, SDD_ERR_INVALID_ARG, "non-finite parameter");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_nrc(c);
    NrcNet& net = c->nrc;
    net = NrcNet{};
    net.T = 1 << d->table_log2;
    net.n_tab = (long long)kNrcLevels * net.T * kNrcFeat;
    net.n_all = n_all;
    const double b = std::exp((std::log(2048.0) - std::log(16.0)) / (kNrcLevels - 1));
    for (int l = 0; l < kNrcLevels; ++l) {
        const int N = (int)std::floor(16.0 * std::pow(b, (double)l));
        net.res[l] = N;
        net.dense[l] = (long long)(N + 1) * (N + 1) * (N + 1) <= (long long)net.T ? 1 : 0;
    }
    for (int a = 0; a < 3; ++a) {
        net.lo[a] = d->aabb_lo[a];
        net.inv_ext[a] = (float)(1.0 / ((double)d->aabb_hi[a] - (double)d->aabb_lo[a]));
    }
    net.lam_lo = d->lambda_lo;
    net.lam_inv = (float)(1.0 / ((double)d->lambda_hi - (double)d->lambda_lo));
    sh_constants(net.shK);
    sdd_status st;
    if ((st = upload(c, &net.p, d->params, (size_t)n_all)) != SDD_OK || (st = dalloc(c, &net.g, (size_t)n_all)) != SDD_OK ||
        (st = dalloc(c, &net.m, (size_t)n_all)) != SDD_OK || (st = dalloc(c, &net.v, (size_t)n_all)) != SDD_OK ||
        (st = dalloc(c, &net.wq, (size_t)kNrcFragsAll * 8)) != SDD_OK ||
        (st = dalloc(c, &net.wf, (size_t)kNrcFrags32)) != SDD_OK || (st = dalloc(c, &c->nrc_loss, 1)) != SDD_OK ||
        (d->table_fp16 && (st = dalloc(c, &c->nrc_t16, (size_t)(net.n_tab / 2))) != SDD_OK)) {
        free_nrc(c);
        return st;
    }
    hipError_t e = nrc_launch_zero(net.g, n_all, c->stream);
    if (e == hipSuccess) e = nrc_launch_zero(net.m, n_all, c->stream);
    if (e == hipSuccess) e = nrc_launch_zero(net.v, n_all, c->stream);
    if (e == hipSuccess) e = nrc_launch_pack(net, c->stream);
    if (e == hipSuccess && c->nrc_t16) e = nrc_launch_tables_f16(net, c->nrc_t16, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        free_nrc(c);
        return hip_fail(c, e, "nrc init");
    }
    c->nrc_train_paths = d->train_paths;
    c->nrc_train_steps = d->train_steps;
    c->nrc_train_batch = d->train_batch;
    c->nrc_precision = d->precision;
    c->nrc_lr = d->lr;
    c->nrc_b1 = d->beta1;
    c->nrc_b2 = d->beta2;
    c->nrc_eps = d->eps;
    c->nrc_t = 0;
    c->nrc_g_dirty = false;
    c->has_nrc = true;
    return SDD_OK;
}

sdd_status sdd_nrc_infer(sdd_ctx* c, int32_t n, const float* x, const float* w, const float* lam, float* y,
                         int32_t precision) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->has_nrc) return fail(c, SDD_ERR_STATE, "sdd_nrc_infer before sdd_nrc_init");
    HIP_TRY(c, nrc_wait_host(c));  // the Adam steps of the last cache render
    if (n < 0 || (n > 0 && (!x || !w || !lam || !y))) return fail(c, SDD_ERR_INVALID_ARG, "bad rows");
    if (precision != 0 && precision != 1) return fail(c, SDD_ERR_INVALID_ARG, "precision must be 0 or 1");
    if (n == 0) return SDD_OK;
    DeviceGuard g(c->device);
    const hipError_t e = precision == 0 ? nrc_launch_infer(c->nrc, n, x, w, lam, y, c->stream)
                                        : nrc_launch_infer_mfma(qnet(c), n, x, w, lam, y, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "nrc infer");
    return SDD_OK;
}

sdd_status sdd_nrc_train_step(sdd_ctx* c, int32_t n, const float* x, const float* w, const float* lam, const float* t,
                              int32_t apply, float* loss) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->has_nrc) return fail(c, SDD_ERR_STATE, "sdd_nrc_train_step before sdd_nrc_init");
    HIP_TRY(c, nrc_wait_host(c));  // the Adam steps of the last cache render
    if (n < 1 || n > kNrcMaxRows) return fail(c, SDD_ERR_INVALID_ARG, "n out of range");
    if (!x || !w || !lam || !t) return fail(c, SDD_ERR_INVALID_ARG, "null rows");
    DeviceGuard g(c->device);
    sdd_status st = nrc_reserve(c, n);
    if (st != SDD_OK) return st;
    NrcBatch b{n, x, w, lam, t, c->nrc_acts, c->nrc_dz, c->nrc_y, c->nrc_dy, c->nrc_loss};
    hipError_t e = c->nrc_g_dirty ? nrc_launch_zero(c->nrc.g, c->nrc.n_all, c->stream) : hipSuccess;
    if (e == hipSuccess) e = nrc_launch_zero(c->nrc_loss, 1, c->stream);
    if (e == hipSuccess) e = nrc_launch_grad(c->nrc, b, c->stream);
    c->nrc_g_dirty = true;  // this step's gradients stay readable (sdd_nrc_get_params)
    if (e == hipSuccess && apply) {
        e = nrc_launch_adam(c->nrc, c->nrc_t + 1, c->nrc_lr, c->nrc_b1, c->nrc_b2, c->nrc_eps, c->stream);
        if (e == hipSuccess) e = nrc_launch_pack(c->nrc, c->stream);
        if (e == hipSuccess && c->nrc_t16) e = nrc_launch_tables_f16(c->nrc, c->nrc_t16, c->stream);
        if (e == hipSuccess) ++c->nrc_t;
    }
    if (e == hipSuccess && loss) {
        e = hipMemcpyAsync(loss, c->nrc_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "nrc train step");
    return SDD_OK;
}

sdd_status sdd_nrc_query(sdd_ctx* c, int32_t n, const float* x4, const float* n4, float* out, int32_t precision) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->has_nrc) return fail(c, SDD_ERR_STATE, "sdd_nrc_query before sdd_nrc_init");
    HIP_TRY(c, nrc_wait_host(c));  // the Adam steps of the last cache render
    if (!c->has_scene) return fail(c, SDD_ERR_STATE, "sdd_nrc_query before sdd_load_scene (wavelengths)");
    if (n < 0 || (n > 0 && (!x4 || !n4 || !out))) return fail(c, SDD_ERR_INVALID_ARG, "bad arguments");
    if (precision != 0 && precision != 1) return fail(c, SDD_ERR_INVALID_ARG, "precision must be 0 or 1");
    if (n == 0) return SDD_OK;
    DeviceGuard g(c->device);
    if (precision == 1) {
        sdd_status st = nrc_ensure_ops(c, n);
        if (st != SDD_OK) return st;
    }
    const NrcOrder ord = nrc_order(c);
    const hipError_t e = nrc_launch_query(precision == 1 ? qnet(c) : c->nrc, n, reinterpret_cast<const float4*>(x4),
                                          reinterpret_cast<const float4*>(n4), c->d_lam, c->nl, c->nlp, out, 0,
                                          precision, c->nrc_hop, c->nrc_sop, precision == 1 ? &ord : nullptr,
                                          c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "nrc query");
    return SDD_OK;
}

sdd_status sdd_nrc_query_noalloc(sdd_ctx* c, int32_t n, const float* x4, const float* n4, float* out) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->has_nrc) return fail(c, SDD_ERR_STATE, "sdd_nrc_query_noalloc before sdd_nrc_init");
    HIP_TRY(c, nrc_wait_host(c));  // the Adam steps of the last cache render
    if (!c->has_scene) return fail(c, SDD_ERR_STATE, "sdd_nrc_query_noalloc before sdd_load_scene (wavelengths)");
    if (n < 0 || (n > 0 && (!x4 || !n4 || !out))) return fail(c, SDD_ERR_INVALID_ARG, "bad arguments");
    if (n > SDD_NRC_NOALLOC_MAX_PATHS)
        return fail(c, SDD_ERR_INVALID_ARG, "n = " + std::to_string(n) + " exceeds the allocation-free query's limit of " +
                                                std::to_string(SDD_NRC_NOALLOC_MAX_PATHS) + " points");
    if (n == 0) return SDD_OK;
    DeviceGuard g(c->device);
    uint4* hop = nullptr;
    uint2* sop = nullptr;
    NrcOrder ord{};
    if (!nrc_query_scratch_layout(c->noalloc_scratch, kNoAllocScratchBytes, n, &hop, &sop, &ord))
        return fail(c, SDD_ERR_INVALID_ARG, "the query's scratch does not fit the static array");
    const hipError_t e = nrc_launch_query(qnet(c), n, reinterpret_cast<const float4*>(x4),
                                          reinterpret_cast<const float4*>(n4), c->d_lam, c->nl, c->nlp, out, 0, 1, hop,
                                          sop, &ord, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "nrc query (allocation-free)");
    return SDD_OK;
}

sdd_status sdd_nrc_last_rows(sdd_ctx* c, int32_t max_rows, float* rows, int32_t* n_rows, int32_t* n_steps,
                             float* loss) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->has_nrc) return fail(c, SDD_ERR_STATE, "sdd_nrc_last_rows before sdd_nrc_init");
    HIP_TRY(c, nrc_wait_host(c));  // the Adam steps of the last cache render
    if (max_rows < 0 || (max_rows > 0 && !rows)) return fail(c, SDD_ERR_INVALID_ARG, "bad arguments");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (n_rows) *n_rows = (int32_t)c->nrc_last_rows;
    if (n_steps) *n_steps = c->nrc_last_steps;
    if (loss) *loss = c->nrc_last_loss;
    const long long m = std::min<long long>(max_rows, c->nrc_last_rows);
    if (m > 0) {
        HIP_TRY(c, hipMemcpyAsync(rows, c->nrc_crows, sizeof(float4) * 2 * (size_t)m, hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return SDD_OK;
}

sdd_status sdd_nrc_get_params(sdd_ctx* c, int32_t which, float* out) {
    if (!c) return SDD_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->has_nrc) return fail(c, SDD_ERR_STATE, "sdd_nrc_get_params before sdd_nrc_init");
    HIP_TRY(c, nrc_wait_host(c));  // the Adam steps of the last cache render
    if (which < 0 || which > 3 || !out) return fail(c, SDD_ERR_INVALID_ARG, "bad arguments");
    DeviceGuard g(c->device);
    const float* src = which == 0 ? c->nrc.p : which == 1 ? c->nrc.g : which == 2 ? c->nrc.m : c->nrc.v;
    HIP_TRY(c, hipMemcpyAsync(out, src, sizeof(float) * (size_t)c->nrc.n_all, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SDD_OK;
}

}  // extern "C"
