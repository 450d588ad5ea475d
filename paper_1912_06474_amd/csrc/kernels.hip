// HIP kernels (gfx950) of the spectral domain-decomposition path tracer.
//
//   k_camgen  primary rays (Sec. 4: one ray per pixel sample), entry cell,
//             append to the per-subdomain extension queues
//   k_trace   one sweep over all non-empty subdomain queues: traverse the
//             cell's BVH over (t_enter, t_exit]; a closest-hit ray that finds
//             nothing (or a shadow ray that is neither blocked nor finished)
//             is handed to the neighbouring cell's queue with its origin,
//             direction and t carried unchanged (Sec. 5, interface condition:
//             continuity of the ray properties)
//   k_shade   per-wavelength interaction at each hit (Eq. 1-3, Sec. 4, 6),
//             shadow ray toward the light, next ray of the path
//   k_flush   per-pixel FP32 accumulation of finished path samples
//   k_resolve FP64 per-pixel mean and spectral -> XYZ reduction
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "kernels.h"
#include "layout.h"

namespace sdd {

// ---------------------------------------------------------------------------
// subdomain grid: point location, entry, exit
// ---------------------------------------------------------------------------
__device__ __forceinline__ int locate_axis(const float* pl, int n, float lo, float inv_h, float x) {
    int i = (int)floorf((x - lo) * inv_h);
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    if (i > 0 && x < pl[i]) --i;
    else if (i < n - 1 && x >= pl[i + 1]) ++i;
    return i;
}

// First cell of a ray and the exclusive lower bound of its parameter range:
// the cell holding the origin (t_enter = 0), or, for an origin outside the
// grid, the cell where the ray enters it.  Returns -1 if it never does.
__device__ __forceinline__ int locate_ray(const GridParams& g, f3 o, f3 d, float& t_enter) {
    const float oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) inside = inside && oo[a] >= g.lo[a] && oo[a] <= g.hi[a];
    float p[3] = {o.x, o.y, o.z};
    t_enter = 0.0f;
    if (!inside) {
        float t0 = 0.0f, t1 = INFINITY;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (dd[a] == 0.0f) {
                if (oo[a] < g.lo[a] || oo[a] > g.hi[a]) return -1;
                continue;
            }
            float ta = (g.lo[a] - oo[a]) / dd[a], tb = (g.hi[a] - oo[a]) / dd[a];
            if (ta > tb) {
                const float t = ta;
                ta = tb;
                tb = t;
            }
            t0 = fmaxf(t0, ta);
            t1 = fminf(t1, tb);
        }
        if (t0 > t1) return -1;
        t_enter = t0;
#pragma unroll
        for (int a = 0; a < 3; ++a) p[a] = fminf(fmaxf(oo[a] + t0 * dd[a], g.lo[a]), g.hi[a]);
    }
    const int ix = locate_axis(g.planes, g.nx, g.lo[0], g.inv_h[0], p[0]);
    const int iy = locate_axis(g.planes + g.off_y, g.ny, g.lo[1], g.inv_h[1], p[1]);
    const int iz = locate_axis(g.planes + g.off_z, g.nz, g.lo[2], g.inv_h[2], p[2]);
    return ix + g.nx * (iy + g.ny * iz);
}

// ---------------------------------------------------------------------------
// camera rays
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_camgen(CamParams P) {
    __shared__ int s_cnt[kMaxCells], s_base[kMaxCells];
    const int pid = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = pid < P.N;
    bool enq = false;
    int cell = 0;
    f3 o{0, 0, 0}, d{0, 0, 1};
    float t_enter = 0.0f;
    if (valid) {
        const long long g = P.g0 + pid;
        const int s = P.s0 + (int)(g / P.WH);
        const int p = (int)(g % P.WH);
        const int px = p % P.W, py = p / P.W;
        const uint4 r = philox4x32_10(make_uint4((uint32_t)p, (uint32_t)s, 0u, 0u), P.key);
        const float x = (float)px + u01(r.x), y = (float)py + u01(r.y);
        const float sx = 2.0f * x / (float)P.W - 1.0f, sy = 1.0f - 2.0f * y / (float)P.H;
        const f3 eye{P.eye[0], P.eye[1], P.eye[2]}, fw{P.fwd[0], P.fwd[1], P.fwd[2]};
        const f3 rt{P.right[0], P.right[1], P.right[2]}, up{P.up[0], P.up[1], P.up[2]};
        if (P.ortho) {
            o = eye + rt * (sx * P.ortho_half_h * P.aspect) + up * (sy * P.ortho_half_h);
            d = fw;
        } else {
            o = eye;
            d = unit3(fw + rt * (sx * P.tan_half * P.aspect) + up * (sy * P.tan_half));
        }
        P.ray_o[pid] = make_float4(o.x, o.y, o.z, 0.0f);
        P.ray_d[pid] = make_float4(d.x, d.y, d.z, 0.0f);
        P.hit[pid] = make_float2(INFINITY, __int_as_float(-1));
        P.flags[pid] = kAlive | kCountE;
        P.sh_state[pid] = kShNone;
        for (int l = 0; l < P.nlp; ++l) {
            P.beta[(size_t)l * P.N + pid] = 1.0f;
            P.Lp[(size_t)l * P.N + pid] = 0.0f;
        }
        cell = locate_ray(P.grid, o, d, t_enter);
        enq = cell >= 0;
    }
    const int slot = block_append(enq, cell, P.ecnt, P.n_cells, s_cnt, s_base);
    if (enq && slot < P.cap) {
        const long long q = (long long)cell * P.cap + slot;
        P.eqa[q] = make_float4(o.x, o.y, o.z, t_enter);
        P.eqb[q] = make_float4(d.x, d.y, d.z, __int_as_float(pid));
        P.eqc[q] = make_int2(-1, __float_as_int(INFINITY));
    }
    const uint64_t m = __ballot(valid);
    if (lane_id() == 0 && m) atomicAdd(&P.stats[kStatExtRays], (unsigned long long)popc64(m));
}

// ---------------------------------------------------------------------------
// traversal of one subdomain (cell) BVH
// ---------------------------------------------------------------------------
struct RayTrav {
    f3 o, d, inv, oinv;
};

__device__ __forceinline__ RayTrav make_trav(f3 o, f3 d) {
    RayTrav r;
    r.o = o;
    r.d = d;
    const float dx = fabsf(d.x) > 1e-20f ? d.x : copysignf(1e-20f, d.x);
    const float dy = fabsf(d.y) > 1e-20f ? d.y : copysignf(1e-20f, d.y);
    const float dz = fabsf(d.z) > 1e-20f ? d.z : copysignf(1e-20f, d.z);
    r.inv = f3{1.0f / dx, 1.0f / dy, 1.0f / dz};
    r.oinv = f3{o.x * r.inv.x, o.y * r.inv.y, o.z * r.inv.z};
    return r;
}

// slab test of one box against [tlo, thi]; returns the entry t (or +inf on a miss)
__device__ __forceinline__ float box_enter(const RayTrav& r, float lox, float hix, float loy, float hiy, float loz,
                                           float hiz, float tlo, float thi) {
    const float ax = fmaf(lox, r.inv.x, -r.oinv.x), bx = fmaf(hix, r.inv.x, -r.oinv.x);
    const float ay = fmaf(loy, r.inv.y, -r.oinv.y), by = fmaf(hiy, r.inv.y, -r.oinv.y);
    const float az = fmaf(loz, r.inv.z, -r.oinv.z), bz = fmaf(hiz, r.inv.z, -r.oinv.z);
    const float tmin = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), tlo));
    const float tmax = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), thi));
    return tmin <= tmax ? tmin : INFINITY;
}

// Moller-Trumbore with inclusive barycentrics; returns false for a parallel
// ray or a miss, else t (may be <= 0: the caller checks the interval).
__device__ __forceinline__ bool tri_test(const RayTrav& r, float4 a, float4 b, float4 c, float& t) {
    const f3 v0 = xyz(a), e1 = xyz(b), e2 = xyz(c);
    const f3 p = cross3(r.d, e2);
    const float det = dot3(e1, p);
    if (det == 0.0f) return false;
    const float idet = 1.0f / det;
    const f3 s = r.o - v0;
    const float u = dot3(s, p) * idet;
    if (!(u >= 0.0f && u <= 1.0f)) return false;
    const f3 q = cross3(s, e1);
    const float v = dot3(r.d, q) * idet;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    t = dot3(e2, q) * idet;
    return true;
}

template <bool SHADOW, bool COUNT>
__device__ __forceinline__ void traverse(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                         const float4* __restrict__ prim_info, int root, const RayTrav& r,
                                         float tlo, float t_exit, float t_max, int exclude, float& thi, int& best,
                                         bool& blocked, int& n_glass, int pid, int* __restrict__ sh_cnt,
                                         float2* __restrict__ sh_glass, int* overflow, int* stk, int* gstk,
                                         int gstride, int& n_nodes, int& n_tris) {
    int sp = 0;
    int link = root;
    // closest hit: thi = t_exit, best = -1 on entry; shadow: thi = min(t_exit, t_max)
    for (;;) {
        if (link >= 0) {
            const float4* nd = nodes + 4 * (size_t)link;
            const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2];
            const int4 n3 = *reinterpret_cast<const int4*>(nd + 3);
            if (COUNT) ++n_nodes;
            const float t0 = box_enter(r, n0.x, n0.y, n0.z, n0.w, n2.x, n2.y, tlo, thi);
            const float t1 = box_enter(r, n1.x, n1.y, n1.z, n1.w, n2.z, n2.w, tlo, thi);
            const bool h0 = t0 != INFINITY, h1 = t1 != INFINITY;
            if (h0 && h1) {
                const bool first0 = t0 <= t1;
                // short stack in LDS, deeper entries in HBM; the builder caps the
                // BVH depth below kStack, so no entry is ever dropped
                const int far = first0 ? n3.y : n3.x;
                if (sp < kLdsStack) stk[sp * kTraceBlock] = far;
                else if (sp < kStack) gstk[(sp - kLdsStack) * gstride] = far;
                ++sp;
                link = first0 ? n3.x : n3.y;
                continue;
            }
            if (h0) {
                link = n3.x;
                continue;
            }
            if (h1) {
                link = n3.y;
                continue;
            }
        } else {
            int ti = ~link;
            for (;;) {
                const float4 a = tris[3 * (size_t)ti], b = tris[3 * (size_t)ti + 1], c = tris[3 * (size_t)ti + 2];
                const int prim = __float_as_int(a.w);
                const int meta = __float_as_int(b.w);
                const int typ = meta & 3;
                if (prim != exclude && !(SHADOW && typ == kEmitter)) {
                    if (COUNT) ++n_tris;
                    float t;
                    if (tri_test(r, a, b, c, t)) {
                        if (!SHADOW) {
                            if (t > tlo && (t < thi || (t == thi && (best < 0 || prim < best)))) {
                                thi = t;
                                best = prim;
                            }
                        } else if (t > tlo && t <= t_exit && t < t_max) {
                            if (typ == kDiffuse) {
                                blocked = true;
                                return;
                            }
                            const f3 ng = xyz(prim_info[prim]);
                            if (n_glass < 0) n_glass = sh_cnt[pid];
                            if (n_glass < kMaxGlass)
                                sh_glass[(size_t)pid * kMaxGlass + n_glass] = make_float2(fabsf(dot3(r.d, ng)), c.w);
                            else
                                atomicExch(overflow, 1);
                            ++n_glass;
                        }
                    }
                }
                if (meta & kLastInLeaf) break;
                ++ti;
            }
        }
        if (sp == 0) break;
        --sp;
        if (sp >= kStack) break;
        link = sp < kLdsStack ? stk[sp * kTraceBlock] : gstk[(sp - kLdsStack) * gstride];
    }
}

// One chunk (up to 64 rays of one cell's queue, one wave): traverse the
// cell's BVH over (t_enter, t_exit] and hand the rays that go on to the
// neighbouring cell's queue.  Reached by all lanes of the wave together.
template <bool SHADOW, bool COUNT>
__device__ __forceinline__ void process_chunk(const TraceParams& P, const QueueSet& Q, int cell, int idx, bool active,
                                              int* stk, int* gstk, int gstride, int& n_visits, int& n_nodes,
                                              int& n_tris) {
    const GridParams& g = P.grid;
    const int ix = cell % g.nx, iy = (cell / g.nx) % g.ny, iz = cell / (g.nx * g.ny);
    const float px0 = g.planes[ix], px1 = g.planes[ix + 1];
    const float py0 = g.planes[g.off_y + iy], py1 = g.planes[g.off_y + iy + 1];
    const float pz0 = g.planes[g.off_z + iz], pz1 = g.planes[g.off_z + iz + 1];
    const int root = P.cell_root[cell];

    bool cont = false;
    int next = 0;
    float4 qa = make_float4(0, 0, 0, 0), qb = make_float4(0, 0, 0, 0);
    int2 qc = make_int2(0, 0);
    if (active) {
        ++n_visits;
        const long long q = (long long)cell * P.cap + idx;
        qa = Q.qa_in[q];
        qb = Q.qb_in[q];
        qc = Q.qc_in[q];
        const f3 o = xyz(qa), d = xyz(qb);
        const int pid = __float_as_int(qb.w);
        const float t_enter = qa.w;
        const float t_max = __int_as_float(qc.y);
        // exit of this cell: nearest far plane, ties x < y < z
        const float tx = d.x > 0.0f ? (px1 - o.x) / d.x : (d.x < 0.0f ? (px0 - o.x) / d.x : INFINITY);
        const float ty = d.y > 0.0f ? (py1 - o.y) / d.y : (d.y < 0.0f ? (py0 - o.y) / d.y : INFINITY);
        const float tz = d.z > 0.0f ? (pz1 - o.z) / d.z : (d.z < 0.0f ? (pz0 - o.z) / d.z : INFINITY);
        int axis = 0;
        float t_exit = tx;
        if (ty < t_exit) {
            t_exit = ty;
            axis = 1;
        }
        if (tz < t_exit) {
            t_exit = tz;
            axis = 2;
        }
        const RayTrav r = make_trav(o, d);
        float thi = SHADOW ? fminf(t_exit, t_max) : t_exit;
        int best = -1;
        bool blocked = false;
        int n_glass = -1;  // pane crossings so far (-1: not loaded yet)
        if (!SHADOW || thi > t_enter)
            traverse<SHADOW, COUNT>(P.nodes, P.tris, P.prim_info, root, r, t_enter, t_exit, t_max, qc.x, thi, best,
                                    blocked, n_glass, pid, P.sh_cnt, P.sh_glass, P.overflow, stk, gstk, gstride,
                                    n_nodes, n_tris);
        bool leave;
        if (!SHADOW) {
            if (best >= 0) P.hit[pid] = make_float2(thi, __int_as_float(best));
            leave = best < 0;
        } else {
            if (blocked) P.sh_state[pid] = kShBlocked;
            else if (n_glass >= 0) P.sh_cnt[pid] = n_glass;
            leave = !blocked && t_exit < t_max;
        }
        if (leave) {
            int nx = ix, ny = iy, nz = iz;
            if (axis == 0) nx += d.x > 0.0f ? 1 : -1;
            else if (axis == 1) ny += d.y > 0.0f ? 1 : -1;
            else nz += d.z > 0.0f ? 1 : -1;
            if (nx >= 0 && nx < g.nx && ny >= 0 && ny < g.ny && nz >= 0 && nz < g.nz) {
                cont = true;
                next = nx + g.nx * (ny + g.ny * nz);
                qa.w = t_exit;  // carried bit-exactly into the neighbour
            }
        }
    }
    const int slot = wave_append(cont, next, Q.cnt_out);
    if (cont && slot < P.cap) {
        const long long q = (long long)next * P.cap + slot;
        Q.qa_out[q] = qa;
        Q.qb_out[q] = qb;
        Q.qc_out[q] = qc;
    }
}

// One sweep over all subdomain queues of both ray kinds (closest-hit rays of
// one depth and shadow rays of the previous one are independent, so they
// share the sweep).  Work is split into 64-ray chunks ordered by (cell, kind);
// the chunk range is cut into kXcd contiguous parts, part x served by the
// workgroups of XCD x (consecutive cells share that XCD's L2).
template <bool COUNT>
__global__ __launch_bounds__(kTraceBlock) void k_trace(TraceParams P) {
    __shared__ int s_pref[2 * kMaxCells + 1];
    __shared__ int s_stack[kLdsStack * kTraceBlock];
    const int G = P.n_cells;
    const int E = 2 * G;  // entry e = 2 * cell + kind
    if (threadIdx.x < 64) {
        // exclusive prefix of the per-entry chunk counts (wave 0, lane-blocked scan)
        const int ln = threadIdx.x;
        const int per = (E + 63) / 64;
        const int c0 = ln * per, c1 = min(c0 + per, E);
        int local = 0;
        for (int e = c0; e < c1; ++e) {
            const int kind = e & 1;
            const int n = P.active[kind] ? P.q[kind].cnt_in[e >> 1] : 0;
            if (n > P.cap) atomicExch(P.overflow, 2);  // never expected: counters are bounded by cap
            local += (n + kChunk - 1) / kChunk;
        }
        int incl = local;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (ln >= o) incl += v;
        }
        int run = incl - local;
        for (int e = c0; e < c1; ++e) {
            s_pref[e] = run;
            const int kind = e & 1;
            const int n = P.active[kind] ? P.q[kind].cnt_in[e >> 1] : 0;
            run += (n + kChunk - 1) / kChunk;
        }
        if (ln == 63) s_pref[E] = incl;
    }
    __syncthreads();
    const int total = s_pref[E];
    if (total == 0) return;
    const int lane = lane_id();
    int* stk = s_stack + threadIdx.x;
    const int gstride = gridDim.x * kTraceBlock;  // entries of one level are contiguous over the grid
    int* gstk = P.gstack + blockIdx.x * kTraceBlock + threadIdx.x;
    const int xcd = blockIdx.x % kXcd;
    int n_nodes = 0, n_tris = 0, n_vis[2] = {0, 0};

    // static XCD-aware striding: the waves of XCD x walk part x of the chunk
    // list round-robin (no atomics, so empty and near-empty sweeps cost only
    // the prologue)
    constexpr int kWavesPerBlock = kTraceBlock / 64;
    const int lw = (blockIdx.x / kXcd) * kWavesPerBlock + (int)(threadIdx.x / 64);
    const int nwx = (gridDim.x / kXcd) * kWavesPerBlock;
    const int lo = (int)((long long)total * xcd / kXcd);
    const int hi = (int)((long long)total * (xcd + 1) / kXcd);
    for (int chunk = lo + lw; chunk < hi; chunk += nwx) {
        int a = 0, b = E;
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if (s_pref[m] <= chunk) a = m;
            else b = m;
        }
        const int e = __builtin_amdgcn_readfirstlane(a);
        const int cell = e >> 1, kind = e & 1;
        const int idx = (chunk - s_pref[e]) * kChunk + lane;
        const bool active = idx < min((long long)P.q[kind].cnt_in[cell], P.cap);
        if (kind == 0)
            process_chunk<false, COUNT>(P, P.q[0], cell, idx, active, stk, gstk, gstride, n_vis[0], n_nodes,
                                        n_tris);
        else
            process_chunk<true, COUNT>(P, P.q[1], cell, idx, active, stk, gstk, gstride, n_vis[1], n_nodes,
                                       n_tris);
    }
    const int v0 = wave_sum(n_vis[0]), v1 = wave_sum(n_vis[1]);
    if (lane == 0) {
        if (v0) atomicAdd(&P.stats[kStatExtVisits], (unsigned long long)v0);
        if (v1) atomicAdd(&P.stats[kStatShadowVisits], (unsigned long long)v1);
    }
    if (COUNT) {
        const int nn = wave_sum(n_nodes), nt = wave_sum(n_tris);
        if (lane == 0) {
            atomicAdd(&P.stats[kStatNodes], (unsigned long long)nn);
            atomicAdd(&P.stats[kStatTris], (unsigned long long)nt);
        }
    }
}

// ---------------------------------------------------------------------------
// shading: per-wavelength interaction, shadow ray, next ray
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kShadeBlock) void k_shade(ShadeParams P) {
    __shared__ int s_cnt[kMaxCells], s_base[kMaxCells];
    const int pid = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = pid < P.N;
    const int N = P.N;
    bool enq_e = false, enq_s = false;
    int cell_e = 0, cell_s = 0;
    f3 xo{0, 0, 0}, dn{0, 0, 1}, ws{0, 0, 1};
    float te = 0.0f, ts = 0.0f, r_sh = 0.0f;
    int prim = -1;
    if (valid) {
        const long long g = P.g0 + pid;
        const int s = P.s0 + (int)(g / P.WH);
        const int p = (int)(g % P.WH);
        const long long log_base = ((long long)p * P.spp_call + (s - P.s0)) * P.max_depth;

        // 1) resolve the shadow ray of the previous vertex
        const int sh = P.sh_state[pid];
        if (sh != kShNone) {
            const bool vis = sh == kShVisible;
            if (P.shadow_log) P.shadow_log[log_base + P.depth - 2] = vis ? 1 : 0;
            if (vis) {
                const float gfac = P.nee_g[pid];
                const int ng = min(P.sh_cnt[pid], kMaxGlass);
                float2 gl[kMaxGlass];
                for (int j = 0; j < ng; ++j) gl[j] = P.sh_glass[(size_t)pid * kMaxGlass + j];
                const float* leL = P.le + (size_t)P.light_mat * P.nlp;
                for (int l = 0; l < P.nl; ++l) {
                    float tr = 1.0f;
                    for (int j = 0; j < ng; ++j) {
                        const int m = __float_as_int(gl[j].y);
                        float Rg, Tg;
                        pane_RT(P.mn[(size_t)m * P.nlp + l], P.mk[(size_t)m * P.nlp + l], P.mat_thick[m],
                                P.lambda_nm[l], gl[j].x, Rg, Tg);
                        tr *= Tg;
                    }
                    P.Lp[(size_t)l * N + pid] += P.beta[(size_t)l * N + pid] * leL[l] * gfac * tr;
                }
            }
            P.sh_state[pid] = kShNone;
        }
        uint32_t fl = P.flags[pid];
        if (!P.final_pass && (fl & kAlive)) {
            const float2 h = P.hit[pid];
            prim = __float_as_int(h.y);
            if (P.hit_log) P.hit_log[log_base + P.depth - 1] = prim;
            if (prim < 0) {
                fl = 0;
            } else {
                const f3 o = xyz(P.ray_o[pid]), d = xyz(P.ray_d[pid]);
                const f3 x = o + d * h.x;
                const float4 pi = P.prim_info[prim];
                const f3 ngm = xyz(pi);
                const int m = __float_as_int(pi.w);
                const float cos_o = -dot3(ngm, d);
                const f3 n = cos_o > 0.0f ? ngm : -ngm;
                const int typ = P.mat_type[m];
                const float* le = P.le + (size_t)m * P.nlp;
                if (typ == kEmitter) {
                    if ((fl & kCountE) && cos_o > 0.0f)
                        for (int l = 0; l < P.nl; ++l) P.Lp[(size_t)l * N + pid] += P.beta[(size_t)l * N + pid] * le[l];
                    fl = 0;
                } else if (typ == kDiffuse) {
                    const float* rho = P.rho + (size_t)m * P.nlp;
                    const bool emit = P.mat_has_le[m] != 0;
                    for (int l = 0; l < P.nl; ++l) {
                        const size_t i = (size_t)l * N + pid;
                        const float b = P.beta[i];
                        if (emit) P.Lp[i] += b * le[l];
                        P.beta[i] = b * rho[l];
                    }
                    const uint4 ub = philox4x32_10(make_uint4((uint32_t)p, (uint32_t)s, (uint32_t)P.depth, 0u), P.key);
                    xo = x + n * kOffset;
                    if (P.light_type != 0) {
                        f3 y{P.lp0[0], P.lp0[1], P.lp0[2]};
                        if (P.light_type == 1)
                            y = y + f3{P.le1[0], P.le1[1], P.le1[2]} * u01(ub.x) + f3{P.le2[0], P.le2[1], P.le2[2]} * u01(ub.y);
                        const f3 w = y - xo;
                        const float r2 = dot3(w, w);
                        const float r = sqrtf(r2);
                        const f3 om = w * (1.0f / r);
                        const float cx = dot3(n, om);
                        const float cy = P.light_type == 1 ? -dot3(f3{P.nL[0], P.nL[1], P.nL[2]}, om) : 1.0f;
                        if (cx > 0.0f && cy > 0.0f) {
                            // (rho/pi) Le cos_x cos_y / r^2 * A (area light); (rho/pi) I cos_x / r^2 (Eq. 3)
                            const float gfac =
                                (P.light_type == 1 ? cx * cy / r2 * P.light_area : cx / r2) * (1.0f / kPi);
                            P.nee_g[pid] = gfac;
                            P.sh_state[pid] = kShVisible;
                            P.sh_cnt[pid] = 0;
                            ws = om;
                            r_sh = r;
                            cell_s = locate_ray(P.grid, xo, ws, ts);
                            enq_s = cell_s >= 0;
                        }
                    }
                    fl &= ~kCountE;
                    if (P.depth == P.max_depth) {
                        fl = 0;
                    } else {
                        const uint4 uc =
                            philox4x32_10(make_uint4((uint32_t)p, (uint32_t)s, (uint32_t)P.depth, 1u), P.key);
                        dn = cosine_dir(n, u01(uc.x), u01(uc.y));
                        enq_e = true;
                    }
                } else {  // glass pane
                    const float c = fabsf(dot3(d, ngm));
                    const float thick = P.mat_thick[m];
                    float sumR = 0.0f, sumT = 0.0f;
                    for (int l = 0; l < P.nl; ++l) {
                        float Rl, Tl;
                        pane_RT(P.mn[(size_t)m * P.nlp + l], P.mk[(size_t)m * P.nlp + l], thick, P.lambda_nm[l], c, Rl,
                                Tl);
                        sumR += Rl;
                        sumT += Tl;
                    }
                    if (!(sumR + sumT > 0.0f) || P.depth == P.max_depth) {
                        fl = 0;
                    } else {
                        const float PR = sumR / (sumR + sumT);
                        const uint4 ub =
                            philox4x32_10(make_uint4((uint32_t)p, (uint32_t)s, (uint32_t)P.depth, 0u), P.key);
                        const bool refl = u01(ub.z) < PR;
                        const float wgt = refl ? 1.0f / PR : 1.0f / (1.0f - PR);
                        for (int l = 0; l < P.nl; ++l) {
                            float Rl, Tl;
                            pane_RT(P.mn[(size_t)m * P.nlp + l], P.mk[(size_t)m * P.nlp + l], thick, P.lambda_nm[l], c,
                                    Rl, Tl);
                            const size_t i = (size_t)l * N + pid;
                            P.beta[i] = P.beta[i] * ((refl ? Rl : Tl) * wgt);
                        }
                        if (refl) {
                            dn = d - ngm * (2.0f * dot3(d, ngm));
                            fl |= kCountE;
                            xo = x + n * kOffset;
                        } else {
                            dn = d;
                            xo = x - n * kOffset;
                        }
                        enq_e = true;
                    }
                }
            }
            if (enq_e) {
                P.ray_o[pid] = make_float4(xo.x, xo.y, xo.z, 0.0f);
                P.ray_d[pid] = make_float4(dn.x, dn.y, dn.z, 0.0f);
                P.hit[pid] = make_float2(INFINITY, __int_as_float(-1));
                cell_e = locate_ray(P.grid, xo, dn, te);
                // a ray that never enters the grid keeps its miss record
                enq_e = cell_e >= 0;
            }
            P.flags[pid] = fl;
        }
    }
    const int slot_e = block_append(enq_e, cell_e, P.ecnt, P.n_cells, s_cnt, s_base);
    if (enq_e && slot_e < P.cap) {
        const long long q = (long long)cell_e * P.cap + slot_e;
        P.eqa[q] = make_float4(xo.x, xo.y, xo.z, te);
        P.eqb[q] = make_float4(dn.x, dn.y, dn.z, __int_as_float(pid));
        P.eqc[q] = make_int2(prim, __float_as_int(INFINITY));
    }
    const int slot_s = block_append(enq_s, cell_s, P.scnt, P.n_cells, s_cnt, s_base);
    if (enq_s && slot_s < P.cap) {
        const long long q = (long long)cell_s * P.cap + slot_s;
        P.sqa[q] = make_float4(xo.x, xo.y, xo.z, ts);
        P.sqb[q] = make_float4(ws.x, ws.y, ws.z, __int_as_float(pid));
        P.sqc[q] = make_int2(prim, __float_as_int(r_sh));
    }
    const uint64_t me = __ballot(enq_e), ms = __ballot(enq_s);
    if (lane_id() == 0) {
        if (me) atomicAdd(&P.stats[kStatExtRays], (unsigned long long)popc64(me));
        if (ms) atomicAdd(&P.stats[kStatShadowRays], (unsigned long long)popc64(ms));
    }
}

// ---------------------------------------------------------------------------
// accumulation and resolve
// ---------------------------------------------------------------------------
// acc[l][p] += path radiance of every sample of pixel p in the batch, in
// increasing sample order (deterministic).
__global__ void k_flush(int N, long long g0, int WH, int nl, const float* __restrict__ Lp, float* __restrict__ acc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int npix = N < WH ? N : WH;
    if (i >= npix) return;
    const long long g = g0 + i;
    const int p = (int)(g % WH);
    for (int l = 0; l < nl; ++l) {
        float a = acc[(size_t)l * WH + p];
        for (long long gg = g; gg < g0 + N; gg += WH) a += Lp[(size_t)l * N + (size_t)(gg - g0)];
        acc[(size_t)l * WH + p] = a;
    }
}

// FP64: mean over samples and XYZ = sum_l w_l cmf_l L_l
__global__ void k_resolve(int WH, int nl, double inv_spp, const float* __restrict__ acc, const double* __restrict__ w,
                          const double* __restrict__ cmf, double* spectral, double* xyz) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= WH) return;
    double X = 0.0, Y = 0.0, Z = 0.0;
    for (int l = 0; l < nl; ++l) {
        const double v = (double)acc[(size_t)l * WH + p] * inv_spp;
        if (spectral) spectral[(size_t)p * nl + l] = v;
        X += w[l] * cmf[3 * l] * v;
        Y += w[l] * cmf[3 * l + 1] * v;
        Z += w[l] * cmf[3 * l + 2] * v;
    }
    if (xyz) {
        xyz[3 * (size_t)p] = X;
        xyz[3 * (size_t)p + 1] = Y;
        xyz[3 * (size_t)p + 2] = Z;
    }
}

__global__ void k_fill_i32(int* p, long long n, int v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_philox(int n, const uint4* ctr, uint2 key, uint4* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox4x32_10(ctr[i], key);
}

// rays for sdd_debug_trace_rays: locate + enqueue, hit initialised to a miss
__global__ void k_debug_rays(int n, const float* o, const float* d, GridParams grid, float2* hit, float4* qa, float4* qb,
                             int2* qc, int* cnt, long long cap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    int cell = 0;
    float te = 0.0f;
    f3 oo{0, 0, 0}, dd{0, 0, 1};
    if (valid) {
        oo = f3{o[3 * i], o[3 * i + 1], o[3 * i + 2]};
        dd = f3{d[3 * i], d[3 * i + 1], d[3 * i + 2]};
        hit[i] = make_float2(INFINITY, __int_as_float(-1));
        cell = locate_ray(grid, oo, dd, te);
    }
    const bool enq = valid && cell >= 0;
    const int slot = wave_append(enq, cell, cnt);
    if (enq && slot < cap) {
        const long long q = (long long)cell * cap + slot;
        qa[q] = make_float4(oo.x, oo.y, oo.z, te);
        qb[q] = make_float4(dd.x, dd.y, dd.z, __int_as_float(i));
        qc[q] = make_int2(-1, __float_as_int(INFINITY));
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_camgen(const CamParams& p, hipStream_t st) {
    if (p.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_camgen, dim3(blocks_for(p.N, 256)), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceParams& p, bool count, int grid_blocks, hipStream_t st) {
    if (count) hipLaunchKernelGGL((k_trace<true>), dim3(grid_blocks), dim3(kTraceBlock), 0, st, p);
    else hipLaunchKernelGGL((k_trace<false>), dim3(grid_blocks), dim3(kTraceBlock), 0, st, p);
    return hipGetLastError();
}

int trace_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<false>, kTraceBlock, 0) != hipSuccess) return 4;
    return nb > 0 ? nb : 1;
}

hipError_t launch_shade(const ShadeParams& p, hipStream_t st) {
    if (p.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_shade, dim3(blocks_for(p.N, kShadeBlock)), dim3(kShadeBlock), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_flush(int N, long long g0, int WH, int nl, const float* Lp, float* acc, hipStream_t st) {
    const int npix = N < WH ? N : WH;
    if (npix <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flush, dim3(blocks_for(npix, 256)), dim3(256), 0, st, N, g0, WH, nl, Lp, acc);
    return hipGetLastError();
}

hipError_t launch_resolve(int WH, int nl, double inv_spp, const float* acc, const double* w, const double* cmf,
                          double* spectral, double* xyz, hipStream_t st) {
    hipLaunchKernelGGL(k_resolve, dim3(blocks_for(WH, 256)), dim3(256), 0, st, WH, nl, inv_spp, acc, w, cmf, spectral,
                       xyz);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_philox(int n, const uint4* ctr, uint2 key, uint4* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, ctr, key, out);
    return hipGetLastError();
}

hipError_t launch_debug_rays(int n, const float* o, const float* d, const GridParams& grid, float2* hit, float4* qa,
                             float4* qb, int2* qc, int* cnt, long long cap, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_rays, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, o, d, grid, hit, qa, qb, qc, cnt,
                       cap);
    return hipGetLastError();
}

}  // namespace sdd
