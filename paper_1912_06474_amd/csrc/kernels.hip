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
//   k_shade   the geometric interaction at each hit (Sec. 4, Eq. 3): shadow
//             ray toward the light, glass branch choice, next ray; one record
//             per vertex
//   k_spectral per-wavelength replay of the vertex records (Eq. 1-3, Sec. 6
//             pane terms) and per-pixel FP32 accumulation
//   k_resolve FP64 per-pixel mean and spectral -> XYZ reduction
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "kernels.h"
#include "layout.h"

namespace sdd {

// ---------------------------------------------------------------------------
// glass terms: uncoated slab or coated pane, by the sign convention of the
// stored cosine cs (> 0: the light arrives on the face the geometric normal
// points out of, where a coating lies)
// ---------------------------------------------------------------------------
// COATED: the scene has coated glass (kernels are instantiated both ways, so
// scenes without coatings keep the small uncoated code)
template <bool COATED>
__device__ __forceinline__ void glass_RT(const float4* pane, const float4* coat, const int* coat_n, int coat_layers,
                                         int nlp, int g, int l, float cs, float& R, float& T) {
    const float4 pc = pane[(size_t)g * nlp + l];
    const int L = COATED ? coat_n[g] : 0;
    if (!COATED || L <= 0) pane_RT(pc, fabsf(cs), R, T);
    else coated_RT(pc, coat + (size_t)g * coat_layers * nlp + l, min(L, coat_layers), nlp, fabsf(cs), cs > 0.0f, R, T);
}

// four consecutive wavelengths l0 .. l0 + 3 (no indexed arrays, so nothing
// leaves registers)
template <bool COATED>
__device__ __forceinline__ void glass_RT4(const float4* pane, const float4* coat, const int* coat_n, int coat_layers,
                                          int nlp, int g, int l0, float cs, float4& R, float4& T) {
    glass_RT<COATED>(pane, coat, coat_n, coat_layers, nlp, g, l0 + 0, cs, R.x, T.x);
    glass_RT<COATED>(pane, coat, coat_n, coat_layers, nlp, g, l0 + 1, cs, R.y, T.y);
    glass_RT<COATED>(pane, coat, coat_n, coat_layers, nlp, g, l0 + 2, cs, R.z, T.z);
    glass_RT<COATED>(pane, coat, coat_n, coat_layers, nlp, g, l0 + 3, cs, R.w, T.w);
}

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
__global__ __launch_bounds__(kShadeBlock) void k_camgen(CamParams P) {
    __shared__ int s_wcnt[(kShadeBlock / 64) * kMaxCells];
    const int lpid = blockIdx.x * blockDim.x + threadIdx.x;  // path of the segment
    const int pid = P.pid_off + lpid;                        // path of the batch
    const int blk = P.pid_off / kShadeBlock + blockIdx.x;    // histogram column
    const bool valid = lpid < P.N;
    bool enq = false;
    int cell = 0;
    f3 o{0, 0, 0}, d{0, 0, 1};
    float t_enter = 0.0f;
    if (valid) {
        const uint32_t q = (uint32_t)(P.pb + lpid);
        const uint32_t qs = fdiv(q, P.fwh);
        const int s = (P.s0p ? *P.s0p : P.s0) + P.sb + (int)qs;
        const int p = (int)(q - qs * (uint32_t)P.WH);  // window pixel (path numbering, training rule)
        const int pf = frame_pixel(P.win, p);            // frame pixel (camera ray, random numbers)
        const int py = (int)(pf / (unsigned)P.W), px = pf - py * P.W;
        const uint4 r = philox4x32_10(make_uint4((uint32_t)pf, (uint32_t)s, 0u, 0u), P.key);
        // the ray in the path state's precision (FP64); traversal gets its FP32 rounding
        const preal x = (preal)px + (preal)u01(r.x), y = (preal)py + (preal)u01(r.y);
        const preal sx = (preal)2 * x / (preal)P.W - (preal)1, sy = (preal)1 - (preal)2 * y / (preal)P.H;
        const pv3 eye{(preal)P.eye[0], (preal)P.eye[1], (preal)P.eye[2]};
        const pv3 fw{(preal)P.fwd[0], (preal)P.fwd[1], (preal)P.fwd[2]};
        const pv3 rt{(preal)P.right[0], (preal)P.right[1], (preal)P.right[2]};
        const pv3 up{(preal)P.up[0], (preal)P.up[1], (preal)P.up[2]};
        pv3 o64 = eye, d64 = fw;
        if (P.ortho) {
            o64 = eye + rt * (sx * (preal)P.ortho_half_h * (preal)P.aspect) + up * (sy * (preal)P.ortho_half_h);
        } else {
            const pv3 v = fw + rt * (sx * (preal)P.tan_half * (preal)P.aspect) + up * (sy * (preal)P.tan_half);
            d64 = v * ((preal)1 / sqrt(dot3(v, v)));
        }
        o = narrow(o64);
        d = narrow(d64);
        P.ray_o[pid] = D4{o64.x, o64.y, o64.z, 0};
        P.ray_d[pid] = D4{d64.x, d64.y, d64.z, 0};
        P.hit[pid] = make_float2(INFINITY, __int_as_float(-1));
        uint32_t fl = kAlive | kCountE;
        if (P.nrc.on && ((uint64_t)(uint32_t)s * (uint64_t)P.WH + (uint64_t)p) % P.nrc.stride == 0) fl |= kTrain;
        P.flags[pid] = fl;
        cell = locate_ray(P.grid, o, d, t_enter);
        enq = cell >= 0;
    }
    const int nb = P.ext_bins;
    const int key = cell * nb + (nb > 1 ? dir_bin(d) : 0);
    const int rank = block_rank(enq, key, P.n_cells * nb, s_wcnt);
    // every slot of the segment's blocks gets a tag (-1 past its last path)
    P.se.tag[pid] = enq ? (key | (rank << 16)) : -1;
    if (enq) {
        P.se.qa[pid] = make_float4(o.x, o.y, o.z, t_enter);
        P.se.qb[pid] = make_float4(d.x, d.y, d.z, __int_as_float(pid));
        P.se.qc[pid] = make_int2(-1, __float_as_int(INFINITY));
    }
    if (!valid) P.flags[pid] = 0;
    if (P.nrc.on) {  // no cache vertex yet (the cache query reads every slot)
        P.nrc.cx[pid] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        P.nrc.cn[pid] = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
    }
    for (int c = threadIdx.x; c < P.n_cells * nb; c += blockDim.x)
        P.se.hist[(long long)c * P.n_blocks + blk] = block_key_total(c, P.n_cells * nb, s_wcnt);
}

// ---------------------------------------------------------------------------
// traversal of one subdomain (cell) BVH
// ---------------------------------------------------------------------------
// A ray prepared for one cell: the plane of lattice coordinate q on axis a
// is met at t = q * sinv.a + boff.a, with sinv = step / d and
// boff = (base - o) / d of the cell's lattice.
struct RayTrav {
    f3 o, d, sinv, boff;
};

__device__ __forceinline__ RayTrav make_trav(f3 o, f3 d, float4 qbase, float4 qstep) {
    RayTrav r;
    r.o = o;
    r.d = d;
    const float dx = fabsf(d.x) > 1e-20f ? d.x : copysignf(1e-20f, d.x);
    const float dy = fabsf(d.y) > 1e-20f ? d.y : copysignf(1e-20f, d.y);
    const float dz = fabsf(d.z) > 1e-20f ? d.z : copysignf(1e-20f, d.z);
    const f3 inv{1.0f / dx, 1.0f / dy, 1.0f / dz};
    r.sinv = f3{qstep.x * inv.x, qstep.y * inv.y, qstep.z * inv.z};
    r.boff = f3{(qbase.x - o.x) * inv.x, (qbase.y - o.y) * inv.y, (qbase.z - o.z) * inv.z};
    return r;
}

// slab test of one quantised child box against [tlo, thi]; returns the entry t
// (or +inf on a miss)
// sx, sy, sz: 16 where the ray runs down that axis (its far plane is the
// low one), else 0; rotating the record's plane pair by it puts the near
// plane in the low half, so no min / max sorts each axis's two t
__device__ __forceinline__ float box_enter(const RayTrav& r, uint4 c, float tlo, float thi, uint32_t sx, uint32_t sy,
                                           uint32_t sz) {
    const uint32_t cx = __builtin_amdgcn_alignbit(c.x, c.x, sx), cy = __builtin_amdgcn_alignbit(c.y, c.y, sy),
                   cz = __builtin_amdgcn_alignbit(c.z, c.z, sz);
    const float nx = fmaf((float)(cx & 0xffffu), r.sinv.x, r.boff.x), fx = fmaf((float)(cx >> 16), r.sinv.x, r.boff.x);
    const float ny = fmaf((float)(cy & 0xffffu), r.sinv.y, r.boff.y), fy = fmaf((float)(cy >> 16), r.sinv.y, r.boff.y);
    const float nz = fmaf((float)(cz & 0xffffu), r.sinv.z, r.boff.z), fz = fmaf((float)(cz >> 16), r.sinv.z, r.boff.z);
    const float tmin = fmaxf(fmaxf(nx, ny), fmaxf(nz, tlo));
    const float tmax = fminf(fminf(fx, fy), fminf(fz, thi));
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

// A value the compiler cannot look through: a load of LDS on one side of a
// branch and of HBM on the other then stay two loads (ds_read and
// global_load) instead of one load through a selected generic pointer, a
// flat access that waits on both memory paths.  The asm is empty: it
// neither reads nor writes memory.
typedef __attribute__((address_space(3))) int lds_int;
typedef __attribute__((address_space(1))) int global_int;
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}
// the same for the four child records of a node read from LDS: the four
// reads are issued back to back and waited for once
__device__ __forceinline__ void opaque4(uint4* c) {
    asm volatile("" : "+v"(c[0].x), "+v"(c[0].y), "+v"(c[0].z), "+v"(c[0].w), "+v"(c[1].x), "+v"(c[1].y),
                 "+v"(c[1].z), "+v"(c[1].w), "+v"(c[2].x), "+v"(c[2].y), "+v"(c[2].z), "+v"(c[2].w), "+v"(c[3].x),
                 "+v"(c[3].y), "+v"(c[3].z), "+v"(c[3].w));
}

// One work item (up to kPool chunks of one cell's queue of one ray kind) on
// one wave, with lane refill.  Each lane traverses the cell's BVH for its ray
// over (t_enter, t_exit] in rounds: node steps until at least half of the
// lanes still taking them have parked a leaf, then the parked leaves.  Once a
// quarter of the lanes have finished their rays (or all of them have), the
// finished lanes store their results, hand the rays that go on to the
// neighbouring cell's queue, and take the item's next rays; the LDS copy of
// the cell's top nodes serves the whole item.  A ray's traversal does not
// depend on which lane or round it runs in.
//  - closest hit: thi = t_exit, best = -1 on entry; the hit does not depend on
//    the visiting order (equal t goes to the lower primitive index);
//  - shadow: thi = min(t_exit, t_max); a diffuse triangle in (tlo, thi] blocks
//    the segment, a pane crossing is recorded in sh_glass (the order of the
//    records changes only the rounding of the product of the pane factors).
template <bool SHADOW, bool COUNT>
__device__ __forceinline__ void trace_item(const TraceParams& P, const QueueSet& Q, int cell, long long first,
                                           int count, const uint4* top, int* stk, int* gstk, int gstride,
                                           int& n_nodes, int& n_tris, int& n_node_steps, int& n_tri_steps,
                                           float4* cc) {
    constexpr int kDone = -2147483647 - 1;  // INT_MIN: no leaf encodes as it (~INT_MAX triangles)
    const GridParams& g = P.grid;
    const int root = P.cell_root[cell];
    {
        // the cell's exit planes and lattice, kept in the wave's LDS slot (read
        // again at each refill rather than held in registers across rounds)
        const int ix = cell % g.nx, iy = (cell / g.nx) % g.ny, iz = cell / (g.nx * g.ny);
        const int lane = lane_id();
        if (lane == 0) {
            cc[0] = make_float4(g.planes[ix], g.planes[ix + 1], g.planes[g.off_y + iy], g.planes[g.off_y + iy + 1]);
            cc[1] = make_float4(g.planes[g.off_z + iz], g.planes[g.off_z + iz + 1], 0.0f, 0.0f);
            cc[2] = P.cell_q[2 * cell];
            cc[3] = P.cell_q[2 * cell + 1];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }

    // the lane's ray: its queue record, its traversal state
    float4 qa = make_float4(0, 0, 0, 0), qb = make_float4(0, 0, 0, 0);
    int2 qc = make_int2(0, 0);
    RayTrav r;
    float t_exit = 0.0f, thi = 0.0f;
    int axis = 0, best = -1, n_glass = -1;
    bool blocked = false, live = false;
    int link = kDone, leaf = 0, sp = 0;
    int cursor = 0;  // rays of the item handed out so far (the same on every lane)

    auto fetch = [&](bool want) {
        const unsigned long long m = __ballot(want);
        const int i = cursor + rank_below(m);
        cursor += popc64(m);
        if (want && i < count) {
            const long long q = (long long)cell * P.cap + first + i;
            qa = Q.qa_in[q];
            qb = Q.qb_in[q];
            qc = Q.qc_in[q];
            const f3 o = xyz(qa), d = xyz(qb);
            const float4 pxy = cc[0], pz = cc[1];
            // exit of this cell: nearest far plane, ties x < y < z
            const float tx = d.x > 0.0f ? (pxy.y - o.x) / d.x : (d.x < 0.0f ? (pxy.x - o.x) / d.x : INFINITY);
            const float ty = d.y > 0.0f ? (pxy.w - o.y) / d.y : (d.y < 0.0f ? (pxy.z - o.y) / d.y : INFINITY);
            const float tz = d.z > 0.0f ? (pz.y - o.z) / d.z : (d.z < 0.0f ? (pz.x - o.z) / d.z : INFINITY);
            axis = 0;
            t_exit = tx;
            if (ty < t_exit) {
                t_exit = ty;
                axis = 1;
            }
            if (tz < t_exit) {
                t_exit = tz;
                axis = 2;
            }
            r = make_trav(o, d, cc[2], cc[3]);
            thi = SHADOW ? fminf(t_exit, __int_as_float(qc.y)) : t_exit;
            best = -1;
            blocked = false;
            n_glass = -1;
            sp = 0;
            leaf = 0;
            link = (!SHADOW || thi > qa.w) ? root : kDone;
            live = true;
        }
    };
    auto pop = [&]() -> int {
        // entries beyond kStack were never stored (the builders' depth cap keeps
        // the stack below it)
        if (sp == 0 || sp > kStack) return kDone;
        --sp;
        int v;
        if (sp < kLdsStack) v = opaque(stk[sp * kTraceBlock]);
        else v = gstk[(sp - kLdsStack) * gstride];
        return v;
    };

    fetch(true);
    while (__ballot(live)) {
        if (live) {
            const float tlo = qa.w;
            // node steps
            while (link >= 0) {
                // the cell's first kTopNodes nodes (breadth-first: its top levels) come from LDS
                const int rel = link - root;
                uint4 ch[kBvhWidth];
                if (rel < kTopNodes) {
#pragma unroll
                    for (int i = 0; i < kBvhWidth; ++i) ch[i] = top[kBvhWidth * rel + i];
                    opaque4(ch);
                } else {
#pragma unroll
                    for (int i = 0; i < kBvhWidth; ++i) ch[i] = P.nodes[kBvhWidth * (size_t)link + i];
                }
                if (COUNT) {
                    ++n_nodes;
                    n_node_steps += first_active_lane();
                }
                float t[kBvhWidth];
                int l[kBvhWidth];
                const uint32_t sx = (__float_as_uint(r.sinv.x) >> 27) & 16u, sy = (__float_as_uint(r.sinv.y) >> 27) & 16u,
                               sz = (__float_as_uint(r.sinv.z) >> 27) & 16u;
#pragma unroll
                for (int i = 0; i < kBvhWidth; ++i) {
                    l[i] = (int)ch[i].w;
                    const float te = box_enter(r, ch[i], tlo, thi, sx, sy, sz);  // tested unconditionally: no branch per child
                    t[i] = l[i] == kEmptyLink ? INFINITY : te;
                }
                // nearest first: sorting network on (t, link), as min / max and selects
                static_assert(kBvhWidth == 4, "the sorting network is written for 4 children");
                auto order = [&](int i, int j) {
                    const bool sw = t[j] < t[i];
                    const float lo = sw ? t[j] : t[i], hi = sw ? t[i] : t[j];
                    const int li = sw ? l[j] : l[i], lj = sw ? l[i] : l[j];
                    t[i] = lo;
                    t[j] = hi;
                    l[i] = li;
                    l[j] = lj;
                };
                order(0, 1);
                order(2, 3);
                order(0, 2);
                order(1, 3);
                order(1, 2);
                // the farther hit children wait on the stack, farthest deepest; the
                // nearest is next (short stack in LDS, deeper entries in HBM)
#pragma unroll
                for (int i = kBvhWidth - 1; i >= 1; --i)
                    if (t[i] != INFINITY) {
                        // typed address spaces keep these two stores apart (no flat store)
                        if (sp < kLdsStack) ((lds_int*)stk)[sp * kTraceBlock] = l[i];
                        else if (sp < kStack) ((global_int*)gstk)[(sp - kLdsStack) * gstride] = l[i];
                        ++sp;
                    }
                link = t[0] != INFINITY ? l[0] : pop();
                if (link < 0 && link != kDone && leaf == 0) {
                    leaf = link;
                    link = pop();
                }
                // leave for the leaf loop once at least half of the lanes here
                // have parked a leaf
                const unsigned long long here = __ballot(true), bare = __ballot(leaf == 0);
                if (2 * __popcll(bare) <= __popcll(here)) break;
            }
            if (leaf == 0 && link < 0 && link != kDone) {
                leaf = link;
                link = pop();
            }
            // triangle tests of the parked leaves (and of leaves met right after them)
            while (leaf < 0) {
                int ti = ~leaf;
                for (;;) {
                    const float4 a = P.tris[3 * (size_t)ti], b = P.tris[3 * (size_t)ti + 1],
                                 c = P.tris[3 * (size_t)ti + 2];
                    const int prim = __float_as_int(a.w);
                    const int meta = __float_as_int(b.w);
                    const int typ = meta & 3;
                    if (prim != qc.x && !(SHADOW && typ == kEmitter)) {
                        if (COUNT) {
                            ++n_tris;
                            n_tri_steps += first_active_lane();
                        }
                        float tt;
                        if (tri_test(r, a, b, c, tt)) {
                            if (!SHADOW) {
                                if (tt > tlo && (tt < thi || (tt == thi && (best < 0 || prim < best)))) {
                                    thi = tt;
                                    best = prim;
                                }
                            } else if (tt > tlo && tt <= t_exit && tt < __int_as_float(qc.y)) {
                                if (typ == kDiffuse) {
                                    blocked = true;
                                    link = kDone;
                                    break;
                                }
                                const int pid = __float_as_int(qb.w);
                                const f3 ng = xyz(P.prim_info[prim]);
                                if (n_glass < 0) n_glass = P.sh_state[pid] >> 4;
                                if (n_glass < kMaxGlass)
                                    P.sh_glass[(size_t)pid * kMaxGlass + n_glass] = make_float2(-dot3(r.d, ng), c.w);
                                else
                                    atomicOr(P.overflow, kOverflowPanes);
                                ++n_glass;
                            }
                        }
                    }
                    if (meta & kLastInLeaf) break;
                    ++ti;
                }
                leaf = 0;
                if (link < 0 && link != kDone) {
                    leaf = link;
                    link = pop();
                }
            }
        }
        // finished rays: results, hand-off and refill, once a quarter of the
        // lanes are done or no lane is still traversing
        const bool done = live && link == kDone;
        const int n_done = popc64(__ballot(done)), n_live = popc64(__ballot(live));
        if (n_done == 0 || (4 * n_done < kChunk && n_done < n_live)) continue;
        bool cont = false;
        int next = 0;
        if (done) {
            const int pid = __float_as_int(qb.w);
            bool leave;
            if (!SHADOW) {
                if (best >= 0) P.hit[pid] = make_float2(thi, __int_as_float(best));
                leave = best < 0;
            } else {
                if (blocked) P.sh_state[pid] = kShBlocked;
                else if (n_glass >= 0) P.sh_state[pid] = kShVisible | (n_glass << 4);
                leave = !blocked && t_exit < __int_as_float(qc.y);
            }
            if (leave) {
                int nx = cell % g.nx, ny = (cell / g.nx) % g.ny, nz = cell / (g.nx * g.ny);
                if (axis == 0) nx += qb.x > 0.0f ? 1 : -1;
                else if (axis == 1) ny += qb.y > 0.0f ? 1 : -1;
                else nz += qb.z > 0.0f ? 1 : -1;
                if (nx >= 0 && nx < g.nx && ny >= 0 && ny < g.ny && nz >= 0 && nz < g.nz) {
                    cont = true;
                    next = nx + g.nx * (ny + g.ny * nz);
                    qa.w = t_exit;  // carried bit-exactly into the neighbour
                }
            }
            live = false;
        }
        const int slot = wave_append(cont, next, Q.cnt_out, kCntStride);
        if (cont && slot < P.cap) {
            const long long q = (long long)next * P.cap + slot;
            Q.qa_out[q] = qa;
            Q.qb_out[q] = qb;
            Q.qc_out[q] = qc;
        }
        if (cursor < count) fetch(done);
    }
}

// One sweep over all subdomain queues of both ray kinds (closest-hit rays of
// one depth and shadow rays of the previous one are independent, so they
// share the sweep).  Work is split into items ordered by (cell, kind): up to
// kItem rays in a sweep with kPool chunks per wave of the grid, one chunk in a
// smaller one.  The item range is cut into kXcd contiguous parts, part x
// served by the workgroups of XCD x (consecutive cells share that XCD's L2).
// A wave works through one item at a time (trace_item: lanes refilled from
// the item as their rays finish).
template <bool COUNT>
__global__ __launch_bounds__(kTraceBlock) __attribute__((amdgpu_waves_per_eu(kTraceWaves, kTraceWaves)))
void k_trace(TraceParams P) {
    extern __shared__ int s_pref[];  // 2 * n_cells + 1 entries (dynamic, so small grids keep occupancy)
    __shared__ int s_stack[kLdsStack * kTraceBlock];
    __shared__ uint4 s_top[(kTraceBlock / 64) * kBvhWidth * kTopNodes];
    __shared__ float4 s_cell[(kTraceBlock / 64) * 4];  // per wave: the current item's cell constants
    const int G = P.n_cells;
    const int E = 2 * G;  // entry e = 2 * cell + kind
    constexpr int kWavesPerBlock = kTraceBlock / 64;
    __shared__ int s_item;  // rays per work item in this sweep
    __shared__ uint32_t s_defer[(2 * kMaxCells + 31) / 32];  // entries that wait for the next sweep
    auto deferred = [&](int e, int n) -> bool {
        if (P.defer_below <= 0 || n <= 0 || n >= P.defer_below) return false;
        const GridParams& g = P.grid;
        const int cell = e >> 1, ix = cell % g.nx, iy = (cell / g.nx) % g.ny, iz = cell / (g.nx * g.ny);
        const int R = max(ix, g.nx - 1 - ix) + max(iy, g.ny - 1 - iy) + max(iz, g.nz - 1 - iz);
        return P.sweep + 1 + R <= P.n_sweeps - 1;
    };
    for (int i = threadIdx.x; i < (E + 31) / 32; i += blockDim.x) s_defer[i] = 0u;
    __syncthreads();
    if (threadIdx.x < 64) {
        // exclusive prefix of the per-entry item counts (wave 0, lane-blocked scan)
        const int ln = threadIdx.x;
        const int per = (E + 63) / 64;
        const int c0 = ln * per, c1 = min(c0 + per, E);
        // items of kPool chunks only when the sweep has kPool chunks per wave of
        // the grid; a smaller sweep keeps one chunk per wave so that all its
        // chunks run at once (every block takes the same decision)
        int chunks = 0;
        for (int e = c0; e < c1; ++e) {
            const int kind = e & 1;
            const int n = P.active[kind] ? P.q[kind].cnt_in[(e >> 1) * kCntStride] : 0;
            chunks += (min((long long)n, P.cap) + kChunk - 1) / kChunk;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) chunks += __shfl_xor(chunks, o);
        const int item = chunks >= kPool * (int)gridDim.x * kWavesPerBlock ? kItem : kChunk;
        if (ln == 0) s_item = item;
        int local = 0;
        for (int e = c0; e < c1; ++e) {
            const int kind = e & 1;
            const int n = P.active[kind] ? P.q[kind].cnt_in[(e >> 1) * kCntStride] : 0;
            if (n > P.cap) atomicOr(P.overflow, kOverflowQueue);  // never expected: counters are bounded by cap
            if (deferred(e, n)) atomicOr(&s_defer[e >> 5], 1u << (e & 31));
            local += (n + item - 1) / item;
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
            const int n = P.active[kind] ? P.q[kind].cnt_in[(e >> 1) * kCntStride] : 0;
            run += (n + item - 1) / item;
        }
        if (ln == 63) s_pref[E] = incl;
    }
    __syncthreads();
    const int total = s_pref[E];
    if (total == 0) return;
    const int item_rays = s_item;
    if (blockIdx.x == 0 && threadIdx.x < 2 && P.active[threadIdx.x]) {
        // every queued ray is traversed exactly once in this sweep (a waiting queue in a later one)
        unsigned long long n = 0;
        for (int c = 0; c < G; ++c) {
            const int e = 2 * c + (int)threadIdx.x;
            if (!((s_defer[e >> 5] >> (e & 31)) & 1u))
                n += (unsigned long long)min((long long)P.q[threadIdx.x].cnt_in[c * kCntStride], P.cap);
        }
        if (n) atomicAdd(&P.stats[threadIdx.x == 0 ? kStatExtVisits : kStatShadowVisits], n);
    }
    const int lane = lane_id();
    int* stk = s_stack + threadIdx.x;
    const int gstride = gridDim.x * kTraceBlock;  // entries of one level are contiguous over the grid
    int* gstk = P.gstack + blockIdx.x * kTraceBlock + threadIdx.x;
    const int xcd = blockIdx.x % kXcd;
    int n_nodes = 0, n_tris = 0, n_node_steps = 0, n_tri_steps = 0;
    uint4* top = s_top + (threadIdx.x / 64) * kBvhWidth * kTopNodes;  // this wave's copy of a cell's top nodes
    int top_cell = -1;

    // static XCD-aware striding: the waves of XCD x walk part x of the item
    // list round-robin (no atomics, so empty and near-empty sweeps cost only
    // the prologue)
    const int lw = (blockIdx.x / kXcd) * kWavesPerBlock + (int)(threadIdx.x / 64);
    const int nwx = (gridDim.x / kXcd) * kWavesPerBlock;
    const int lo = (int)((long long)total * xcd / kXcd);
    const int hi = (int)((long long)total * (xcd + 1) / kXcd);
    for (int item = lo + lw; item < hi; item += nwx) {
        int a = 0, b = E;
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if (s_pref[m] <= item) a = m;
            else b = m;
        }
        const int e = __builtin_amdgcn_readfirstlane(a);
        const int cell = e >> 1, kind = e & 1;
        if ((s_defer[e >> 5] >> (e & 31)) & 1u) {
            // the queue waits: its rays go unchanged to its own queue of the next sweep
            const QueueSet& Q = P.q[kind];
            const long long first = (long long)(item - s_pref[e]) * item_rays;
            const int count = (int)min((long long)item_rays,
                                       min((long long)Q.cnt_in[cell * kCntStride], P.cap) - first);
            for (int b = 0; b < count; b += 64) {
                const bool on = b + lane < count;
                const long long q = (long long)cell * P.cap + first + b + lane;
                float4 qa = make_float4(0, 0, 0, 0), qb = make_float4(0, 0, 0, 0);
                int2 qc = make_int2(0, 0);
                if (on) {
                    qa = Q.qa_in[q];
                    qb = Q.qb_in[q];
                    qc = Q.qc_in[q];
                }
                const int slot = wave_append(on, cell, Q.cnt_out, kCntStride);
                if (on && slot < P.cap) {
                    const long long o = (long long)cell * P.cap + slot;
                    Q.qa_out[o] = qa;
                    Q.qb_out[o] = qb;
                    Q.qc_out[o] = qc;
                }
            }
            continue;
        }
        if (cell != top_cell) {
            // the wave is done with the previous cell's copy (its traversals
            // have returned), so it can be overwritten; LDS operations of one
            // wave complete in order
            top_cell = cell;
            const int nn = kBvhWidth * min(P.cell_nodes[cell], kTopNodes);
            const uint4* src = P.nodes + kBvhWidth * (size_t)P.cell_root[cell];
            for (int i = lane; i < nn; i += 64) top[i] = src[i];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
        const long long first = (long long)(item - s_pref[e]) * item_rays;
        const int count = (int)min((long long)item_rays,
                                   min((long long)P.q[kind].cnt_in[cell * kCntStride], P.cap) - first);
        if (kind == 0)
            trace_item<false, COUNT>(P, P.q[0], cell, first, count, top, stk, gstk, gstride, n_nodes, n_tris,
                                     n_node_steps, n_tri_steps, s_cell + 4 * (threadIdx.x / 64));
        else
            trace_item<true, COUNT>(P, P.q[1], cell, first, count, top, stk, gstk, gstride, n_nodes, n_tris,
                                    n_node_steps, n_tri_steps, s_cell + 4 * (threadIdx.x / 64));
    }
    if (COUNT) {
        const int nn = wave_sum(n_nodes), nt = wave_sum(n_tris);
        const int ns = wave_sum(n_node_steps), nts = wave_sum(n_tri_steps);
        if (lane == 0) {
            atomicAdd(&P.stats[kStatNodes], (unsigned long long)nn);
            atomicAdd(&P.stats[kStatTris], (unsigned long long)nt);
            atomicAdd(&P.stats[kStatNodeSteps], (unsigned long long)ns);
            atomicAdd(&P.stats[kStatTriSteps], (unsigned long long)nts);
        }
    }
}

// ---------------------------------------------------------------------------
// shading: the geometric part of the interaction at each hit
// ---------------------------------------------------------------------------
// One thread per path.  A single geometric path carries every wavelength
// (panes do not bend rays, diffuse bounces are wavelength independent), so
// this kernel decides the path and records each vertex; k_spectral applies the
// per-wavelength factors afterwards.  Per hit (Sec. 4 inverse ray tracing):
//  - emitter: counted (one-sided) if no diffuse vertex came since the camera or
//    since the last glass reflection, then the path ends;
//  - diffuse: one shadow ray toward the light (Eq. 3 for a point light, a
//    uniform area sample of the parallelogram), then a cosine-weighted bounce;
//  - glass pane: reflect with probability P_R = mean R / (mean R + mean T) of
//    the pane's Fresnel slab terms (Eq. 1, Sec. 6), else transmit straight on.
// R and T summed over the wavelengths for the pane hits of a wave, shared out
// over all of its lanes (a hit's slab terms, or a coated pane's transfer
// matrices, at every wavelength would otherwise run on its lane alone while
// the others wait).
// The (hit, wavelength) pairs go out 64 per round, hits in rank order; each
// hit's lane then adds its pairs from the wave's LDS slots in wavelength
// order, the order of a lone lane's loop, so the sums are the same.  Every
// lane of the wave calls this.
template <bool COATED>
__device__ __forceinline__ void wave_pane_sums(bool need, int m, float c, const float4* pane, const ShadeParams& P,
                                               int* owner, float2* rt, float& sumR, float& sumT) {
    const unsigned long long own = __ballot(need);
    if (own == 0) return;
    const int lane = lane_id(), n_own = popc64(own), rank = rank_below(own);
    if (need) owner[rank] = lane;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    const int nl = P.nl, total = n_own * nl;
    for (int base = 0; base < total; base += 64) {
        const int q = base + lane;
        const int orank = min(q / nl, n_own - 1);
        const int o = owner[orank];
        const int mo = __shfl(m, o);
        const float co = __shfl(c, o);
        float R = 0.0f, T = 0.0f;
        if (q < total) glass_RT<COATED>(pane, P.coat, P.coat_n, P.coat_layers, P.nlp, mo, q - orank * nl, co, R, T);
        rt[lane] = make_float2(R, T);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (need) {
            const int lo = max(rank * nl - base, 0), hi = min((rank + 1) * nl - base, 64);
            for (int k = lo; k < hi; ++k) {
                const float2 v = rt[k];
                sumR += v.x;
                sumT += v.y;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

template <bool COATED>
__global__ __launch_bounds__(kShadeBlock) void k_shade(ShadeParams P) {
    __shared__ int s_wcnt[(kShadeBlock / 64) * kMaxCells];
    __shared__ float4 s_pane[kLdsPane];
    __shared__ int s_gown[kShadeBlock];     // per wave: lanes of its pane hits by rank
    __shared__ float2 s_grt[kShadeBlock];   // per wave: R and T of one round of pairs
    const int n_pane = P.n_glass * P.nlp;
    const bool pane_lds = n_pane <= kLdsPane;
    if (pane_lds)
        for (int i = threadIdx.x; i < n_pane; i += blockDim.x) s_pane[i] = P.pane[i];
    __syncthreads();
    const float4* pane = pane_lds ? s_pane : P.pane;
    const int lpid = blockIdx.x * blockDim.x + threadIdx.x;  // path of the segment
    const int pid = P.pid_off + lpid;                        // path of the batch
    const int blk = P.pid_off / kShadeBlock + blockIdx.x;    // histogram column
    const bool valid = lpid < P.N;
    bool enq_e = false, enq_s = false;
    int cell_e = 0, cell_s = 0;
    f3 xo{0, 0, 0}, dn{0, 0, 1}, ws{0, 0, 1};
    float te = 0.0f, ts = 0.0f, r_sh = 0.0f;
    int prim = -1;
    // the hit and the FP64 ray are loaded with the flags, before the branches
    // that need them, so their latencies overlap; past depth 2 of a cache
    // render most paths have ended in the cache, and those are read only
    // when their flags say they live
    uint32_t fl = 0;
    float2 h = make_float2(0.0f, 0.0f);
    D4 ro{}, rd{};
    if (valid) {
        if (!(P.nrc.on && P.depth > 2)) {
            fl = P.flags[pid];
            h = P.hit[pid];
            ro = P.ray_o[pid];
            rd = P.ray_d[pid];
        } else {
            fl = P.flags[pid];
            if (fl & kAlive) {
                h = P.hit[pid];
                ro = P.ray_o[pid];
                rd = P.ray_d[pid];
            }
        }
    }
    const bool alive = valid && (fl & kAlive);
    if (alive) prim = __float_as_int(h.y);
    const bool last_depth = P.depth == P.max_depth;
    // the hit's material and geometry (the pane sums below need them on
    // every lane of the wave before the branches on the material)
    const pv3 o{ro.x, ro.y, ro.z}, d{rd.x, rd.y, rd.z};
    float4 pi = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int typ = -1, m = 0, emits = 0;
    pv3 ng{0, 0, 1}, n{0, 0, 1}, x{0, 0, 0};
    preal cos_o = 0;
    if (alive && prim >= 0) {
        pi = P.prim_info[prim];
        const int word = __float_as_int(pi.w);
        typ = (word >> kMatTypeShift) & 3;
        // material, or compact glass index for glass (with this render's substitution)
        m = word & kMatIdMask;
        if (typ == kGlass && m == P.glass_from) m = P.glass_to;
        emits = (word & kMatEmits) ? kVEmits : 0;
        // geometry in the path state's precision (FP64) from the triangle's
        // vertices: N = (v1 - v0) x (v2 - v0), the hit point on its plane
        // x = o + t d with t = N.(v0 - o) / N.d (the FP32 traversal t only
        // chose the triangle), the side the ray came from
        const pv3 v0 = state3(P.prim_v[3 * (size_t)prim]);
        const pv3 N =
            cross3(state3(P.prim_v[3 * (size_t)prim + 1]) - v0, state3(P.prim_v[3 * (size_t)prim + 2]) - v0);
        const preal nn = dot3(N, N), nd = dot3(N, d);
        ng = nn > (preal)0 ? N * ((preal)1 / sqrt(nn)) : state3(xyz(pi));
        cos_o = -dot3(ng, d);
        n = cos_o > (preal)0 ? ng : ng * (preal)-1;
        x = nd != (preal)0 ? o + d * (dot3(N, v0 - o) / nd) : o + d * (preal)h.x;
    }
    // a pane hit: signed cosine, > 0 when the ray meets the normal-side (coated) face
    const bool pane_hit = alive && prim >= 0 && typ == kGlass;
    float pane_c = 0.0f;
    if (pane_hit) {
        const float cabs = (float)fabs(dot3(d, ng));
        pane_c = cos_o > (preal)0 ? cabs : -cabs;
    }
    float sumR = 0.0f, sumT = 0.0f;  // over the wavelengths, for a pane hit before the last depth
    const int wv = threadIdx.x / 64;
    wave_pane_sums<COATED>(pane_hit && !last_depth, m, pane_c, pane, P, s_gown + 64 * wv, s_grt + 64 * wv, sumR, sumT);
    if (alive) {
        {
            const uint32_t q = (uint32_t)(P.pb + lpid);
            const uint32_t qs = fdiv(q, P.fwh);
            const int s0 = P.s0p ? *P.s0p : P.s0;
            const int s = s0 + P.sb + (int)qs;
            const int p = (int)(q - qs * (uint32_t)P.WH);
            const int pf = frame_pixel(P.win, p);
            if (P.hit_log) P.hit_log[((long long)p * P.spp_call + (s - s0)) * P.max_depth + P.depth - 1] = prim;
            int4 rec = make_int4(kVNone, 0, 0, 0);
            int sh = kShNone;
            if (prim < 0) {
                fl = 0;  // no sky dome: a miss carries nothing
            } else {
                pv3 xo64 = x, dn64 = d;
                if (typ == kEmitter) {
                    rec.x = ((fl & kCountE) && cos_o > (preal)0) ? (kVEmit | kVLast | (m << kVIdShift)) : kVNone;
                    fl = 0;
                } else if (typ == kDiffuse) {
                    const uint4 ub = philox4x32_10(make_uint4((uint32_t)pf, (uint32_t)s, (uint32_t)P.depth, 0u), P.key);
                    xo64 = x + n * (preal)kOffset;
                    xo = narrow(xo64);
                    float gfac = 0.0f;
                    if (P.light_type != 0) {
                        // light sample and geometry term
                        pv3 y{(preal)P.lp0[0], (preal)P.lp0[1], (preal)P.lp0[2]};
                        if (P.light_type == 1)
                            y = y + pv3{(preal)P.le1[0], (preal)P.le1[1], (preal)P.le1[2]} * (preal)u01(ub.x) +
                                pv3{(preal)P.le2[0], (preal)P.le2[1], (preal)P.le2[2]} * (preal)u01(ub.y);
                        const pv3 w = y - xo64;
                        const preal r2 = dot3(w, w);
                        const preal r = sqrt(r2);
                        const pv3 om = w * ((preal)1 / r);
                        const preal cx = dot3(n, om);
                        const preal cy =
                            P.light_type == 1 ? -dot3(pv3{(preal)P.nL[0], (preal)P.nL[1], (preal)P.nL[2]}, om) : (preal)1;
                        if (cx > (preal)0 && cy > (preal)0) {
                            // (rho/pi) Le cos_x cos_y / r^2 * A (area light); (rho/pi) I cos_x / r^2 (Eq. 3)
                            gfac = (float)((P.light_type == 1 ? cx * cy / r2 * (preal)P.light_area : cx / r2) *
                                           (preal)(1.0 / 3.14159265358979323846));
                            sh = kShVisible;
                            ws = narrow(om);
                            r_sh = (float)r;
                            cell_s = locate_ray(P.grid, xo, ws, ts);
                            enq_s = cell_s >= 0;
                        }
                    }
                    // radiance cache: a path other than a training path ends here from depth 2 on
                    const bool to_cache = P.nrc.on && P.depth >= 2 && !(fl & kTrain);
                    const bool stop = last_depth || to_cache;
                    rec = make_int4(kVDiffuse | (stop ? kVLast : 0) | emits | (m << kVIdShift), to_cache ? 1 : 0,
                                    0, __float_as_int(gfac));
                    if (P.nrc.on && P.depth >= 2 && (to_cache || !last_depth)) {
                        const float4 xf = make_float4((float)x.x, (float)x.y, (float)x.z, 1.0f);
                        const float4 nf = make_float4((float)n.x, (float)n.y, (float)n.z, 0.0f);
                        if (to_cache) {
                            P.nrc.cx[pid] = xf;
                            P.nrc.cn[pid] = nf;
                        } else {  // a vertex of a training path that continues
                            const uint64_t qc = (uint64_t)(uint32_t)(s - s0) * (uint64_t)P.WH + (uint64_t)p;
                            const size_t slot = (size_t)(qc / P.nrc.stride) * P.max_depth + (P.depth - 1);
                            P.nrc.tx[slot] = xf;
                            P.nrc.tn[slot] = nf;
                        }
                    }
                    fl &= ~kCountE;
                    if (stop) {
                        fl = 0;
                    } else {
                        const uint4 uc =
                            philox4x32_10(make_uint4((uint32_t)pf, (uint32_t)s, (uint32_t)P.depth, 1u), P.key);
                        dn64 = cosine_dir_state(n, (preal)u01(uc.x), (preal)u01(uc.y));
                        enq_e = true;
                    }
                } else {  // glass pane: R and T summed over the wavelengths above
                    const float c = pane_c;
                    if (!(sumR + sumT > 0.0f) || last_depth) {
                        rec.x = kVGlassT | kVLast | (m << kVIdShift);
                        fl = 0;
                    } else {
                        const float PR = sumR / (sumR + sumT);
                        const uint4 ub =
                            philox4x32_10(make_uint4((uint32_t)pf, (uint32_t)s, (uint32_t)P.depth, 0u), P.key);
                        const bool refl = u01(ub.z) < PR;
                        rec = make_int4((refl ? kVGlassR : kVGlassT) | (m << kVIdShift), __float_as_int(c),
                                        __float_as_int(PR), 0);
                        if (refl) {
                            dn64 = d - ng * ((preal)2 * dot3(d, ng));
                            fl |= kCountE;
                            xo64 = x + n * (preal)kOffset;
                        } else {
                            xo64 = x - n * (preal)kOffset;
                        }
                        enq_e = true;
                    }
                }
                if (enq_e) {
                    P.ray_o[pid] = D4{xo64.x, xo64.y, xo64.z, 0};
                    P.ray_d[pid] = D4{dn64.x, dn64.y, dn64.z, 0};
                    xo = narrow(xo64);
                    dn = narrow(dn64);
                }
            }
            P.vrec[pid] = rec;
            if ((rec.x & 7) == kVDiffuse) P.sh_state[pid] = sh;
            if (enq_e) {
                P.hit[pid] = make_float2(INFINITY, __int_as_float(-1));
                cell_e = locate_ray(P.grid, xo, dn, te);
                // a ray that never enters the grid keeps its miss record
                enq_e = cell_e >= 0;
            }
            P.flags[pid] = fl;
        }
    }
    // stage both rays in path order; k_route scatters them into the queues
    // every slot of the segment's blocks gets a tag (-1 past its last path)
    const int nb = P.ext_bins;
    const int key_e = cell_e * nb + (nb > 1 ? dir_bin(dn) : 0);
    const int rank_e = block_rank(enq_e, key_e, P.n_cells * nb, s_wcnt);
    P.se.tag[pid] = enq_e ? (key_e | (rank_e << 16)) : -1;
    if (enq_e) {
        P.se.qa[pid] = make_float4(xo.x, xo.y, xo.z, te);
        P.se.qb[pid] = make_float4(dn.x, dn.y, dn.z, __int_as_float(pid));
        P.se.qc[pid] = make_int2(prim, __float_as_int(INFINITY));
    }
    for (int c = threadIdx.x; c < P.n_cells * nb; c += blockDim.x)
        P.se.hist[(long long)c * P.n_blocks + blk] = block_key_total(c, P.n_cells * nb, s_wcnt);
    const int rank_s = block_rank(enq_s, cell_s, P.n_cells, s_wcnt);
    P.ss.tag[pid] = enq_s ? (cell_s | (rank_s << 16)) : -1;
    if (enq_s) {
        P.ss.qa[pid] = make_float4(xo.x, xo.y, xo.z, ts);
        P.ss.qb[pid] = make_float4(ws.x, ws.y, ws.z, __int_as_float(pid));
        P.ss.qc[pid] = make_int2(prim, __float_as_int(r_sh));
    }
    for (int c = threadIdx.x; c < P.n_cells; c += blockDim.x)
        P.ss.hist[(long long)c * P.n_blocks + blk] = block_key_total(c, P.n_cells, s_wcnt);
}

// ---------------------------------------------------------------------------
// routing of staged rays into the per-cell queues (count -> scan -> scatter)
// ---------------------------------------------------------------------------
// One workgroup per (kind, cell): exclusive scan, in block order, of the
// per-block counts; the cell's total becomes its queue length.
// One workgroup per (kind, routing key): exclusive scan, in block order, of
// the key's per-block counts; the key's total goes to ktot and is added to its
// cell's queue length.  A cell's keys (direction bins) follow each other in
// its queue: k_route adds the totals of the cell's lower bins.
__global__ __launch_bounds__(256) void k_route_scan(RouteParams P) {
    __shared__ int s_part[256];
    const int per_kind = P.n_cells * kExtBins;
    const int kind = blockIdx.x / per_kind, key = blockIdx.x % per_kind;
    if (!P.active[kind] || key >= P.n_cells * P.nbin[kind]) return;
    int* h = P.st[kind].hist + (long long)key * P.n_blocks;
    const int nb = P.n_blocks;
    const int per = (nb + 255) / 256;
    const int b0 = threadIdx.x * per, b1 = min(b0 + per, nb);
    int local = 0;
    for (int b = b0; b < b1; ++b) local += h[b];
    s_part[threadIdx.x] = local;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int v = threadIdx.x >= o ? s_part[threadIdx.x - o] : 0;
        __syncthreads();
        s_part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = s_part[threadIdx.x] - local;
    for (int b = b0; b < b1; ++b) {
        const int v = h[b];
        h[b] = run;
        run += v;
    }
    if (threadIdx.x == 255) {
        const int total = s_part[255];
        P.ktot[kind][key] = total;
        if (total) {
            atomicAdd(&P.cnt[kind][(key / P.nbin[kind]) * kCntStride], total);  // queue lengths start at zero per batch
            if (P.count[kind])
                atomicAdd(&P.stats[kind == 0 ? kStatExtRays : kStatShadowRays], (unsigned long long)total);
        }
    }
}

// Workgroup i runs on XCD i % 8; path block pb = x * per + j goes to the j-th
// workgroup of XCD x, so each XCD routes a contiguous range of path blocks.
// A key's runs from consecutive path blocks are adjacent in its queue, and
// when one XCD writes them its L2 merges them into whole lines instead of
// several XCDs writing back parts of the same lines.
// The block's records of one kind are staged in LDS in key order (a key's
// records by rank), so that consecutive threads write consecutive slots of a
// key's run in its cell's queue: whole lines instead of scattered 40-byte
// records.  Every record goes to the slot it would get on its own thread.
__global__ __launch_bounds__(kShadeBlock) void k_route(RouteParams P) {
    __shared__ int s_off[kShadeBlock];     // per key: exclusive prefix of the block's counts
    __shared__ int s_key[kShadeBlock];     // per staged record: its key
    __shared__ float4 s_qa[kShadeBlock], s_qb[kShadeBlock];
    __shared__ int2 s_qc[kShadeBlock];
    __shared__ int s_wsum[kShadeBlock / 64];
    const int per = gridDim.x / kXcd;  // the grid is a multiple of kXcd
    const int pb = (int)(blockIdx.x % kXcd) * per + (int)(blockIdx.x / kXcd);
    if (pb >= P.n_blocks) return;      // whole block: before any barrier
    const int t = threadIdx.x;
    const int pid = pb * kShadeBlock + t;
    const bool valid = pid < P.N;
#pragma unroll
    for (int kind = 0; kind < 2; ++kind) {
        if (!P.active[kind]) continue;  // uniform
        const Stage& S = P.st[kind];
        const int nbin = P.nbin[kind], n_keys = P.n_cells * nbin;
        const int tag = valid ? S.tag[pid] : -1;
        const int key = tag & 0xFFFF, rank = tag >> 16;
        // the block's count per key (the key's highest rank + 1), then their prefix
        s_off[t] = 0;
        __syncthreads();
        if (tag >= 0 && key < kShadeBlock) atomicMax(&s_off[key], rank + 1);
        __syncthreads();
        const int c = s_off[t];  // keys beyond n_keys stay 0
        int incl = c;            // block-wide inclusive scan over the keys
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane_id() >= o) incl += v;
        }
        if (lane_id() == 63) s_wsum[t / 64] = incl;
        __syncthreads();
        int wbase = 0;
        for (int w = 0; w < t / 64; ++w) wbase += s_wsum[w];
        const int n_staged = [&] { int n = 0; for (int w = 0; w < kShadeBlock / 64; ++w) n += s_wsum[w]; return n; }();
        __syncthreads();
        s_off[t] = wbase + incl - c;
        __syncthreads();
        if (tag >= 0 && key < kShadeBlock && n_keys <= kShadeBlock) {
            const int at = s_off[key] + rank;
            s_key[at] = key;
            s_qa[at] = S.qa[pid];
            s_qb[at] = S.qb[pid];
            s_qc[at] = S.qc[pid];
        }
        __syncthreads();
        if (t < n_staged && n_keys <= kShadeBlock) {
            const int k = s_key[t], cell = k / nbin;
            long long slot = (long long)S.hist[(long long)k * P.n_blocks + pb] + (t - s_off[k]);
            for (int k2 = cell * nbin; k2 < k; ++k2) slot += P.ktot[kind][k2];  // the cell's lower bins
            if (slot >= 0 && slot < P.cap && cell < P.n_cells) {  // always: defence only
                const long long q = (long long)cell * P.cap + slot;
                P.qa[kind][q] = s_qa[t];
                P.qb[kind][q] = s_qb[t];
                P.qc[kind][q] = s_qc[t];
            }
        }
        if (n_keys > kShadeBlock && tag >= 0) {  // more keys than staging slots (not with the library's grids)
            const int cell = key / nbin;
            long long slot = (long long)S.hist[(long long)key * P.n_blocks + pb] + rank;
            for (int k2 = cell * nbin; k2 < key; ++k2) slot += P.ktot[kind][k2];
            if (slot >= 0 && slot < P.cap && cell < P.n_cells) {
                const long long q = (long long)cell * P.cap + slot;
                P.qa[kind][q] = S.qa[pid];
                P.qb[kind][q] = S.qb[pid];
                P.qc[kind][q] = S.qc[pid];
            }
        }
        __syncthreads();  // the staging is reused by the next kind
    }
}

// ---------------------------------------------------------------------------
// per-wavelength replay of the path histories and per-pixel accumulation
// ---------------------------------------------------------------------------
// One thread per (pixel p, group of 4 wavelengths): for every sample of p in
// the batch (increasing sample order, so the FP32 sums are deterministic)
// rebuild the path throughput beta(l) from the vertex records and add
//   emission:  beta Le                       (emitters, diffuse emitters)
//   shadow ray: beta rho Le_light g T_panes  (after the Lambert factor rho)
// Glass vertices multiply beta by R/P_R or T/(1-P_R) (Eq. 1, Sec. 6 slab).
// Vertices are replayed in predicated blocks of 2 so that all their records
// and table values are loaded before the (sequential) arithmetic (one at a
// time in scenes with coated panes, whose glass code is too large to unroll).

__device__ __forceinline__ float4 f4mul(float4 a, float4 b) { return make_float4(a.x * b.x, a.y * b.y, a.z * b.z, a.w * b.w); }
__device__ __forceinline__ float4 f4fma(float4 a, float4 b, float4 c) {
    return make_float4(a.x * b.x + c.x, a.y * b.y + c.y, a.z * b.z + c.z, a.w * b.w + c.w);
}
__device__ __forceinline__ float4 f4scale(float4 a, float s) { return make_float4(a.x * s, a.y * s, a.z * s, a.w * s); }

template <bool COATED>
__global__ __launch_bounds__(256) void k_spectral(SpectralParams P) {
    // records replayed per block: two (90 VGPRs, 5 waves per SIMD) hide the
    // loads' latency better than four (128 VGPRs, 4 waves); the coated pane
    // code is too large to unroll, so coated scenes go one vertex at a time
    constexpr int kVBlock = COATED ? 1 : 2;
    __shared__ float4 s_pane[kLdsPane];
    const int n_pane = P.n_glass * P.nlp;
    const bool pane_lds = n_pane <= kLdsPane;
    if (pane_lds)
        for (int i = threadIdx.x; i < n_pane; i += blockDim.x) s_pane[i] = P.pane[i];
    __syncthreads();
    const float4* pane = pane_lds ? s_pane : P.pane;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int npix = P.N < P.WH ? P.N : P.WH;
    if (t >= (uint32_t)npix * (uint32_t)P.ngrp) return;
    const int i = (int)fdiv(t, P.fgrp), grp = (int)t - i * P.ngrp;
    const int l0 = 4 * grp;
    const uint32_t q = (uint32_t)(P.pb + i);
    const uint32_t qs = fdiv(q, P.fwh);
    const int p = (int)(q - qs * (uint32_t)P.WH);
    const int s0 = P.s0p ? *P.s0p : P.s0;
    int s = s0 + P.sb + (int)qs;  // sample of the first path of p in the batch
    const float4 leL = *reinterpret_cast<const float4*>(P.le + (size_t)P.light_mat * P.nlp + l0);
    float4* accp = reinterpret_cast<float4*>(P.acc + (size_t)p * P.nlp + l0);
    float4 a = *accp;
    for (int pid = P.pid_off + i; pid < P.pid_off + P.N; pid += P.WH, ++s) {
        float4 beta = make_float4(1.0f, 1.0f, 1.0f, 1.0f), L = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        bool live = true;
        for (int d0 = 0; d0 < P.max_depth && live; d0 += kVBlock) {
            int4 v[kVBlock];
            int shs[kVBlock];
#pragma unroll
            for (int j = 0; j < kVBlock; ++j) {
                const bool in = d0 + j < P.max_depth;
                const size_t vi = (size_t)(in ? d0 + j : 0) * P.N_all + pid;  // always a valid address
                v[j] = in ? P.vrec[vi] : make_int4(kVNone, 0, 0, 0);
                shs[j] = in ? P.sh_state[vi] : kShNone;
            }
            // which records of the block belong to the path: only those are
            // dereferenced (records past the path's end are stale or unwritten)
            bool on[kVBlock];
            bool run = live;
#pragma unroll
            for (int j = 0; j < kVBlock; ++j) {
                run = run && (v[j].x & 7) != kVNone;
                on[j] = run;
                run = run && !(v[j].x & kVLast);
            }
            float4 rho[kVBlock], le[kVBlock];
#pragma unroll
            for (int j = 0; j < kVBlock; ++j) {
                const int kind = v[j].x & 7;
                const int m = min(max(v[j].x >> kVIdShift, 0), P.n_mats - 1);
                const bool dif = on[j] && kind == kVDiffuse;
                const bool emit = on[j] && (kind == kVEmit || (kind == kVDiffuse && (v[j].x & kVEmits)));
                rho[j] = dif ? *reinterpret_cast<const float4*>(P.rho + (size_t)m * P.nlp + l0)
                             : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
                le[j] = emit ? *reinterpret_cast<const float4*>(P.le + (size_t)m * P.nlp + l0)
                             : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int j = 0; j < kVBlock; ++j) {
                const int x = v[j].x, kind = x & 7;
                if (!on[j]) continue;
                L = f4fma(beta, le[j], L);
                if (kind == kVDiffuse) {
                    beta = f4mul(beta, rho[j]);
                    const float gfac = __int_as_float(v[j].w);
                    if (gfac > 0.0f && (shs[j] & 15) == kShVisible) {
                        float4 trv = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
                        const int ng = min(shs[j] >> 4, kMaxGlass);
                        for (int k = 0; k < ng; ++k) {
                            const size_t vi = (size_t)(d0 + j) * P.N_all + pid;
                            const float2 gl = P.sh_glass[vi * kMaxGlass + k];
                            int gi = min(max(__float_as_int(gl.y), 0), P.n_glass - 1);
                            if (gi == P.glass_from) gi = P.glass_to;
                            float4 Rg, Tg;
                            glass_RT4<COATED>(pane, P.coat, P.coat_n, P.coat_layers, P.nlp, gi, l0, gl.x, Rg, Tg);
                            trv = f4mul(trv, Tg);
                        }
                        L = f4fma(f4scale(f4mul(beta, leL), gfac), trv, L);
                    }
                    if (P.lhat && v[j].y == 1) {  // the path's cache vertex: beta (after rho) times the cache
                        // cache values tiled by 16 paths: [pid / 16][l][pid % 16]
                        const float* lh = P.lhat + (size_t)(pid >> 4) * P.nlp * 16 + (size_t)l0 * 16 + (pid & 15);
                        L = f4fma(beta, make_float4(lh[0], lh[16], lh[32], lh[48]), L);
                    }
                } else if ((kind == kVGlassR || kind == kVGlassT) && !(x & kVLast)) {
                    const int gi = min(max(x >> kVIdShift, 0), P.n_glass - 1);
                    const float PR = __int_as_float(v[j].z);
                    const float c = __int_as_float(v[j].y);
                    float4 Rl, Tl;
                    glass_RT4<COATED>(pane, P.coat, P.coat_n, P.coat_layers, P.nlp, gi, l0, c, Rl, Tl);
                    beta = f4mul(beta, kind == kVGlassR ? f4scale(Rl, 1.0f / PR) : f4scale(Tl, 1.0f / (1.0f - PR)));
                }
            }
            live = run;
            if (P.shadow_log && grp == 0) {
                int* sl = P.shadow_log + ((long long)p * P.spp_call + (s - s0)) * P.max_depth;
#pragma unroll
                for (int j = 0; j < kVBlock; ++j)
                    if (on[j] && (v[j].x & 7) == kVDiffuse && __int_as_float(v[j].w) > 0.0f)
                        sl[d0 + j] = (shs[j] & 15) == kShVisible ? 1 : 0;
            }
        }
        a = make_float4(a.x + L.x, a.y + L.y, a.z + L.z, a.w + L.w);
    }
    *accp = a;
}

// ---------------------------------------------------------------------------
// radiance-cache training rows
// ---------------------------------------------------------------------------
// One thread per training path.  For each diffuse vertex v of depth >= 2 that
// continued the path, at one wavelength l drawn for (p, s, depth, 3): the
// target is the radiance the path carries back into v along its continuation,
// R(v + 1), where R(k) = Le_k + f_k (N_k + R(k + 1)) over the later records k
// (f the record's throughput factor -- rho, R / P_R or T / (1 - P_R) -- and N
// the light sample of a diffuse record), exactly the terms the spectral
// replay adds for those records.
template <bool COATED>
__global__ __launch_bounds__(256) void k_nrc_rows(NrcRowParams P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const long long j = P.j0 + i;
    const long long qc = P.r + j * (long long)P.stride;
    const int pid = P.pid_off + (int)(qc - P.q0);
    const int s = P.s0 + (int)(qc / P.WH), p = frame_pixel(P.win, (int)(qc % P.WH));
    const int D = P.max_depth;
    bool live = true;
    for (int v = 0; v < D; ++v) {
        const int4 rv = live ? P.vrec[(size_t)v * P.N_all + pid] : make_int4(kVNone, 0, 0, 0);
        const bool on = live && (rv.x & 7) != kVNone;
        if (v >= 1) {
            const size_t row = (size_t)j * (D - 1) + (v - 1);
            const bool ok = on && (rv.x & 7) == kVDiffuse && !(rv.x & kVLast);
            P.row_ok[row] = ok ? 1 : 0;
            if (ok) {
                const uint4 u = philox4x32_10(make_uint4((uint32_t)p, (uint32_t)s, (uint32_t)(v + 1), 3u), P.key);
                const int l = (int)(u.x % (uint32_t)P.nl);
                float R = 0.0f, f = 1.0f;
                for (int k = v + 1; k < D; ++k) {
                    const int4 rk = P.vrec[(size_t)k * P.N_all + pid];
                    const int kind = rk.x & 7;
                    if (kind == kVNone) break;
                    const int m = min(max(rk.x >> kVIdShift, 0), P.n_mats - 1);
                    if (kind == kVEmit) {
                        R += f * P.le[(size_t)m * P.nlp + l];
                    } else if (kind == kVDiffuse) {
                        if (rk.x & kVEmits) R += f * P.le[(size_t)m * P.nlp + l];
                        f *= P.rho[(size_t)m * P.nlp + l];
                        const float gfac = __int_as_float(rk.w);
                        const int shs = P.sh_state[(size_t)k * P.N_all + pid];
                        if (gfac > 0.0f && (shs & 15) == kShVisible) {
                            float trv = 1.0f;
                            const int ng = min(shs >> 4, kMaxGlass);
                            for (int q = 0; q < ng; ++q) {
                                const float2 gl = P.sh_glass[((size_t)k * P.N_all + pid) * kMaxGlass + q];
                                int gi = min(max(__float_as_int(gl.y), 0), P.n_glass - 1);
                                if (gi == P.glass_from) gi = P.glass_to;
                                float Rg, Tg;
                                glass_RT<COATED>(P.pane, P.coat, P.coat_n, P.coat_layers, P.nlp, gi, l, gl.x, Rg, Tg);
                                trv *= Tg;
                            }
                            R += f * P.le[(size_t)P.light_mat * P.nlp + l] * gfac * trv;
                        }
                    } else if (!(rk.x & kVLast)) {  // glass, reflected or transmitted
                        const int gi = min(max(rk.x >> kVIdShift, 0), P.n_glass - 1);
                        const float PR = __int_as_float(rk.z), c = __int_as_float(rk.y);
                        float Rl, Tl;
                        glass_RT<COATED>(P.pane, P.coat, P.coat_n, P.coat_layers, P.nlp, gi, l, c, Rl, Tl);
                        f *= kind == kVGlassR ? Rl / PR : Tl / (1.0f - PR);
                    }
                    if (rk.x & kVLast) break;
                }
                const float4 x = P.tx[(size_t)j * D + v], n = P.tn[(size_t)j * D + v];
                P.rows[2 * row] = make_float4(x.x, x.y, x.z, P.lam_nm[l]);
                P.rows[2 * row + 1] = make_float4(n.x, n.y, n.z, R);
            }
        }
        live = on && !(rv.x & kVLast);
    }
}

// FP64: mean over samples and XYZ = sum_l w_l cmf_l L_l
// 64 pixels per block: their accumulator rows (contiguous, nlp a multiple of
// 4) are staged in LDS (dynamic, 64 nlp floats, so short spectra keep many
// blocks per CU) with 16-byte loads, the spectral means are written as one
// contiguous run, and one thread per (pixel, X/Y/Z) forms XYZ from the
// products w_l cmf_l staged once per block
constexpr int kResolvePix = 64;
__global__ __launch_bounds__(256) void k_resolve(int WH, int nl, int nlp, double inv_spp, const float* __restrict__ acc,
                                                 const double* __restrict__ w, const double* __restrict__ cmf,
                                                 double* spectral, double* xyz) {
    extern __shared__ float4 s_acc4[];  // kResolvePix * nlp / 4
    __shared__ double s_wc[3 * 128];    // w_l cmf_l, l < nl <= 128
    const float* s_acc = reinterpret_cast<const float*>(s_acc4);
    const int p0 = blockIdx.x * kResolvePix;
    const int np = min(kResolvePix, WH - p0);
    const float4* src = reinterpret_cast<const float4*>(acc + (size_t)p0 * nlp);
    for (int e = threadIdx.x; e < np * nlp / 4; e += blockDim.x) s_acc4[e] = src[e];
    if (xyz)
        for (int e = threadIdx.x; e < 3 * nl; e += blockDim.x) s_wc[e] = w[e / 3] * cmf[e];
    __syncthreads();
    if (spectral) {
        double* dst = spectral + (size_t)p0 * nl;
        for (int e = threadIdx.x; e < np * nl; e += blockDim.x) {
            const int pp = e / nl, l = e - pp * nl;
            dst[e] = (double)s_acc[pp * nlp + l] * inv_spp;
        }
    }
    if (xyz && (int)threadIdx.x < 3 * np) {
        const int pp = threadIdx.x / 3, k = threadIdx.x - 3 * pp;
        double X = 0.0;
        for (int l = 0; l < nl; ++l) {
            const double v = (double)s_acc[pp * nlp + l] * inv_spp;
            X += s_wc[3 * l + k] * v;
        }
        xyz[3 * (size_t)p0 + threadIdx.x] = X;  // pixel p0 + pp, component k
    }
}

__global__ void k_fill_i32(int* p, long long n, int v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fold_flags(FlagFold f) {
    const int i = threadIdx.x;
    if (i < f.n) atomicOr(f.dst[i], *f.src);
}

__global__ void k_pane(int n, const float4* pc, const float* c, float2* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float R, T;
    pane_RT(pc[i], c[i], R, T);
    out[i] = make_float2(R, T);
}

__global__ void k_glass(int n, GlassTable tab, const int4* q, float2* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int4 v = q[i];
    float R, T;
    if (tab.coat_n) glass_RT<true>(tab.pane, tab.coat, tab.coat_n, tab.coat_layers, tab.nlp, v.x, v.y, __int_as_float(v.z), R, T);
    else glass_RT<false>(tab.pane, tab.coat, tab.coat_n, tab.coat_layers, tab.nlp, v.x, v.y, __int_as_float(v.z), R, T);
    out[i] = make_float2(R, T);
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
    const int slot = wave_append(enq, cell, cnt, kCntStride);
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
    hipLaunchKernelGGL(k_camgen, dim3(blocks_for(p.N, kShadeBlock)), dim3(kShadeBlock), 0, st, p);
    return hipGetLastError();
}

static size_t trace_lds_bytes(int n_cells) { return sizeof(int) * (size_t)(2 * n_cells + 1); }

hipError_t launch_trace(const TraceParams& p, bool count, int grid_blocks, hipStream_t st) {
    const size_t lds = trace_lds_bytes(p.n_cells);
    if (count) hipLaunchKernelGGL((k_trace<true>), dim3(grid_blocks), dim3(kTraceBlock), lds, st, p);
    else hipLaunchKernelGGL((k_trace<false>), dim3(grid_blocks), dim3(kTraceBlock), lds, st, p);
    return hipGetLastError();
}

int trace_blocks_per_cu(int n_cells) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<false>, kTraceBlock, trace_lds_bytes(n_cells)) !=
        hipSuccess)
        return 4;
    return nb > 0 ? nb : 1;
}

hipError_t launch_shade(const ShadeParams& p, hipStream_t st) {
    if (p.N <= 0) return hipSuccess;
    if (p.coat_n) hipLaunchKernelGGL(k_shade<true>, dim3(blocks_for(p.N, kShadeBlock)), dim3(kShadeBlock), 0, st, p);
    else hipLaunchKernelGGL(k_shade<false>, dim3(blocks_for(p.N, kShadeBlock)), dim3(kShadeBlock), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_route(const RouteParams& p, hipStream_t st) {
    if (p.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_route_scan, dim3(2 * p.n_cells * kExtBins), dim3(256), 0, st, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int per = (p.n_blocks + kXcd - 1) / kXcd;
    hipLaunchKernelGGL(k_route, dim3(per * kXcd), dim3(kShadeBlock), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_spectral(const SpectralParams& p, hipStream_t st) {
    const int npix = p.N < p.WH ? p.N : p.WH;
    const long long n = (long long)npix * p.ngrp;
    if (n <= 0) return hipSuccess;
    if (p.coat_n) hipLaunchKernelGGL(k_spectral<true>, dim3(blocks_for(n, 256)), dim3(256), 0, st, p);
    else hipLaunchKernelGGL(k_spectral<false>, dim3(blocks_for(n, 256)), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_nrc_rows(const NrcRowParams& p, hipStream_t st) {
    if (p.n <= 0) return hipSuccess;
    if (p.coat_n) hipLaunchKernelGGL(k_nrc_rows<true>, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p);
    else hipLaunchKernelGGL(k_nrc_rows<false>, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_resolve(int WH, int nl, int nlp, double inv_spp, const float* acc, const double* w,
                          const double* cmf, double* spectral, double* xyz, hipStream_t st) {
    if (nlp > 128 || nlp % 4 != 0 || nl > nlp) return hipErrorInvalidValue;  // the LDS staging's shape
    hipLaunchKernelGGL(k_resolve, dim3(blocks_for(WH, kResolvePix)), dim3(256), sizeof(float) * kResolvePix * nlp, st,
                       WH, nl, nlp, inv_spp, acc, w, cmf, spectral, xyz);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fold_flags(const int* src, int* const* dst, int n, hipStream_t st) {
    for (int i0 = 0; i0 < n; i0 += kFoldMax) {
        FlagFold f{};
        f.src = src;
        f.n = n - i0 < kFoldMax ? n - i0 : kFoldMax;
        for (int i = 0; i < f.n; ++i) f.dst[i] = dst[i0 + i];
        hipLaunchKernelGGL(k_fold_flags, dim3(1), dim3(64), 0, st, f);
    }
    return hipGetLastError();
}

hipError_t launch_pane(int n, const float4* pc, const float* c, float2* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pane, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, pc, c, out);
    return hipGetLastError();
}

hipError_t launch_glass(int n, const GlassTable& tab, const int4* q, float2* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_glass, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, tab, q, out);
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
