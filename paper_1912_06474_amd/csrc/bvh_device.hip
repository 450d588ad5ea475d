// Device build of the subdomain references and per-subdomain BVHs: a linear
// BVH per cell (Morton order of the reference centroids, hierarchy from the
// longest common prefixes of neighbouring codes, Karras, HPG 2012), with
// bottom-up boxes, emitted in the same layout as the host SAH builder
// (layout.h): breadth-first inner nodes per cell with quantised children,
// triangle records in leaf order, per-cell lattice.  Closest hits do not
// depend on the BVH, so both builders give the same images.
//
// Steps (one stream, no host round trip except the reference total):
//   k_ref_count / scan / k_ref_emit  references of every triangle in every
//                                    cell its padded box overlaps (as the host)
//   radix sort by (cell, Morton code)
//   k_cell_start                     first sorted reference of every cell
//   k_lbvh_nodes                     children of every internal node
//   k_lbvh_boxes                     boxes bottom-up (the second child to
//                                    arrive at a node forms its union)
//   k_emit_cell                      one workgroup per cell: lattice, then the
//                                    breadth-first walk that turns small or
//                                    deep subtrees into leaves and writes nodes
//   k_emit_tris                      triangle records, last-in-leaf flags
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "bvh_device.h"
#include "layout.h"

namespace sdd {

namespace {

__device__ __forceinline__ float down_f(double v) {
    float f = (float)v;
    if ((double)f > v) f = nextafterf(f, -INFINITY);
    return f;
}
__device__ __forceinline__ float up_f(double v) {
    float f = (float)v;
    if ((double)f < v) f = nextafterf(f, INFINITY);
    return f;
}

// cells [i0, i1] of one axis overlapped by [lo, hi]: i0 = number of interior
// planes below lo, i1 = number of interior planes at or below hi
__device__ __forceinline__ void axis_range(const float* pl, int n, double lo, double hi, int& i0, int& i1) {
    i0 = 0;
    while (i0 < n - 1 && (double)pl[i0 + 1] < lo) ++i0;
    i1 = n - 1;
    while (i1 > 0 && (double)pl[i1] > hi) --i1;
}

__device__ __forceinline__ void tri_box(const float4* prim_v, int i, double lo[3], double hi[3]) {
    for (int a = 0; a < 3; ++a) {
        lo[a] = INFINITY;
        hi[a] = -INFINITY;
    }
    for (int j = 0; j < 3; ++j) {
        const float4 v = prim_v[3 * (size_t)i + j];
        const double p[3] = {v.x, v.y, v.z};
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], p[a]);
            hi[a] = fmax(hi[a], p[a]);
        }
    }
}

__global__ void k_ref_count(DevBuildArgs A, int* count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.T) return;
    double lo[3], hi[3];
    tri_box(A.prim_v, i, lo, hi);
    const float* pl[3] = {A.planes, A.planes + A.n[0] + 1, A.planes + A.n[0] + 1 + A.n[1] + 1};
    int c = 1;
    for (int a = 0; a < 3; ++a) {
        int i0, i1;
        axis_range(pl[a], A.n[a], lo[a] - A.cpad, hi[a] + A.cpad, i0, i1);
        c *= max(0, i1 - i0 + 1);
    }
    count[i] = c;
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_ref_emit(DevBuildArgs A, const int* offset, float4* ref_lo, float4* ref_hi,
                           unsigned long long* key, int* val) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.T) return;
    double lo[3], hi[3];
    tri_box(A.prim_v, i, lo, hi);
    const float* pl[3] = {A.planes, A.planes + A.n[0] + 1, A.planes + A.n[0] + 1 + A.n[1] + 1};
    int r0[3], r1[3];
    for (int a = 0; a < 3; ++a) axis_range(pl[a], A.n[a], lo[a] - A.cpad, hi[a] + A.cpad, r0[a], r1[a]);
    int k = offset[i];
    for (int iz = r0[2]; iz <= r1[2]; ++iz)
        for (int iy = r0[1]; iy <= r1[1]; ++iy)
            for (int ix = r0[0]; ix <= r1[0]; ++ix) {
                const int ci[3] = {ix, iy, iz};
                float bl[3], bh[3];
                uint32_t code = 0;
                for (int a = 0; a < 3; ++a) {
                    const double clo = (double)pl[a][ci[a]] - A.cpad, chi = (double)pl[a][ci[a] + 1] + A.cpad;
                    bl[a] = down_f(fmax(lo[a], clo) - A.npad);
                    bh[a] = up_f(fmin(hi[a], chi) + A.npad);
                    // Morton coordinate of the centroid within the padded cell
                    const double cen = 0.5 * ((double)bl[a] + (double)bh[a]);
                    const double u = (cen - clo) / (chi - clo);
                    const uint32_t q = (uint32_t)fmin(1023.0, fmax(0.0, u * 1024.0));
                    code |= spread10(q) << (2 - a);
                }
                const int cell = ix + A.n[0] * (iy + A.n[1] * iz);
                ref_lo[k] = make_float4(bl[0], bl[1], bl[2], __int_as_float(i));
                ref_hi[k] = make_float4(bh[0], bh[1], bh[2], __int_as_float(cell));
                key[k] = ((unsigned long long)cell << 30) | code;
                val[k] = k;
                ++k;
            }
}

// first sorted reference of each cell (cell_start[G] = total)
__global__ void k_cell_start(int G, long long total, const unsigned long long* key, int* cell_start) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > G) return;
    long long a = 0, b = total;  // first index with key >> 30 >= c
    while (a < b) {
        const long long m = (a + b) >> 1;
        if ((long long)(key[m] >> 30) < c) a = m + 1;
        else b = m;
    }
    cell_start[c] = (int)a;
}

// common prefix length of sorted codes i and j of one cell (index tie-break)
__device__ __forceinline__ int delta(const unsigned long long* key, int s, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    const uint32_t a = (uint32_t)(key[s + i] & 0x3fffffffu), b = (uint32_t)(key[s + j] & 0x3fffffffu);
    return a != b ? __clz(a ^ b) : 32 + __clz((uint32_t)(i ^ j));
}

// internal node j (sorted position j, not the last of its cell) of cell c:
// child links >= 0 are internal nodes, < 0 encode leaf position -(p + 1)
__global__ void k_lbvh_nodes(long long total, const unsigned long long* key, const int* cell_start, int2* child,
                             int2* range, int* parent) {
    const long long jj = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= total) return;
    const int j = (int)jj;
    const int c = (int)(key[j] >> 30);
    const int s = cell_start[c], n = cell_start[c + 1] - s;
    const int i = j - s;
    if (i >= n - 1) return;
    // direction and extent of the range (Karras 2012)
    const int d = delta(key, s, n, i, i + 1) - delta(key, s, n, i, i - 1) >= 0 ? 1 : -1;
    const int dmin = delta(key, s, n, i, i - d);
    int lmax = 2;
    while (delta(key, s, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(key, s, n, i, i + (l + t) * d) > dmin) l += t;
    const int jo = i + l * d;
    const int dnode = delta(key, s, n, i, jo);
    int sp = 0;
    for (int t = (l + 1) >> 1;; t = (t + 1) >> 1) {
        if (delta(key, s, n, i, i + (sp + t) * d) > dnode) sp += t;
        if (t == 1) break;
    }
    const int gamma = i + sp * d + min(d, 0);
    const int first = min(i, jo), last = max(i, jo);
    const int lc = first == gamma ? -(s + gamma + 1) : s + gamma;
    const int rc = last == gamma + 1 ? -(s + gamma + 1 + 1) : s + gamma + 1;
    child[j] = make_int2(lc, rc);
    range[j] = make_int2(s + first, s + last);
    // parents: internal nodes in parent[0 .. total), leaves in parent[total ..)
    parent[lc >= 0 ? lc : total + (-lc - 1)] = j;
    parent[rc >= 0 ? rc : total + (-rc - 1)] = j;
}

__global__ void k_lbvh_boxes(long long total, const unsigned long long* key, const int* cell_start, const int* val,
                             const float4* ref_lo, const float4* ref_hi, const int2* child, const int* parent,
                             int* arrive, float4* box_lo, float4* box_hi, int* error) {
    const long long jj = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= total) return;
    const int j = (int)jj;
    const int c = (int)(key[j] >> 30);
    const int s = cell_start[c], n = cell_start[c + 1] - s;
    if (n < 2) return;
    int p = parent[total + j];
    // a binary radix tree over n leaves is at most n - 1 levels deep
    for (int steps = 0;; ++steps) {
        if (p < s || p >= s + n - 1 || steps >= n) {
            atomicExch(error, 1);  // never expected: the hierarchy is inconsistent
            return;
        }
        __threadfence();
        if (atomicAdd(&arrive[p], 1) == 0) return;  // the sibling subtree is not done yet
        __threadfence();
        const int2 ch = child[p];
        float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f), hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
        const int cc[2] = {ch.x, ch.y};
        for (int k = 0; k < 2; ++k) {
            float4 a, b;
            if (cc[k] >= 0) {
                a = box_lo[cc[k]];
                b = box_hi[cc[k]];
            } else {
                const int r = val[-cc[k] - 1];
                a = ref_lo[r];
                b = ref_hi[r];
            }
            lo = make_float4(fminf(lo.x, a.x), fminf(lo.y, a.y), fminf(lo.z, a.z), 0.0f);
            hi = make_float4(fmaxf(hi.x, b.x), fmaxf(hi.y, b.y), fmaxf(hi.z, b.z), 0.0f);
        }
        box_lo[p] = lo;
        box_hi[p] = hi;
        if (p == s) return;  // root of the cell
        p = parent[p];
    }
}

// per-cell lattice: fmaf(q, step, base) for q in [0, 65535] covers [lo, hi]
__device__ __forceinline__ void lattice(float lo, float hi, float& base, float& step) {
    base = lo;
    if (!(hi > lo)) {
        step = 0.0f;
        return;
    }
    step = up_f(((double)hi - (double)lo) / 65535.0);
    while (fmaf(65535.0f, step, base) < hi) step = nextafterf(step, INFINITY);
}
__device__ __forceinline__ uint32_t quant_lo(float v, float base, float step) {
    if (!(step > 0.0f)) return 0;
    const double q = floor(((double)v - (double)base) / (double)step);
    int qi = (int)fmin(65535.0, fmax(0.0, q));
    while (qi > 0 && fmaf((float)qi, step, base) > v) --qi;
    return (uint32_t)qi;
}
__device__ __forceinline__ uint32_t quant_hi(float v, float base, float step) {
    if (!(step > 0.0f)) return 0;
    const double q = ceil(((double)v - (double)base) / (double)step);
    int qi = (int)fmin(65535.0, fmax(0.0, q));
    while (qi < 65535 && fmaf((float)qi, step, base) < v) ++qi;
    return (uint32_t)qi;
}

constexpr int kEmitBlock = 256;

// One workgroup per cell: breadth-first walk over the cell's LBVH.  A child
// becomes a leaf (its whole sorted range) if it holds at most leaf_max
// references or sits at the depth cap; otherwise it becomes the next
// breadth-first inner node.  Node k of cell c is stored at node_base[c] + k.
__global__ __launch_bounds__(kEmitBlock) void k_emit_cell(DevBuildArgs A, const int* cell_start, const int* val,
                                                          const float4* ref_lo, const float4* ref_hi,
                                                          const int2* child, const int2* range,
                                                          const float4* box_lo, const float4* box_hi,
                                                          int* level_a, int* level_b, int* last_flag, uint4* nodes,
                                                          float4* cell_q, int* cell_root, int* cell_nodes,
                                                          int* max_depth, int* error) {
    __shared__ int s_scan[kEmitBlock];
    __shared__ float s_q[6];
    const int c = blockIdx.x;
    const int s = cell_start[c], n = cell_start[c + 1] - s;
    const int base = s + c;  // n + 1 node slots per cell
    if (threadIdx.x == 0) {
        float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        if (n == 1) {
            const float4 a = ref_lo[val[s]], b = ref_hi[val[s]];
            lo[0] = a.x; lo[1] = a.y; lo[2] = a.z;
            hi[0] = b.x; hi[1] = b.y; hi[2] = b.z;
        } else if (n >= 2) {
            const float4 a = box_lo[s], b = box_hi[s];
            lo[0] = a.x; lo[1] = a.y; lo[2] = a.z;
            hi[0] = b.x; hi[1] = b.y; hi[2] = b.z;
        }
        for (int a = 0; a < 3; ++a) {
            float qb = 0.0f, qs = 0.0f;
            if (n > 0) lattice(lo[a], hi[a], qb, qs);
            s_q[a] = qb;
            s_q[3 + a] = qs;
        }
        cell_q[2 * c] = make_float4(s_q[0], s_q[1], s_q[2], 0.0f);
        cell_q[2 * c + 1] = make_float4(s_q[3], s_q[4], s_q[5], 0.0f);
        cell_root[c] = base;
    }
    __syncthreads();
    const float qb[3] = {s_q[0], s_q[1], s_q[2]}, qs[3] = {s_q[3], s_q[4], s_q[5]};
    auto quant = [&](float4 lo, float4 hi, int link, uint4& out) {
        const float l[3] = {lo.x, lo.y, lo.z}, h[3] = {hi.x, hi.y, hi.z};
        uint32_t w[3];
        for (int a = 0; a < 3; ++a)
            w[a] = link == kEmptyLink ? 0u : (quant_lo(l[a], qb[a], qs[a]) | (quant_hi(h[a], qb[a], qs[a]) << 16));
        out = make_uint4(w[0], w[1], w[2], (uint32_t)link);
    };
    if (n <= A.leaf_max) {
        // the root is a leaf (or the cell is empty): one wrapper node
        if (threadIdx.x == 0) {
            uint4 c0, c1;
            if (n > 0) {
                float4 lo, hi;
                if (n >= 2) {
                    lo = box_lo[s];
                    hi = box_hi[s];
                } else {
                    lo = ref_lo[val[s]];
                    hi = ref_hi[val[s]];
                }
                quant(lo, hi, ~s, c0);
                last_flag[s + n - 1] = 1;
            } else {
                quant(make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0), kEmptyLink, c0);
            }
            quant(make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0), kEmptyLink, c1);
            nodes[2 * (size_t)base] = c0;
            nodes[2 * (size_t)base + 1] = c1;
            cell_nodes[c] = 1;
        }
        return;
    }
    // level lists hold internal node ids (sorted positions); level 0 = root s
    int* cur = level_a + s;
    int* nxt = level_b + s;
    if (threadIdx.x == 0) cur[0] = s;
    int n_cur = 1, first_k = 0, depth = 0;
    __syncthreads();
    while (n_cur > 0) {
        int n_next = 0;
        const int next_k0 = first_k + n_cur;  // breadth-first index of the next level's first node
        for (int b0 = 0; b0 < n_cur; b0 += kEmitBlock) {
            const int t = b0 + (int)threadIdx.x;
            int node = -1, links[2] = {0, 0}, inner[2] = {0, 0};
            if (t < n_cur && first_k + t < n - 1) {
                node = cur[t];
                const int2 ch = child[node];
                const int cc[2] = {ch.x, ch.y};
                for (int k = 0; k < 2; ++k) {
                    if (cc[k] >= 0) {
                        const int2 rg = range[cc[k]];
                        inner[k] = (rg.y - rg.x + 1 > A.leaf_max) && (depth + 1 < kMaxBvhDepth - 1);
                    }
                }
            }
            // block-wide exclusive scan of inner-child counts
            const int mine = inner[0] + inner[1];
            s_scan[threadIdx.x] = mine;
            __syncthreads();
            for (int o = 1; o < kEmitBlock; o <<= 1) {
                const int v = threadIdx.x >= (unsigned)o ? s_scan[threadIdx.x - o] : 0;
                __syncthreads();
                s_scan[threadIdx.x] += v;
                __syncthreads();
            }
            const int excl = s_scan[threadIdx.x] - mine;
            const int chunk_total = s_scan[kEmitBlock - 1];
            if (node >= 0) {
                const int2 ch = child[node];
                const int cc[2] = {ch.x, ch.y};
                int slot = n_next + excl;
                uint4 rec[2];
                for (int k = 0; k < 2; ++k) {
                    float4 lo, hi;
                    if (cc[k] >= 0) {
                        lo = box_lo[cc[k]];
                        hi = box_hi[cc[k]];
                        if (inner[k]) {
                            // a cell has at most n - 1 inner nodes
                            if (next_k0 + slot >= n - 1) {
                                atomicExch(error, 2);
                                links[k] = kEmptyLink;
                            } else {
                                nxt[slot] = cc[k];
                                links[k] = base + next_k0 + slot;
                                ++slot;
                            }
                        } else {
                            const int2 rg = range[cc[k]];
                            links[k] = ~rg.x;
                            last_flag[rg.y] = 1;
                        }
                    } else {
                        const int p = -cc[k] - 1;
                        lo = ref_lo[val[p]];
                        hi = ref_hi[val[p]];
                        links[k] = ~p;
                        last_flag[p] = 1;
                    }
                    quant(lo, hi, links[k], rec[k]);
                }
                const size_t at = 2 * (size_t)(base + first_k + t);
                nodes[at] = rec[0];
                nodes[at + 1] = rec[1];
            }
            n_next = min(n_next + chunk_total, n - 1 - next_k0);
            __syncthreads();
        }
        first_k += n_cur;
        n_cur = n_next;
        int* tmp = cur;
        cur = nxt;
        nxt = tmp;
        ++depth;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cell_nodes[c] = first_k;
        atomicMax(max_depth, depth);
    }
}

__global__ void k_emit_tris(long long total, const int* val, const float4* ref_lo, const float4* prim_v,
                            const float4* prim_info, const int* last_flag, float4* tris) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= total) return;
    const int prim = __float_as_int(ref_lo[val[p]].w);
    const float4 v0 = prim_v[3 * (size_t)prim], v1 = prim_v[3 * (size_t)prim + 1], v2 = prim_v[3 * (size_t)prim + 2];
    const int word = __float_as_int(prim_info[prim].w);
    const int typ = (word >> kMatTypeShift) & 3;
    const int gi = typ == kGlass ? (word & kMatIdMask) : -1;
    const int meta = typ | (last_flag[p] ? kLastInLeaf : 0);
    tris[3 * p] = make_float4(v0.x, v0.y, v0.z, __int_as_float(prim));
    tris[3 * p + 1] = make_float4((float)((double)v1.x - v0.x), (float)((double)v1.y - v0.y),
                                  (float)((double)v1.z - v0.z), __int_as_float(meta));
    tris[3 * p + 2] = make_float4((float)((double)v2.x - v0.x), (float)((double)v2.y - v0.y),
                                  (float)((double)v2.z - v0.z), __int_as_float(gi));
}

__global__ void k_fill(int* p, long long n, int v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t dev_count_refs(const DevBuildArgs& a, int* count, int* offset, void* tmp, size_t& tmp_bytes,
                          hipStream_t st) {
    if (!tmp) return hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, count, offset, a.T, st);
    hipLaunchKernelGGL(k_ref_count, dim3(nblk(a.T, 256)), dim3(256), 0, st, a, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, count, offset, a.T, st);
}

hipError_t dev_sort_bytes(long long total, size_t& tmp_bytes) {
    return hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, (const unsigned long long*)nullptr,
                                              (unsigned long long*)nullptr, (const int*)nullptr, (int*)nullptr,
                                              (int)total, 0, 64, (hipStream_t)0);
}

hipError_t dev_build(const DevBuildArgs& a, const DevBuildBufs& b, hipStream_t st) {
    const long long total = b.total;
    hipLaunchKernelGGL(k_ref_emit, dim3(nblk(a.T, 256)), dim3(256), 0, st, a, b.offset, b.ref_lo, b.ref_hi, b.key_in,
                       b.val_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int end_bit = 30;
    while ((1LL << (end_bit - 30)) <= a.G) ++end_bit;
    size_t tb = b.tmp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(b.tmp, tb, b.key_in, b.key, b.val_in, b.val, (int)total, 0, end_bit, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_start, dim3(nblk(a.G + 1, 256)), dim3(256), 0, st, a.G, total, b.key, b.cell_start);
    hipLaunchKernelGGL(k_fill, dim3(nblk(total, 256)), dim3(256), 0, st, b.arrive, total, 0);
    hipLaunchKernelGGL(k_fill, dim3(nblk(total, 256)), dim3(256), 0, st, b.last_flag, total, 0);
    hipLaunchKernelGGL(k_fill, dim3(nblk(2 * total, 256)), dim3(256), 0, st, b.parent, 2 * total, -1);
    hipLaunchKernelGGL(k_lbvh_nodes, dim3(nblk(total, 256)), dim3(256), 0, st, total, b.key, b.cell_start, b.child,
                       b.range, b.parent);
    hipLaunchKernelGGL(k_lbvh_boxes, dim3(nblk(total, 256)), dim3(256), 0, st, total, b.key, b.cell_start, b.val,
                       b.ref_lo, b.ref_hi, b.child, b.parent, b.arrive, b.box_lo, b.box_hi, b.error);
    hipLaunchKernelGGL(k_emit_cell, dim3(a.G), dim3(kEmitBlock), 0, st, a, b.cell_start, b.val, b.ref_lo, b.ref_hi,
                       b.child, b.range, b.box_lo, b.box_hi, b.level_a, b.level_b, b.last_flag, b.nodes, b.cell_q,
                       b.cell_root, b.cell_nodes, b.max_depth, b.error);
    hipLaunchKernelGGL(k_emit_tris, dim3(nblk(total, 256)), dim3(256), 0, st, total, b.val, b.ref_lo, a.prim_v,
                       a.prim_info, b.last_flag, b.tris);
    return hipGetLastError();
}

}  // namespace sdd
