// Binary BVH -> 4-wide BVH, on the device (see bvh_wide.h).
//
// Depths come from pointer jumping over the parent links: after round k every
// node knows its 2^k-th ancestor and the distance to it, so ceil(log2(depth
// cap)) rounds give every node its depth with no per-level launches.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "bvh_wide.h"
#include "layout.h"

namespace sdd {

namespace {

constexpr int kWideBlock = 256;
constexpr int kJumpRounds = 6;  // 2^6 > kMaxBvhDepth
static_assert((1 << kJumpRounds) > kMaxBvhDepth, "pointer jumping must reach the root");

__device__ __forceinline__ bool inner_link(int l) { return l >= 0 && l != kEmptyLink; }

// grid (chunks, cells): the nodes of cell blockIdx.y; marks them as belonging
// to a cell and records the parent of every inner child
__global__ void k_widen_parent(WidenBufs B) {
    const int c = blockIdx.y;
    const int k = blockIdx.x * kWideBlock + threadIdx.x;
    if (k >= B.cell_nodes[c]) return;
    const int n = B.cell_root[c] + k;
    B.dist[0][n] = 0;  // in a cell (the distance is set by k_widen_init)
    for (int i = 0; i < 2; ++i) {
        const int l = (int)B.nodes2[2 * (size_t)n + i].w;
        if (inner_link(l)) B.anc[0][l] = n;
    }
}

__global__ void k_widen_init(WidenBufs B) {
    const int n = blockIdx.x * kWideBlock + threadIdx.x;
    if (n >= B.n2) return;
    if (B.dist[0][n] >= 0) B.dist[0][n] = B.anc[0][n] >= 0 ? 1 : 0;
}

__global__ void k_widen_jump(WidenBufs B, int from) {
    const int n = blockIdx.x * kWideBlock + threadIdx.x;
    if (n >= B.n2) return;
    const int* ai = B.anc[from];
    const int* di = B.dist[from];
    int* ao = B.anc[from ^ 1];
    int* dout = B.dist[from ^ 1];
    const int a = ai[n], d = di[n];
    if (d >= 0 && a >= 0) {
        ao[n] = ai[a];
        dout[n] = d + di[a];
    } else {
        ao[n] = a;
        dout[n] = d;
    }
}

__global__ void k_widen_flag(WidenBufs B, int from) {
    const int n = blockIdx.x * kWideBlock + threadIdx.x;
    if (n > B.n2) return;
    const int d = n < B.n2 ? B.dist[from][n] : -1;
    B.flag[n] = (d >= 0 && (d & 1) == 0) ? 1 : 0;
}

__global__ void k_widen_emit(WidenBufs B, uint4* nodes4) {
    const int n = blockIdx.x * kWideBlock + threadIdx.x;
    if (n >= B.n2 || !B.flag[n]) return;
    uint4 out[4];
    int k = 0;
    for (int i = 0; i < 2; ++i) {
        const uint4 r = B.nodes2[2 * (size_t)n + i];
        const int l = (int)r.w;
        if (l == kEmptyLink) continue;
        if (l < 0) {
            out[k++] = r;  // a leaf stays a child
            continue;
        }
        for (int q = 0; q < 2; ++q) {
            uint4 g = B.nodes2[2 * (size_t)l + q];
            const int gl = (int)g.w;
            if (gl == kEmptyLink) continue;
            if (gl >= 0) g.w = (unsigned)B.idx[gl];  // an even-depth node: its 4-wide index
            out[k++] = g;
        }
    }
    const size_t j = (size_t)B.idx[n];
    for (int i = 0; i < 4; ++i)
        nodes4[4 * j + i] = i < k ? out[i] : make_uint4(0u, 0u, 0u, (unsigned)kEmptyLink);
}

__global__ void k_widen_cells(WidenBufs B, int* cell_root4, int* cell_nodes4) {
    const int c = blockIdx.x * kWideBlock + threadIdx.x;
    if (c >= B.G) return;
    const int r = B.cell_root[c];
    cell_root4[c] = B.idx[r];
    cell_nodes4[c] = B.idx[r + B.cell_nodes[c]] - B.idx[r];
}

int blocks(long long n) { return (int)((n + kWideBlock - 1) / kWideBlock); }

}  // namespace

hipError_t widen_mark(WidenBufs& b, hipStream_t st) {
    if (!b.tmp) return hipcub::DeviceScan::ExclusiveSum(nullptr, b.tmp_bytes, b.flag, b.idx, b.n2 + 1, st);
    hipError_t e = hipMemsetAsync(b.anc[0], 0xff, sizeof(int) * (size_t)b.n2, st);  // -1: no parent
    if (e == hipSuccess) e = hipMemsetAsync(b.dist[0], 0xff, sizeof(int) * (size_t)b.n2, st);  // -1: no cell
    if (e != hipSuccess) return e;
    if (b.max_cell_nodes > 0)
        hipLaunchKernelGGL(k_widen_parent, dim3(blocks(b.max_cell_nodes), b.G), dim3(kWideBlock), 0, st, b);
    hipLaunchKernelGGL(k_widen_init, dim3(blocks(b.n2)), dim3(kWideBlock), 0, st, b);
    int from = 0;
    for (int r = 0; r < kJumpRounds; ++r, from ^= 1)
        hipLaunchKernelGGL(k_widen_jump, dim3(blocks(b.n2)), dim3(kWideBlock), 0, st, b, from);
    hipLaunchKernelGGL(k_widen_flag, dim3(blocks(b.n2 + 1LL)), dim3(kWideBlock), 0, st, b, from);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipcub::DeviceScan::ExclusiveSum(b.tmp, b.tmp_bytes, b.flag, b.idx, b.n2 + 1, st);
}

hipError_t widen_emit(const WidenBufs& b, uint4* nodes4, int* cell_root4, int* cell_nodes4, hipStream_t st) {
    hipLaunchKernelGGL(k_widen_emit, dim3(blocks(b.n2)), dim3(kWideBlock), 0, st, b, nodes4);
    hipLaunchKernelGGL(k_widen_cells, dim3(blocks(b.G)), dim3(kWideBlock), 0, st, b, cell_root4, cell_nodes4);
    return hipGetLastError();
}

}  // namespace sdd
