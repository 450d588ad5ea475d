// Device build of the subdomain grid's references and per-cell BVHs
// (bvh_device.hip); the host computes the grid planes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace sdd {

struct DevBuildArgs {
    int T;                    // triangles
    const float4* prim_v;     // [T][3] vertices
    const float4* prim_info;  // [T] (normal, material word)
    const float* planes;      // device: nx+1, ny+1, nz+1 planes
    int n[3];                 // cells per axis
    int G;                    // cells
    double cpad, npad;        // reference and child-box padding (m)
    int leaf_max;
};

struct DevBuildBufs {
    long long total;          // references
    int* count;               // [T]
    int* offset;              // [T]
    float4* ref_lo;           // [total] (box lo, prim bits)
    float4* ref_hi;           // [total] (box hi, cell bits)
    unsigned long long* key_in;  // [total] cell << 30 | Morton code
    unsigned long long* key;     // [total] sorted
    int* val_in;              // [total]
    int* val;                 // [total] sorted reference index
    int* cell_start;          // [G + 1]
    int2* child;              // [total] internal node children
    int2* range;              // [total] internal node sorted range
    int* parent;              // [2 total] parents of internal nodes, then of leaves
    int* arrive;              // [total]
    float4* box_lo;           // [total]
    float4* box_hi;           // [total]
    int* level_a;             // [total]
    int* level_b;             // [total]
    int* last_flag;           // [total]
    uint4* nodes;             // [2 (total + G)] output nodes (n + 1 slots per cell)
    float4* cell_q;           // [2 G]
    int* cell_root;           // [G]
    int* cell_nodes;          // [G]
    int* max_depth;           // [1]
    int* error;               // [1] non-zero if the hierarchy came out inconsistent
    float4* tris;             // [3 total]
    void* tmp;                // scan / sort scratch
    size_t tmp_bytes;
};

// With tmp == nullptr: only sets tmp_bytes for the scan.  Otherwise counts the
// references of every triangle and their exclusive prefix.
hipError_t dev_count_refs(const DevBuildArgs& a, int* count, int* offset, void* tmp, size_t& tmp_bytes,
                          hipStream_t st);
// scratch bytes of the reference sort
hipError_t dev_sort_bytes(long long total, size_t& tmp_bytes);
// everything after the count: references, sort, hierarchy, boxes, layout
hipError_t dev_build(const DevBuildArgs& a, const DevBuildBufs& b, hipStream_t st);

}  // namespace sdd
