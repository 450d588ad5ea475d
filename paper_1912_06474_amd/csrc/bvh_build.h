// Host builder of the subdomain grid and the per-subdomain BVHs.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sdd {

struct HostF4 {
    float x, y, z, w;
};

struct GridBvh {
    int nx = 1, ny = 1, nz = 1;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    std::vector<float> planes;      // nx+1, ny+1, nz+1 planes (float)
    std::vector<uint32_t> nodes;    // 8 words per node: two quantised children (layout.h)
    std::vector<HostF4> cell_q;     // 2 per cell: quantisation base, step (layout.h)
    std::vector<HostF4> tris;       // 3 per reference
    std::vector<int32_t> cell_root; // per cell
    std::vector<int32_t> cell_refs; // references per cell
    std::vector<int32_t> cell_nodes;// nodes per cell
    int64_t n_refs = 0;
    int max_depth = 0;
};

struct BuildInput {
    const float* verts;       // [V][3]
    int n_verts;
    const int32_t* tris;      // [T][3]
    int n_tris;
    const int32_t* tri_mat;   // [T]
    const int32_t* mat_type;  // [M]
    const int32_t* glass_of;  // [M] compact glass index or -1 (may be null: no glass)
    const int32_t* mat_emits; // [M] nonzero if the material emits (may be null)
    int nx, ny, nz;
    int leaf_max;
    int sah_bins;
};

// Returns false and fills err on failure.
bool build_grid_bvh(const BuildInput& in, GridBvh& out, std::string& err);

// Only the subdomain grid (planes, lo, hi) and the scene extent, whose
// fractions pad references (1e-4) and child boxes (2e-6).
bool grid_planes(const BuildInput& in, GridBvh& out, double& ext, std::string& err);

// Unit geometric normal (v1 - v0) x (v2 - v0) of every triangle, in double
// then rounded, with the material word (layout.h) in w (as int bits).
void triangle_info(const BuildInput& in, std::vector<HostF4>& info);

}  // namespace sdd
