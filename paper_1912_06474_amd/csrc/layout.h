// Data layout in HBM and kernel parameter blocks, shared by the host runtime
// and the HIP kernels.
//
// Per-subdomain acceleration data (built on the host, one BVH per grid cell):
//   nodes  float4[4 * n_nodes]  64 B per inner node (both child boxes + links):
//          n0 = (c0.lo.x, c0.hi.x, c0.lo.y, c0.hi.y)
//          n1 = (c1.lo.x, c1.hi.x, c1.lo.y, c1.hi.y)
//          n2 = (c0.lo.z, c0.hi.z, c1.lo.z, c1.hi.z)
//          n3 = (link0, link1, 0, 0) as int: link >= 0 inner node index,
//               link < 0 leaf starting at triangle ~link
//          Nodes of each cell are stored breadth-first (root first).
//   tris   float4[3 * n_refs]   48 B per triangle reference, in leaf order:
//          (v0, prim), (e1, meta), (e2, mat) with meta = type | last_in_leaf << 2
//   cell_root int[n_cells]      root node of each cell (always an inner node)
//   planes float[nx+1 + ny+1 + nz+1]  cell boundary planes per axis
//
// Ray queues (segmented by cell, `cap` slots per cell), structure of arrays:
//   qa float4 (o.x, o.y, o.z, t_enter)   qb float4 (d.x, d.y, d.z, path id)
//   qc int2   (excluded prim, t_max bits)
// Path state, indexed by path id within a batch (N paths):
//   ray_o / ray_d float4, hit float2 (t, prim), flags u32, nee_g float,
//   sh_state / sh_cnt int, sh_glass float2[4 per path] (cos, mat),
//   beta / Lp float[n_lambda_pad][N] (wavelength-major, coalesced per lambda).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdd {

constexpr int kTraceBlock = 128;  // threads per traversal workgroup
constexpr int kStack = 40;        // traversal stack entries per lane (total)
constexpr int kLdsStack = 16;     // of which the first kLdsStack live in LDS, the rest in HBM
constexpr int kMaxBvhDepth = kStack;  // the builder never exceeds the stack
constexpr int kChunk = 64;        // rays per scheduling chunk (one wave)
constexpr int kXcd = 8;           // XCDs of an MI355X; workgroup i runs on XCD i % 8
constexpr int kMaxGlass = 4;      // pane crossings recorded per shadow segment
constexpr int kMaxCells = 512;
constexpr int kShadeBlock = 256;

enum : int { kDiffuse = 0, kGlass = 1, kEmitter = 2 };
enum : uint32_t { kAlive = 1u, kCountE = 2u };
enum : int { kShNone = 0, kShVisible = 1, kShBlocked = 2 };
constexpr int kLastInLeaf = 4;

enum Stat : int {
    kStatExtRays = 0,
    kStatShadowRays,
    kStatExtVisits,
    kStatShadowVisits,
    kStatNodes,
    kStatTris,
    kStatCount
};

struct GridParams {
    const float* planes;  // [nx+1][ny+1][nz+1] concatenated
    int nx, ny, nz;
    int off_y, off_z;     // offsets of the y / z planes in `planes`
    float lo[3], hi[3];   // grid box (= first / last planes)
    float inv_h[3];       // cells per metre, for the initial guess of point location
};

// one segmented queue pair (input of this sweep, output for the next)
struct QueueSet {
    const float4* qa_in;
    const float4* qb_in;
    const int2* qc_in;
    const int* cnt_in;
    float4* qa_out;
    float4* qb_out;
    int2* qc_out;
    int* cnt_out;
};

struct TraceParams {
    QueueSet q[2];        // [0] closest-hit rays, [1] shadow rays
    int active[2];        // which of the two sets holds work in this sweep
    long long cap;        // slots per cell
    int n_cells;
    GridParams grid;
    const float4* nodes;
    const float4* tris;
    const int* cell_root;
    const float4* prim_info;  // (unit geometric normal, mat bits)
    // closest-hit output
    float2* hit;
    // shadow outputs
    int* sh_state;
    int* sh_cnt;
    float2* sh_glass;
    int* overflow;
    int* gstack;          // spill stack: (kStack - kLdsStack) entries per thread of the grid
    unsigned long long* stats;
};

struct ShadeParams {
    int N;                 // paths in this batch
    long long g0;          // first global path index of the batch
    int W, WH;
    int s0;                // first sample index of this call
    int spp_call;
    int depth, max_depth;
    int final_pass;        // 1: only resolve the pending shadow rays
    uint2 key;
    // path state
    uint32_t* flags;
    float4* ray_o;
    float4* ray_d;
    float2* hit;
    float* beta;
    float* Lp;
    float* nee_g;
    int* sh_state;
    int* sh_cnt;
    const float2* sh_glass;
    // scene
    const float4* prim_info;
    const int* mat_type;
    const int* mat_has_le;
    const float* mat_thick;
    const float* rho;      // [M][nlp]
    const float* mn;
    const float* mk;
    const float* le;
    const float* lambda_nm;
    int nl, nlp;
    int light_type;
    float lp0[3], le1[3], le2[3], nL[3];
    float light_area;
    int light_mat;
    GridParams grid;
    int n_cells;
    // queues written
    float4* eqa;
    float4* eqb;
    int2* eqc;
    int* ecnt;
    float4* sqa;
    float4* sqb;
    int2* sqc;
    int* scnt;
    long long cap;
    int* hit_log;
    int* shadow_log;
    unsigned long long* stats;
};

struct CamParams {
    int N;
    long long g0;
    int W, H, WH;
    int s0;
    uint2 key;
    int ortho;
    float eye[3], fwd[3], right[3], up[3];
    float tan_half, aspect, ortho_half_h;
    int nlp;
    uint32_t* flags;
    float4* ray_o;
    float4* ray_d;
    float2* hit;
    float* beta;
    float* Lp;
    int* sh_state;
    GridParams grid;
    int n_cells;
    float4* eqa;
    float4* eqb;
    int2* eqc;
    int* ecnt;
    long long cap;
    unsigned long long* stats;
};

}  // namespace sdd
