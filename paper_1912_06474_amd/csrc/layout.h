// Data layout in HBM and kernel parameter blocks, shared by the host runtime
// and the HIP kernels.
//
// Per-subdomain acceleration data (built on the host, one BVH per grid cell):
//   nodes  uint4[4 * n_nodes]   64 B per 4-wide inner node, one 16 B record per child:
//          (lo.x | hi.x << 16, lo.y | hi.y << 16, lo.z | hi.z << 16, link)
//          with 16-bit lattice coordinates: coordinate = base + q * step of
//          the node's cell (cell_q), rounded outward; link >= 0 inner node
//          index, link < 0 leaf starting at triangle ~link, kEmptyLink none
//          (a node's empty records come last).  Nodes of each cell are stored
//          breadth-first (root first).  The builders emit binary nodes (two
//          records, same format), which bvh_wide.hip widens.
//   cell_q float4[2 * n_cells]   lattice of each cell: (base.xyz, 0), (step.xyz, 0)
//   tris   float4[3 * n_refs]   48 B per triangle reference, in leaf order:
//          (v0, prim), (e1, meta), (e2, glass index) with meta = type | last_in_leaf << 2
//          and the compact glass-material index (-1 for other materials)
//   prim_v float4[T][3]          triangle vertices (FP64 shading geometry)
//   prim_info float4[T]          (unit geometric normal, mat word) with
//          mat word = id | type << 24 | emits << 26, id = material index, or
//          the compact glass index for glass
//   pane   float4[n_glass][nlp]  per glass material and wavelength: the pane
//          constants (n^2 - k^2, 2 n k, 1 / n^2, 4 pi k d / lambda)
//   coat   float4[n_glass][Lc][nlp] coating layers of each glass (from the air
//          side of the coated face): (Re N^2, Im N^2, 2 pi d / lambda, 0);
//          coat_n int[n_glass] layers in use (absent when no glass is coated)
//   cell_root int[n_cells]      root node of each cell (always an inner node)
//   planes float[nx+1 + ny+1 + nz+1]  cell boundary planes per axis
//
// Ray queues (segmented by cell, `cap` slots per cell), structure of arrays:
//   qa float4 (o.x, o.y, o.z, t_enter)   qb float4 (d.x, d.y, d.z, path id)
//   qc int2   (excluded prim, t_max bits)
// Path state, indexed by path id within a batch (N paths):
//   ray_o / ray_d D4 (FP64 origin and direction: shading geometry), hit
//   float2 (FP32 t, prim: traversal result), flags u32.  The queue records
//   carry the FP32-rounded ray that traversal tests.
// Path history, indexed [depth][path]: one geometric path carries every
// wavelength, so the per-wavelength factors are not stored per bounce; each
// surface vertex leaves a record that k_spectral replays once per wavelength:
//   vrec int4     (kind | last << 3 | emits << 4 | id << 5, glass cos, glass P_R, NEE g)
//   sh_state int  shadow ray of that vertex: none / visible (| panes << 4) / blocked
//   sh_glass float2[kMaxGlass] (cos, glass index) of the panes the shadow ray crossed
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdd {

constexpr int kTraceBlock = 128;  // threads per traversal workgroup
constexpr int kBvhWidth = 4;      // child records per node the traversal reads
constexpr int kMaxBvhDepth = 40;  // depth cap of the binary builders (a node at the cap becomes a leaf)
// traversal stack entries per lane (total): a 4-wide node pushes at most 3
// siblings, and the widened tree has at most kMaxBvhDepth / 2 + 1 inner levels
constexpr int kStack = 64;
static_assert(3 * (kMaxBvhDepth / 2 + 1) <= kStack, "the traversal stack must hold every pushed sibling");
constexpr int kLdsStack = 8;      // of which the first kLdsStack live in LDS, the rest in HBM
// queue fill counters are kCntStride ints apart (one 128-B line each): the
// appends of every wave in the device are atomics on them, and counters
// sharing a line would serialise all of them on that line
constexpr int kCntStride = 32;
constexpr int kTopNodes = 32;     // breadth-first top nodes (128 records) of the current cell kept in LDS per wave
constexpr int kTraceWaves = 8;    // waves per SIMD the trace kernel is compiled for (registers <= 64)
constexpr int kChunk = 64;        // rays per scheduling chunk (one wave)
constexpr int kPool = 2;          // chunks per work item (one wave refills its lanes from them)
constexpr int kItem = kChunk * kPool;
constexpr int kXcd = 8;           // XCDs of an MI355X; workgroup i runs on XCD i % 8
constexpr int kMaxGlass = 4;      // pane crossings recorded per shadow segment
// bits of the overflow flag the trace kernel raises (atomic OR)
constexpr int kOverflowPanes = 1;  // a shadow segment crossed more than kMaxGlass panes
constexpr int kOverflowQueue = 2;  // a subdomain queue count exceeded its capacity
constexpr int kFoldMax = 32;       // destinations per flag-fold launch
constexpr int kMaxCells = 512;
constexpr int kShadeBlock = 512;

constexpr int kMaxBatch = 1 << 24;  // paths per batch (32-bit path arithmetic in the kernels)

// unsigned division by a launch-invariant divisor d (Hacker's Delight,
// round-up multiplier): n / d = (umulhi(n, m) + n) >> l for n < 2^31
struct FastDiv {
    uint32_t d, m, l;
};
inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return FastDiv{d, (uint32_t)m, l};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) { return (__umulhi(n, f.m) + n) >> f.l; }

// A render traces the pixels of a window of its frame: the paths, the
// accumulator and the logs are numbered over the window's pixels, while the
// camera ray and the random numbers belong to the pixel's place in the frame.
struct PixWindow {
    int fw;      // frame width
    int x0, y0;  // window origin in the frame
    int cw;      // window width; 0: the window is the whole frame
};
// frame pixel index of window pixel pl
__host__ __device__ inline int frame_pixel(const PixWindow& w, int pl) {
    if (w.cw == 0) return pl;
    const int ly = pl / w.cw;
    return (w.y0 + ly) * w.fw + w.x0 + (pl - ly * w.cw);
}

// vector of the per-path ray state (w unused): FP64, 32 B (FP32, 16 B, in the
// SDD_PATH_STATE_F32 measurement build)
#ifdef SDD_PATH_STATE_F32
struct alignas(16) D4 {
    float x, y, z, w;
};
#else
struct alignas(32) D4 {
    double x, y, z, w;
};
#endif

enum : int { kDiffuse = 0, kGlass = 1, kEmitter = 2 };
enum : uint32_t { kAlive = 1u, kCountE = 2u, kTrain = 4u };
enum : int { kShNone = 0, kShVisible = 1, kShBlocked = 2 };  // | pane count << 4 when visible
constexpr int kLastInLeaf = 4;
constexpr int kEmptyLink = 0x7fffffff;  // child slot without a subtree
// vertex record kinds
enum : int { kVNone = 0, kVDiffuse = 1, kVGlassR = 2, kVGlassT = 3, kVEmit = 4 };
constexpr int kVLast = 8, kVEmits = 16, kVIdShift = 5;
constexpr int kMatTypeShift = 24, kMatEmits = 1 << 26, kMatIdMask = (1 << 24) - 1;
constexpr int kLdsPane = 512;     // pane constants staged in LDS when n_glass * nlp fits
// closest-hit rays are routed by (cell, direction quadrant: signs of x and y)
// when cells * kExtBins keys fit the per-block ranking table, so a cell's queue
// holds its rays grouped by direction and a wave's rays tend to traverse alike
// (4 bins measured a little faster than the 8 octants on the room scenes)
constexpr int kExtBins = 4;

enum Stat : int {
    kStatExtRays = 0,
    kStatShadowRays,
    kStatExtVisits,
    kStatShadowVisits,
    kStatNodes,
    kStatTris,
    kStatNodeSteps,  // wave-level steps (counted by the first active lane)
    kStatTriSteps,
    kStatNrcRows,    // (path, wavelength) rows of BF16 render queries (cache vertices only)
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

// rays produced in path order (by camgen / shade), before routing into the
// per-cell queues: record + tag (cell | rank-in-block << 16, or -1), plus
// per-block histograms hist[cell][block] (blocks of kShadeBlock paths)
struct Stage {
    float4* qa;
    float4* qb;
    int2* qc;
    int* tag;
    int* hist;
};

struct TraceParams {
    QueueSet q[2];        // [0] closest-hit rays, [1] shadow rays
    int active[2];        // which of the two sets holds work in this sweep
    long long cap;        // slots per cell
    int n_cells;
    GridParams grid;
    const uint4* nodes;
    const float4* cell_q;
    const float4* tris;
    const int* cell_root;
    const int* cell_nodes;    // inner nodes per cell
    const float4* prim_info;  // (unit geometric normal, mat bits)
    // closest-hit output
    float2* hit;
    // shadow outputs (arrays of the shadow rays' depth)
    int* sh_state;
    float2* sh_glass;
    int* overflow;
    int* gstack;          // spill stack: (kStack - kLdsStack) entries per thread of the grid
    unsigned long long* stats;
    // deferral (the paper's load-balancing rule, Sec. 5): in sweep `sweep` of
    // n_sweeps, a queue with fewer than defer_below rays (0: never) waits for
    // the next sweep when even its worst-placed ray still drains: sweep + 1 +
    // R(cell) <= n_sweeps - 1, R the most cell boundaries a ray can still cross
    int defer_below;
    int sweep, n_sweeps;
};
constexpr int kMaxDeferExtra = 4;  // sweeps per depth a deferral schedule may add

// Radiance-cache rendering.  Training paths ((s * WH + p) % stride == 0,
// s the absolute sample index) are traced in full; every other path ends at
// its first diffuse vertex of depth >= 2, where the cache value is added.
struct NrcPaths {
    int on;
    uint32_t stride;
    float4* cx;  // [N_all] cache vertex position (w = 1 once set)
    float4* cn;  // [N_all] its geometric normal, on the side the ray arrived from
    float4* tx;  // [slots][D] vertices of training paths (position)
    float4* tn;  // [slots][D] (normal)
};

struct ShadeParams {
    int N;                 // paths of this render segment
    int pid_off;           // its first path in the batch (a multiple of kShadeBlock)
    int glass_from, glass_to;  // compact glass index substituted for this render (-1: none)
    int pb, sb;            // pixel and sample of the batch's first path
    FastDiv fwh;           // division by WH
    int W, WH;             // frame width; pixels of the render's window
    PixWindow win;
    int s0;                // first sample index of this call
    const int* s0p;        // if set, read the first sample index here (graph replays)
    int spp_call;
    int depth, max_depth;
    uint2 key;
    // path state
    uint32_t* flags;
    D4* ray_o;
    D4* ray_d;
    float2* hit;
    // history of this depth
    int4* vrec;
    int* sh_state;
    // scene
    const float4* prim_info;
    const float4* prim_v;  // [T][3] vertices
    const float4* pane;    // [n_glass][nlp]
    const float4* coat;    // [n_glass][coat_layers][nlp] coating layers, or null
    const int* coat_n;     // [n_glass] layers per glass, or null (no coatings)
    int coat_layers;
    int n_glass;
    int nl, nlp;
    int light_type;
    double lp0[3], le1[3], le2[3], nL[3];  // light corner, edges, unit front normal
    double light_area;
    GridParams grid;
    int n_cells;
    Stage se, ss;          // next closest-hit rays, shadow rays
    int ext_bins;          // direction bins per cell of the closest-hit routing (1 or kExtBins)
    int n_blocks;          // histogram stride (blocks per batch)
    int* hit_log;
    unsigned long long* stats;
    NrcPaths nrc;
};

struct CamParams {
    int N;                 // paths of this render segment
    int pid_off;           // its first path in the batch (a multiple of kShadeBlock)
    int pb, sb;
    FastDiv fwh;
    int W, H, WH;          // frame size (camera); pixels of the render's window
    PixWindow win;
    int s0;
    const int* s0p;        // if set, read the first sample index here (graph replays)
    uint2 key;
    int ortho;
    double eye[3], fwd[3], right[3], up[3];
    double tan_half, aspect, ortho_half_h;
    uint32_t* flags;
    D4* ray_o;
    D4* ray_d;
    float2* hit;
    GridParams grid;
    int n_cells;
    Stage se;
    int ext_bins;          // direction bins per cell of the closest-hit routing (1 or kExtBins)
    int n_blocks;
    unsigned long long* stats;
    NrcPaths nrc;
};

// scan of the block histograms and scatter of staged rays into the queues
struct RouteParams {
    int N;
    int n_blocks;
    int n_cells;
    long long cap;
    int active[2];
    int nbin[2];           // routing keys per cell (key = cell * nbin + bin; rays of a cell ordered by bin)
    Stage st[2];
    float4* qa[2];
    float4* qb[2];
    int2* qc[2];
    int* cnt[2];           // per-cell totals of the routed queues (zero on entry; the scan adds)
    int* ktot[2];          // per-key totals, [n_cells * nbin]
    int count[2];          // add the routed rays of this kind to the ray statistics
    unsigned long long* stats;
};

// the glass tables of a scene, as the debug entry point sees them
// dst[i] |= *src for i < n: a call's overflow flag folded into its renders' flags
struct FlagFold {
    const int* src;
    int* dst[kFoldMax];
    int n;
};

struct GlassTable {
    const float4* pane;
    const float4* coat;
    const int* coat_n;
    int coat_layers;
    int nlp;
};

// replay of the path histories, one thread per (pixel, wavelength)
struct SpectralParams {
    int N;                 // paths of this render segment
    int pid_off;           // its first path in the batch
    int N_all;             // paths in the batch (stride of the history arrays)
    int glass_from, glass_to;  // compact glass index substituted for this render (-1: none)
    int pb, sb;
    FastDiv fwh;
    int ngrp;              // wavelength groups of 4 (nlp / 4)
    FastDiv fgrp;
    int WH;
    int s0, spp_call;
    const int* s0p;        // if set, read the first sample index here (graph replays)
    int max_depth;
    const int4* vrec;      // [D][N]
    const int* sh_state;   // [D][N]
    const float2* sh_glass;// [D][N][kMaxGlass]
    const float4* pane;    // [n_glass][nlp]
    const float4* coat;    // [n_glass][coat_layers][nlp] coating layers, or null
    const int* coat_n;     // [n_glass] layers per glass, or null (no coatings)
    int coat_layers;
    int n_glass;
    int n_mats;
    const float* rho;      // [M][nlp]
    const float* le;
    int nl, nlp;
    int light_mat;
    float* acc;            // [WH][nlp]
    int* shadow_log;
    const float* lhat;     // [N_all / 16][nlp][16] cache values at the paths' cache vertices, or null
};

// training rows of the radiance cache from the training paths of one batch
// segment: one row per diffuse vertex of depth >= 2 that continued the path
struct NrcRowParams {
    int n;                 // training paths in the segment
    long long j0;          // first training slot (call-wide numbering)
    long long r;           // call path index of slot j: r + j * stride
    uint32_t stride;
    long long q0;          // call path index of the segment's first path
    int pid_off;           // batch position of that path
    int N_all;
    int WH, s0;            // pixels of the render's window
    PixWindow win;
    uint2 key;
    int max_depth, nl, nlp, n_glass, n_mats;
    int glass_from, glass_to;
    const int4* vrec;
    const int* sh_state;
    const float2* sh_glass;
    const float4* pane;
    const float4* coat;
    const int* coat_n;
    int coat_layers;
    const float* rho;
    const float* le;
    int light_mat;
    const float* lam_nm;   // [nl]
    const float4* tx;      // [slots][D]
    const float4* tn;
    float4* rows;          // [slots][D - 1][2]: (x, lambda nm), (n, target)
    int* row_ok;           // [slots][D - 1]
};

}  // namespace sdd
