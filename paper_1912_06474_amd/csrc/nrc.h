// Learned radiance cache: device state and kernel launchers (nrc.hip).
//
// Network: input 64 = multiresolution hash encoding of the position (16
// levels x 2 features) + real spherical harmonics of the direction (bands
// 0..3, 16) + one-blob encoding of the wavelength (16 bins); 5 hidden ReLU
// layers of 64; one linear output (radiance at that wavelength).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdd {

constexpr int kNrcLevels = 16;
constexpr int kNrcFeat = 2;
constexpr int kNrcHash = kNrcLevels * kNrcFeat;  // 32
constexpr int kNrcSh = 16;
constexpr int kNrcBlob = 16;
constexpr int kNrcIn = 64;
constexpr int kNrcHid = 64;
constexpr int kNrcLayers = 5;
constexpr int kNrcW = kNrcLayers * kNrcHid * kNrcHid;  // hidden weights (out, in)
// BF16 weights in matrix-core operand order: [layer][out tile 4][k step 2][lane 64] x 8 values,
// then the output layer as one 16-row tile (row 0 = wo, rows 1..15 zero): [k step 2][lane 64] x 8
constexpr int kNrcFrags = kNrcLayers * 4 * 2 * 64;
constexpr int kNrcFragsAll = kNrcFrags + 2 * 64;
constexpr int kNrcFrags32 = 2 * kNrcLayers * 4 * 16 * 64;  // FP32 training fragments (one float per lane)

// flat parameter space: tables [L][T][F] | W [5][64][64] | b [5][64] | wo [64] | bo
struct NrcNet {
    float* p;          // parameters (FP32 master copy)
    float* g;          // gradients (same layout)
    float* m;          // Adam first moments
    float* v;          // Adam second moments
    uint16_t* wq;      // [kNrcFragsAll][8] BF16 weights, operand order (refreshed by nrc_launch_pack)
    float* wf;         // [2][5][4][16][64] FP32 hidden weights in training operand order: W, then W^T
    const uint32_t* t16;  // FP16 pairs of the tables, one per entry (nullptr: gathers read the FP32 tables)
    long long n_tab;   // L * T * F
    long long n_all;   // all parameters
    int T;             // table entries per level (power of two)
    int res[kNrcLevels];
    int dense[kNrcLevels];    // (res + 1)^3 <= T: direct indexing
    float lo[3], inv_ext[3];  // position normalisation to [0, 1]^3
    float lam_lo, lam_inv;    // wavelength normalisation to [0, 1]
    float shK[kNrcSh];        // spherical-harmonic normalisation K_l^|m|, (l, m) order
    __host__ __device__ long long off_W() const { return n_tab; }
    __host__ __device__ long long off_b() const { return n_tab + kNrcW; }
    __host__ __device__ long long off_wo() const { return n_tab + kNrcW + kNrcLayers * kNrcHid; }
    __host__ __device__ long long off_bo() const { return off_wo() + kNrcHid; }
};

// one training batch on the device
struct NrcBatch {
    int n;              // rows
    const float* x;     // [n][3] positions (m)
    const float* w;     // [n][3] unit directions
    const float* lam;   // [n] wavelengths (nm)
    const float* t;     // [n] targets
    float* acts;        // [6][64][n] input features and hidden activations (feature-major)
    float* dz;          // [5][64][n] pre-activation gradients (feature-major)
    float* y;           // [n] outputs
    float* dy;          // [n] dloss / dy
    float* loss;        // [1] accumulated loss (mean over the rows)
};

// Order of the operand gathers: the paths sorted by the Morton code of
// their (normalised) cache vertex, so that neighbouring gathers share table
// lines in the caches.  keys and vals hold 2 x n entries each (the sort's two
// buffers); temp is the sort's scratch, nrc_order_temp_bytes(n) bytes.  The
// operands of every path still go to that path's own slots, so the order
// changes no result.
struct NrcOrder {
    uint32_t* keys;
    int* vals;
    void* temp;
    size_t temp_bytes;
};
size_t nrc_order_temp_bytes(int n);

// FP32 forward of n rows (device arrays)
hipError_t nrc_launch_infer(const NrcNet& net, int n, const float* x, const float* w, const float* lam, float* y,
                            hipStream_t st);
// BF16 matrix-core forward (FP32 accumulation); needs net.wq packed from the current weights
hipError_t nrc_launch_infer_mfma(const NrcNet& net, int n, const float* x, const float* w, const float* lam,
                                 float* y, hipStream_t st);
// Position of the cache value of (path, wavelength l) in an [n][nlp] array:
// row-major, or tiled by 16 paths, [path / 16][l][path % 16], which the query
// writes in whole 64-byte runs (16 paths of one wavelength) -- the render's
// layout.  n must be a multiple of 16 for the tiled form.
__host__ __device__ inline size_t nrc_lhat_index(long long path, int l, int nlp, int tiled) {
    return tiled ? (size_t)(path >> 4) * (size_t)nlp * 16 + (size_t)l * 16 + (size_t)(path & 15)
                 : (size_t)path * nlp + l;
}

// cache values of n paths at nl wavelengths, lhat[nrc_lhat_index(path, l)], for the
// cache vertex (cx, cn) of each path (precision 0: FP32, 1: BF16 matrix cores,
// which stage the paths' operands in hop, sop: nrc_query_ops_paths(n) entries
// each -- 4 lane groups of 16 B and 8 B per path; unused for precision 0)
long long nrc_query_ops_paths(int n);
hipError_t nrc_launch_query(const NrcNet& net, int n, const float4* cx, const float4* cn, const float* lam, int nl,
                            int nlp, float* lhat, int tiled, int precision, uint4* hop, uint2* sop,
                            const NrcOrder* ord, hipStream_t st);
// the two stages of the BF16 query: operand gathers (in the order of ord, or
// path order if ord is null), then the matrix-core network
hipError_t nrc_launch_query_operands(const NrcNet& net, int n, const float4* cx, const float4* cn, uint4* hop,
                                     uint2* sop, const NrcOrder* ord, hipStream_t st);
// n_dev (device, nullable): the number of rows to evaluate, read by the kernel
// (at most n); cp (nullable): row r is the cache vertex of path cp[r], whose
// values go to lhat[nrc_lhat_index(cp[r], l)]; rows_stat (nullable) gains
// rows * nl
hipError_t nrc_launch_query_mfma(const NrcNet& net, int n, const uint4* hop, const uint2* sop, const float* lam,
                                 int nl, int nlp, float* lhat, int tiled, hipStream_t st, const int* n_dev = nullptr,
                                 const int* cp = nullptr, unsigned long long* rows_stat = nullptr);
// Operands of a render's cache query, only for the paths that own a cache
// vertex (cx[p].w == 1) among its n paths.  flags and rank (n + 1 ints each)
// number those paths in path order: rank[p] is path p's row, rank[n] the
// number of rows; cp[row] = p.  The gathers run in the Morton order of ord
// (31-bit keys: paths without a cache vertex sort last), the operands go to
// the path's row, so rows keep path order and the query's stores stay runs of
// neighbouring paths.  ord->temp must hold nrc_order_temp_bytes(n) and
// nrc_scan_temp_bytes(n + 1) bytes.
hipError_t nrc_launch_cache_operands(const NrcNet& net, int n, const float4* cx, const float4* cn, uint4* hop,
                                     uint2* sop, const NrcOrder* ord, int* flags, int* rank, int* cp,
                                     hipStream_t st);
size_t nrc_scan_temp_bytes(int n);
// Allocation-free BF16 query: its scratch (operand staging, sort keys and
// values, the sort's temporary storage) lives in one file-scope device array
// of kNoAllocScratchBytes per GPU, held until the process ends.
constexpr size_t kNoAllocScratchBytes = 12u << 20;
constexpr int kNoAllocMaxPaths = 1 << 16;
// device address of that array on `device` (must be the current device);
// resolved once per device and cached
hipError_t nrc_noalloc_scratch(int device, void** out);
// carve the scratch of an n-path BF16 query out of [base, base + cap), every
// part 256-byte aligned; false if it does not fit
bool nrc_query_scratch_layout(void* base, size_t cap, int n, uint4** hop, uint2** sop, NrcOrder* ord);

// stable compaction of the training rows (pairs of float4) whose flag is set;
// with temp == nullptr only sets *temp_bytes
hipError_t nrc_select_rows(const float4* rows, const int* ok, int n, float4* out, int* d_count, void* temp,
                           size_t* temp_bytes, hipStream_t st);
// training batch k of S (rows (k + i S) m, i < n) of the compacted rows into SoA arrays
hipError_t nrc_launch_unpack(const float4* rows, int k, int S, int m, int n, float* x, float* w, float* lam, float* t,
                             hipStream_t st);
// BF16 operand-order copy of the hidden weights into net.wq
hipError_t nrc_launch_pack(const NrcNet& net, hipStream_t st);
// forward, loss, backward, gradient reduction (gradients are accumulated in net.g)
hipError_t nrc_launch_grad(const NrcNet& net, const NrcBatch& b, hipStream_t st);
// Adam step t (>= 1) over all parameters; clear: leave the gradients at zero
// for the next step's accumulation (else they stay readable)
hipError_t nrc_launch_adam(const NrcNet& net, int t, float lr, float b1, float b2, float eps, hipStream_t st,
                           bool clear = false);
hipError_t nrc_launch_zero(float* p, long long n, hipStream_t st);
// FP16 copy of the tables (round to nearest even): t16[i] holds features 2i, 2i+1
hipError_t nrc_launch_tables_f16(const NrcNet& net, uint32_t* t16, hipStream_t st);

}  // namespace sdd
