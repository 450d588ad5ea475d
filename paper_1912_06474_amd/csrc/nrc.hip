// Learned radiance cache on the device: FP32 training and inference, and a
// BF16 matrix-core (MFMA) inference path with FP32 accumulation.
//
// Encodings, each from its definition:
//  - multiresolution hash encoding (Mueller et al. 2022): level l has
//    resolution N_l; the 8 lattice corners around the position are looked
//    up, directly (c.x + c.y (N+1) + c.z (N+1)^2) when the level's lattice
//    fits the table, else by the spatial hash (c.x * 1) ^ (c.y * 2654435761)
//    ^ (c.z * 805459861) mod T, and blended trilinearly;
//  - real spherical harmonics, bands 0..3: K_l^m P_l^|m|(cos theta) times
//    sqrt2 cos(m phi) (m > 0), 1 (m = 0) or sqrt2 sin(|m| phi) (m < 0); the
//    associated Legendre functions come from their recurrences (no
//    Condon-Shortley phase), K_l^m from the host in double;
//  - one-blob wavelength encoding: 16 Gaussian bins exp(-(16 u - (i + 1/2))^2 / 2).
// Loss: relative L2, (y - t)^2 / (y^2 + 0.01) with y^2 held constant
// (Mueller et al. 2021).  Optimiser: Adam (Kingma and Ba 2015).
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <mutex>

#include <cmath>

#include "nrc.h"

namespace sdd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// encodings
// ---------------------------------------------------------------------------

__device__ __forceinline__ void sh_features(const float* K, float x, float y, float z, float* out) {
    const float ct = z, st = sqrtf(fmaxf(0.0f, 1.0f - z * z));
    // cos(m phi), sin(m phi) of the azimuth phi = atan2(y, x) by the angle-sum
    // recurrence from cos phi = x / rho, sin phi = y / rho (phi = 0 on the pole)
    const float rho = sqrtf(x * x + y * y);
    const float c1 = rho > 0.0f ? x / rho : 1.0f, s1 = rho > 0.0f ? y / rho : 0.0f;
    float cm[4], sm[4];
    cm[0] = 1.0f;
    sm[0] = 0.0f;
#pragma unroll
    for (int m = 1; m < 4; ++m) {
        cm[m] = cm[m - 1] * c1 - sm[m - 1] * s1;
        sm[m] = sm[m - 1] * c1 + cm[m - 1] * s1;
    }
    float P[4][4];  // P[l][m], m <= l
    float pmm = 1.0f;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (m > 0) pmm *= (float)(2 * m - 1) * st;
        P[m][m] = pmm;
        if (m + 1 < 4) P[m + 1][m] = ct * (float)(2 * m + 1) * pmm;
#pragma unroll
        for (int l = m + 2; l < 4; ++l)
            P[l][m] = ((float)(2 * l - 1) * ct * P[l - 1][m] - (float)(l + m - 1) * P[l - 2][m]) / (float)(l - m);
    }
    int k = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int m = -l; m <= l; ++m, ++k) {
            const int am = m < 0 ? -m : m;
            const float base = K[k] * P[l][am];
            out[k] = m > 0 ? 1.41421356237309515f * base * cm[am]
                           : (m < 0 ? 1.41421356237309515f * base * sm[am] : base);
        }
}

__device__ __forceinline__ float blob_bin(const NrcNet& net, float lam, int i) {
    const float u = (lam - net.lam_lo) * net.lam_inv * (float)kNrcBlob;
    const float d = u - ((float)i + 0.5f);
    return expf(-0.5f * d * d);
}

__device__ __forceinline__ uint32_t corner_slot(int N, int dense, int T, int cx, int cy, int cz) {
    if (dense) return (uint32_t)(cx + (N + 1) * (cy + (N + 1) * cz));
    const uint32_t h = (uint32_t)cx ^ ((uint32_t)cy * 2654435761u) ^ ((uint32_t)cz * 805459861u);
    return h & (uint32_t)(T - 1);
}

__device__ __forceinline__ void level_setup(int N, const float xn[3], int i0[3], float f[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float p = xn[a] * (float)N;
        int i = (int)floorf(p);
        i = i < 0 ? 0 : (i > N - 1 ? N - 1 : i);
        i0[a] = i;
        f[a] = p - (float)i;
    }
}

__device__ __forceinline__ float corner_weight(const float f[3], int c) {
    return ((c & 1) ? f[0] : 1.0f - f[0]) * ((c & 2) ? f[1] : 1.0f - f[1]) * ((c & 4) ? f[2] : 1.0f - f[2]);
}

__device__ __forceinline__ void normalise(const NrcNet& net, const float* x, float xn[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) xn[a] = fminf(1.0f, fmaxf(0.0f, (x[a] - net.lo[a]) * net.inv_ext[a]));
}

// both features of level l (resolution N) at the normalised position xn
__device__ __forceinline__ float2 hash_level(const NrcNet& net, int l, int N, int dense, const float xn[3]) {
    int i0[3];
    float f[3];
    level_setup(N, xn, i0, f);
    const float2* tab = reinterpret_cast<const float2*>(net.p) + (size_t)l * net.T;
    const uint32_t* tab16 = net.t16 ? net.t16 + (size_t)l * net.T : nullptr;
    float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float w = corner_weight(f, c);
        const uint32_t s = corner_slot(N, dense, net.T, i0[0] + (c & 1), i0[1] + ((c >> 1) & 1), i0[2] + (c >> 2));
        float2 e;
        if (tab16) {
            const uint32_t h = tab16[s];
            e = make_float2((float)__builtin_bit_cast(_Float16, (uint16_t)(h & 0xffffu)),
                            (float)__builtin_bit_cast(_Float16, (uint16_t)(h >> 16)));
        } else {
            e = tab[s];
        }
        a0 += w * e.x;
        a1 += w * e.y;
    }
    return make_float2(a0, a1);
}

__device__ __forceinline__ void features(const NrcNet& net, const float* x, const float* w, float lam, float* f) {
    float xn[3];
    normalise(net, x, xn);
#pragma unroll
    for (int l = 0; l < kNrcLevels; ++l) {
        const float2 e = hash_level(net, l, net.res[l], net.dense[l], xn);
        f[2 * l] = e.x;
        f[2 * l + 1] = e.y;
    }
    sh_features(net.shK, w[0], w[1], w[2], f + kNrcHash);
#pragma unroll
    for (int i = 0; i < kNrcBlob; ++i) f[kNrcHash + kNrcSh + i] = blob_bin(net, lam, i);
}

// a[4 g + j] by selects on register values (an indexed read would place a in scratch)
__device__ __forceinline__ float pick4(const float* a, int g, int j) {
    float v0 = a[j], v1 = a[4 + j], v2 = a[8 + j], v3 = a[12 + j];
    asm volatile("" : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(v3));
    const float lo = (g & 1) ? v1 : v0, hi = (g & 1) ? v3 : v2;
    return (g & 2) ? hi : lo;
}

// ---------------------------------------------------------------------------
// FP32 network, one row per thread; weights are read at wave-uniform
// addresses (scalar loads shared by the wave)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void layer(const float* __restrict__ W, const float* __restrict__ b, const float* in,
                                      float* out) {
#pragma unroll
    for (int i = 0; i < kNrcHid; ++i) {
        float s = b[i];
#pragma unroll
        for (int j = 0; j < kNrcHid; ++j) s = fmaf(W[i * kNrcHid + j], in[j], s);
        out[i] = fmaxf(s, 0.0f);
    }
}

__device__ __forceinline__ float output(const NrcNet& net, const float* h) {
    const float* wo = net.p + net.off_wo();
    float s = net.p[net.off_bo()];
#pragma unroll
    for (int j = 0; j < kNrcHid; ++j) s = fmaf(wo[j], h[j], s);
    return s;
}

__global__ __launch_bounds__(256) void k_infer(NrcNet net, int n, const float* x, const float* w, const float* lam,
                                               float* y) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    float h[kNrcHid], g[kNrcHid];
    features(net, x + 3 * (size_t)r, w + 3 * (size_t)r, lam[r], h);
    const float* W = net.p + net.off_W();
    const float* b = net.p + net.off_b();
    for (int k = 0; k < kNrcLayers; ++k) {
        layer(W + k * kNrcHid * kNrcHid, b + k * kNrcHid, h, g);
#pragma unroll
        for (int j = 0; j < kNrcHid; ++j) h[j] = g[j];
    }
    y[r] = output(net, h);
}

// ---------------------------------------------------------------------------
// Training on the FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// As in the BF16 path each layer is computed transposed, Z^T = W H^T, on 16 x
// 16 tiles (16 features x 16 rows); a step of 4 contraction slots takes one
// value per lane group, and step t, group g stands for input feature
// F(t, g) = 16 (t / 4) + 4 g + t % 4.  Lane (g, c) then holds, for row c of
// each column tile, exactly the features {16 mt + 4 g + i} a D tile gives it,
// so activations chain from layer to layer in registers.  The backward pass
// is the same product with W^T.  Activations and pre-activation gradients are
// also stored feature-major for the weight-gradient reduction.  A wave covers
// 64 rows (4 column tiles).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int frag_feature(int q, int g) { return 16 * (q >> 2) + 4 * g + (q & 3); }

constexpr int kTrainBlock = 64;

__global__ __launch_bounds__(kTrainBlock) void k_train_fwd_mfma(NrcNet net, NrcBatch b) {
    __shared__ float s_loss[kTrainBlock / 64];
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, wv = threadIdx.x >> 6;
    const int n = b.n;
    const size_t nn = (size_t)n;
    const long long base = ((long long)blockIdx.x * (kTrainBlock / 64) + wv) * 64;
    float contrib = 0.0f;
    if (base < n) {
        float h[4][16];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const long long row = base + nt * 16 + c;
            const long long rr = min(row, (long long)n - 1);
            float xn[3];
            normalise(net, b.x + 3 * rr, xn);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int l = (q < 2 ? 0 : 8) + 2 * g + (q & 1);
                const float2 e = hash_level(net, l, net.res[l], net.dense[l], xn);
                h[nt][2 * q] = e.x;
                h[nt][2 * q + 1] = e.y;
            }
            float sh[kNrcSh];
            sh_features(net.shK, b.w[3 * rr], b.w[3 * rr + 1], b.w[3 * rr + 2], sh);
            const float lm = b.lam[rr];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                h[nt][8 + i] = pick4(sh, g, i);
                h[nt][12 + i] = blob_bin(net, lm, 4 * g + i);
            }
            if (row < n)
#pragma unroll
                for (int q = 0; q < 16; ++q) b.acts[(size_t)frag_feature(q, g) * nn + row] = h[nt][q];
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll 1
        for (int k = 0; k < kNrcLayers; ++k) {
            const float* wf = net.wf + (size_t)k * 4 * 16 * 64 + lane;
            const float* bk = net.p + net.off_b() + k * kNrcHid;
            f32x4 acc[4][4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const f32x4 bias = {bk[16 * mt + 4 * g], bk[16 * mt + 4 * g + 1], bk[16 * mt + 4 * g + 2],
                                    bk[16 * mt + 4 * g + 3]};
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc[nt][mt] = bias;
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const float a = wf[(mt * 16 + t) * 64];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
                        acc[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, h[nt][t], acc[nt][mt], 0, 0, 0);
                }
            }
            float* a_out = b.acts + (size_t)(k + 1) * kNrcHid * nn;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const long long row = base + nt * 16 + c;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) h[nt][4 * mt + i] = fmaxf(acc[nt][mt][i], 0.0f);
                if (row < n)
#pragma unroll
                    for (int q = 0; q < 16; ++q) a_out[(size_t)frag_feature(q, g) * nn + row] = h[nt][q];
            }
        }
        const float* wo = net.p + net.off_wo();
        const float bo = net.p[net.off_bo()];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            float s = 0.0f;
#pragma unroll
            for (int q = 0; q < 16; ++q) s = fmaf(wo[frag_feature(q, g)], h[nt][q], s);
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            const long long row = base + nt * 16 + c;
            if (g == 0 && row < n) {
                const float y = s + bo, t = b.t[row];
                const float den = y * y + 0.01f;
                b.y[row] = y;
                b.dy[row] = 2.0f * (y - t) / den / (float)n;
                contrib += (y - t) * (y - t) / den / (float)n;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) contrib += __shfl_xor(contrib, o);
    if (lane == 0) s_loss[wv] = contrib;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w2 = 0; w2 < kTrainBlock / 64; ++w2) t += s_loss[w2];
        atomicAdd(b.loss, t);
    }
}

__global__ __launch_bounds__(kTrainBlock) void k_train_bwd_mfma(NrcNet net, NrcBatch b) {
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, wv = threadIdx.x >> 6;
    const int n = b.n;
    const size_t nn = (size_t)n;
    const long long base = ((long long)blockIdx.x * (kTrainBlock / 64) + wv) * 64;
    if (base >= n) return;
    const float* wo = net.p + net.off_wo();
    float d[4][16];  // gradient w.r.t. the current layer's output, fragment layout
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const long long row = base + nt * 16 + c;
        const float dy = row < n ? b.dy[row] : 0.0f;
#pragma unroll
        for (int q = 0; q < 16; ++q) d[nt][q] = dy * wo[frag_feature(q, g)];
    }
#pragma unroll 1
    for (int k = kNrcLayers - 1; k >= 0; --k) {
        const float* a_k = b.acts + (size_t)(k + 1) * kNrcHid * nn;
        float* z_k = b.dz + (size_t)k * kNrcHid * nn;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const long long row = base + nt * 16 + c;
            const long long rr = min(row, (long long)n - 1);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const size_t at = (size_t)frag_feature(q, g) * nn;
                d[nt][q] = a_k[at + rr] > 0.0f ? d[nt][q] : 0.0f;
                if (row < n) z_k[at + row] = d[nt][q];
            }
        }
        const float* wf = net.wf + (size_t)(kNrcLayers + k) * 4 * 16 * 64 + lane;  // W_k^T fragments
        f32x4 acc[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[nt][mt] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const float a = wf[(mt * 16 + t) * 64];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, d[nt][t], acc[nt][mt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) d[nt][4 * mt + i] = acc[nt][mt][i];
    }
    // d is now dloss / d(input features); its slots 0..7 are hash levels 2g, 2g+1, 8+2g, 9+2g
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const long long row = base + nt * 16 + c;
        if (row >= n) continue;
        float xn[3];
        normalise(net, b.x + 3 * row, xn);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int l = (q < 2 ? 0 : 8) + 2 * g + (q & 1);
            const int N = net.res[l];
            int i0[3];
            float f[3];
            level_setup(N, xn, i0, f);
            float2* gt = reinterpret_cast<float2*>(net.g) + (size_t)l * net.T;
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) {
                const float wc = corner_weight(f, cc);
                const uint32_t sl = corner_slot(N, net.dense[l], net.T, i0[0] + (cc & 1), i0[1] + ((cc >> 1) & 1),
                                                i0[2] + (cc >> 2));
                float* gp = reinterpret_cast<float*>(gt + sl);
                atomicAdd(gp, wc * d[nt][2 * q]);
                atomicAdd(gp + 1, wc * d[nt][2 * q + 1]);
            }
        }
    }
}

// weight gradients of layer k (k < 5: hidden layer, k == 5: output layer):
// sums over a chunk of rows of dz_k[i][r] acts_k[j][r], accumulated in net.g
constexpr int kRowTile = 64;
__global__ __launch_bounds__(256) void k_train_wgrad(NrcNet net, NrcBatch b, int rows_per_block) {
    __shared__ float s_dz[kNrcHid][kRowTile + 1];
    __shared__ float s_a[kNrcHid][kRowTile + 1];
    const int k = blockIdx.y;
    const int r0 = blockIdx.x * rows_per_block, r1 = min(b.n, r0 + rows_per_block);
    const size_t n = (size_t)b.n;
    const int i = threadIdx.x >> 2, j0 = (threadIdx.x & 3) * 16;
    const bool out_layer = k == kNrcLayers;
    const int n_i = out_layer ? 1 : kNrcHid;
    float acc[16];
    float accb = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
    const float* A = b.acts + (size_t)k * kNrcHid * n;  // inputs of layer k (acts[5] for the output layer)
    const float* Z = out_layer ? b.dy : b.dz + (size_t)k * kNrcHid * n;
    for (int rt = r0; rt < r1; rt += kRowTile) {
        const int nr = min(kRowTile, r1 - rt);
        for (int e = threadIdx.x; e < kNrcHid * kRowTile; e += blockDim.x) {
            const int f = e / kRowTile, rr = e % kRowTile;
            const bool in = rr < nr;
            s_a[f][rr] = in ? A[(size_t)f * n + rt + rr] : 0.0f;
            s_dz[f][rr] = (in && f < n_i) ? Z[(size_t)f * n + rt + rr] : 0.0f;
        }
        __syncthreads();
        if (i < n_i) {
            for (int rr = 0; rr < nr; ++rr) {
                const float zz = s_dz[i][rr];
                accb += zz;
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[q] = fmaf(zz, s_a[j0 + q][rr], acc[q]);
            }
        }
        __syncthreads();
    }
    if (i < n_i) {
        float* gW = out_layer ? net.g + net.off_wo()
                              : net.g + net.off_W() + (size_t)k * kNrcHid * kNrcHid + (size_t)i * kNrcHid;
#pragma unroll
        for (int q = 0; q < 16; ++q) atomicAdd(gW + j0 + q, acc[q]);
        if (j0 == 0) atomicAdd(out_layer ? net.g + net.off_bo() : net.g + net.off_b() + k * kNrcHid + i, accb);
    }
}

__global__ void k_adam(NrcNet net, float lr, float b1, float b2, float eps, float c1, float c2, int clear) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= net.n_all) return;
    const float g = net.g[i];
    if (clear) net.g[i] = 0.0f;  // ready for the next step's accumulation
    const float m = b1 * net.m[i] + (1.0f - b1) * g;
    const float v = b2 * net.v[i] + (1.0f - b2) * g * g;
    net.m[i] = m;
    net.v[i] = v;
    net.p[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

__global__ void k_tables_f16(const float* p, long long n_pairs, uint32_t* t16) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pairs) return;
    const float2 v = reinterpret_cast<const float2*>(p)[i];
    const uint16_t lo = __builtin_bit_cast(uint16_t, (_Float16)v.x), hi = __builtin_bit_cast(uint16_t, (_Float16)v.y);
    t16[i] = (uint32_t)lo | ((uint32_t)hi << 16);
}

__global__ void k_zero(float* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// ---------------------------------------------------------------------------
// BF16 matrix-core forward.
//
// Each layer is computed transposed, Z^T = W H^T, with v_mfma_f32_16x16x32_bf16:
// A = a 16 x 32 tile of W (16 output features x 32 inputs), B = a 32 x 16
// tile of H^T (32 inputs x 16 rows), D = 16 output features x 16 rows.  Lane
// l of a wave holds operand rows / columns l % 16 and 8 k slots of group
// g = l / 16, and D values (rows 4 g + i, column l % 16).  A layer's D tiles
// therefore already hold, per lane, the 16 features {16 mt + 4 g + i} of one
// data row; they become the next layer's B operand without leaving
// registers if the contraction index is permuted: k step s, slot j of group
// g stands for input feature 16 (2 s + j / 4) + 4 g + j % 4 (A and B use the
// same slot-to-k map, so the product is the plain one).  The weights are
// stored in that order (k_pack) and staged in LDS.  A wave evaluates 64 rows
// (4 column tiles), so each weight fragment read from LDS feeds 4 MFMAs.
// Input features follow the same permutation: in step 0 group g holds hash
// levels 2g, 2g+1, 8+2g, 9+2g; in step 1 the harmonics 4g..4g+3 and the
// wavelength bins 4g..4g+3.  The output layer runs on the matrix cores too,
// as a 16-row tile whose row 0 is wo (the others zero): the output of a
// column is D row 0, held by the lanes of group 0.
// ---------------------------------------------------------------------------

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

// relu(a), relu(b) rounded to BF16: rounding keeps the sign, so the ReLU is a
// signed 16-bit max with 0 on the rounded bit patterns (negative values and
// -0 become +0), one packed integer op per pair
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s16x2 relu_bf16x2(float a, float b) {
    const bf16x2 p = __builtin_convertvector((f32x2){a, b}, bf16x2);
    return __builtin_elementwise_max(__builtin_bit_cast(s16x2, p), (s16x2){0, 0});
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 relu_pack8(f32x4 a, f32x4 b) {
    const u32x4 q = {__builtin_bit_cast(uint32_t, relu_bf16x2(a[0], a[1])),
                     __builtin_bit_cast(uint32_t, relu_bf16x2(a[2], a[3])),
                     __builtin_bit_cast(uint32_t, relu_bf16x2(b[0], b[1])),
                     __builtin_bit_cast(uint32_t, relu_bf16x2(b[2], b[3]))};
    return __builtin_bit_cast(bf16x8, q);
}

constexpr int kMfmaBlock = 256;
constexpr int kMfmaRowsPerWave = 64;

// LDS of a matrix-core block: the BF16 weight fragments, biases and level table
struct MfmaLds {
    bf16x8 w[kNrcFragsAll];
    __align__(16) float b[kNrcLayers * kNrcHid];
    int res[kNrcLevels], dense[kNrcLevels];
};

__device__ __forceinline__ void mfma_stage(const NrcNet& net, MfmaLds& L) {
    const bf16x8* wq = reinterpret_cast<const bf16x8*>(net.wq);
    for (int e = threadIdx.x; e < kNrcFragsAll; e += kMfmaBlock) L.w[e] = wq[e];
    for (int e = threadIdx.x; e < kNrcLayers * kNrcHid; e += kMfmaBlock) L.b[e] = net.p[net.off_b() + e];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int l = 0; l < kNrcLevels; ++l) {  // static indexes: kernel arguments stay out of scratch
            L.res[l] = net.res[l];
            L.dense[l] = net.dense[l];
        }
    }
    __syncthreads();
}

// step-0 operand of one row: hash levels 2g, 2g+1, 8+2g, 9+2g
__device__ __forceinline__ bf16x8 mfma_hash_operand(const NrcNet& net, const MfmaLds& L, int g, const float xn[3]) {
    bf16x8 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int l = (q < 2 ? 0 : 8) + 2 * g + (q & 1);
        const float2 e = hash_level(net, l, L.res[l], L.dense[l], xn);
        v[2 * q] = (__bf16)e.x;
        v[2 * q + 1] = (__bf16)e.y;
    }
    return v;
}

// Layer 0 is split by input: its path part (hash levels and harmonics, step
// 0 and the harmonic slots of step 1, started from the bias) and its
// wavelength part (the one-blob slots of step 1, started from 0), added in
// FP32.  A BF16 product is exact in FP32, so only the summation order
// differs from one chain, and it is the same for every kernel that uses these
// functions.  The cache query then computes the path part once per path and
// the wavelength part once per wavelength for all paths.
__device__ __forceinline__ void mfma_layer0_path(const MfmaLds& L, int lane, int g, const bf16x8 (&h)[4],
                                                 const bf16x8 (&sh)[4], f32x4 (&P)[4][4]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const f32x4 bias = *reinterpret_cast<const f32x4*>(&L.b[16 * mt + 4 * g]);
        const bf16x8 a0 = L.w[(mt * 2 + 0) * 64 + lane];
        const bf16x8 a1 = L.w[(mt * 2 + 1) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            P[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, h[nt], bias, 0, 0, 0);
            P[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, sh[nt], P[nt][mt], 0, 0, 0);
        }
    }
}

// wavelength part of layer 0 for one B operand (one-blob slots, harmonic slots zero)
__device__ __forceinline__ f32x4 mfma_layer0_lambda(const MfmaLds& L, int lane, int mt, bf16x8 bl) {
    const bf16x8 a1 = L.w[(mt * 2 + 1) * 64 + lane];
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bl, (f32x4){0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
}

// hidden layers 1..4 and the output layer from layer 0's pre-activations
// z0[nt][mt] (4 column tiles); y[nt] is the output of column c of tile nt in
// the lanes of group 0
__device__ __forceinline__ void mfma_rest(const MfmaLds& L, int lane, int g, const f32x4 (&z0)[4][4], float bo,
                                          float (&y)[4]) {
    bf16x8 b0[4], b1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        b0[nt] = relu_pack8(z0[nt][0], z0[nt][1]);
        b1[nt] = relu_pack8(z0[nt][2], z0[nt][3]);
    }
    for (int k = 1; k < kNrcLayers; ++k) {
        // output tiles in pairs, each pair packed to the next operand before
        // the next pair (fewer live accumulators; same products and order)
        bf16x8 nb[2][4];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            f32x4 acc[4][2];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int mt = 2 * half + m;
                const f32x4 bias = *reinterpret_cast<const f32x4*>(&L.b[k * kNrcHid + 16 * mt + 4 * g]);
                const bf16x8 a0 = L.w[((k * 4 + mt) * 2 + 0) * 64 + lane];
                const bf16x8 a1 = L.w[((k * 4 + mt) * 2 + 1) * 64 + lane];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    acc[nt][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0[nt], bias, 0, 0, 0);
                    acc[nt][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1[nt], acc[nt][m], 0, 0, 0);
                }
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) nb[half][nt] = relu_pack8(acc[nt][0], acc[nt][1]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            b0[nt] = nb[0][nt];
            b1[nt] = nb[1][nt];
        }
    }
    const bf16x8 o0 = L.w[kNrcFrags + lane], o1 = L.w[kNrcFrags + 64 + lane];
    const f32x4 c0 = {g == 0 ? bo : 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o0, b0[nt], c0, 0, 0, 0);
        o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o1, b1[nt], o, 0, 0, 0);
        y[nt] = o[0];
    }
}

// the network from its input operands b0 (step 0), b1 (step 1: harmonics in
// slots 0..3, one-blob in slots 4..7), 4 column tiles
__device__ __forceinline__ void mfma_forward(const MfmaLds& L, int lane, int g, const bf16x8 (&b0)[4],
                                             const bf16x8 (&b1)[4], float bo, float (&y)[4]) {
    bf16x8 shq[4], blq[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const u32x4 v = __builtin_bit_cast(u32x4, b1[nt]);
        shq[nt] = __builtin_bit_cast(bf16x8, (u32x4){v[0], v[1], 0u, 0u});
        blq[nt] = __builtin_bit_cast(bf16x8, (u32x4){0u, 0u, v[2], v[3]});
    }
    f32x4 z0[4][4];
    mfma_layer0_path(L, lane, g, b0, shq, z0);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) z0[nt][mt] = z0[nt][mt] + mfma_layer0_lambda(L, lane, mt, blq[nt]);
    mfma_rest(L, lane, g, z0, bo, y);
}

__global__ __launch_bounds__(kMfmaBlock) void k_infer_mfma(NrcNet net, int n, const float* x, const float* w,
                                                          const float* lam, float* y) {
    __shared__ MfmaLds L;
    __shared__ bf16x8 s_in[kMfmaBlock / 64][4][2][64];  // per-lane parking of the input operands
    mfma_stage(net, L);
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, wv = threadIdx.x >> 6;
    const long long base = ((long long)blockIdx.x * (kMfmaBlock / 64) + wv) * kMfmaRowsPerWave;
    if (base >= n) return;  // whole wave idle (no barrier follows)
    // features, one column tile at a time (a rolled loop bounds the live
    // gathers); each lane parks its operands in its own LDS slots
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt) {
        const long long row = min(base + nt * 16 + c, (long long)n - 1);
        float xn[3];
        normalise(net, x + 3 * row, xn);
        const bf16x8 v0 = mfma_hash_operand(net, L, g, xn);
        float sh[kNrcSh];
        sh_features(net.shK, w[3 * row], w[3 * row + 1], w[3 * row + 2], sh);
        const float lm = lam[row];
        bf16x8 v1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v1[j] = (__bf16)pick4(sh, g, j);
            v1[4 + j] = (__bf16)blob_bin(net, lm, 4 * g + j);
        }
        s_in[wv][nt][0][lane] = v0;
        s_in[wv][nt][1][lane] = v1;
    }
    bf16x8 b0[4], b1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        b0[nt] = s_in[wv][nt][0][lane];
        b1[nt] = s_in[wv][nt][1][lane];
    }
    float out[4];
    mfma_forward(L, lane, g, b0, b1, net.p[net.off_bo()], out);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const long long row = base + nt * 16 + c;
        if (g == 0 && row < n) y[row] = out[nt];
    }
}

// Operands of the cache query, one thread per path: for each lane group g of
// the matrix layout, the step-0 operand (hash levels 2g, 2g+1, 8+2g, 9+2g,
// 8 BF16) and the harmonics 4g..4g+3 (4 BF16), stored where lane (g, c) of
// the path's 16-column tile reads them: hop[(tile * 4 + g) * 16 + c],
// sop[(tile * 4 + g) * 16 + c].  A plain gather kernel at full occupancy; the
// matrix kernel then needs no parking space and no gathers.
__device__ __forceinline__ void query_operands(const NrcNet& net, float4 x4, float4 n4, int row, uint4* hop,
                                               uint2* sop) {
    const float xp[3] = {x4.x, x4.y, x4.z};
    float xn[3];
    normalise(net, xp, xn);
    float sh[kNrcSh];
    sh_features(net.shK, n4.x, n4.y, n4.z, sh);
    const size_t slot = (size_t)(row >> 4) * 64 + (row & 15);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int l = (q < 2 ? 0 : 8) + 2 * g + (q & 1);
            const float2 e = hash_level(net, l, net.res[l], net.dense[l], xn);
            w[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){e.x, e.y}, bf16x2));
        }
        hop[slot + 16 * g] = make_uint4(w[0], w[1], w[2], w[3]);
        sop[slot + 16 * g] = make_uint2(
            __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){sh[4 * g], sh[4 * g + 1]}, bf16x2)),
            __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){sh[4 * g + 2], sh[4 * g + 3]}, bf16x2)));
    }
}

__global__ __launch_bounds__(256) void k_query_operands(NrcNet net, int n, const float4* cx, const float4* cn,
                                                        uint4* hop, uint2* sop, const int* order) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int p = order ? order[i] : i;  // a permutation of 0 .. n-1
    query_operands(net, cx[p], cn[p], p, hop, sop);
}

// a render's query: gathers in Morton order, operands to the path's row
__global__ __launch_bounds__(256) void k_cache_operands(NrcNet net, int n, const float4* cx, const float4* cn,
                                                        uint4* hop, uint2* sop, const int* order, const int* flags,
                                                        const int* rank, int* cp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int p = order[i];
    if (!flags[p]) return;  // no cache vertex (these sort last)
    const int r = rank[p];
    cp[r] = p;
    query_operands(net, cx[p], cn[p], r, hop, sop);
}

// 30-bit Morton code of the normalised cache vertex (10 bits per axis)
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint32_t morton_key(const NrcNet& net, float4 x4) {
    const float xp[3] = {x4.x, x4.y, x4.z};
    float xn[3];
    normalise(net, xp, xn);
    uint32_t m = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float q = fminf(fmaxf(xn[a] * 1024.0f, 0.0f), 1023.0f);  // NaN -> 0
        m |= spread3((uint32_t)q) << a;
    }
    return m;
}

__global__ __launch_bounds__(256) void k_query_keys(NrcNet net, int n, const float4* cx, uint32_t* keys, int* vals) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    keys[p] = morton_key(net, cx[p]);
    vals[p] = p;
}

// keys of a render's query: paths without a cache vertex get bit 30 (last in
// a 31-bit sort); flags[p] marks the others, flags[n] = 0 closes the scan
__global__ __launch_bounds__(256) void k_cache_keys(NrcNet net, int n, const float4* cx, uint32_t* keys, int* vals,
                                                    int* flags) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > n) return;
    if (p == n) {
        flags[n] = 0;
        return;
    }
    const float4 x4 = cx[p];
    const bool has = x4.w == 1.0f;
    keys[p] = has ? morton_key(net, x4) : (1u << 30);
    vals[p] = p;
    flags[p] = has;
}

// Cache values of n paths at every wavelength: lhat[path][l], from the
// operands of k_query_operands (n rounded up to whole 64-path waves there).
// Per wavelength only the one-blob slots change, so layer 0's path part is
// computed once and its wavelength part once per wavelength.  LDS holds only
// the weights, so three blocks fit a CU.  Same products and summation order
// as k_infer_mfma.
__global__ __launch_bounds__(kMfmaBlock) __attribute__((amdgpu_waves_per_eu(3)))
void k_query_mfma(NrcNet net, int n, const uint4* hop, const uint2* sop, const float* lam, int nl, int nlp,
                  float* lhat, int tiled, const int* n_dev, const int* cp, unsigned long long* rows_stat) {
    if (n_dev) n = min(n, *n_dev);
    if (rows_stat && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(rows_stat, (unsigned long long)n * nl);
    const long long first_row = (long long)blockIdx.x * kMfmaBlock / 64 * kMfmaRowsPerWave;
    if (first_row >= n) return;  // whole block idle (before the staging barrier)
    __shared__ MfmaLds L;
    mfma_stage(net, L);
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, wv = threadIdx.x >> 6;
    const long long base = ((long long)blockIdx.x * (kMfmaBlock / 64) + wv) * kMfmaRowsPerWave;
    if (base >= n) return;  // whole wave idle (no barrier follows)
    // where each tile's column c goes: lhat[dst[nt] + l * lstep] (no store for dst < 0)
    long long dst[4];
    const int lstep = tiled ? 16 : 1;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const long long row = base + nt * 16 + c;
        dst[nt] = row < n ? (long long)nrc_lhat_index(cp ? (long long)cp[row] : row, 0, nlp, tiled) : -1;
    }
    bf16x8 hq[4];           // step-0 operand per tile
    uint2 shq[4];           // harmonics per tile
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const size_t slot = (size_t)((base >> 4) + nt) * 64 + 16 * g + c;
        hq[nt] = __builtin_bit_cast(bf16x8, hop[slot]);
        shq[nt] = sop[slot];
    }
    const float bo = net.p[net.off_bo()];
    // layer 0's path part, once for all wavelengths
    f32x4 P[4][4];
    {
        bf16x8 shop[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) shop[nt] = __builtin_bit_cast(bf16x8, (u32x4){shq[nt].x, shq[nt].y, 0u, 0u});
        mfma_layer0_path(L, lane, g, hq, shop, P);
    }
    for (int l = 0; l < nl; ++l) {
        // keeps the weight fragments' LDS reads inside the loop (hoisted out of
        // it they would hold 160 registers)
        asm volatile("" ::: "memory");
        const float lm = lam[l];
        // the wavelength's bins 4g..4g+3, the same for every path
        const uint32_t bl0 = __builtin_bit_cast(
            uint32_t, __builtin_convertvector((f32x2){blob_bin(net, lm, 4 * g), blob_bin(net, lm, 4 * g + 1)}, bf16x2));
        const uint32_t bl1 = __builtin_bit_cast(
            uint32_t,
            __builtin_convertvector((f32x2){blob_bin(net, lm, 4 * g + 2), blob_bin(net, lm, 4 * g + 3)}, bf16x2));
        const bf16x8 blq = __builtin_bit_cast(bf16x8, (u32x4){0u, 0u, bl0, bl1});
        // layer 0's wavelength part: every column of the tile holds the same bins
        f32x4 z0[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const f32x4 q = mfma_layer0_lambda(L, lane, mt, blq);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) z0[nt][mt] = P[nt][mt] + q;
        }
        float out[4];
        mfma_rest(L, lane, g, z0, bo, out);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            if (g == 0 && dst[nt] >= 0) lhat[dst[nt] + (long long)l * lstep] = out[nt];
    }
}

// FP32 cache values, one thread per (path, wavelength), as k_infer
__global__ __launch_bounds__(256) void k_query(NrcNet net, int n, const float4* cx, const float4* cn, const float* lam,
                                               int nl, int nlp, float* lhat, int tiled) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)n * nl) return;
    const int path = (int)(t / nl), l = (int)(t - (long long)path * nl);
    const float4 x4 = cx[path], n4 = cn[path];
    const float xp[3] = {x4.x, x4.y, x4.z}, wp[3] = {n4.x, n4.y, n4.z};
    float h[kNrcHid], g[kNrcHid];
    features(net, xp, wp, lam[l], h);
    const float* W = net.p + net.off_W();
    const float* b = net.p + net.off_b();
    for (int k = 0; k < kNrcLayers; ++k) {
        layer(W + k * kNrcHid * kNrcHid, b + k * kNrcHid, h, g);
#pragma unroll
        for (int j = 0; j < kNrcHid; ++j) h[j] = g[j];
    }
    lhat[nrc_lhat_index(path, l, nlp, tiled)] = output(net, h);
}

// training batch k of S: rows (k + i S) m, i < n, of the compacted rows, into SoA
__global__ void k_unpack(const float4* rows, int k, int S, int m, int n, float* x, float* w, float* lam, float* t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t src = ((size_t)k + (size_t)i * S) * m;
    const float4 a = rows[2 * src], b = rows[2 * src + 1];
    x[3 * (size_t)i] = a.x;
    x[3 * (size_t)i + 1] = a.y;
    x[3 * (size_t)i + 2] = a.z;
    lam[i] = a.w;
    w[3 * (size_t)i] = b.x;
    w[3 * (size_t)i + 1] = b.y;
    w[3 * (size_t)i + 2] = b.z;
    t[i] = b.w;
}

struct NrcRow {
    float4 a, b;
};

// weights -> BF16 operand order: hidden fragment e = ((k * 4 + mt) * 2 + s) * 64 + lane,
// output fragment kNrcFrags + s * 64 + lane (row 0 = wo, rows 1..15 zero)
__global__ void k_pack(NrcNet net) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kNrcFragsAll) return;
    const bool out = e >= kNrcFrags;
    const int f = out ? e - kNrcFrags : e;
    const int lane = f & 63, s = (f >> 6) & 1, mt = (f >> 7) & 3, k = f >> 9;
    const int g = lane >> 4;
    const int m = out ? (lane & 15) : 16 * mt + (lane & 15);
    const float* W = out ? net.p + net.off_wo()
                         : net.p + net.off_W() + (size_t)k * kNrcHid * kNrcHid + (size_t)m * kNrcHid;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int in = 16 * (2 * s + j / 4) + 4 * g + (j & 3);
        const float v = out && m != 0 ? 0.0f : W[in];
        net.wq[(size_t)e * 8 + j] = __builtin_bit_cast(uint16_t, (__bf16)v);
    }
}

// hidden weights -> FP32 training fragments: [dir][k][mt][t][lane], dir 0 = W
// (A[16 mt + c][F(t, g)]), dir 1 = W^T (A[16 mt + c][F(t, g)] = W[F(t, g)][16 mt + c])
__global__ void k_pack32(NrcNet net) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kNrcFrags32) return;
    const int lane = e & 63, t = (e >> 6) & 15, mt = (e >> 10) & 3, kk = e >> 12;  // kk = dir * 5 + k
    const int dir = kk / kNrcLayers, k = kk % kNrcLayers;
    const int m = 16 * mt + (lane & 15), fin = frag_feature(t, lane >> 4);
    const float* W = net.p + net.off_W() + (size_t)k * kNrcHid * kNrcHid;
    net.wf[e] = dir == 0 ? W[m * kNrcHid + fin] : W[fin * kNrcHid + m];
}

inline unsigned nblocks(long long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t nrc_launch_infer(const NrcNet& net, int n, const float* x, const float* w, const float* lam, float* y,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_infer, dim3(nblocks(n, 256)), dim3(256), 0, st, net, n, x, w, lam, y);
    return hipGetLastError();
}

hipError_t nrc_launch_infer_mfma(const NrcNet& net, int n, const float* x, const float* w, const float* lam,
                                 float* y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int rows_per_block = (kMfmaBlock / 64) * kMfmaRowsPerWave;
    hipLaunchKernelGGL(k_infer_mfma, dim3(nblocks(n, rows_per_block)), dim3(kMfmaBlock), 0, st, net, n, x, w, lam,
                       y);
    return hipGetLastError();
}

long long nrc_query_ops_paths(int n) { return ((long long)n + kMfmaRowsPerWave - 1) / kMfmaRowsPerWave * kMfmaRowsPerWave; }

hipError_t nrc_launch_query(const NrcNet& net, int n, const float4* cx, const float4* cn, const float* lam, int nl,
                            int nlp, float* lhat, int tiled, int precision, uint4* hop, uint2* sop,
                            const NrcOrder* ord, hipStream_t st) {
    if (n <= 0 || nl <= 0) return hipSuccess;
    if (precision == 0) {
        hipLaunchKernelGGL(k_query, dim3(nblocks((long long)n * nl, 256)), dim3(256), 0, st, net, n, cx, cn, lam, nl,
                           nlp, lhat, tiled);
        return hipGetLastError();
    }
    hipError_t e = nrc_launch_query_operands(net, n, cx, cn, hop, sop, ord, st);
    if (e != hipSuccess) return e;
    return nrc_launch_query_mfma(net, n, hop, sop, lam, nl, nlp, lhat, tiled, st);
}

// sort keys are 31 bits: 30 of Morton code, and bit 30 for paths without a
// cache vertex (render queries)
constexpr int kOrderBits = 31;

size_t nrc_order_temp_bytes(int n) {
    size_t bytes = 0;
    hipcub::DoubleBuffer<uint32_t> kb(nullptr, nullptr);
    hipcub::DoubleBuffer<int> vb(nullptr, nullptr);
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kb, vb, n, 0, kOrderBits) != hipSuccess) return 0;
    return bytes;
}

size_t nrc_scan_temp_bytes(int n) {
    size_t bytes = 0;
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const int*)nullptr, (int*)nullptr, n) != hipSuccess)
        return 0;
    return bytes;
}

hipError_t nrc_launch_cache_operands(const NrcNet& net, int n, const float4* cx, const float4* cn, uint4* hop,
                                     uint2* sop, const NrcOrder* ord, int* flags, int* rank, int* cp,
                                     hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!ord || nrc_order_temp_bytes(n) > ord->temp_bytes || nrc_scan_temp_bytes(n + 1) > ord->temp_bytes)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cache_keys, dim3(nblocks((long long)n + 1, 256)), dim3(256), 0, st, net, n, cx, ord->keys,
                       ord->vals, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = ord->temp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(ord->temp, bytes, (const int*)flags, rank, n + 1, st);
    if (e != hipSuccess) return e;
    hipcub::DoubleBuffer<uint32_t> kb(ord->keys, ord->keys + n);
    hipcub::DoubleBuffer<int> vb(ord->vals, ord->vals + n);
    bytes = ord->temp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(ord->temp, bytes, kb, vb, n, 0, kOrderBits, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cache_operands, dim3(nblocks(n, 256)), dim3(256), 0, st, net, n, cx, cn, hop, sop,
                       (const int*)vb.Current(), (const int*)flags, (const int*)rank, cp);
    return hipGetLastError();
}

hipError_t nrc_launch_query_operands(const NrcNet& net, int n, const float4* cx, const float4* cn, uint4* hop,
                                     uint2* sop, const NrcOrder* ord, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int* order = nullptr;
    if (ord) {
        if (nrc_order_temp_bytes(n) > ord->temp_bytes) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_query_keys, dim3(nblocks(n, 256)), dim3(256), 0, st, net, n, cx, ord->keys, ord->vals);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipcub::DoubleBuffer<uint32_t> kb(ord->keys, ord->keys + n);
        hipcub::DoubleBuffer<int> vb(ord->vals, ord->vals + n);
        size_t bytes = ord->temp_bytes;
        e = hipcub::DeviceRadixSort::SortPairs(ord->temp, bytes, kb, vb, n, 0, kOrderBits, st);
        if (e != hipSuccess) return e;
        order = vb.Current();  // the buffer the last pass wrote (chosen on the host)
    }
    hipLaunchKernelGGL(k_query_operands, dim3(nblocks(n, 256)), dim3(256), 0, st, net, n, cx, cn, hop, sop, order);
    return hipGetLastError();
}

hipError_t nrc_launch_query_mfma(const NrcNet& net, int n, const uint4* hop, const uint2* sop, const float* lam,
                                 int nl, int nlp, float* lhat, int tiled, hipStream_t st, const int* n_dev,
                                 const int* cp, unsigned long long* rows_stat) {
    if (n <= 0 || nl <= 0) return hipSuccess;
    const int rows_per_block = (kMfmaBlock / 64) * kMfmaRowsPerWave;
    hipLaunchKernelGGL(k_query_mfma, dim3(nblocks(n, rows_per_block)), dim3(kMfmaBlock), 0, st, net, n, hop, sop,
                       lam, nl, nlp, lhat, tiled, n_dev, cp, rows_stat);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free query
// ---------------------------------------------------------------------------
// Host code never passes this array's name to a kernel or copy: in host code
// it is a stand-in, not a device address.  nrc_noalloc_scratch resolves the
// address once per device, with that device current, and the caller passes
// that address on.  Every call on a GPU shares its array: calls that overlap
// on one GPU race.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t nrc_noalloc_scratch(int device, void** out) {
    if (!out || device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

bool nrc_query_scratch_layout(void* base, size_t cap, int n, uint4** hop, uint2** sop, NrcOrder* ord) {
    if (!base || n <= 0) return false;
    const size_t need = (size_t)nrc_query_ops_paths(n);
    // the sort runs on n keys; its need is not monotonic in the size, so ask for n itself
    const size_t tb = nrc_order_temp_bytes(n);
    if (tb == 0) return false;
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t off = 0;
    char* b = static_cast<char*>(base);
    const size_t o_hop = off;
    off = up(off + 4 * need * sizeof(uint4));
    const size_t o_sop = off;
    off = up(off + 4 * need * sizeof(uint2));
    const size_t o_keys = off;
    off = up(off + 2 * need * sizeof(uint32_t));
    const size_t o_vals = off;
    off = up(off + 2 * need * sizeof(int));
    const size_t o_temp = off;
    off = up(off + tb);
    if (off > cap) return false;
    *hop = reinterpret_cast<uint4*>(b + o_hop);
    *sop = reinterpret_cast<uint2*>(b + o_sop);
    ord->keys = reinterpret_cast<uint32_t*>(b + o_keys);
    ord->vals = reinterpret_cast<int*>(b + o_vals);
    ord->temp = b + o_temp;
    ord->temp_bytes = tb;
    return true;
}

hipError_t nrc_select_rows(const float4* rows, const int* ok, int n, float4* out, int* d_count, void* temp,
                           size_t* temp_bytes, hipStream_t st) {
    return hipcub::DeviceSelect::Flagged(temp, *temp_bytes, reinterpret_cast<const NrcRow*>(rows), ok,
                                         reinterpret_cast<NrcRow*>(out), d_count, n, st);
}

hipError_t nrc_launch_unpack(const float4* rows, int k, int S, int m, int n, float* x, float* w, float* lam, float* t,
                             hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack, dim3(nblocks(n, 256)), dim3(256), 0, st, rows, k, S, m, n, x, w, lam, t);
    return hipGetLastError();
}

hipError_t nrc_launch_pack(const NrcNet& net, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3(nblocks(kNrcFragsAll, 256)), dim3(256), 0, st, net);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pack32, dim3(nblocks(kNrcFrags32, 256)), dim3(256), 0, st, net);
    return hipGetLastError();
}

hipError_t nrc_launch_grad(const NrcNet& net, const NrcBatch& b, hipStream_t st) {
    if (b.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_train_fwd_mfma, dim3(nblocks(b.n, kTrainBlock)), dim3(kTrainBlock), 0, st, net, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_train_bwd_mfma, dim3(nblocks(b.n, kTrainBlock)), dim3(kTrainBlock), 0, st, net, b);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int rows_per_block = 256;  // 2^14 rows: 64 x 6 blocks, enough to fill the device
    hipLaunchKernelGGL(k_train_wgrad, dim3(nblocks(b.n, rows_per_block), kNrcLayers + 1), dim3(256), 0, st, net, b,
                       rows_per_block);
    return hipGetLastError();
}

hipError_t nrc_launch_adam(const NrcNet& net, int t, float lr, float b1, float b2, float eps, hipStream_t st,
                           bool clear) {
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(nblocks(net.n_all, 256)), dim3(256), 0, st, net, lr, b1, b2, eps, c1, c2,
                       clear ? 1 : 0);
    return hipGetLastError();
}

hipError_t nrc_launch_tables_f16(const NrcNet& net, uint32_t* t16, hipStream_t st) {
    const long long pairs = net.n_tab / 2;
    if (pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tables_f16, dim3(nblocks(pairs, 256)), dim3(256), 0, st, (const float*)net.p, pairs, t16);
    return hipGetLastError();
}

hipError_t nrc_launch_zero(float* p, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(nblocks(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace sdd
