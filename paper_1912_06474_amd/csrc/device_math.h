// Device-side math for the spectral ray tracer (gfx950, FP32 unless stated).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdd {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kOffset = 1e-4f;  // origin offset (m) toward the side the new ray leaves

// ---------------------------------------------------------------------------
// small float3 helpers
// ---------------------------------------------------------------------------
struct f3 {
    float x, y, z;
};
__device__ __forceinline__ f3 mk3(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return f3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return f3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return f3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ f3 operator-(f3 a) { return f3{-a.x, -a.y, -a.z}; }
__device__ __forceinline__ float dot3(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross3(f3 a, f3 b) {
    return f3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ f3 unit3(f3 a) { return a * (1.0f / sqrtf(dot3(a, a))); }
__device__ __forceinline__ f3 xyz(float4 v) { return f3{v.x, v.y, v.z}; }

// double-precision vectors for the shading geometry
struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return d3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 operator*(d3 a, double s) { return d3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dot3(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross3(d3 a, d3 b) {
    return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ d3 wide(f3 a) { return d3{a.x, a.y, a.z}; }
__device__ __forceinline__ d3 wide(float4 a) { return d3{a.x, a.y, a.z}; }
__device__ __forceinline__ f3 narrow(d3 a) { return f3{(float)a.x, (float)a.y, (float)a.z}; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32
// multiplies with the published multipliers and Weyl key increments.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

// top 24 bits -> [0, 1); exact in FP32
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-8f; }

// Polarisation-averaged reflectance R and transmittance T of a pane: an
// incoherent slab of thickness d with complex index n + i k (Eq. 1) on both
// faces, incidence cosine c from air.  pc holds per-(material, wavelength)
// constants (n^2 - k^2, 2 n k, 1 / n^2, 4 pi k d / lambda).
// Face reflectance: with u + i v = sqrt(n~^2 - sin^2) (principal root, the
// n~ cos(theta_t) of complex Snell) and n~^2 c = P + i Q,
//   R_s = ((c - u)^2 + v^2) / ((c + u)^2 + v^2)
//   R_p = ((P - u)^2 + (Q - v)^2) / ((P + u)^2 + (Q + v)^2).
// Internal attenuation tau = exp(-4 pi k d / (lambda cos theta_r)) with
// theta_r from real Snell (Beer-Lambert), and the sum over internal
// reflections T = (1-R)^2 tau / (1 - R^2 tau^2),
// R_slab = R + (1-R)^2 R tau^2 / (1 - R^2 tau^2), per polarisation.
__device__ __forceinline__ void pane_RT(float4 pc, float c, float& R_out, float& T_out) {
    const float s2 = 1.0f - c * c;
    const float A = pc.x - s2, B = pc.y;
    const float m = sqrtf(A * A + B * B);
    float u, v;
    if (A >= 0.0f) {
        u = sqrtf(0.5f * (m + A));
        v = u > 0.0f ? B / (2.0f * u) : 0.0f;
    } else {
        v = sqrtf(0.5f * (m - A));
        u = B / (2.0f * v);
    }
    const float P = pc.x * c, Q = pc.y * c;
    const float rs_den = (c + u) * (c + u) + v * v;
    const float rp_den = (P + u) * (P + u) + (Q + v) * (Q + v);
    const float Rf[2] = {rs_den > 0.0f ? ((c - u) * (c - u) + v * v) / rs_den : 1.0f,
                         rp_den > 0.0f ? ((P - u) * (P - u) + (Q - v) * (Q - v)) / rp_den : 1.0f};
    const float cosr2 = 1.0f - s2 * pc.z;
    const float tau = cosr2 > 0.0f ? expf(-pc.w / sqrtf(cosr2)) : 0.0f;
    const float tau2 = tau * tau;
    float Rsum = 0.0f, Tsum = 0.0f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float Ri = Rf[i];
        const float den = 1.0f - Ri * Ri * tau2;
        if (den <= 0.0f) {
            Rsum += 1.0f;
            continue;
        }
        const float a = (1.0f - Ri) * (1.0f - Ri) / den;
        Tsum += a * tau;
        Rsum += Ri + a * Ri * tau2;
    }
    R_out = 0.5f * Rsum;
    T_out = 0.5f * Tsum;
}

// Cosine-weighted direction about the unit normal n (pdf cos/pi), with the
// orthonormal basis of Duff et al. (JCGT 2017); the branch sign is +1 for
// both signed zeros of n.z.
__device__ __forceinline__ f3 cosine_dir(f3 n, float u0, float u1) {
    const float s = n.z >= 0.0f ? 1.0f : -1.0f;
    const float a = -1.0f / (s + n.z);
    const float b = n.x * n.y * a;
    const f3 b1{1.0f + s * n.x * n.x * a, s * b, -s * n.x};
    const f3 b2{b, s + n.y * n.y * a, -n.y};
    const float r = sqrtf(u0);
    float sp, cp;
    sincosf(2.0f * kPi * u1, &sp, &cp);
    const float lz = sqrtf(1.0f - u0);
    return b1 * (r * cp) + b2 * (r * sp) + n * lz;
}

// ---------------------------------------------------------------------------
// wave-level helpers (64-wide)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// number of set bits of m below this lane
__device__ __forceinline__ int rank_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Multi-split append: every lane with `active` gets a unique slot in the
// segment `key` of a segmented queue whose per-segment fill counters are
// `counts`.  One atomic per distinct key in the wave (ballot + mbcnt).  Must
// be reached by all lanes of the wave together.
__device__ __forceinline__ int wave_append(bool active, int key, int* counts) {
    int slot = -1;
    uint64_t pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int lk = __builtin_amdgcn_readlane(key, leader);
        const uint64_t m = __ballot(active && key == lk);
        int base = 0;
        if (lane_id() == leader) base = atomicAdd(&counts[lk], popc64(m));
        base = __builtin_amdgcn_readlane(base, leader);
        if (active && key == lk) {
            slot = base + rank_below(m);
            active = false;
        }
        pending &= ~m;
    }
    return slot;
}

// Stable workgroup multi-split rank: every thread with `active` gets its
// rank among the threads of the block with the same key, in thread order
// (per wave: ballot + mbcnt; across waves: prefix of the per-wave counts held
// in s_wcnt[wave][n_seg]).  Afterwards s_wcnt[0][k] holds nothing useful; the
// block's count of key k is returned by block_key_total.  Every thread of the
// block must call it (it synchronises the block).
__device__ __forceinline__ int block_rank(bool active, int key, int n_seg, int* s_wcnt) {
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();  // earlier readers of s_wcnt are done
    for (int i = threadIdx.x; i < nw * n_seg; i += blockDim.x) s_wcnt[i] = 0;
    __syncthreads();
    int rank = 0;
    uint64_t pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int lk = __builtin_amdgcn_readlane(key, leader);
        const uint64_t m = __ballot(active && key == lk);
        if (lane_id() == leader) s_wcnt[w * n_seg + lk] = popc64(m);
        if (active && key == lk) rank = rank_below(m);
        pending &= ~m;
    }
    __syncthreads();
    if (active)
        for (int v = 0; v < w; ++v) rank += s_wcnt[v * n_seg + key];
    return rank;
}

__device__ __forceinline__ int block_key_total(int key, int n_seg, const int* s_wcnt) {
    const int nw = (blockDim.x + 63) >> 6;
    int t = 0;
    for (int v = 0; v < nw; ++v) t += s_wcnt[v * n_seg + key];
    return t;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

}  // namespace sdd
