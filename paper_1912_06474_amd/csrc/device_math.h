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

// ---------------------------------------------------------------------------
// complex FP32 arithmetic for the Fresnel terms of n + i k (Eq. 1)
// ---------------------------------------------------------------------------
struct cf {
    float re, im;
};
__device__ __forceinline__ cf cmul(cf a, cf b) { return cf{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
// Smith's division
__device__ __forceinline__ cf cdiv(cf a, cf b) {
    if (fabsf(b.re) >= fabsf(b.im)) {
        const float r = b.im / b.re, den = b.re + b.im * r;
        return cf{(a.re + a.im * r) / den, (a.im - a.re * r) / den};
    }
    const float r = b.re / b.im, den = b.im + b.re * r;
    return cf{(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
// principal square root (Re >= 0), stable form
__device__ __forceinline__ cf csqrt_principal(cf z) {
    const float m = hypotf(z.re, z.im);
    if (m == 0.0f) return cf{0.0f, 0.0f};
    if (z.re >= 0.0f) {
        const float a = sqrtf(0.5f * (m + z.re));
        return cf{a, z.im / (2.0f * a)};
    }
    float b = copysignf(sqrtf(0.5f * (m - z.re)), z.im);
    return cf{z.im / (2.0f * b), b};
}

// Polarisation-averaged reflectance R and transmittance T of a pane: an
// incoherent slab of thickness thick (m) with index n + i k on both faces,
// incidence cosine c from air.  Per polarisation: Fresnel R of the face
// (complex Snell, principal cos theta_t), internal attenuation
// tau = exp(-4 pi k / lambda * thick / cos theta_r) with theta_r from real
// Snell, and the sum over internal reflections
//   T = (1-R)^2 tau / (1 - R^2 tau^2),  Rs = R + (1-R)^2 R tau^2 / (1 - R^2 tau^2).
__device__ __forceinline__ void pane_RT(float n, float k, float thick, float lambda_nm, float c, float& R_out,
                                        float& T_out) {
    const cf nt{n, k};
    const cf sin2t = cdiv(cf{1.0f - c * c, 0.0f}, cmul(nt, nt));
    const cf cost = csqrt_principal(cf{1.0f - sin2t.re, -sin2t.im});
    const cf ntc = cmul(nt, cost);
    const cf rs = cdiv(cf{c - ntc.re, -ntc.im}, cf{c + ntc.re, ntc.im});
    const cf nc{nt.re * c, nt.im * c};
    const cf rp = cdiv(cf{nc.re - cost.re, nc.im - cost.im}, cf{nc.re + cost.re, nc.im + cost.im});
    const float Rf[2] = {rs.re * rs.re + rs.im * rs.im, rp.re * rp.re + rp.im * rp.im};
    const float cosr2 = 1.0f - (1.0f - c * c) / (n * n);
    float tau = 0.0f;
    if (cosr2 > 0.0f) {
        const float alpha = 4.0f * kPi * k / (lambda_nm * 1e-9f);
        tau = expf(-alpha * thick / sqrtf(cosr2));
    }
    float Rsum = 0.0f, Tsum = 0.0f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float Ri = Rf[i];
        const float den = 1.0f - Ri * Ri * tau * tau;
        if (den <= 0.0f) {
            Rsum += 1.0f;
            continue;
        }
        const float a = (1.0f - Ri) * (1.0f - Ri);
        Tsum += a * tau / den;
        Rsum += Ri + a * Ri * tau * tau / den;
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

// Workgroup multi-split append: per-segment histogram in LDS (s_cnt, s_base:
// n_seg ints each), then one global atomic per non-empty segment of the
// workgroup, issued by different threads in parallel.  Every thread of the
// block must call it (it synchronises the block).
__device__ __forceinline__ int block_append(bool active, int key, int* counts, int n_seg, int* s_cnt, int* s_base) {
    for (int i = threadIdx.x; i < n_seg; i += blockDim.x) s_cnt[i] = 0;
    __syncthreads();
    const int local = active ? atomicAdd(&s_cnt[key], 1) : 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n_seg; i += blockDim.x) {
        const int c = s_cnt[i];
        if (c) s_base[i] = atomicAdd(&counts[i], c);
    }
    __syncthreads();
    return active ? s_base[key] + local : -1;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

}  // namespace sdd
