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

// Precision of the per-path ray state and of the shading geometry built on it
// (camera ray, hit point on the triangle's plane, normal, light sample and
// NEE geometry, bounce directions): FP64 in the library.  Compiled with
// SDD_PATH_STATE_F32 (a measurement build, libsdd_f32state.so) they are FP32,
// state storage included, so that build states what FP32 state costs in
// accuracy against the FP64 oracle and what FP64 state costs in time.
#ifdef SDD_PATH_STATE_F32
using preal = float;
using pv3 = f3;
__device__ __forceinline__ pv3 state3(f3 a) { return a; }
__device__ __forceinline__ pv3 state3(float4 a) { return f3{a.x, a.y, a.z}; }
__device__ __forceinline__ f3 narrow(f3 a) { return a; }
#else
using preal = double;
using pv3 = d3;
__device__ __forceinline__ pv3 state3(f3 a) { return wide(a); }
__device__ __forceinline__ pv3 state3(float4 a) { return wide(a); }
#endif

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

// ---------------------------------------------------------------------------
// complex arithmetic (FP32) for coherent coatings
// ---------------------------------------------------------------------------
struct cpx {
    float re, im;
};
__device__ __forceinline__ cpx cadd(cpx a, cpx b) { return cpx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cpx csub(cpx a, cpx b) { return cpx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cpx cmul(cpx a, cpx b) { return cpx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cpx cscale(cpx a, float s) { return cpx{a.re * s, a.im * s}; }
__device__ __forceinline__ float cabs2(cpx a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ cpx cdiv(cpx a, cpx b) {
    const float inv = 1.0f / cabs2(b);
    return cpx{(a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv};
}
// principal square root (re >= 0)
__device__ __forceinline__ cpx csqrt_p(cpx z) {
    const float m = sqrtf(z.re * z.re + z.im * z.im);
    if (z.re >= 0.0f) {
        const float u = sqrtf(0.5f * (m + z.re));
        return cpx{u, u > 0.0f ? z.im / (2.0f * u) : 0.0f};
    }
    const float v = copysignf(sqrtf(0.5f * (m - z.re)), z.im);
    return cpx{z.im / (2.0f * v), v};
}
// cos and sin of a complex argument a + i b
__device__ __forceinline__ void csincos(cpx z, cpx& sn, cpx& cs) {
    float s, c;
    sincosf(z.re, &s, &c);
    const float ep = expf(z.im), em = 1.0f / ep;
    const float ch = 0.5f * (ep + em), sh = 0.5f * (ep - em);
    sn = cpx{s * ch, c * sh};
    cs = cpx{c * ch, -s * sh};
}

// 2 x 2 complex matrix, right-multiplied by a layer's characteristic matrix
// [[cos D, -i sin D / eta], [-i eta sin D, cos D]]
struct CMat {
    cpx m11{1.0f, 0.0f}, m12{0.0f, 0.0f}, m21{0.0f, 0.0f}, m22{1.0f, 0.0f};
    __device__ __forceinline__ void times_layer(cpx cs, cpx sn, cpx eta) {
        const cpx t12 = cdiv(sn, eta), t21 = cmul(eta, sn);
        const cpx a12{t12.im, -t12.re}, a21{t21.im, -t21.re};  // times -i
        const cpx n11 = cadd(cmul(m11, cs), cmul(m12, a21)), n12 = cadd(cmul(m11, a12), cmul(m12, cs));
        const cpx n21 = cadd(cmul(m21, cs), cmul(m22, a21)), n22 = cadd(cmul(m21, a12), cmul(m22, cs));
        m11 = n11;
        m12 = n12;
        m21 = n21;
        m22 = n22;
    }
};

// Pane with a coherent coating of L layers on its coated face (thin-film
// optics by characteristic matrices; the index is n + i k with fields
// ~ exp(-i omega t)).  pc: substrate pane constants as for pane_RT; lay[j *
// stride]: per layer (Re N^2, Im N^2, 2 pi d / lambda); c: incidence cosine
// in air; coated_side: the light arrives on the coated face.  With beta^2 =
// 1 - c^2, every medium has w = sqrt(N^2 - beta^2) (= N cos theta, principal
// root) and admittance w (s) or N^2 / w (p); a layer's matrix is
// [[cos D, -i sin D / eta], [-i eta sin D, cos D]], D = (2 pi d / lambda) w.
// With M = M_1 ... M_L, the stack seen from air gives B = m11 + m12 eta_s,
// C = m21 + m22 eta_s, r = (eta_0 B - C) / (eta_0 B + C),
// T = 4 eta_0 Re(eta_s) / |eta_0 B + C|^2; seen from the substrate the
// product runs backwards, which for these matrices swaps m11 and m22.  The
// two faces then combine incoherently through the substrate (Beer-Lambert
// tau as for the uncoated pane), per polarisation, and (s + p) / 2 is taken.
__device__ __forceinline__ void coated_RT(float4 pc, const float4* lay, int L, int stride, float c, bool coated_side,
                                          float& R_out, float& T_out) {
    if (!(c > 1e-6f)) {
        R_out = 1.0f;
        T_out = 0.0f;
        return;
    }
    const float b2 = 1.0f - c * c;
    const cpx Ns2{pc.x, pc.y};
    const cpx ws = csqrt_p(cpx{pc.x - b2, pc.y});
    // product matrices for s and p
    CMat ms, mp;
    for (int j = 0; j < L; ++j) {
        const float4 q = lay[(size_t)j * stride];
        const cpx N2{q.x, q.y};
        const cpx w = csqrt_p(cpx{q.x - b2, q.y});
        cpx sn, cs;
        csincos(cscale(w, q.z), sn, cs);
        ms.times_layer(cs, sn, w);
        mp.times_layer(cs, sn, cdiv(N2, w));
    }
    const float cosr2 = 1.0f - b2 * pc.z;
    const float tau = cosr2 > 0.0f ? expf(-pc.w / sqrtf(cosr2)) : 0.0f;
    const float tau2 = tau * tau;
    float Rsum = 0.0f, Tsum = 0.0f;
#pragma unroll
    for (int pol = 0; pol < 2; ++pol) {
        const CMat& M = pol ? mp : ms;
        const float e0 = pol ? 1.0f / c : c;
        const cpx em = pol ? cdiv(Ns2, ws) : ws;
        // coated face from air
        const cpx B = cadd(M.m11, cmul(M.m12, em)), C = cadd(M.m21, cmul(M.m22, em));
        const cpx den = cadd(cscale(B, e0), C);
        const float inv_den = 1.0f / cabs2(den);
        const float Rc = cabs2(csub(cscale(B, e0), C)) * inv_den;
        const float Tc = 4.0f * e0 * em.re * inv_den;
        // coated face from the substrate (reversed product: m11 <-> m22)
        const cpx B2 = cadd(M.m22, cscale(M.m12, e0)), C2 = cadd(M.m21, cscale(M.m11, e0));
        const cpx den2 = cadd(cmul(em, B2), C2);
        const float Rc2 = cabs2(csub(cmul(em, B2), C2)) / cabs2(den2);
        // bare face
        const float Rb = cabs2(csub(cpx{e0, 0.0f}, em)) / cabs2(cadd(cpx{e0, 0.0f}, em));
        const float Tb = 1.0f - Rb;
        const float dn = 1.0f - Rc2 * Rb * tau2;
        if (!(dn > 0.0f)) {
            Rsum += 1.0f;
            continue;
        }
        if (coated_side) {
            Tsum += Tc * tau * Tb / dn;
            Rsum += Rc + Tc * Tc * Rb * tau2 / dn;
        } else {
            Tsum += Tb * tau * Tc / dn;
            Rsum += Rb + Tb * Tb * Rc2 * tau2 / dn;
        }
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

// The same in FP64 (the path's shading geometry).
__device__ __forceinline__ d3 cosine_dir64(d3 n, double u0, double u1) {
    const double s = n.z >= 0.0 ? 1.0 : -1.0;
    const double a = -1.0 / (s + n.z);
    const double b = n.x * n.y * a;
    const d3 b1{1.0 + s * n.x * n.x * a, s * b, -s * n.x};
    const d3 b2{b, s + n.y * n.y * a, -n.y};
    const double r = sqrt(u0);
    double sp, cp;
    sincos(2.0 * 3.14159265358979323846 * u1, &sp, &cp);
    const double lz = sqrt(1.0 - u0);
    return b1 * (r * cp) + b2 * (r * sp) + n * lz;
}

#ifdef SDD_PATH_STATE_F32
__device__ __forceinline__ pv3 cosine_dir_state(pv3 n, preal u0, preal u1) { return cosine_dir(n, u0, u1); }
#else
__device__ __forceinline__ pv3 cosine_dir_state(pv3 n, preal u0, preal u1) { return cosine_dir64(n, u0, u1); }
#endif

// ---------------------------------------------------------------------------
// wave-level helpers (64-wide)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }
// 1 on the lowest active lane of the wave, 0 elsewhere (wave-level counting)
__device__ __forceinline__ int first_active_lane() {
    return (int)(lane_id() == (int)__builtin_ctzll(__builtin_amdgcn_read_exec()));
}

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// number of set bits of m below this lane
__device__ __forceinline__ int rank_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Multi-split append: every lane with `active` gets a unique slot in the
// segment `key` of a segmented queue whose per-segment fill counters are
// counts[key * stride].  The active lanes are grouped by key (ballot per
// distinct key); each group's lowest lane takes the group's slots with one
// atomic, and the leaders' atomics go out as one instruction, so the wave
// waits on memory once.  A lane's slot is its leader's base plus its rank in
// the group.  Must be reached by all lanes of the wave together.
__device__ __forceinline__ int wave_append(bool active, int key, int* counts, int stride) {
    int leader = 0, rank = 0, n_key = 0;
    uint64_t pending = __ballot(active);
    while (pending) {
        const int l = __ffsll((unsigned long long)pending) - 1;
        const int lk = __builtin_amdgcn_readlane(key, l);
        const uint64_t m = __ballot(active && key == lk);
        if (active && key == lk) {
            leader = l;
            rank = rank_below(m);
        }
        if (lane_id() == l) n_key = popc64(m);
        pending &= ~m;
    }
    int base = 0;
    if (active && lane_id() == leader) base = atomicAdd(&counts[(size_t)key * stride], n_key);
    base = __shfl(base, leader);
    return active ? base + rank : -1;
}

// Stable workgroup multi-split rank: every thread with `active` gets its
// rank among the threads of the block with the same key, in thread order
// (per wave: ballot + mbcnt; across waves: prefix of the per-wave counts held
// in s_wcnt[wave][n_seg]).  Afterwards s_wcnt[0][k] holds nothing useful; the
// block's count of key k is returned by block_key_total.  Every thread of the
// block must call it (it synchronises the block).
// direction bin of the closest-hit routing: sign bits of x and y
__device__ __forceinline__ int dir_bin(f3 d) { return (d.x < 0.0f ? 1 : 0) | (d.y < 0.0f ? 2 : 0); }

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
