// Device-side Gaussian test matrix Omega, generated on the fly and never stored.
//
// The method only needs i.i.d. N(0,1) entries (§2.4, Alg. 1 input) and the
// paper notes they can be produced on the fly, column-wise or in blocks (§3.1).
// This library fixes the generator so that every kernel, every launch shape and
// every request sees the same Omega for the same (seed, mode):
//   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (seed lo, seed hi),
//   counter = (c lo, c hi, k / 4, mode), c = unfolding column (row of Omega),
//   four output words -> u = (w + 1/2) 2^-32 -> two Box-Muller pairs giving the
//   normals of columns 4 (k/4) .. 4 (k/4) + 3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rt {

struct PhiloxOut { uint32_t w0, w1, w2, w3; };

// Ten rounds of the 4x32 Philox bijection.  Each round forms the 64-bit
// products of words 0 and 2 with the two multipliers, feeds the high halves
// (xored with the other two words and the round key) and the low halves into
// the next state, and advances the key by the two Weyl increments.  Each
// product is one 32 x 32 -> 64-bit multiply.
__device__ __forceinline__ PhiloxOut philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                  uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = (uint32_t)pb; c2 = n2; c3 = (uint32_t)pa;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return PhiloxOut{c0, c1, c2, c3};
}

__device__ __forceinline__ PhiloxOut omega_words(uint64_t seed, uint32_t mode, uint64_t c, uint32_t q) {
    return philox_block((uint32_t)c, (uint32_t)(c >> 32), q, mode, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// -2 ln u for u = (w + 1/2) 2^-32, single precision, without branches.
// u <= 1/2: the hardware base-2 logarithm (relative error about 1e-7 there).
// u > 1/2: the complement v = 1 - u = (~w + 1/2) 2^-32 is formed from the
// integer, and ln(1 - v) = -2 atanh(s) with s = v / (2 - v) <= 1/3 is summed
// as its odd power series to s^15 (remainder below 2^-24 relative), which keeps
// full relative accuracy as u -> 1.
__device__ __forceinline__ float neg2_log_uniform_f32(uint32_t w) {
    const float u = fmaf((float)w, 0x1p-32f, 0x1p-33f);
    const float lo = -2.0f * 0.693147180559945309f * __builtin_amdgcn_logf(u);
    const float v = fmaf((float)(~w), 0x1p-32f, 0x1p-33f);
    const float sv = v * __builtin_amdgcn_rcpf(2.0f - v);
    const float z = sv * sv;
    float p = 1.0f / 15.0f;
    p = fmaf(p, z, 1.0f / 13.0f);
    p = fmaf(p, z, 1.0f / 11.0f);
    p = fmaf(p, z, 1.0f / 9.0f);
    p = fmaf(p, z, 1.0f / 7.0f);
    p = fmaf(p, z, 1.0f / 5.0f);
    p = fmaf(p, z, 1.0f / 3.0f);
    p = fmaf(p, z, 1.0f);
    const float hi = 4.0f * sv * p;
    return w < 0x80000000u ? lo : hi;
}

__device__ __forceinline__ float uniform_f32(uint32_t w) { return fmaf((float)w, 0x1p-32f, 0x1p-33f); }

// Four normals, single precision (used by the FP32 and BF16 paths).  The
// angle 2 pi u goes to the hardware sine and cosine, which take their argument
// in revolutions (absolute error about 1.3e-7 on (0, 1)); square roots are the
// hardware ones (relative error about 1e-7).
__device__ __forceinline__ void omega4_f32(uint64_t seed, uint32_t mode, uint64_t c, uint32_t q, float z[4]) {
    PhiloxOut w = omega_words(seed, mode, c, q);
    const float ra = __builtin_amdgcn_sqrtf(neg2_log_uniform_f32(w.w0));
    const float rb = __builtin_amdgcn_sqrtf(neg2_log_uniform_f32(w.w2));
    const float ua = uniform_f32(w.w1), ub = uniform_f32(w.w3);
    z[0] = ra * __builtin_amdgcn_cosf(ua);
    z[1] = ra * __builtin_amdgcn_sinf(ua);
    z[2] = rb * __builtin_amdgcn_cosf(ub);
    z[3] = rb * __builtin_amdgcn_sinf(ub);
}

// Four normals, double precision (used by the FP64 path).
__device__ __forceinline__ void omega4_f64(uint64_t seed, uint32_t mode, uint64_t c, uint32_t q, double z[4]) {
    PhiloxOut w = omega_words(seed, mode, c, q);
    const double s = 0x1p-32;
    double u0 = ((double)w.w0 + 0.5) * s, u1 = ((double)w.w1 + 0.5) * s;
    double u2 = ((double)w.w2 + 0.5) * s, u3 = ((double)w.w3 + 0.5) * s;
    double ra = sqrt(-2.0 * log(u0));
    double rb = sqrt(-2.0 * log(u2));
    double sa, ca, sb, cb;
    sincospi(2.0 * u1, &sa, &ca);
    sincospi(2.0 * u3, &sb, &cb);
    z[0] = ra * ca; z[1] = ra * sa; z[2] = rb * cb; z[3] = rb * sb;
}

template <typename T> struct OmegaGen;
template <> struct OmegaGen<float> {
    static __device__ __forceinline__ void gen4(uint64_t seed, uint32_t mode, uint64_t c, uint32_t q, float z[4]) {
        omega4_f32(seed, mode, c, q, z);
    }
};
template <> struct OmegaGen<double> {
    static __device__ __forceinline__ void gen4(uint64_t seed, uint32_t mode, uint64_t c, uint32_t q, double z[4]) {
        omega4_f64(seed, mode, c, q, z);
    }
};

}  // namespace rt
