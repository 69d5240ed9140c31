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
// the next state, and advances the key by the two Weyl increments.
__device__ __forceinline__ PhiloxOut philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                  uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo_a = 0xD2511F53u * c0;
        const uint32_t hi_a = __umulhi(0xD2511F53u, c0);
        const uint32_t lo_b = 0xCD9E8D57u * c2;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi_b ^ c1 ^ k0;
        const uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0; c1 = lo_b; c2 = n2; c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return PhiloxOut{c0, c1, c2, c3};
}

__device__ __forceinline__ PhiloxOut omega_words(uint64_t seed, uint32_t mode, uint64_t c, uint32_t q) {
    return philox_block((uint32_t)c, (uint32_t)(c >> 32), q, mode, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ln u for u = (w + 1/2) 2^-32, single precision.  For u > 1/2 the complement
// 1 - u = (~w + 1/2) 2^-32 is formed exactly from the integer and log1p keeps
// full relative accuracy near u = 1.
__device__ __forceinline__ float log_uniform_f32(uint32_t w) {
    if (w < 0x80000000u) {
        return logf(fmaf((float)w, 0x1p-32f, 0x1p-33f));
    }
    return log1pf(-fmaf((float)(~w), 0x1p-32f, 0x1p-33f));
}

__device__ __forceinline__ float uniform_f32(uint32_t w) { return fmaf((float)w, 0x1p-32f, 0x1p-33f); }

// Four normals, single precision (used by the FP32 and BF16 paths).
__device__ __forceinline__ void omega4_f32(uint64_t seed, uint32_t mode, uint64_t c, uint32_t q, float z[4]) {
    PhiloxOut w = omega_words(seed, mode, c, q);
    float ra = sqrtf(-2.0f * log_uniform_f32(w.w0));
    float rb = sqrtf(-2.0f * log_uniform_f32(w.w2));
    float sa, ca, sb, cb;
    sincospif(2.0f * uniform_f32(w.w1), &sa, &ca);
    sincospif(2.0f * uniform_f32(w.w3), &sb, &cb);
    z[0] = ra * ca; z[1] = ra * sa; z[2] = rb * cb; z[3] = rb * sb;
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
