// Sketch Y = X_(n) Omega (§2.4 Alg. 1 step 1; Alg. 3 step 4) of float32 data on
// the bfloat16 matrix cores: at float32 accuracy (NP = 3), or as the bfloat16
// sketch (NP = 2).
//
// NP = 3: every float32 operand is split exactly into three bfloat16 pieces,
// x = h + m + l: h keeps the top 8 significant bits of x (truncation), m the top
// 8 of the remainder x - h, l the remaining at most 8 bits.  The product x w is
// formed from the six piece products whose weight is at least 2^-16 of it
// (hh, hm, mh, hl, lh, mm); each is exact in the float32 accumulator, and the
// three dropped ones (ml, lm, ll) together stay below 3 * 2^-24 |x w|, so the
// result carries float32 accuracy.
//
// NP = 2 (the bfloat16 sketch): two pieces per operand, x = h + m + r with the
// same truncations (|r| < 2^-15 |x|), and the three products of weight above
// 2^-16 (hh, hm, mh), the bf16x3 scheme of Henry, Tang and Heinecke (ARITH
// 2019): a relative rounding near 2^-15 instead of the 2^-8 of operands rounded
// once to bfloat16.
//
// v_mfma_f32_16x16x32_bf16 runs at 16 x the
// rate of the float32 MFMA, so even six products per product leave the kernel
// bound by its memory traffic rather than by the matrix cores.
//
// Layout.  A wave owns RM blocks of 16 rows; a workgroup (eight waves) shares
// the Omega tile of KC = 32 or 64 unfolding columns (one or two MFMA steps of
// 32; the 64-column tile gives each row a 256-byte run per step, which reads
// faster when a workgroup holds 128 rows).  In MFMA step j, lane l = 16 g + i
// supplies row i of X at the eight unfolding columns (KC / 4) g + 8 j .. + 7
// (two 16-byte loads straight into registers; R % 8 == 0 keeps them in one
// l-slab) and,
// as the B operand, Omega at the same eight columns for sketch column i of a
// 16-column block; the accumulator of lane l holds Y[4 g + v][i], v = 0..3.
// Omega is generated once per tile per workgroup (Philox4x32-10 + Box-Muller,
// the same values as every other sketch kernel), split or rounded, and stored as
// NP bfloat16 planes, each [sketch column n][k] (k pairs packed in a word, four
// words of padding after every two columns; one 16-byte LDS read per operand).
// X is read through a buffer descriptor sized to the tensor (at most 0x7fff0000
// bytes), so rows past J and columns past L R load zeros: their offsets are
// pushed past the end without wrapping.  Split-K partial sums go to
// partial[split][row][0 .. ell) and are added in a fixed order afterwards, like
// those of the other sketch kernels.
#include "rt_kernels.hpp"
#include "rt_philox.hpp"

namespace rt {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int X6_KC = 32;     // unfolding columns per MFMA step (one 16x16x32 K block)
constexpr int X6_WPG = 8;     // waves per workgroup

__device__ __forceinline__ f4 mfma_bf16(u4 a, u4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// x = h + m + l exactly; each piece a float32 whose low 16 bits are zero, i.e.
// a bfloat16 value in the high half
__device__ __forceinline__ void split3(float x, uint32_t& h, uint32_t& m, uint32_t& l) {
    h = __float_as_uint(x) & 0xffff0000u;
    const float r = x - __uint_as_float(h);
    m = __float_as_uint(r) & 0xffff0000u;
    l = __float_as_uint(r - __uint_as_float(m));
}
// the first two pieces of split3 (x - h - m is left out)
__device__ __forceinline__ void split2(float x, uint32_t& h, uint32_t& m) {
    h = __float_as_uint(x) & 0xffff0000u;
    m = __float_as_uint(x - __uint_as_float(h)) & 0xffff0000u;
}
// two bfloat16 (the high halves of a and b) in one word, a in the low half
__device__ __forceinline__ uint32_t pack2(uint32_t a, uint32_t b) { return (a >> 16) | (b & 0xffff0000u); }

// NP = 3: the float32 products from three pieces per operand, six MFMAs per
// block; NP = 2: the bfloat16 sketch from two pieces, three MFMAs per block.
template <int NB, int RM, int NP, int KC>
__global__ __launch_bounds__(64 * X6_WPG) void sketch_x6_kernel(const float* __restrict__ X, int64_t L, int64_t J, int64_t R,
                                                        int ell, int64_t col0, uint64_t seed, uint32_t mode,
                                                        int64_t tiles_per_split, float* __restrict__ partial,
                                                        double* __restrict__ nrm2_partial) {
    constexpr int NTH = 64 * X6_WPG;
    constexpr int MT = 16 * RM * X6_WPG;              // rows per workgroup
    // words per bfloat16 plane: row n (16 k pairs) at n * 16 + (n / 2) * 4, the
    // padding keeps the generation's stores and the 16-byte reads apart in the banks
    constexpr int NG = KC / X6_KC;                    // MFMA steps (8-column groups per lane) per tile
    constexpr int PL = NB * 16 * (KC / 2) + NB * 8 * 4;
    __shared__ __align__(16) uint32_t om[2][NP * PL];
    __shared__ double red[X6_WPG];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, i16 = lane & 15;
    const int64_t K = L * R;
    const int64_t ntiles = (K + KC - 1) / KC;
    const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_split;
    const int64_t t_end = t_begin + tiles_per_split < ntiles ? t_begin + tiles_per_split : ntiles;
    const int64_t wrow0 = (int64_t)blockIdx.y * MT + wave * 16 * RM;
    const int64_t qbase = col0 / 4;                  // col0 % 4 == 0
    const int nq4 = (ell + 3) / 4;

    for (int e = tid; e < 2 * NP * PL; e += NTH) (&om[0][0])[e] = 0u;

    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(X), (short)0, (int)(K * J * 4), 0x00020000);
    uint32_t rowbyte[RM];
#pragma unroll
    for (int rm = 0; rm < RM; ++rm) {
        const int64_t row = wrow0 + rm * 16 + i16;
        rowbyte[rm] = row < J ? (uint32_t)(row * R * 4) : 0x7fff0000u;   // >= the tensor size
    }
    // (l, r) of this lane group's first column 8 g of the next tile to load
    int64_t cl = 0, cr = 0;
    {
        const int64_t c = t_begin * KC + (KC / 4) * g;
        cl = c / R;
        cr = c - cl * R;
    }
    // a lane's NG groups of eight columns, (KC / 4) g + 8 j, each inside one l-slab
    auto load = [&](int64_t tile, f4 (&v)[RM][2 * NG]) {
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const bool wrap = cr + 8 * j >= R;
            const int64_t clj = wrap ? cl + 1 : cl, crj = wrap ? cr + 8 * j - R : cr + 8 * j;
            const uint32_t base = (tile < t_end && clj < L) ? (uint32_t)((clj * J * R + crj) * 4) : 0x7ffffff0u;
#pragma unroll
            for (int rm = 0; rm < RM; ++rm) {
                v[rm][2 * j] =
                    __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xr, rowbyte[rm] + base, 0, 0));
                v[rm][2 * j + 1] =
                    __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xr, rowbyte[rm] + base + 16, 0, 0));
            }
        }
        cr += KC;
        while (cr >= R) { cr -= R; ++cl; }
    };
    // Omega of a tile: item (k pair kp, quad q) = columns 2 kp, 2 kp + 1 of sketch
    // columns 4 q .. 4 q + 3, each value split into the three planes
    auto gen = [&](int64_t tile, int buf) {
        for (int it = tid; it < (KC / 2) * nq4; it += NTH) {
            const int kp = it % (KC / 2), q = it / (KC / 2);
            const uint64_t c = (uint64_t)(tile * KC + 2 * kp);
            float za[4], zb[4];
            omega4_f32(seed, mode, c, (uint32_t)(qbase + q), za);
            omega4_f32(seed, mode, c + 1, (uint32_t)(qbase + q), zb);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int n = 4 * q + u;
                const int w = n * (KC / 2) + (n >> 1) * 4 + kp;
                if (NP == 2) {
                    uint32_t ha, ma, hb, mb;
                    split2(za[u], ha, ma);
                    split2(zb[u], hb, mb);
                    om[buf][w] = pack2(ha, hb);
                    om[buf][PL + w] = pack2(ma, mb);
                } else {
                    uint32_t ha, ma, la, hb, mb, lb;
                    split3(za[u], ha, ma, la);
                    split3(zb[u], hb, mb, lb);
                    om[buf][w] = pack2(ha, hb);
                    om[buf][PL + w] = pack2(ma, mb);
                    om[buf][2 * PL + w] = pack2(la, lb);
                }
            }
        }
    };

    f4 acc[RM][NB];
#pragma unroll
    for (int rm = 0; rm < RM; ++rm)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[rm][nb] = f4{0.f, 0.f, 0.f, 0.f};
    double nrm = 0.0;

    auto compute = [&](const f4 (&vv)[RM][2 * NG], int buf) {
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        u4 bh[NB], bm[NB], bl[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int n = nb * 16 + i16;
            const int w = n * (KC / 2) + (n >> 1) * 4 + (KC / 8) * g + 4 * j;
            bh[nb] = *reinterpret_cast<const u4*>(&om[buf][w]);
            if (NP >= 2) bm[nb] = *reinterpret_cast<const u4*>(&om[buf][PL + w]);
            if (NP == 3) bl[nb] = *reinterpret_cast<const u4*>(&om[buf][2 * PL + w]);
        }
        u4 ah[RM], am[RM], al[RM];
#pragma unroll
        for (int rm = 0; rm < RM; ++rm) {
            const f4 v0 = vv[rm][2 * j], v1 = vv[rm][2 * j + 1];
            const float x[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
            if (NP == 2) {
                uint32_t h[8], m[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) split2(x[e], h[e], m[e]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    ah[rm][j] = pack2(h[2 * j], h[2 * j + 1]);
                    am[rm][j] = pack2(m[2 * j], m[2 * j + 1]);
                }
            } else {
                uint32_t h[8], m[8], l[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) split3(x[e], h[e], m[e], l[e]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    ah[rm][j] = pack2(h[2 * j], h[2 * j + 1]);
                    am[rm][j] = pack2(m[2 * j], m[2 * j + 1]);
                    al[rm][j] = pack2(l[2 * j], l[2 * j + 1]);
                }
            }
            if (nrm2_partial) {
#pragma unroll
                for (int e = 0; e < 8; ++e) nrm = fma((double)x[e], (double)x[e], nrm);
            }
        }
        if (NP == 2) {
            // the two smaller products first
#pragma unroll
            for (int rm = 0; rm < RM; ++rm)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[rm][nb] = mfma_bf16(am[rm], bh[nb], acc[rm][nb]);
#pragma unroll
            for (int rm = 0; rm < RM; ++rm)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[rm][nb] = mfma_bf16(ah[rm], bm[nb], acc[rm][nb]);
        }
        if (NP == 3) {
            // the five smaller products first, the accumulators of all blocks in between
#pragma unroll
            for (int rm = 0; rm < RM; ++rm)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[rm][nb] = mfma_bf16(am[rm], bm[nb], acc[rm][nb]);
#pragma unroll
            for (int rm = 0; rm < RM; ++rm)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[rm][nb] = mfma_bf16(al[rm], bh[nb], acc[rm][nb]);
#pragma unroll
            for (int rm = 0; rm < RM; ++rm)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[rm][nb] = mfma_bf16(ah[rm], bl[nb], acc[rm][nb]);
#pragma unroll
            for (int rm = 0; rm < RM; ++rm)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[rm][nb] = mfma_bf16(am[rm], bh[nb], acc[rm][nb]);
#pragma unroll
            for (int rm = 0; rm < RM; ++rm)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[rm][nb] = mfma_bf16(ah[rm], bm[nb], acc[rm][nb]);
        }
#pragma unroll
        for (int rm = 0; rm < RM; ++rm)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[rm][nb] = mfma_bf16(ah[rm], bh[nb], acc[rm][nb]);
      }
    };

    // X NSET - 1 tiles ahead in registers (NSET register sets in rotation),
    // Omega one tile ahead in the other of two buffers; one barrier per tile
    // hands the Omega buffers over.  Loads past t_end read nothing (their
    // offsets are out of range), so they are issued unconditionally.
    constexpr int NSET = 2;
    f4 xs[NSET][RM][2 * NG];
#pragma unroll
    for (int s = 0; s + 1 < NSET; ++s) load(t_begin + s, xs[s]);
    __syncthreads();                                   // the zeroed planes before any generation
    if (t_begin < t_end) gen(t_begin, 0);
    __syncthreads();
    for (int64_t t = t_begin; t < t_end; t += NSET) {
#pragma unroll
        for (int s = 0; s < NSET; ++s) {
            const int64_t tt = t + s;
            load(tt + NSET - 1, xs[(s + NSET - 1) % NSET]);
            if (tt >= t_end) break;
            const int par = (int)((tt - t_begin) & 1);
            if (tt + 1 < t_end) gen(tt + 1, par ^ 1);
            compute(xs[s], par);
            __syncthreads();
        }
    }

#pragma unroll
    for (int rm = 0; rm < RM; ++rm)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = wrow0 + rm * 16 + 4 * g + v;
            if (row < J) {
                float* dst = partial + ((int64_t)blockIdx.x * J + row) * ell;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int n = nb * 16 + i16;
                    if (n < ell) dst[n] = acc[rm][nb][v];
                }
            }
        }
    if (nrm2_partial) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        if (lane == 0) red[wave] = nrm;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < X6_WPG; ++w) t += red[w];
            nrm2_partial[blockIdx.y * gridDim.x + blockIdx.x] = t;
        }
    }
}

template <int NB, int NP, int KC>
hipError_t x6_by_rm(int rm, dim3 grid, const float* X, Shape3 s, int ell, int64_t col0, uint64_t seed, uint32_t mode,
                    int64_t tps, float* partial, double* nrm2, hipStream_t st) {
    switch (rm) {
        case 1:
            hipLaunchKernelGGL((sketch_x6_kernel<NB, 1, NP, KC>), grid, dim3(64 * X6_WPG), 0, st, X, s.L, s.J, s.R, ell,
                               col0, seed, mode, tps, partial, nrm2);
            return hipGetLastError();
        case 2:
            hipLaunchKernelGGL((sketch_x6_kernel<NB, 2, NP, KC>), grid, dim3(64 * X6_WPG), 0, st, X, s.L, s.J, s.R, ell,
                               col0, seed, mode, tps, partial, nrm2);
            return hipGetLastError();
        case 4:
            hipLaunchKernelGGL((sketch_x6_kernel<NB, 4, NP, KC>), grid, dim3(64 * X6_WPG), 0, st, X, s.L, s.J, s.R, ell,
                               col0, seed, mode, tps, partial, nrm2);
            return hipGetLastError();
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace

bool sketch_x6_ok(Shape3 s, int ell, int64_t col0, const void* X) {
    const int64_t bytes = s.L * s.J * s.R * 4;
    // (below 65 rows a workgroup of 128 rows would idle most of its waves; the
    // LDS-staged float32 kernel serves those modes)
    return s.J > 64 && ell >= 1 && ell <= 64 && col0 % 4 == 0 && s.R % 8 == 0 && ((uintptr_t)X & 15) == 0 &&
           bytes <= 0x7fff0000LL;
}

void plan_sketch_x6(SketchPlan& p, Shape3 s, int ell, bool bf16, int rb, int wgs) {
    p.kind = bf16 ? 4 : 3;
    p.rb = rb == 1 || rb == 2 || rb == 4 ? rb : (s.J <= 128 ? 1 : 2);   // 16-row blocks per wave
    p.rw = 0;
    p.nq = (ell + 15) / 16;
    p.ldp = ell;
    // tiles of 64 columns (two MFMA steps, 256-byte runs per row) for the
    // bfloat16 sketch over 128-row workgroups, where they read faster; 32 otherwise
    p.kc = bf16 && p.rb == 1 ? 2 * X6_KC : X6_KC;
    const int64_t mt = 16 * p.rb * X6_WPG;
    const int64_t K = s.L * s.R;
    const int64_t ntl = (K + p.kc - 1) / p.kc;
    p.nrowtile = (int)((s.J + mt - 1) / mt);
    int64_t want = (wgs > 0 ? wgs : 2048 / X6_WPG) / p.nrowtile;   // built-in: two waves per SIMD
    if (want < 1) want = 1;
    if (want > ntl) want = ntl;
    p.tiles_per_split = (ntl + want - 1) / want;
    p.nsplit = (int)((ntl + p.tiles_per_split - 1) / p.tiles_per_split);
    p.partial_elems = (size_t)p.nsplit * (size_t)s.J * (size_t)p.ldp;
    p.nwg = p.nsplit * p.nrowtile;
}

hipError_t launch_sketch_f32_x6(const SketchPlan& p, const float* X, Shape3 s, int ell, int64_t col0, uint64_t seed,
                                uint32_t mode, float* partial, double* nrm2, hipStream_t stream) {
    if ((p.kind != 3 && p.kind != 4) || !sketch_x6_ok(s, ell, col0, X)) return hipErrorInvalidValue;
    const dim3 grid(p.nsplit, p.nrowtile);
    const int64_t tps = p.tiles_per_split;
#define RT_X6(NBV)                                                                                                  \
    return p.kind == 3   ? x6_by_rm<NBV, 3, X6_KC>(p.rb, grid, X, s, ell, col0, seed, mode, tps, partial, nrm2, stream) \
           : p.kc == X6_KC ? x6_by_rm<NBV, 2, X6_KC>(p.rb, grid, X, s, ell, col0, seed, mode, tps, partial, nrm2, stream) \
                         : x6_by_rm<NBV, 2, 2 * X6_KC>(p.rb, grid, X, s, ell, col0, seed, mode, tps, partial, nrm2, stream)
    switch (p.nq) {
        case 1: RT_X6(1);
        case 2: RT_X6(2);
        case 3: RT_X6(3);
        case 4: RT_X6(4);
        default: return hipErrorInvalidValue;
    }
#undef RT_X6
}

}  // namespace rt
