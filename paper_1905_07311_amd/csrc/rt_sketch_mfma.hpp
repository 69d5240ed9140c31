// FP32 MFMA sketch kernel Y = X_(n) Omega (§2.4 Alg. 1 step 1, Alg. 3 step 4),
// with Omega generated on the fly (Philox4x32-10 + Box-Muller, never stored).
//
// v_mfma_f32_4x4x1_16b_f32 computes sixteen independent 4x4 outer products:
// lane l = 4 blk + t supplies A[blk][t] and B[blk][t], and accumulator register
// v of lane l receives D[blk][v][t] (layout checked on the device).  Here the
// sixteen blocks are sixteen groups of four rows of X and every block uses the
// same B = four columns of one Omega row, so the narrow side (ell = r + p) is
// padded to a multiple of 4 only.
//
// The B operand is the same for all blocks, so a lane's Omega values are
// re-read from LDS for every MFMA group; each wave holds RB row blocks (64 RB
// rows) of Y so that one Omega register feeds RB MFMAs.  A workgroup of four
// waves owns MT = 64 RB RW rows; the CW = 4 / RW waves of one row block split
// the columns of each tile and their sums are added through LDS at the end.
//
// Per 32-column tile: X is loaded one tile ahead into registers with coalesced
// 16-byte loads (along the rows when R % 4 == 0, along the columns when
// R == 1) and stored to LDS; Omega for the next tile is generated into
// registers by the whole workgroup, one or two Philox blocks per thread.
// Partial sums per split of the unfolding columns go to
// partial[split][row][0 .. 4 NQ) and are added in a fixed order afterwards.
#pragma once
#include "rt_kernels.hpp"
#include "rt_philox.hpp"

namespace rt {
namespace skm {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;         // unfolding columns per tile
constexpr int XLD = KC + 4;    // row stride (floats) of a tile stored by rows

enum { LOAD_ROWS = 0, LOAD_COLS = 1 };

typedef short s4 __attribute__((ext_vector_type(4)));

// Workgroup barrier for LDS hand-offs only: waits for this wave's LDS operations
// (lgkmcnt) but leaves its global loads in flight, unlike __syncthreads(), whose
// fence also waits for every outstanding vector memory operation and so would
// drain the prefetched tile at each barrier.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

template <int RB, int RW, int LOADER>
struct TileShape {
    static constexpr int CW = 4 / RW;                      // waves per row block
    static constexpr int MT = 64 * RB * RW;                // rows per workgroup
    static constexpr int NLOAD = MT * KC / 4 / 256;        // float4 loads per thread per tile
    static constexpr int TLD = MT + 4;                     // column stride of a tile stored by columns
    static constexpr int XSZ = LOADER == LOAD_ROWS ? MT * XLD : KC * TLD;
    static constexpr int JC = 2 * RW;                      // quads per epilogue chunk
};

// X viewed as (L, J, R) row-major; unfolding column c = l R + r.
// LOAD_ROWS needs R % 4 == 0 (four columns of a load lie in one l-slab); LOAD_COLS needs
// R == 1 and J % 4 == 0.  16-byte alignment of X; ell <= 4 NQ <= 64; the
// Omega blocks of columns [col0, col0 + ell) number at most 16.
// EXPL (LOAD_ROWS, float32 only): Omega is read from Om, an (L, ell, R) tensor with
// Omega[l R + r][k] = Om[(l ell + k) R + r] (the subspace-iteration product
// Y = X_(n) Z, Z = Om_(n)^T), instead of generated; seed, mode and col0 unused.
template <int RB, int RW, int NQ, int LOADER, bool EXPL = false>
__global__ __launch_bounds__(256) void sketch_f32_kernel(const float* __restrict__ X, int64_t L, int64_t J,
                                                         int64_t R, int ell, int64_t col0, uint64_t seed,
                                                         uint32_t mode, int64_t tiles_per_split,
                                                         float* __restrict__ partial,
                                                         double* __restrict__ nrm2_partial,
                                                         const float* __restrict__ Om = nullptr) {
    static_assert(!EXPL || LOADER == LOAD_ROWS, "explicit Omega: rows loader only");
    typedef TileShape<RB, RW, LOADER> S;
    constexpr int CW = S::CW, MT = S::MT, NLOAD = S::NLOAD, TLD = S::TLD, JC = S::JC;
    constexpr int NQP = (NQ + 3) / 4 * 4;  // Omega row length in LDS (16-byte reads)
    constexpr int LDP = 4 * NQ;            // partial row length
    __shared__ __align__(16) float xs[S::XSZ];
    // Omega tile: [c][t][j] = Omega[c][4 j + t], then a sink
    __shared__ __align__(16) float os[KC * 4 * NQP + 4];
    __shared__ double red[4];
    static_assert(4 * 64 * RB * JC * 4 <= S::XSZ, "epilogue buffer exceeds the tile");

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int blk = lane >> 2, t = lane & 3;
    const int rw = wave % RW, cw = wave / RW;
    const int64_t K = L * R;
    const int64_t ntiles = (K + KC - 1) / KC;
    const int64_t row0 = (int64_t)blockIdx.y * MT;
    const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_split;
    const int64_t t_end = t_begin + tiles_per_split < ntiles ? t_begin + tiles_per_split : ntiles;
    const int64_t qbase = col0 / 4;
    const int nqblk = (int)((col0 + ell - 1) / 4 - qbase + 1);
    const int shift = (int)(col0 - 4 * qbase);  // sketch column k is Omega column col0 + k

    f4 acc[RB][NQ];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < NQ; ++j) acc[rb][j] = f4{0.f, 0.f, 0.f, 0.f};
    double nrm = 0.0;
    f4 pre[NLOAD];
    float opre[8];

    // whole tiles (all MT rows present, all KC columns inside K) load without
    // per-element guards
    const bool rows_full = row0 + MT <= J;
    // LOAD_ROWS: a thread always loads the four columns 4 (tid & 7) .. + 3 of a
    // tile, which lie in one l-slab since R % 4 == 0; their (l, r) is advanced by
    // KC per tile (tiles are loaded in order)
    int64_t cur_l = 0, cur_r = 0;
    if (LOADER == LOAD_ROWS) {
        const int64_t cg = t_begin * KC + 4 * (tid & 7);
        cur_l = cg / R;
        cur_r = cg - cur_l * R;
    }
    auto load_tile = [&](int64_t tile) {
        const int64_t c0 = tile * KC;
        const bool full = rows_full && c0 + KC <= K;
        if (LOADER == LOAD_ROWS) {
            const float* base = X + (cur_l * J + row0) * R + cur_r;
            const int cc = 4 * (tid & 7);
            if (full) {
#pragma unroll
                for (int it = 0; it < NLOAD; ++it) {
                    const int e = tid + 256 * it;
                    pre[it] = *reinterpret_cast<const f4*>(base + (int64_t)(e >> 3) * R);
                }
            } else {
#pragma unroll
                for (int it = 0; it < NLOAD; ++it) {
                    const int e = tid + 256 * it;
                    const int rr = e >> 3;
                    f4 v = f4{0.f, 0.f, 0.f, 0.f};
                    if (row0 + rr < J && c0 + cc < K) v = *reinterpret_cast<const f4*>(base + (int64_t)rr * R);
                    pre[it] = v;
                }
            }
            cur_r += KC;
            while (cur_r >= R) { cur_r -= R; ++cur_l; }
        } else {
            const float* base = X + c0 * J + row0;
            if (full) {
#pragma unroll
                for (int it = 0; it < NLOAD; ++it) {
                    const int e = tid + 256 * it;
                    pre[it] = *reinterpret_cast<const f4*>(base + (int64_t)(e / (MT / 4)) * J + 4 * (e % (MT / 4)));
                }
            } else {
#pragma unroll
                for (int it = 0; it < NLOAD; ++it) {
                    const int e = tid + 256 * it;
                    const int cc = e / (MT / 4), rr = 4 * (e % (MT / 4));
                    f4 v = f4{0.f, 0.f, 0.f, 0.f};
                    if (row0 + rr < J && c0 + cc < K) v = *reinterpret_cast<const f4*>(base + (int64_t)cc * J + rr);
                    pre[it] = v;
                }
            }
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int it = 0; it < NLOAD; ++it) {
            const int e = tid + 256 * it;
            if (LOADER == LOAD_ROWS) {
                const int rr = e >> 3, cc = 4 * (e & 7);
                *reinterpret_cast<f4*>(&xs[rr * XLD + cc]) = pre[it];
            } else {
                const int cc = e / (MT / 4), rr = 4 * (e % (MT / 4));
                *reinterpret_cast<f4*>(&xs[cc * TLD + rr]) = pre[it];
            }
        }
    };
    // sum of squares of the staged tile in fp64 (each square exact)
    auto norm_tile = [&]() {
#pragma unroll
        for (int it = 0; it < NLOAD; ++it) {
            const f4 v = pre[it];
            const double x = v.x, y = v.y, z = v.z, w = v.w;
            nrm = fma(w, w, fma(z, z, fma(y, y, fma(x, x, nrm))));
        }
    };
    auto gen_omega = [&](int64_t tile, int h) {
        const int e = tid + 256 * h;
        if (EXPL) {
            // row k = e / 8 of Om, columns 4 (e % 8) .. + 3 of the tile (one l-slab)
            const int k = e >> 3;
            const int64_t c = tile * KC + 4 * (tid & 7);
            f4 v = f4{0.f, 0.f, 0.f, 0.f};
            if (k < ell && c < K) {
                int64_t l, r;
                if (K <= 0xffffffffll) {
                    const uint32_t q = (uint32_t)c / (uint32_t)R;
                    l = q;
                    r = c - (int64_t)q * R;
                } else {
                    l = c / R;
                    r = c - l * R;
                }
                v = *reinterpret_cast<const f4*>(Om + (l * ell + k) * R + r);
            }
            opre[4 * h + 0] = v.x; opre[4 * h + 1] = v.y; opre[4 * h + 2] = v.z; opre[4 * h + 3] = v.w;
            return;
        }
        if (e < KC * nqblk) {
            const int cc = e % KC, qi = e / KC;
            float z[4];
            omega4_f32(seed, mode, (uint64_t)(tile * KC + cc), (uint32_t)(qbase + qi), z);
            opre[4 * h + 0] = z[0]; opre[4 * h + 1] = z[1]; opre[4 * h + 2] = z[2]; opre[4 * h + 3] = z[3];
        }
    };
    // columns outside [0, ell) of a generated block go to the sink slot
    auto store_omega = [&]() {
        if (EXPL) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = (tid + 256 * h) >> 3, cq = tid & 7;
                if (k < ell) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) os[((4 * cq + u) * 4 + (k & 3)) * NQP + (k >> 2)] = opre[4 * h + u];
                }
            }
            return;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + 256 * h;
            if (e < KC * nqblk) {
                const int cc = e % KC, qi = e / KC;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = 4 * qi + u - shift;
                    const bool in = k >= 0 && k < ell;
                    os[in ? (cc * 4 + (k & 3)) * NQP + (k >> 2) : KC * 4 * NQP] = opre[4 * h + u];
                }
            }
        }
    };

    // Omega columns ell .. 4 NQP - 1 of the LDS tile stay zero
    for (int e = tid; e < KC * 4 * NQP; e += 256) os[e] = 0.f;
    if (t_begin < t_end) {
        load_tile(t_begin);
        gen_omega(t_begin, 0);
        gen_omega(t_begin, 1);
    }
    for (int64_t tile = t_begin; tile < t_end; ++tile) {
        lds_barrier();
        store_tile();
        if (nrm2_partial) norm_tile();
        store_omega();
        lds_barrier();
        const bool more = tile + 1 < t_end;
        if (more) load_tile(tile + 1);
#pragma unroll
        for (int m = 0; m < 8 / CW; ++m) {
            const int c4 = 4 * (cw + CW * m);
            float a[RB][4];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int row = rw * 64 * RB + rb * 64 + 4 * blk + t;
                if (LOADER == LOAD_ROWS) {
                    const f4 v = *reinterpret_cast<const f4*>(&xs[row * XLD + c4]);
                    a[rb][0] = v.x; a[rb][1] = v.y; a[rb][2] = v.z; a[rb][3] = v.w;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) a[rb][u] = xs[(c4 + u) * TLD + row];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float* orow = &os[((c4 + u) * 4 + t) * NQP];
                float bv[NQP];
#pragma unroll
                for (int j4 = 0; j4 < NQP; j4 += 4) {
                    const f4 v = *reinterpret_cast<const f4*>(orow + j4);
                    bv[j4] = v.x; bv[j4 + 1] = v.y; bv[j4 + 2] = v.z; bv[j4 + 3] = v.w;
                }
#pragma unroll
                for (int j = 0; j < NQ; ++j)
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) acc[rb][j] = mfma4(a[rb][u], bv[j], acc[rb][j]);
            }
            // Omega of the next tile, spread over the first two column groups
            if (more && m < 2) gen_omega(tile + 1, m);
        }
        if (more && 8 / CW < 2) gen_omega(tile + 1, 1);
    }

    // Epilogue: the CW waves of a row block add their sums through LDS, JC quads
    // at a time; each (row, quad) of the partial is written as one 16-byte store.
    float* buf = xs;
    for (int j0 = 0; j0 < NQ; j0 += JC) {
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < JC; ++jj) {
            const int j = j0 + jj;
            if (j < NQ) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        buf[((((wave * RB + rb) * 4 + v) * 16 + blk) * JC + jj) * 4 + t] = acc[rb][j][v];
            }
        }
        __syncthreads();
        constexpr int NITEM = JC * 64 * RB * RW;
        for (int e = tid; e < NITEM; e += 256) {
            const int jj = e % JC;
            int rest = e / JC;
            const int v = rest & 3;
            rest >>= 2;
            const int b = rest & 15;
            rest >>= 4;
            const int rb = rest % RB, rw2 = rest / RB;
            const int j = j0 + jj;
            const int64_t i = row0 + rw2 * 64 * RB + rb * 64 + 4 * b + v;
            if (j < NQ && i < J) {
                f4 s = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const int w = c * RW + rw2;
                    s += *reinterpret_cast<const f4*>(&buf[((((w * RB + rb) * 4 + v) * 16 + b) * JC + jj) * 4]);
                }
                *reinterpret_cast<f4*>(&partial[((int64_t)blockIdx.x * J + i) * LDP + 4 * j]) = s;
            }
        }
    }
    if (nrm2_partial) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        __syncthreads();
        if (lane == 0) red[wave] = nrm;
        __syncthreads();
        if (tid == 0) nrm2_partial[blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

}  // namespace skm
}  // namespace rt
