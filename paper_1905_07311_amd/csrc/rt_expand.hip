// Mode-n expansion of a Tucker core, the step of reconstruction X_hat =
// G x_1 A_1 ... x_d A_d (§2.1, the Tucker format): on the (L, r, R) view of the
// current tensor and a factor A (I x r, row-major),
//     out[l, i, q] = sum_k A[i, k] G[l, k, q]     (out viewed as (L, I, R)).
// The output is much larger than its inputs (I >> r), so the kernels are laid
// out for the output stream: lanes own consecutive output entries (coalesced
// 4- or 8-byte stores), the operand that varies along the lanes sits in
// registers, and the other one is read from LDS as a broadcast.
//   * R == 1 (the last mode), float64: out (L x I) = G (L x r) A^T: lane i
//     holds A[i, :] in registers, a block of G rows is staged in LDS.
//   * R == 1, float32: the same product on the matrix cores
//     (v_mfma_f32_16x16x4f32), A's block staged in LDS, G's rows in registers,
//     results passed through LDS so that stores cover whole cache lines.
//   * R > 1, float32: per l the slab A G[l] on the matrix cores, A's block
//     staged in LDS, a block of G[l]'s columns in registers, results passed
//     through LDS so that consecutive lanes store consecutive addresses.
//   * R >= 64, float64: lane q holds G[l, :, q] in registers, a block of A rows
//     is staged in LDS.
//   * 1 < R < 64, float64: lanes own consecutive entries of one l's I x R output
//     slab, G[l] staged in LDS once per workgroup, rows of A read through the
//     cache.
// Each output is a dot product of length r summed in order k = 0, 1, ...,
// except on the matrix cores (the hardware's order, float32).
#include "rt_kernels.hpp"

namespace rt {

namespace {

constexpr int EX_T = 256;     // threads per workgroup
constexpr int EX_LB = 32;     // G rows (R == 1) or A rows (R > 1) staged per workgroup
typedef float f4 __attribute__((ext_vector_type(4)));

// Four outputs of a lane at a time (independent chains), each summed in order k.
template <typename T, int RK>
__device__ __forceinline__ void dot4(const T* v, const T (*rows)[RK], int n, T* dst, int64_t dst_step) {
    int m = 0;
    for (; m + 4 <= n; m += 4) {
        T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
        for (int k = 0; k < RK; ++k) {
            s0 += v[k] * rows[m][k];
            s1 += v[k] * rows[m + 1][k];
            s2 += v[k] * rows[m + 2][k];
            s3 += v[k] * rows[m + 3][k];
        }
        dst[m * dst_step] = s0;
        dst[(m + 1) * dst_step] = s1;
        dst[(m + 2) * dst_step] = s2;
        dst[(m + 3) * dst_step] = s3;
    }
    for (; m < n; ++m) {
        T s0 = T(0);
#pragma unroll
        for (int k = 0; k < RK; ++k) s0 += v[k] * rows[m][k];
        dst[m * dst_step] = s0;
    }
}

// grid: x = blocks of EX_LB rows of G, y = blocks of EX_T output columns i
template <typename T, int RK>
__global__ __launch_bounds__(EX_T) void expand_last_kernel(const T* __restrict__ G, int64_t L, int r,
                                                           const T* __restrict__ A, int64_t I, T* __restrict__ out) {
    __shared__ T gs[EX_LB][RK];
    const int64_t i = (int64_t)blockIdx.y * EX_T + threadIdx.x;
    const int64_t l0 = (int64_t)blockIdx.x * EX_LB;
    T a[RK];
#pragma unroll
    for (int k = 0; k < RK; ++k) a[k] = (i < I && k < r) ? A[i * r + k] : T(0);
    for (int e = threadIdx.x; e < EX_LB * RK; e += EX_T) {
        const int ll = e / RK, k = e % RK;
        gs[ll][k] = (l0 + ll < L && k < r) ? G[(l0 + ll) * r + k] : T(0);
    }
    __syncthreads();
    if (i >= I) return;
    const int lmax = (int)(L - l0 < EX_LB ? L - l0 : EX_LB);
    dot4<T, RK>(a, gs, lmax, out + l0 * I + i, I);
}

// grid: x = (l, block of EX_T columns q) flattened, y = blocks of EX_LB rows i
template <typename T, int RK>
__global__ __launch_bounds__(EX_T) void expand_rows_kernel(const T* __restrict__ G, int64_t L, int r, int64_t R,
                                                           const T* __restrict__ A, int64_t I, T* __restrict__ out) {
    __shared__ T as[EX_LB][RK];
    const int64_t nqb = (R + EX_T - 1) / EX_T;
    const int64_t l = blockIdx.x / nqb;
    const int64_t q = (blockIdx.x - l * nqb) * EX_T + threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.y * EX_LB;
    T g[RK];
#pragma unroll
    for (int k = 0; k < RK; ++k) g[k] = (q < R && k < r) ? G[(l * r + k) * R + q] : T(0);
    for (int e = threadIdx.x; e < EX_LB * RK; e += EX_T) {
        const int ii = e / RK, k = e % RK;
        as[ii][k] = (i0 + ii < I && k < r) ? A[(i0 + ii) * r + k] : T(0);
    }
    __syncthreads();
    if (q >= R) return;
    const int imax = (int)(I - i0 < EX_LB ? I - i0 : EX_LB);
    dot4<T, RK>(g, as, imax, out + (l * I + i0) * R + q, R);
}

// 1 < R < 64: for a fixed l the output is one contiguous I x R slab.  A
// workgroup takes EX_SC consecutive entries of one l's slab: G[l, :, :] (r x R)
// is staged in LDS once, and lane t computes entries t, t + EX_T, ... as
// (i, q) = (e / R, e % R) from row i of A (read through the cache; the R lanes
// that share i read the same row) and column q of the staged block.
constexpr int EX_SC = EX_T * 16;   // slab entries per workgroup

// grid: x = (l, block of EX_SC slab entries) flattened
template <typename T, int RK>
__global__ __launch_bounds__(EX_T) void expand_slab_kernel(const T* __restrict__ G, int64_t L, int r, int64_t R,
                                                           const T* __restrict__ A, int64_t I, T* __restrict__ out) {
    __shared__ T gs[RK][64];
    const int64_t slab = I * R;
    const int64_t nb = (slab + EX_SC - 1) / EX_SC;
    const int64_t l = blockIdx.x / nb;
    const int64_t t0 = (blockIdx.x - l * nb) * EX_SC;
    for (int e = threadIdx.x; e < RK * 64; e += EX_T) {
        const int k = e / 64, q = e % 64;
        gs[k][q] = (k < r && q < R) ? G[(l * r + k) * R + q] : T(0);
    }
    __syncthreads();
    const int Ri = (int)R;
    for (int u = 0; u < EX_SC / EX_T; ++u) {
        const int64_t t = t0 + u * EX_T + threadIdx.x;
        if (t >= slab) break;
        const int64_t i = t / Ri;
        const int q = (int)(t - i * Ri);
        const T* arow = A + i * r;
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < RK; ++k) acc += (k < r ? arow[k] : T(0)) * gs[k][q];
        out[l * slab + t] = acc;
    }
}

// Float32 expansion on the matrix cores (v_mfma_f32_16x16x4f32).  A 16 x 16
// tile is D[m][n] = sum_k A[i0 + m][k] B[k][n]: the factor A is the first
// operand (M = rows i), the second is G's rows (the last mode, R == 1: B[k][n]
// = G[l0 + n][k], D = out^T) or a block of G[l]'s columns (R > 1: B[k][n] =
// G[l][k][q0 + n], D = out[l] rows i, columns q).  For this instruction lane
// 16 g + j supplies the first operand's row j at k-slot g, the second
// operand's column j at k-slot g, and holds D[4 g + v][j] in component v.
// The r (<= 4 KS) terms are dealt to the four k-slots in contiguous runs: in
// MFMA step s, slot g carries k = g KS + s, so a lane's KS values of a row
// are contiguous.  The factor stays in registers: a workgroup's four waves own
// consecutive runs of 16 NT rows of A (loaded once), and walk the same
// sequence of units (row tiles of G, or (l, column block) pairs) grid-stride,
// so that together they write whole contiguous runs of the output; each
// wave's tiles go through a wave-private LDS buffer and leave as stores of
// consecutive addresses.  Sums are in the hardware's order (float32, within
// rounding of the ordered sum).

// The first operand of NT tiles of A: rows i_lo + 16 t + j, k = g KS .. g KS + KS - 1.
template <int KS, int NT>
__device__ __forceinline__ void load_factor(const float* __restrict__ A, int64_t I, int r, int64_t i_lo, int g,
                                            int j, float (&a)[NT][KS]) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int64_t i = i_lo + 16 * t + j;
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) {
            const int k = g * KS + s2;
            a[t][s2] = (i < I && k < r) ? A[i * r + k] : 0.f;
        }
    }
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// R == 1.  Wave w of the workgroup owns columns [ib + 16 NT w, ib + 16 NT (w + 1)),
// ib = blockIdx.y * 64 NT; a unit is one tile of 16 rows of G (its operand
// loaded one unit ahead).  Buffer: 16 rows l x 16 NT columns i; a store
// instruction then covers 64 / (4 NT) ... rows of 64 NT contiguous bytes each.
template <int KS, int NT>
__global__ __launch_bounds__(256) void expand_last_mfma_kernel(const float* __restrict__ G, int64_t L, int r,
                                                               const float* __restrict__ A, int64_t I,
                                                               float* __restrict__ out) {
    constexpr int TW = 16 * NT + 4;               // floats per buffer row
    constexpr int LPR = 4 * NT;                   // lanes per output row (four floats each)
    constexpr int RPI = 64 / LPR;                 // rows per store instruction
    __shared__ __align__(16) float tb[4][16 * TW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int64_t i_lo = (int64_t)blockIdx.y * 64 * NT + 16 * NT * wave;
    float a[NT][KS];
    load_factor<KS, NT>(A, I, r, i_lo, g, j, a);
    float* tw = tb[wave];
    const bool vec = (I & 3) == 0;
    const int64_t ntiles = (L + 15) / 16;
    float gb[KS], gn[KS];
    auto load_g = [&](int64_t tile, float (&dst)[KS]) {
        const int64_t l = tile * 16 + j;
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) {
            const int k = g * KS + s2;
            dst[s2] = (tile < ntiles && l < L && k < r) ? G[l * r + k] : 0.f;
        }
    };
    int64_t tile = blockIdx.x;
    load_g(tile, gb);
    const int rr = lane / LPR, cc = lane % LPR;
    for (; tile < ntiles; tile += gridDim.x) {
        load_g(tile + gridDim.x, gn);
        if (i_lo < I) {
            f4 acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                acc[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s2 = 0; s2 < KS; ++s2)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][s2], gb[s2], acc[t], 0, 0, 0);
            }
            // acc[t][v] = out[l0 + j][i_lo + 16 t + 4 g + v] -> tw[j][16 t + 4 g + v]
#pragma unroll
            for (int t = 0; t < NT; ++t) *reinterpret_cast<f4*>(tw + j * TW + 16 * t + 4 * g) = acc[t];
            wave_lds_sync();
            const int64_t l0 = tile * 16;
            const int64_t ic = i_lo + 4 * cc;
#pragma unroll
            for (int p = 0; p < 16 / RPI; ++p) {
                const int m = RPI * p + rr;
                const f4 v = *reinterpret_cast<const f4*>(tw + m * TW + 4 * cc);
                const int64_t l = l0 + m;
                if (l >= L || ic >= I) continue;
                float* dst = out + l * I + ic;
                if (vec && ic + 3 < I) {
                    *reinterpret_cast<f4*>(dst) = v;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (ic + u < I) dst[u] = v[u];
                }
            }
            wave_lds_sync();
        }
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) gb[s2] = gn[s2];
    }
}

// R > 1.  Wave w owns rows [ib + 16 NT w, ib + 16 NT (w + 1)) of A; a unit is
// (l, block of 16 NQ columns q), its operand loaded one unit ahead.  Buffer:
// 16 NT rows i x 16 NQ columns q; the block's W = min(16 NQ, R - q0) columns of
// those rows are stored with consecutive lanes on consecutive columns (one
// contiguous run of the wave's rows when the block spans R).
template <int KS, int NT, int NQ>
__global__ __launch_bounds__(256) void expand_mid_mfma_kernel(const float* __restrict__ G, int64_t L, int r,
                                                              int64_t R, const float* __restrict__ A, int64_t I,
                                                              float* __restrict__ out) {
    constexpr int TW = 16 * NQ + 1;
    __shared__ float tb[4][16 * NT * TW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int64_t i_lo = (int64_t)blockIdx.y * 64 * NT + 16 * NT * wave;
    float a[NT][KS];
    load_factor<KS, NT>(A, I, r, i_lo, g, j, a);
    float* tw = tb[wave];
    const int64_t nqb = (R + 16 * NQ - 1) / (16 * NQ);
    const int64_t units = L * nqb;
    const int rows = (int)(I - i_lo < 16 * NT ? (I - i_lo > 0 ? I - i_lo : 0) : 16 * NT);
    float gb[NQ][KS], gn[NQ][KS];
    auto load_g = [&](int64_t u, float (&dst)[NQ][KS]) {
        const int64_t l = u / nqb;
        const int64_t q0 = (u - l * nqb) * 16 * NQ;
#pragma unroll
        for (int t = 0; t < NQ; ++t)
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2) {
                const int k = g * KS + s2;
                const int64_t q = q0 + 16 * t + j;
                dst[t][s2] = (u < units && k < r && q < R) ? G[(l * r + k) * R + q] : 0.f;
            }
    };
    int64_t u = blockIdx.x;
    load_g(u, gb);
    for (; u < units; u += gridDim.x) {
        load_g(u + gridDim.x, gn);
        if (rows > 0) {
            const int64_t l = u / nqb;
            const int64_t q0 = (u - l * nqb) * 16 * NQ;
            const int W = (int)(R - q0 < 16 * NQ ? R - q0 : 16 * NQ);
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int tq = 0; tq < NQ; ++tq) {
                    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s2 = 0; s2 < KS; ++s2)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][s2], gb[tq][s2], acc, 0, 0, 0);
                    // acc[v] = out[l][i_lo + 16 t + 4 g + v][q0 + 16 tq + j]
#pragma unroll
                    for (int v = 0; v < 4; ++v) tw[(16 * t + 4 * g + v) * TW + 16 * tq + j] = acc[v];
                }
            wave_lds_sync();
            // entry e = lane + 64 it of the rows x W block: (m, c) = (e / W, e % W),
            // advanced by 64 = dm W + dc per step
            const int dm = 64 / W, dc = 64 - dm * W;
            int m = lane / W, c = lane - m * W;
            float* base = out + (l * I + i_lo) * R + q0;
            while (m < rows) {
                base[(int64_t)m * R + c] = tw[m * TW + c];
                m += dm;
                c += dc;
                if (c >= W) { c -= W; ++m; }
            }
            wave_lds_sync();
        }
#pragma unroll
        for (int tq = 0; tq < NQ; ++tq)
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2) gb[tq][s2] = gn[tq][s2];
    }
}

// Workgroups per launch (two per CU), units grid-stride: for the 512^3 float32
// last mode 144 us against 153 us with 1024 and 178 us with 256 workgroups.
constexpr int XM_WGS = 512;

template <int KS, int NT, int NQ>
hipError_t expand_mid_mfma(Shape3 s, const float* G, const float* A, int64_t I, float* out, hipStream_t st) {
    const int64_t ny = (I + 64 * NT - 1) / (64 * NT);
    const int64_t units = s.L * ((s.R + 16 * NQ - 1) / (16 * NQ));
    int64_t gx = (XM_WGS + ny - 1) / ny;
    gx = gx < units ? gx : units;
    const dim3 grid((unsigned)gx, (unsigned)ny);
    hipLaunchKernelGGL((expand_mid_mfma_kernel<KS, NT, NQ>), grid, dim3(256), 0, st, G, s.L, (int)s.J, s.R, A, I,
                       out);
    return hipGetLastError();
}

// the block of q columns: one to four tiles; rows of A per wave: 16 NT with NT NQ = 8
template <int KS>
hipError_t expand_mid_nq(Shape3 s, const float* G, const float* A, int64_t I, float* out, hipStream_t st) {
    switch (s.R <= 16 ? 1 : s.R <= 32 ? 2 : 4) {
        case 1: return expand_mid_mfma<KS, 8, 1>(s, G, A, I, out, st);
        case 2: return expand_mid_mfma<KS, 4, 2>(s, G, A, I, out, st);
        default: return expand_mid_mfma<KS, 2, 4>(s, G, A, I, out, st);
    }
}

template <int KS>
hipError_t expand_last_mfma(Shape3 s, const float* G, const float* A, int64_t I, float* out, hipStream_t st) {
    constexpr int NT = 8;     // 128 columns per wave, 512 per workgroup
    const int64_t ny = (I + 64 * NT - 1) / (64 * NT);
    const int64_t ntiles = (s.L + 15) / 16;
    int64_t gx = (XM_WGS + ny - 1) / ny;
    gx = gx < ntiles ? gx : ntiles;
    const dim3 grid((unsigned)gx, (unsigned)ny);
    hipLaunchKernelGGL((expand_last_mfma_kernel<KS, NT>), grid, dim3(256), 0, st, G, s.L, (int)s.J, A, I, out);
    return hipGetLastError();
}

template <int KS>
hipError_t expand_f32_ks(Shape3 s, const float* G, const float* A, int64_t I, float* out, hipStream_t st) {
    return s.R == 1 ? expand_last_mfma<KS>(s, G, A, I, out, st) : expand_mid_nq<KS>(s, G, A, I, out, st);
}

// float32, any R: the matrix-core kernels, r padded to a multiple of 4
hipError_t expand_f32(Shape3 s, const float* G, const float* A, int64_t I, float* out, hipStream_t st) {
    switch ((s.J + 3) / 4) {
        case 1: return expand_f32_ks<1>(s, G, A, I, out, st);
        case 2: return expand_f32_ks<2>(s, G, A, I, out, st);
        case 3: return expand_f32_ks<3>(s, G, A, I, out, st);
        case 4: return expand_f32_ks<4>(s, G, A, I, out, st);
        case 5: return expand_f32_ks<5>(s, G, A, I, out, st);
        case 6: return expand_f32_ks<6>(s, G, A, I, out, st);
        case 7: return expand_f32_ks<7>(s, G, A, I, out, st);
        case 8: return expand_f32_ks<8>(s, G, A, I, out, st);
        case 9: return expand_f32_ks<9>(s, G, A, I, out, st);
        case 10: return expand_f32_ks<10>(s, G, A, I, out, st);
        case 11: return expand_f32_ks<11>(s, G, A, I, out, st);
        case 12: return expand_f32_ks<12>(s, G, A, I, out, st);
        case 13: return expand_f32_ks<13>(s, G, A, I, out, st);
        case 14: return expand_f32_ks<14>(s, G, A, I, out, st);
        case 15: return expand_f32_ks<15>(s, G, A, I, out, st);
        default: return expand_f32_ks<16>(s, G, A, I, out, st);
    }
}

template <typename T, int RK>
hipError_t expand_rk(Shape3 s, const T* G, const T* A, int64_t I, T* out, hipStream_t st) {
    const int r = (int)s.J;
    if (s.R > 1 && s.R < 64) {
        const dim3 grid((unsigned)(((I * s.R + EX_SC - 1) / EX_SC) * s.L));
        hipLaunchKernelGGL((expand_slab_kernel<T, RK>), grid, dim3(EX_T), 0, st, G, s.L, r, s.R, A, I, out);
    } else if (s.R == 1) {
        const dim3 grid((unsigned)((s.L + EX_LB - 1) / EX_LB), (unsigned)((I + EX_T - 1) / EX_T));
        hipLaunchKernelGGL((expand_last_kernel<T, RK>), grid, dim3(EX_T), 0, st, G, s.L, r, A, I, out);
    } else {
        const dim3 grid((unsigned)(((s.R + EX_T - 1) / EX_T) * s.L), (unsigned)((I + EX_LB - 1) / EX_LB));
        hipLaunchKernelGGL((expand_rows_kernel<T, RK>), grid, dim3(EX_T), 0, st, G, s.L, r, s.R, A, I, out);
    }
    return hipGetLastError();
}

// the core dimension padded to a multiple of 8 (zero padding costs FMAs only)
template <typename T>
hipError_t expand_t(Shape3 s, const T* G, const T* A, int64_t I, T* out, hipStream_t st) {
    switch ((s.J + 7) / 8) {
        case 1: return expand_rk<T, 8>(s, G, A, I, out, st);
        case 2: return expand_rk<T, 16>(s, G, A, I, out, st);
        case 3: return expand_rk<T, 24>(s, G, A, I, out, st);
        case 4: return expand_rk<T, 32>(s, G, A, I, out, st);
        case 5: return expand_rk<T, 40>(s, G, A, I, out, st);
        case 6: return expand_rk<T, 48>(s, G, A, I, out, st);
        case 7: return expand_rk<T, 56>(s, G, A, I, out, st);
        default: return expand_rk<T, 64>(s, G, A, I, out, st);
    }
}

}  // namespace

// grid limits: x < 2^31, y < 2^16
bool expand_ok(Shape3 s, int64_t I) {
    if (s.J < 1 || s.J > LMAX || I < 1) return false;
    if (s.R == 1) return (s.L + EX_LB - 1) / EX_LB < 0x7fffffffLL && (I + 127) / 128 < 65536;
    if (s.R < 64) return ((I * s.R + EX_SC - 1) / EX_SC) * s.L < 0x7fffffffLL && (I + 127) / 128 < 65536;
    return ((s.R + EX_T - 1) / EX_T) * s.L < 0x7fffffffLL && (I + EX_LB - 1) / EX_LB < 65536;
}

hipError_t launch_expand(Dt dt, const void* G, Shape3 s, const void* A, int64_t I, void* out, hipStream_t stream) {
    if (!expand_ok(s, I)) return hipErrorInvalidValue;
    if (dt == Dt::F64) return expand_t<double>(s, (const double*)G, (const double*)A, I, (double*)out, stream);
    return expand_f32(s, (const float*)G, (const float*)A, I, (float*)out, stream);
}

}  // namespace rt
