// MFMA projection B = X x_n Q^T on gfx950 (§2.4 Alg. 1 step 3; also the core
// update G <- U^T G of Alg. 3) for float32 data.
//
// v_mfma_f32_4x4x1_16b_f32: sixteen independent 4x4 outer products per
// instruction, so the narrow side of this skinny contraction (ell = r + p rows
// of Q^T) is padded to a multiple of 4 only (ell = 35 -> 36).  Operand layout
// (checked on the device): lane l = 4 blk + t holds A[blk][t] and B[blk][t];
// accumulator register v of lane l holds D[blk][v][t].
//
// A wave owns 256 consecutive unfolding columns (four per lane, so every row of
// the strip is one 1 KiB load) and streams all J rows of them from HBM, eight
// rows in flight; Q^T is held in LDS.  The MFMA blocks are sixteen groups of
// four columns, the four lanes' adjacent columns are four separate accumulator
// sets.  The result is stored in the (L, ell, R) layout directly.  When R == 1
// each lane streams one row of the (L, J) matrix instead.
#include "rt_kernels.hpp"
#include "rt_philox.hpp"

namespace rt {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int MK_NQ = 16;  // max column quads (ell <= 64)

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// ---- projection -------------------------------------------------------------------------

constexpr int PM_DEPTH = 16;  // rows of the strip in flight per lane (a shallower ring leaves HBM idle)
// Rows of Q staged in LDS at a time: as many as fit in 96 KiB (one workgroup per
// CU with the widest strips) or 48 KiB, so that for the usual mode sizes all of
// Q is staged once and the load ring is never drained by a barrier mid-strip.
template <int QW, int SETS>
struct PmChunk {
    static constexpr int bytes = SETS == 4 ? 96 * 1024 : 48 * 1024;
    static constexpr int rows = (bytes / (16 * QW)) / 16 * 16;
};
constexpr int PR1_QCH = 128;  // the same for the last-mode kernel

// B[l, k, r] = sum_i Q[i, k] G[l, i, r].  Each wave owns a strip of 64 * SETS
// consecutive unfolding columns, SETS adjacent columns per lane (one vector load
// per row), and streams all J rows of the strip.  Requires R % SETS == 0.
// NQ: column quads of the output (ell <= 4 NQ).
// gridDim.y > 1 splits the contraction: block row y sums the rows
// [y jchunk, (y + 1) jchunk) of the mode and writes its partial result at
// B + y * split_stride (the caller then adds the partials in a fixed order).
template <int NQ, int SETS, int DEPTH = PM_DEPTH, bool ROLL = false>
__global__ __launch_bounds__(256) void project_mfma_kernel(const float* __restrict__ G, int64_t L, int64_t Jfull,
                                                           int64_t ldj, int64_t R, const float* __restrict__ Qfull,
                                                           int64_t ldq, int ell, float* __restrict__ Bbase, int64_t ldk,
                                                           int64_t koff, double* __restrict__ nrm2_partial,
                                                           int64_t jchunk, int64_t split_stride) {
    const int64_t jb = (int64_t)blockIdx.y * jchunk;
    const int64_t J = (Jfull - jb < jchunk ? Jfull - jb : jchunk);
    const float* Q = Qfull + jb * ldq;
    float* B = Bbase + (int64_t)blockIdx.y * split_stride;
    typedef float vec __attribute__((ext_vector_type(SETS)));
    constexpr int QW = (NQ + 3) / 4 * 4;                    // padded quads per Q row in LDS
    constexpr int PM_QCH = PmChunk<QW, SETS>::rows;
    __shared__ __align__(16) float qs[PM_QCH * 4 * QW];     // [i][t][j] = Q[i][4 j + t]
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int t = lane & 3;
    const int64_t K = L * R;
    constexpr int SW = 64 * SETS;                           // strip width (columns)
    const int64_t nstrips = (K + SW - 1) / SW;
    double nrm = 0.0;
    // set s of lane l holds B[4 j + v][c + s] in register v of acc[s][j]
    auto store = [&](const f4 (&acc)[SETS][NQ], int64_t l, int64_t r) {
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = 4 * j + v;
                if (k < ell) {
                    vec o;
#pragma unroll
                    for (int s = 0; s < SETS; ++s) o[s] = acc[s][j][v];
                    *reinterpret_cast<vec*>(B + (l * ldk + koff + k) * R + r) = o;
                    if (nrm2_partial)
#pragma unroll
                        for (int s = 0; s < SETS; ++s) nrm += (double)o[s] * o[s];
                }
            }
        }
    };
    // ROLL, for short modes (the launch checks: no contraction split, J <= 64,
    // all of Q staged at once, J a multiple of the ring depth): Q is staged once,
    // and the load ring rolls on from one strip of the wave into its next, so the
    // loads never drain between strips.  The ring slot d always holds row d of
    // the current group of DEPTH rows.
    if constexpr (ROLL) {
        for (int e = tid; e < PM_QCH * 4 * QW; e += 256) {
            const int ii = e / (4 * QW), tt = (e / QW) & 3, j = e % QW;
            const int k = 4 * j + tt;
            qs[e] = (ii < J && k < ell) ? Q[ii * ldq + k] : 0.f;
        }
        __syncthreads();
        const int64_t sstep = (int64_t)gridDim.x * 4;
        // the strip's first-row pointer (G itself for a strip past the end: its
        // loads stay inside the first J rows and are never used)
        auto strip_ptr = [&](int64_t strip, bool& ok, int64_t& l, int64_t& r) -> const float* {
            const int64_t c = strip * SW + SETS * lane;
            ok = strip < nstrips && c < K;
            l = 0;
            r = 0;
            if (ok) { l = c / R; r = c - l * R; }
            return ok ? G + l * ldj * R + r : G;
        };
        int64_t strip = (int64_t)blockIdx.x * 4 + wave;
        bool ok;
        int64_t l, r;
        const float* gq = strip_ptr(strip, ok, l, r);
        vec ring[DEPTH];
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) ring[d] = *reinterpret_cast<const vec*>(gq + (int64_t)d * R);
        for (; strip < nstrips; strip += sstep) {
            bool okn;
            int64_t ln, rn;
            const float* gn = strip_ptr(strip + sstep, okn, ln, rn);
            f4 acc[SETS][NQ];
#pragma unroll
            for (int s = 0; s < SETS; ++s)
#pragma unroll
                for (int j = 0; j < NQ; ++j) acc[s][j] = f4{0.f, 0.f, 0.f, 0.f};
            for (int ii = 0; ii < J; ii += DEPTH) {
                const bool last = ii + DEPTH >= J;
#pragma unroll
                for (int d = 0; d < DEPTH; ++d) {
                    const vec x = ring[d];
                    const float* src = last ? gn + (int64_t)d * R : gq + (int64_t)(ii + DEPTH + d) * R;
                    ring[d] = *reinterpret_cast<const vec*>(src);
                    const float* qrow = &qs[((ii + d) * 4 + t) * QW];
                    float av[QW];
#pragma unroll
                    for (int j4 = 0; j4 < QW; j4 += 4) {
                        const f4 q = *reinterpret_cast<const f4*>(qrow + j4);
                        av[j4] = q.x; av[j4 + 1] = q.y; av[j4 + 2] = q.z; av[j4 + 3] = q.w;
                    }
#pragma unroll
                    for (int j = 0; j < NQ; ++j)
#pragma unroll
                        for (int s = 0; s < SETS; ++s) acc[s][j] = mfma4(av[j], x[s], acc[s][j]);
                }
            }
            if (ok) store(acc, l, r);
            gq = gn;
            ok = okn;
            l = ln;
            r = rn;
        }
    } else
    for (int64_t s0 = (int64_t)blockIdx.x * 4; s0 < nstrips; s0 += (int64_t)gridDim.x * 4) {
        const int64_t strip = s0 + wave;
        const int64_t c = strip * SW + SETS * lane;          // this lane's columns c .. c + SETS - 1
        const bool valid = strip < nstrips && c < K;
        int64_t l = 0, r = 0;
        if (valid) { l = c / R; r = c - l * R; }
        const float* gp = G + (l * ldj + jb) * R + r;
        f4 acc[SETS][NQ];
#pragma unroll
        for (int s = 0; s < SETS; ++s)
#pragma unroll
            for (int j = 0; j < NQ; ++j) acc[s][j] = f4{0.f, 0.f, 0.f, 0.f};
        for (int64_t i0 = 0; i0 < J; i0 += PM_QCH) {
            const int rows = (int)((J - i0) < PM_QCH ? (J - i0) : PM_QCH);
            __syncthreads();
            for (int e = tid; e < PM_QCH * 4 * QW; e += 256) {
                const int ii = e / (4 * QW), tt = (e / QW) & 3, j = e % QW;
                const int k = 4 * j + tt;
                qs[e] = (ii < rows && k < ell) ? Q[(i0 + ii) * ldq + k] : 0.f;
            }
            __syncthreads();
            // Ring of DEPTH rows in flight.  The loads are unconditional (row index
            // clamped to the chunk, lanes without a column read column 0), so the
            // compiler keeps DEPTH of them outstanding instead of draining the queue
            // at every row; the rows past the chunk are loaded but never used.
            const float* gq = valid ? gp + i0 * R : G;
            vec ring[DEPTH];
#pragma unroll
            for (int d = 0; d < DEPTH; ++d)
                ring[d] = *reinterpret_cast<const vec*>(gq + (int64_t)(d < rows ? d : rows - 1) * R);
            auto step = [&](int row, const vec& x) {
                const float* qrow = &qs[(row * 4 + t) * QW];
                float av[QW];
#pragma unroll
                for (int j4 = 0; j4 < QW; j4 += 4) {
                    const f4 q = *reinterpret_cast<const f4*>(qrow + j4);
                    av[j4] = q.x; av[j4 + 1] = q.y; av[j4 + 2] = q.z; av[j4 + 3] = q.w;
                }
#pragma unroll
                for (int j = 0; j < NQ; ++j)
#pragma unroll
                    for (int s = 0; s < SETS; ++s) acc[s][j] = mfma4(av[j], x[s], acc[s][j]);
            };
            const int nfull = rows / DEPTH * DEPTH;
            for (int ii = 0; ii < nfull; ii += DEPTH) {
#pragma unroll
                for (int d = 0; d < DEPTH; ++d) {
                    const vec x = ring[d];
                    const int nxt = ii + DEPTH + d;
                    ring[d] = *reinterpret_cast<const vec*>(gq + (int64_t)(nxt < rows ? nxt : rows - 1) * R);
                    step(ii + d, x);
                }
            }
#pragma unroll
            for (int d = 0; d < DEPTH; ++d)
                if (nfull + d < rows) step(nfull + d, ring[d]);
        }
        if (valid) store(acc, l, r);
    }
    if (nrm2_partial) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        __syncthreads();
        if (lane == 0) red[wave] = nrm;
        __syncthreads();
        if (tid == 0) nrm2_partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// ring depth per strip width (measured on a 512 x 262144 unfolding: 16 rows for
// 4 columns per lane, 8 rows for 2)
template <int SETS>
struct PmDepth { static constexpr int value = SETS == 2 ? 8 : 16; };

template <int NQ, int SETS>
hipError_t launch_pm(const ProjectPlan& p, const float* G, Shape3 s, int64_t ldj, const float* Q, int64_t ldq, int ell,
                     float* B, int64_t ldk, int64_t koff, double* nrm2, hipStream_t stream) {
    constexpr int D = PmDepth<SETS>::value;
    constexpr int QCH = PmChunk<(NQ + 3) / 4 * 4, SETS>::rows;
    // the rolling ring pays off for short modes only (measured: 48 rows gain,
    // 128 and 512 rows lose)
    if (p.nsplit == 1 && s.J <= 64 && s.J <= QCH && s.J % D == 0)
        hipLaunchKernelGGL((project_mfma_kernel<NQ, SETS, D, true>), dim3(p.nwg, 1), dim3(256), 0, stream, G, s.L,
                           s.J, ldj, s.R, Q, ldq, ell, B, ldk, koff, nrm2, p.jchunk, p.split_stride);
    else
        hipLaunchKernelGGL((project_mfma_kernel<NQ, SETS, D, false>), dim3(p.nwg, p.nsplit), dim3(256), 0, stream,
                           G, s.L, s.J, ldj, s.R, Q, ldq, ell, B, ldk, koff, nrm2, p.jchunk, p.split_stride);
    return hipGetLastError();
}

// Projection of the last mode (R == 1): B[l, k] = sum_i G[l, i] Q[i, k], a plain
// row-major (L x J) times (J x ell) product.  Each wave owns 64 rows l (sixteen
// MFMA blocks of four rows); every lane streams its own row of G, four
// consecutive i at a time (one 16-byte load when J % 4 == 0), and Q^T sits in
// LDS in chunks of QCH rows.
template <int NQ>
__global__ __launch_bounds__(256) void project_r1_mfma_kernel(const float* __restrict__ Gfull, int64_t L, int64_t Jfull,
                                                              int64_t ldj, const float* __restrict__ Qfull, int64_t ldq,
                                                              int ell, float* __restrict__ Bbase, int64_t ldk, int64_t koff,
                                                              double* __restrict__ nrm2_partial, int64_t jchunk,
                                                              int64_t split_stride) {
    const int64_t jb = (int64_t)blockIdx.y * jchunk;
    const int64_t J = (Jfull - jb < jchunk ? Jfull - jb : jchunk);
    const float* G = Gfull + jb;
    const float* Q = Qfull + jb * ldq;
    float* B = Bbase + (int64_t)blockIdx.y * split_stride;
    constexpr int QW = (NQ + 3) / 4 * 4;
    __shared__ __align__(16) float qs[PR1_QCH * 4 * QW];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int blk = lane >> 2, t = lane & 3;
    const int64_t l = (int64_t)blockIdx.x * 256 + wave * 64 + lane;     // the row this lane streams
    const bool lvalid = l < L;
    const float* grow = G + (lvalid ? l : 0) * ldj;
    const bool vec4 = (J % 4 == 0) && (ldj % 4 == 0) && ((((uintptr_t)G) & 15) == 0) && (jb % 4 == 0);
    f4 acc[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int64_t i0 = 0; i0 < J; i0 += PR1_QCH) {
        const int rows = (int)((J - i0) < PR1_QCH ? (J - i0) : PR1_QCH);
        __syncthreads();
        for (int e = tid; e < PR1_QCH * 4 * QW; e += 256) {
            const int ii = e / (4 * QW), tt = (e / QW) & 3, j = e % QW;
            const int k = 4 * j + tt;
            qs[e] = (ii < rows && k < ell) ? Q[(i0 + ii) * ldq + k] : 0.f;
        }
        __syncthreads();
        for (int ii = 0; ii < rows; ii += 4) {
            // this lane's four G values G[l, i0+ii .. +3]; the MFMA block of lane
            // (blk, t) uses A = G[4 blk + v, i] via the lane that owns row 4 blk + v
            f4 x = f4{0.f, 0.f, 0.f, 0.f};
            if (lvalid) {
                if (vec4 && ii + 3 < rows) x = *reinterpret_cast<const f4*>(grow + i0 + ii);
                else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) x[u] = (ii + u < rows) ? grow[i0 + ii + u] : 0.f;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (ii + u < rows) {
                    const float* qrow = &qs[((ii + u) * 4 + t) * QW];
                    float bv[QW];
#pragma unroll
                    for (int j4 = 0; j4 < QW; j4 += 4) {
                        const f4 q = *reinterpret_cast<const f4*>(qrow + j4);
                        bv[j4] = q.x; bv[j4 + 1] = q.y; bv[j4 + 2] = q.z; bv[j4 + 3] = q.w;
                    }
#pragma unroll
                    for (int j = 0; j < NQ; ++j) acc[j] = mfma4(x[u], bv[j], acc[j]);
                }
            }
        }
    }
    // lane (blk, t) holds B[4 blk + v][4 j + t] in register v of acc[j]
    double nrm = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t lr = (int64_t)blockIdx.x * 256 + wave * 64 + 4 * blk + v;
        if (lr < L) {
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                const int k = 4 * j + t;
                if (k < ell) {
                    const float o = acc[j][v];
                    B[lr * ldk + koff + k] = o;
                    nrm += (double)o * o;
                }
            }
        }
    }
    if (nrm2_partial) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        __syncthreads();
        if (lane == 0) red[wave] = nrm;
        __syncthreads();
        if (tid == 0) nrm2_partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

template <int NQ>
hipError_t launch_pr1(const ProjectPlan& p, const float* G, Shape3 s, int64_t ldj, const float* Q, int64_t ldq, int ell,
                      float* B, int64_t ldk, int64_t koff, double* nrm2, hipStream_t stream) {
    hipLaunchKernelGGL((project_r1_mfma_kernel<NQ>), dim3(p.nwg, p.nsplit), dim3(256), 0, stream, G, s.L, s.J, ldj, Q,
                       ldq, ell, B, ldk, koff, nrm2, p.jchunk, p.split_stride);
    return hipGetLastError();
}

// B[l, koff + k, r] = sum_{s < nsplit} part[s][l][k][r] (in fp64, s = 0, 1, ...,
// rounded once), k < ell; optionally sum B^2 (fp64) per workgroup.
__global__ __launch_bounds__(256) void project_reduce_kernel(const float* __restrict__ part, int nsplit,
                                                             int64_t L, int ell, int64_t R, float* __restrict__ B,
                                                             int64_t ldk, int64_t koff, double* __restrict__ nrm2_partial) {
    __shared__ double red[4];
    const int64_t n = L * ell * R;
    const int64_t stride = n;
    const bool contiguous = ldk == ell && koff == 0;   // B has the partials' layout
    double nrm = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        double acc[8];
        double sum = 0.0;
        for (int s0 = 0; s0 < nsplit; s0 += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] = (s0 + u < nsplit) ? (double)part[(int64_t)(s0 + u) * stride + e] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) sum += acc[u];
        }
        const float v = (float)sum;
        if (contiguous) {
            B[e] = v;
        } else {
            const uint64_t lk = (uint64_t)e / (uint64_t)R;
            const int64_t r = e - (int64_t)lk * R;
            const int64_t l = (int64_t)(lk / (uint64_t)ell), k = (int64_t)lk - l * ell;
            B[(l * ldk + koff + k) * R + r] = v;
        }
        nrm += (double)v * v;
    }
    if (nrm2_partial) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
        __syncthreads();
        if (threadIdx.x == 0) nrm2_partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

}  // namespace

// Columns per lane: wide strips for large unfoldings (fewer LDS reads of Q per
// MFMA), narrow ones for small unfoldings (more waves).
int project_sets(Shape3 s, int ell) {
    const int nq = (ell + 3) / 4;
    const int64_t K = s.L * s.R;
    if (nq <= 10 && s.R % 4 == 0 && K >= ((int64_t)1 << 18)) return 4;
    if (s.R % 2 == 0 && K >= ((int64_t)1 << 16)) return 2;
    return 1;
}

bool project_mfma_ok(Shape3 s, int ell, const void* G, const void* B, int64_t koff) {
    if (ell > 4 * MK_NQ || s.R < 2) return false;
    const int sets = project_sets(s, ell);
    const uintptr_t al = 4u * (uintptr_t)sets - 1u;
    return (((uintptr_t)G & al) == 0) && (((uintptr_t)B & al) == 0) && ((koff * s.R) % sets == 0);
}

// Split of the contraction so that the launch has >= ~1024 waves, chunks of at
// least 32 rows (a multiple of 4).
static void split_plan(ProjectPlan& p, int64_t waves, Shape3 s, int ell) {
    int nsplit = 1;
    while (waves * nsplit < 1024 && s.J / (2 * nsplit) >= 32) nsplit *= 2;
    p.nsplit = nsplit;
    p.jchunk = nsplit > 1 ? ((s.J + nsplit - 1) / nsplit + 3) / 4 * 4 : s.J;
    p.nsplit = (int)((s.J + p.jchunk - 1) / p.jchunk);
    p.split_stride = s.L * (int64_t)ell * s.R;
    p.partial_elems = p.nsplit > 1 ? (size_t)p.nsplit * (size_t)p.split_stride : 0;
}

void plan_project_mfma(ProjectPlan& p, Shape3 s, int ell) {
    p.sets = project_sets(s, ell);
    const int64_t nstrips = (s.L * s.R + 64 * p.sets - 1) / (64 * p.sets);
    int64_t g = (nstrips + 3) / 4;
    if (g > 2048) g = 2048;
    p.nwg = (int)(g < 1 ? 1 : g);
    split_plan(p, nstrips, s, ell);
}

hipError_t launch_project_mfma(const ProjectPlan& p, const float* G, Shape3 s, int64_t ldj, const float* Q, int64_t ldq,
                               int ell, float* B, int64_t ldk, int64_t koff, double* nrm2, hipStream_t stream) {
    const int nq = (ell + 3) / 4;
    const int sets = p.sets;
#define RT_PM(NQV, S) return launch_pm<NQV, S>(p, G, s, ldj, Q, ldq, ell, B, ldk, koff, nrm2, stream)
    if (sets == 4) {
        if (nq <= 2) RT_PM(2, 4);
        if (nq <= 4) RT_PM(4, 4);
        if (nq <= 7) RT_PM(7, 4);
        if (nq <= 9) RT_PM(9, 4);
        RT_PM(10, 4);
    }
    if (sets == 2) {
        if (nq <= 4) RT_PM(4, 2);
        if (nq <= 9) RT_PM(9, 2);
        if (nq <= 12) RT_PM(12, 2);
        RT_PM(16, 2);
    }
    if (nq <= 4) RT_PM(4, 1);
    if (nq <= 9) RT_PM(9, 1);
    if (nq <= 12) RT_PM(12, 1);
    RT_PM(16, 1);
#undef RT_PM
}

void plan_project_r1_mfma(ProjectPlan& p, Shape3 s, int ell) {
    int64_t g = (s.L + 255) / 256;
    p.nwg = (int)(g < 1 ? 1 : g);
    p.sets = 1;
    split_plan(p, 4 * g, s, ell);
}

hipError_t launch_project_r1_mfma(const ProjectPlan& p, const float* G, Shape3 s, int64_t ldj, const float* Q,
                                  int64_t ldq, int ell, float* B, int64_t ldk, int64_t koff, double* nrm2,
                                  hipStream_t stream) {
    const int nq = (ell + 3) / 4;
#define RT_PR1(NQV) return launch_pr1<NQV>(p, G, s, ldj, Q, ldq, ell, B, ldk, koff, nrm2, stream)
    if (nq <= 2) RT_PR1(2);
    if (nq <= 4) RT_PR1(4);
    if (nq <= 7) RT_PR1(7);
    if (nq <= 9) RT_PR1(9);
    if (nq <= 12) RT_PR1(12);
    RT_PR1(16);
#undef RT_PR1
}

int plan_project_reduce(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 1024) g = 1024;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_project_reduce(const float* part, int nsplit, Shape3 s, int ell, float* B, int64_t ldk, int64_t koff,
                                 double* nrm2, int nwg, hipStream_t stream) {
    hipLaunchKernelGGL(project_reduce_kernel, dim3(nwg), dim3(256), 0, stream, part, nsplit, s.L, ell, s.R, B, ldk,
                       koff, nrm2);
    return hipGetLastError();
}

}  // namespace rt
