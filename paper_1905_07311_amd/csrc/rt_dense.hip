// Small dense FP64 kernels of the hot path, each run by one workgroup:
//   * orth      - Q = orth(Y) for the J x ell sketch (§2.4 Alg. 1 step 2): CholeskyQR2
//                 (Fukaya et al. 2014) with an acceptance test on the Cholesky pivots,
//                 falling back to Householder QR when the sketch is too ill-conditioned
//                 or numerically rank deficient (Householder always returns ell
//                 orthonormal columns, so a rank-deficient sketch is padded with
//                 zero-weight orthonormal directions).
//   * truncate  - thin SVD of B through the eigendecomposition of the fp64 Gram
//                 B B^T (parallel cyclic Jacobi), rank choice and the factor
//                 A_n = Q U_B(:, 1:k) (Alg. 1 steps 4-6; adaptive truncation rule).
//   * block_orth- one block of the adaptive range finder (§4): block Gram-Schmidt
//                 against the basis so far, done twice, then Householder QR and a
//                 one-sided Jacobi SVD of the small R factor to drop the directions
//                 whose singular values fall below drop * ||Y||_F.
// All matrices are row-major; the workgroup has 256 threads; ell <= LMAX = 64.
#include <float.h>
#include <math.h>

#include "rt_kernels.hpp"

// Phase timestamps for offline tuning builds; empty in the library.
#ifndef RT_DENSE_TRACE
#define RT_DENSE_TRACE(slot)
#define RT_DENSE_TRACE_VAL(slot, v)
#endif

namespace rt {

namespace {

constexpr int NT = 512;              // threads of every dense kernel (8 waves)
constexpr int NRG = NT / LMAX;       // row groups of the Householder column sweeps
constexpr int LDW = LMAX + 1;
typedef double Mat[LMAX][LDW];

__device__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double readlane64(double v, int l) {
    const unsigned long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// v moved across lanes by the DPP control CTRL for the rows in RMASK; lanes of
// the other rows get 0.
template <int CTRL, int RMASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, RMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, RMASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes of a wave through DPP (every lane active), returned to
// every lane: quad swaps, half-row and row mirrors give every lane its row's
// sum; row_bcast:15 and row_bcast:31 carry rows 0-2 into row 3, whose lane 63
// ends with the total (a fixed order, so the same bits on every call).
__device__ __forceinline__ double wave_total(double v) {
    v += dpp_f64<0xb1, 0xf>(v);     // quad_perm [1,0,3,2]
    v += dpp_f64<0x4e, 0xf>(v);     // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xf>(v);    // row_half_mirror
    v += dpp_f64<0x140, 0xf>(v);    // row_mirror
    v += dpp_f64<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return readlane64(v, 63);
}

// Sum over aligned groups of G = 8 or 16 lanes through DPP, returned to every
// lane of the group.
template <int G>
__device__ __forceinline__ double group_total(double v) {
    v += dpp_f64<0xb1, 0xf>(v);     // quad_perm [1,0,3,2]
    v += dpp_f64<0x4e, 0xf>(v);     // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xf>(v);    // row_half_mirror: 8-lane sums
    if (G == 16) v += dpp_f64<0x140, 0xf>(v);    // row_mirror: 16-lane sums
    return v;
}


// dst[e] = src(e) for e < n by `nthr` threads with PER loads in flight per
// thread (all issued before the first store), for the small staging copies.
template <int PER, typename F, typename G>
__device__ __forceinline__ void batched_copy(int n, int tid, int nthr, F load, G store) {
    for (int e0 = 0; e0 < n; e0 += PER * nthr) {
        double v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = e0 + u * nthr + tid;
            v[u] = e < n ? load(e) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = e0 + u * nthr + tid;
            if (e < n) store(e, v[u]);
        }
    }
}

// Sum over the workgroup (every thread gets the result).
__device__ __forceinline__ double blk_sum(double v, double* red) {
    const int tid = threadIdx.x;
    v = wave_sum(v);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < NT / 64; ++w) r += red[w];
    __syncthreads();
    return r;
}

// W = Y^T Y (n x n) for Y (J x n, row stride ldy) in global memory.  Each thread
// owns one 4x4 tile of the upper triangle and every G-th row (G a power of two,
// the G threads of a tile adjacent in one wave); rows are loaded two at a time
// so that 16 loads are in flight per thread, and the G partial tiles are summed
// with shuffles.
__device__ __attribute__((noinline)) void blk_gram(const double* Y, int64_t J, int n, int64_t ldy, Mat& W) {
    const int tid = threadIdx.x;
    const int nt = (n + 3) / 4;
    const int npt = nt * (nt + 1) / 2;
    int G = 64;
    while (G > 1 && G * npt > NT) G >>= 1;
    const int pr = tid / G, g = tid % G;
    if (pr < npt) {
        int ti = 0, rem = pr;
        while (rem >= nt - ti) { rem -= nt - ti; ++ti; }
        const int tj = ti + rem;
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        int64_t i = g;
        for (; i + G < J; i += 2 * G) {
            double x[2][4], y[2][4];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double* row = Y + (i + u * G) * ldy;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    x[u][a] = (4 * ti + a < n) ? row[4 * ti + a] : 0.0;
                    y[u][a] = (4 * tj + a < n) ? row[4 * tj + a] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] += x[u][a] * y[u][b];
        }
        for (; i < J; i += G) {
            const double* row = Y + i * ldy;
            double x[4], y[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                x[a] = (4 * ti + a < n) ? row[4 * ti + a] : 0.0;
                y[a] = (4 * tj + a < n) ? row[4 * tj + a] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double v = acc[a][b];
                for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                acc[a][b] = v;
            }
        if (g == 0) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int r = 4 * ti + a, c = 4 * tj + b;
                    if (r < n && c < n) { W[r][c] = acc[a][b]; W[c][r] = acc[a][b]; }
                }
        }
    }
    __syncthreads();
}

// In-place Cholesky W + shift I = L L^T (lower triangle), one barrier per
// elimination step: every thread reads the pivot and updates its share of the
// trailing triangle with W[i][j] -= W[i][k] W[j][k] / W[k][k] (a 32 x 16 grid of
// threads covers the trailing block); the columns are scaled by
// 1/sqrt(pivot) at the end and invd[k] = 1 / L[k][k] is left for the solves.
// Returns false on a non-positive or non-finite pivot; *min_ratio = min_k
// pivot_k / W_kk(original), the squared sine of the angle between column k and
// the span of the previous columns.
template <int NTH = NT>
__device__ bool blk_cholesky(Mat& W, int n, double shift, double* diag0, double* min_ratio, int* flag, double* invd) {
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;      // (NTH / 16) x 16 grid of threads
    __syncthreads();
    if (tid < n) {
        diag0[tid] = W[tid][tid];
        W[tid][tid] += shift;
    }
    __syncthreads();
    double mr = 1.0;
    bool ok = true;
    for (int k = 0; k < n; ++k) {
        const double piv = W[k][k];
        if (!(piv > 0.0) || !isfinite(piv) || !(diag0[k] + shift > 0.0)) { ok = false; break; }
        mr = fmin(mr, piv / (diag0[k] + shift));
        const double rp = 1.0 / piv;
        for (int i = k + 1 + ty; i < n; i += NTH / 16) {
            const double wik = W[i][k] * rp;
            for (int j = k + 1 + tx; j <= i; j += 16) W[i][j] -= wik * W[j][k];
        }
        __syncthreads();
    }
    if (ok) {
        if (tid < n) invd[tid] = 1.0 / sqrt(W[tid][tid]);
        __syncthreads();
        for (int i = ty; i < n; i += NTH / 16)
            for (int k = tx; k < i; k += 16) W[i][k] *= invd[k];
        __syncthreads();
        if (tid < n) W[tid][tid] = 1.0 / invd[tid];
    }
    __syncthreads();
    if (tid == 0) { flag[0] = ok ? 0 : 1; min_ratio[0] = mr; }
    __syncthreads();
    return ok;
}

// Y <- Y R^{-1} with R = L^T (L lower, in W; invd = 1 / diag(L)), row by row
// (right-looking): z_j = y_j / L[j][j], then y_k -= z_j L[k][j] for k > j, with the
// row held in registers and L read with wave-uniform (broadcast) LDS accesses.
template <int NR>
__device__ void blk_trsm_rows(double* Y, int64_t J, int n, int64_t ldy, const Mat& W, const double* invd) {
    const int tid = threadIdx.x;
    for (int64_t i = tid; i < J; i += NT) {
        double y[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) y[j] = (j < n) ? Y[i * ldy + j] : 0.0;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (j < n) {
                const double zj = y[j] * invd[j];
                y[j] = zj;
#pragma unroll
                for (int k = j + 1; k < NR; ++k) {
                    y[k] -= zj * W[k][j];
                    if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);   // bound the hoisted loads
                }
            }
            __builtin_amdgcn_sched_barrier(0);   // keep the column loads of step j local
        }
#pragma unroll
        for (int j = 0; j < NR; ++j)
            if (j < n) Y[i * ldy + j] = y[j];
    }
    __syncthreads();
}

// Householder QR of A (J x n, ld), overwritten by the explicit thin Q (J x n).
// Returns in rdiag[k] the diagonal of R.  Works for any rank: a zero column gets
// the identity reflector, so Q always has n orthonormal columns.
__device__ void blk_householder_q(double* A, int64_t J, int n, int64_t lda, double* V /* J x n scratch */,
                                  double* tau, double* v0, double* rdiag, double* red, double* wbuf) {
    const int tid = threadIdx.x;
    const int rg = tid / LMAX, jj = tid % LMAX;
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int64_t i = k + tid; i < J; i += NT) { const double x = A[i * lda + k]; s += x * x; }
        s = blk_sum(s, red);
        if (tid == 0) {
            const double x0 = A[(int64_t)k * lda + k];
            const double alpha = sqrt(s);
            if (alpha == 0.0) {
                tau[k] = 0.0; v0[k] = 0.0; rdiag[k] = 0.0;
            } else {
                const double beta = (x0 >= 0.0) ? -alpha : alpha;
                const double vk = x0 - beta;
                const double vtv = s - x0 * x0 + vk * vk;
                tau[k] = vtv > 0.0 ? 2.0 / vtv : 0.0;
                v0[k] = vk;
                rdiag[k] = beta;
            }
        }
        __syncthreads();
        // copy the reflector into V[:, k] (rows >= k)
        for (int64_t i = k + tid; i < J; i += NT) V[i * n + k] = (i == k) ? v0[k] : A[i * lda + k];
        __syncthreads();
        // apply H_k to the trailing columns j > k
        const double tk = tau[k];
        if (tk != 0.0) {
            double w = 0.0;
            const int j = jj;
            if (j > k && j < n)
                for (int64_t i = k + rg; i < J; i += NRG) w += V[i * n + k] * A[i * lda + j];
            wbuf[rg * LDW + jj] = w;
            __syncthreads();
            if (rg == 0) {
                double t = 0.0;
                for (int g = 0; g < NRG; ++g) t += wbuf[g * LDW + jj];
                wbuf[NRG * LDW + jj] = t * tk;
            }
            __syncthreads();
            if (j > k && j < n) {
                const double f = wbuf[NRG * LDW + j];
                for (int64_t i = k + rg; i < J; i += NRG) A[i * lda + j] -= f * V[i * n + k];
            }
            __syncthreads();
        }
    }
    // explicit Q = H_0 H_1 ... H_{n-1} [I; 0]
    for (int64_t e = tid; e < J * n; e += NT) {
        const int64_t i = e / n;
        const int j = (int)(e % n);
        A[i * lda + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;            // uniform: tau lives in shared memory
        double w = 0.0;
        const int j = jj;
        if (j >= k && j < n)
            for (int64_t i = k + rg; i < J; i += NRG) w += V[i * n + k] * A[i * lda + j];
        wbuf[rg * LDW + jj] = w;
        __syncthreads();
        if (rg == 0) {
            double t = 0.0;
            for (int g = 0; g < NRG; ++g) t += wbuf[g * LDW + jj];
            wbuf[NRG * LDW + jj] = t * tk;
        }
        __syncthreads();
        if (j >= k && j < n) {
            const double f = wbuf[NRG * LDW + j];
            for (int64_t i = k + rg; i < J; i += NRG) A[i * lda + j] -= f * V[i * n + k];
        }
        __syncthreads();
    }
}

// Jacobi rotation (c, s) for the 2 x 2 symmetric block [[app, apq], [apq, aqq]]
// under A <- R^T A R with R = [c s; -s c].  Rotations with apq^2 <= 1e-36 |app aqq|
// are skipped.  The tangent of the smaller angle is formed in single precision
// from the block scaled by a power of two (an inexact angle only slows
// convergence down to the single-precision level per rotation); c = 1 / sqrt(1 +
// t^2) is refined from the single-precision reciprocal square root by two
// Newton steps and s = t c, so the rotation is orthogonal to double precision
// and the similarity is exact up to rounding.
__device__ __forceinline__ void jrot(double app, double aqq, double apq, double& c, double& s) {
    c = 1.0; s = 0.0;
    const double aa = fabs(apq);
    if (!(aa > 1e-300) || !(aa * aa > 1e-36 * fabs(app * aqq))) return;
    const double d = aqq - app;
    const int e = ilogb(fmax(fabs(d), aa));
    const float df = (float)ldexp(d, -e), af = (float)ldexp(apq, -e);
    const float r = __builtin_amdgcn_sqrtf(df * df + 4.0f * af * af);
    const float tf = 2.0f * af * __builtin_amdgcn_rcpf(df >= 0.0f ? df + r : df - r);
    const double t = (double)tf;
    const double x = fma(t, t, 1.0);
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    y = y * fma(-0.5 * x, y * y, 1.5);
    y = y * fma(-0.5 * x, y * y, 1.5);
    c = y;
    s = t * y;
}

// Rank positions: perm[t] = index of the t-th largest diagonal entry (ties by index).
__device__ void blk_sort_desc(const Mat& A, int n, int* perm, double* lam) {
    const int tid = threadIdx.x;
    if (tid < n) {
        const double v = A[tid][tid];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double w = A[j][j];
            if (w > v || (w == v && j < tid)) ++rank;
        }
        perm[rank] = tid;
        lam[rank] = v;
    }
    __syncthreads();
}

struct DenseShared {
    Mat W;
    Mat M2;
    Mat stage;
    double red[NT];
    double wbuf[(NRG + 1) * LDW];
    double diag0[LMAX];
    double invd[LMAX];
    double tau[LMAX];
    double v0[LMAX];
    double rdiag[LMAX];
    double minr[1];
    int pairs[LMAX + 2];
    int perm[LMAX];
    int flag[4];
};

template <int NR>
__device__ void cholqr_apply(double* Y, int64_t J, int ell, DenseShared& S) {
    blk_trsm_rows<NR>(Y, J, ell, ell, S.W, S.invd);
}

// gate: when non-null the kernel runs only if gate[0] != 0 (the multi-workgroup
// CholeskyQR2 below did not accept the sketch); Y is then the original sketch.
template <int NR>
__global__ __launch_bounds__(NT) void orth_kernel(double* __restrict__ Y, int64_t J, int ell, float* __restrict__ Qf,
                                                  double* __restrict__ V, double accept_ratio,
                                                  uint32_t* __restrict__ status, const int* __restrict__ gate) {
    if (gate && gate[0] == 0) return;
    __shared__ DenseShared S;
    const int tid = threadIdx.x;
    uint32_t st = 0;
    if (tid == 0) S.flag[1] = 0;
    // keep a copy of Y for the Householder fallback
    double* Ycopy = V + J * (int64_t)ell;
    double nonfinite = 0.0, fro = 0.0;
    const int64_t tot = J * (int64_t)ell;
    for (int64_t e0 = tid; e0 < tot; e0 += 8 * NT) {
        double y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u] = (e0 + u * NT < tot) ? Y[e0 + u * NT] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (e0 + u * NT < tot) {
                Ycopy[e0 + u * NT] = y[u];
                if (!isfinite(y[u])) nonfinite += 1.0;
                else fro += y[u] * y[u];
            }
        }
    }
    nonfinite = blk_sum(nonfinite, S.red);
    fro = blk_sum(fro, S.red);
    RT_DENSE_TRACE(1);
    bool ok = nonfinite == 0.0 && fro > 0.0;
    if (nonfinite != 0.0) st |= 4u;
    if (ok) {
        // CholeskyQR2: accepted when the first factorisation keeps every pivot
        // ratio >= accept_ratio (kappa(Y) ~ 1/sqrt(ratio)) and the second one is
        // nearly orthogonal already (ratio >= 1/2).
        blk_gram(Y, J, ell, ell, S.W);
        RT_DENSE_TRACE(2);
        ok = blk_cholesky(S.W, ell, 0.0, S.diag0, S.minr, S.flag, S.invd) && S.minr[0] >= accept_ratio;
        RT_DENSE_TRACE(3);
        if (!ok) {
            // shifted CholeskyQR3 (Fukaya et al. 2020): factor Y^T Y + s I with
            // s = 11 (J ell + ell (ell + 1)) u ||Y||_F^2, which bounds kappa of
            // Y R^-1 by O(u^-1/2), then CholeskyQR2 on the result.
            blk_gram(Y, J, ell, ell, S.W);
            const double shift = 11.0 * ((double)J * ell + (double)ell * (ell + 1)) * 0x1p-53 * fro;
            ok = blk_cholesky(S.W, ell, shift, S.diag0, S.minr, S.flag, S.invd);
            if (ok) {
                cholqr_apply<NR>(Y, J, ell, S);
                blk_gram(Y, J, ell, ell, S.W);
                ok = blk_cholesky(S.W, ell, 0.0, S.diag0, S.minr, S.flag, S.invd) && S.minr[0] >= accept_ratio;
                // a direction of Y far below sqrt(shift) leaves a pivot ratio near u:
                // Y was numerically rank deficient and Q holds padding directions
                if (ok && S.minr[0] < 1e-6) st |= 1u;
            }
        }
        if (ok) {
            cholqr_apply<NR>(Y, J, ell, S);
            RT_DENSE_TRACE(4);
            blk_gram(Y, J, ell, ell, S.W);
            RT_DENSE_TRACE(5);
            ok = blk_cholesky(S.W, ell, 0.0, S.diag0, S.minr, S.flag, S.invd) && S.minr[0] >= 0.5;
            RT_DENSE_TRACE(6);
            if (ok) cholqr_apply<NR>(Y, J, ell, S);
            RT_DENSE_TRACE(7);
        }
    }
    if (!ok) {
        // Householder QR of the original sketch: unconditionally orthonormal
        for (int64_t e = tid; e < J * ell; e += NT) Y[e] = isfinite(Ycopy[e]) ? Ycopy[e] : 0.0;
        __syncthreads();
        blk_householder_q(Y, J, ell, ell, V, S.tau, S.v0, S.rdiag, S.red, S.wbuf);
        st |= 2u;
        if (tid == 0) {
            double mx = 0.0;
            for (int k = 0; k < ell; ++k) mx = fmax(mx, fabs(S.rdiag[k]));
            for (int k = 0; k < ell; ++k)
                if (!(fabs(S.rdiag[k]) > 1e-12 * mx)) S.flag[1] = 1;
        }
        if (tid == 0 && S.flag[1]) st |= 1u;
    }
    __syncthreads();
    if (Qf)
        for (int64_t e = tid; e < J * ell; e += NT) Qf[e] = (float)Y[e];
    if (tid == 0 && status) status[0] = st;
}

// One adaptive block: Y (J x b) <- (I - Q Q^T) Y twice, then the kept left singular
// vectors of Y are appended to Qall (ld = ldq) at column k.
__global__ __launch_bounds__(NT) void block_orth_kernel(double* __restrict__ Y, int64_t J, int b,
                                                        double* __restrict__ Qall, int ldq, int k, double drop,
                                                        double* __restrict__ V, int* __restrict__ knew,
                                                        float* __restrict__ Qf, const double* __restrict__ y0_ext) {
    __shared__ DenseShared S;
    const int tid = threadIdx.x;
    // y0 = ||Y||_F before the projections (or the caller's, when Y was already
    // projected against earlier basis columns)
    double s = 0.0;
    for (int64_t e = tid; e < J * b; e += NT) s += Y[e] * Y[e];
    const double ys = sqrt(blk_sum(s, S.red));
    const double y0 = y0_ext ? y0_ext[0] : ys;
    // two passes of block Gram-Schmidt: C = Q^T Y (k x b), Y -= Q C
    for (int pass = 0; pass < 2 && k > 0; ++pass) {
        for (int e = tid; e < k * b; e += NT) {
            const int a = e / b, j = e % b;
            double c = 0.0;
            for (int64_t i = 0; i < J; ++i) c += Qall[i * ldq + a] * Y[i * b + j];
            S.W[a][j] = c;
        }
        __syncthreads();
        for (int64_t e = tid; e < J * b; e += NT) {
            const int64_t i = e / b;
            const int j = (int)(e % b);
            double c = 0.0;
            for (int a = 0; a < k; ++a) c += Qall[i * ldq + a] * S.W[a][j];
            Y[e] -= c;
        }
        __syncthreads();
    }
    // Householder QR: V (J x b) keeps the reflectors; R's upper triangle is built
    // from the reflected columns before Q is formed, so save it first.
    // Copy Y to the scratch tail to recover R = Q^T Y afterwards.
    double* Ysave = V + J * (int64_t)b;
    for (int64_t e = tid; e < J * b; e += NT) Ysave[e] = Y[e];
    __syncthreads();
    blk_householder_q(Y, J, b, b, V, S.tau, S.v0, S.rdiag, S.red, S.wbuf);
    // R = Q^T Ysave (b x b)
    for (int e = tid; e < b * b; e += NT) {
        const int a = e / b, j = e % b;
        double c = 0.0;
        for (int64_t i = 0; i < J; ++i) c += Y[i * b + a] * Ysave[i * b + j];
        S.M2[a][j] = c;                       // R (upper up to rounding)
    }
    __syncthreads();
    // one-sided Jacobi on M = R^T: rotate columns of M (rows of R); accumulate in Vr
    if (tid == 0) {
        // M[i][j] = R[j][i]
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) { S.stage[i][j] = S.M2[j][i]; S.W[i][j] = (i == j) ? 1.0 : 0.0; }
        for (int sweep = 0; sweep < 60; ++sweep) {
            bool rotated = false;
            for (int p = 0; p < b - 1; ++p)
                for (int q = p + 1; q < b; ++q) {
                    double al = 0.0, be = 0.0, ga = 0.0;
                    for (int i = 0; i < b; ++i) {
                        al += S.stage[i][p] * S.stage[i][p];
                        be += S.stage[i][q] * S.stage[i][q];
                        ga += S.stage[i][p] * S.stage[i][q];
                    }
                    if (fabs(ga) <= 1e-15 * sqrt(al * be) || ga == 0.0) continue;
                    rotated = true;
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                    for (int i = 0; i < b; ++i) {
                        const double mp = S.stage[i][p], mq = S.stage[i][q];
                        S.stage[i][p] = c * mp - sn * mq;
                        S.stage[i][q] = sn * mp + c * mq;
                        const double vp = S.W[i][p], vq = S.W[i][q];
                        S.W[i][p] = c * vp - sn * vq;
                        S.W[i][q] = sn * vp + c * vq;
                    }
                }
            if (!rotated) break;
        }
        // singular values = column norms of M V; keep sigma > drop * y0, in decreasing order
        double sig[LMAX];
        for (int j = 0; j < b; ++j) {
            double n2 = 0.0;
            for (int i = 0; i < b; ++i) n2 += S.stage[i][j] * S.stage[i][j];
            sig[j] = sqrt(n2);
        }
        int kept = 0;
        bool used[LMAX];
        for (int j = 0; j < b; ++j) used[j] = false;
        for (int t = 0; t < b; ++t) {
            int best = -1;
            for (int j = 0; j < b; ++j)
                if (!used[j] && (best < 0 || sig[j] > sig[best])) best = j;
            used[best] = true;
            if (sig[best] > drop * y0 && y0 > 0.0) S.perm[kept++] = best;
        }
        S.flag[0] = kept;
    }
    __syncthreads();
    const int kept = S.flag[0];
    // new basis columns: Qy * Vr[:, perm[t]]  (Qy in Y, J x b); columns
    // k + kept .. k + b - 1 are zero-filled
    for (int64_t e = tid; e < J * b; e += NT) {
        const int64_t i = e / b;
        const int t = (int)(e % b);
        double c = 0.0;
        if (t < kept) {
            const int j = S.perm[t];
            for (int a = 0; a < b; ++a) c += Y[i * b + a] * S.W[a][j];
        }
        Qall[i * ldq + k + t] = c;
        if (Qf) Qf[i * ldq + k + t] = (float)c;
    }
    if (tid == 0) knew[0] = kept;
}



// ---- truncation (Alg. 1 steps 4-6) --------------------------------------------------------
// Three launches: the eigen-decomposition of the ell x ell Gram W = B B^T and
// the rank choice by one workgroup; A = Q U (J x k) by ceil(J / 64) workgroups,
// each also reporting per column its entry of largest magnitude; and the sign
// fix (each column of A and U flipped so that its largest-|.| entry, lowest
// row on ties, is positive) applied to A and written into U.

// ---- parallel cyclic Jacobi -----------------------------------------------------------
// Round-robin pairing of m = n + (n odd) indices: in step `step` (0 .. m - 2)
// pair t joins indices a and b as below (index m - 1 stays fixed, the others
// rotate), every index once per step; p < q.
__device__ __forceinline__ void jpair(int step, int t, int m, int& p, int& q) {
    int a, b;
    if (t == 0) { a = m - 1; b = step; }
    else {
        a = step + t; if (a >= m - 1) a -= m - 1;
        b = step - t + (m - 1); if (b >= m - 1) b -= m - 1;
    }
    p = a < b ? a : b;
    q = a < b ? b : a;
}

// jrot without early exits (identity where jrot would skip)
__device__ __forceinline__ void jrot_nb(double app, double aqq, double apq, double& c, double& s) {
    const double aa = fabs(apq);
    const bool skip = !(aa > 1e-300) || !(aa * aa > 1e-36 * fabs(app * aqq));
    const double d = aqq - app;
    const int e = ilogb(fmax(fmax(fabs(d), aa), 1e-300));
    const float df = (float)ldexp(d, -e), af = (float)ldexp(apq, -e);
    const float r = __builtin_amdgcn_sqrtf(df * df + 4.0f * af * af);
    const float den = df >= 0.0f ? df + r : df - r;
    const float tf = 2.0f * af * __builtin_amdgcn_rcpf(den == 0.0f ? 1.0f : den);
    const double t = (double)tf;
    const double x = fma(t, t, 1.0);
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    y = y * fma(-0.5 * x, y * y, 1.5);
    y = y * fma(-0.5 * x, y * y, 1.5);
    c = skip ? 1.0 : y;
    s = skip ? 0.0 : t * y;
}

// Parallel cyclic Jacobi, two phases per step: wave 0 computes the rotations
// of the step's pairs from their diagonal blocks (once per pair) into LDS, then
// every thread applies R^T A R to its 2 x 2 blocks of A and V R to its 2 x 2
// blocks of V in place (rows of pair bi, columns of pair bj; the blocks of a
// step are disjoint).  When n is odd, index n is a phantom whose row and column
// stay zero, so its rotations are the identity.  Stops when the off-diagonal sum
// of squares is <= tol ||A||_F^2 (checked once per sweep).  A's diagonal then
// holds the eigenvalues and V's columns the eigenvectors.
__device__ __forceinline__ int jacobi_2p(Mat& A, int n, Mat& V, double tol, double* red, double* cs, int* pq) {
    const int tid = threadIdx.x;
    const int m = (n % 2) ? n + 1 : n;
    const int half = m / 2;
    const int nblk = half * half;
    for (int e = tid; e < m * m; e += NT) {
        const int i = e / m, j = e % m;
        V[i][j] = (i == j && i < n) ? 1.0 : 0.0;
        if (i >= n || j >= n) A[i][j] = 0.0;
    }
    double tot = 0.0;
    for (int e = tid; e < n * n; e += NT) tot += A[e / n][e % n] * A[e / n][e % n];
    tot = blk_sum(tot, red);
    if (tot == 0.0 || n < 2) return 0;
    const bool own0 = tid < nblk, own1 = tid + NT < nblk;
    const int bi0 = own0 ? tid / half : 0, bj0 = own0 ? tid % half : 0;
    const int bi1 = own1 ? (tid + NT) / half : 0, bj1 = own1 ? (tid + NT) % half : 0;
    int sweeps = 0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        for (int step = 0; step < m - 1; ++step) {
            if (tid < half) {
                int p, q;
                jpair(step, tid, m, p, q);
                double c, sn;
                jrot_nb(A[p][p], A[q][q], A[p][q], c, sn);
                cs[2 * tid] = c;
                cs[2 * tid + 1] = sn;
                pq[tid] = p | (q << 8);
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u == 0 ? own0 : own1) {
                    const int bi = u == 0 ? bi0 : bi1, bj = u == 0 ? bj0 : bj1;
                    const int pqi = pq[bi], pqj = pq[bj];
                    const int pi = pqi & 255, qi = pqi >> 8, pj = pqj & 255, qj = pqj >> 8;
                    const double2 rsi = *reinterpret_cast<const double2*>(&cs[2 * bi]);
                    const double2 rsj = *reinterpret_cast<const double2*>(&cs[2 * bj]);
                    const double ci = rsi.x, si = rsi.y, cj = rsj.x, sj = rsj.y;
                    const double a = A[pi][pj], b = A[pi][qj], c = A[qi][pj], d = A[qi][qj];
                    const double vpp = V[pi][pj], vpq = V[pi][qj], vqp = V[qi][pj], vqq = V[qi][qj];
                    const double a1 = ci * a - si * c, b1 = ci * b - si * d;
                    const double c1 = si * a + ci * c, d1 = si * b + ci * d;
                    A[pi][pj] = a1 * cj - b1 * sj;
                    A[pi][qj] = a1 * sj + b1 * cj;
                    A[qi][pj] = c1 * cj - d1 * sj;
                    A[qi][qj] = c1 * sj + d1 * cj;
                    V[pi][pj] = cj * vpp - sj * vpq;
                    V[pi][qj] = sj * vpp + cj * vpq;
                    V[qi][pj] = cj * vqp - sj * vqq;
                    V[qi][qj] = sj * vqp + cj * vqq;
                }
            }
            __syncthreads();
        }
        ++sweeps;
        double off = 0.0;
        for (int e = tid; e < n * n; e += NT) {
            const int i = e / n, j = e - i * n;
            if (i != j) off += A[i][j] * A[i][j];
        }
        off = blk_sum(off, red);
        if (off <= tol * tot) break;
    }
    RT_DENSE_TRACE_VAL(9, sweeps);
    return sweeps;
}

// ---- adaptive block step for blocks of at most 16 columns ----------------------------
// The same result as block_orth_kernel, with Y (J x b) staged in LDS (row stride
// b | 1): y0 = ||Y||_F, two passes of block Gram-Schmidt against Qall[:, :k],
// then a parallel one-sided (Hestenes) Jacobi on the columns of Y: in each step
// of the round-robin schedule wave t rotates the columns of pair t (sums of
// squares and the inner product over the rows reduced through DPP) so that they
// become orthogonal; a sweep without a rotation ends it.  The columns of Y are
// then Y's left singular vectors times its singular values (the column norms);
// those with sigma > drop * y0 are appended, normalised, in decreasing order.
constexpr int BO_MAXB = 16;
constexpr int BO_MAXE = 8192;    // J * (b | 1) doubles staged

struct BlockOrthShared {
    double Y[BO_MAXE];
    double C[LMAX][BO_MAXB + 1];
    double red[NT];
    double sig[BO_MAXB];
    int perm[BO_MAXB];
    int flag[3];
};

// Rotation (c, s) of the one-sided Jacobi step for columns p, q with Gram
// entries al = |y_p|^2, be = |y_q|^2, ga = y_p . y_q (ga != 0):
// t = 2 ga / (d + sign(d) sqrt(d^2 + 4 ga^2)), d = be - al, the smaller of the
// two angles that make the rotated columns orthogonal; c = 1 / sqrt(1 + t^2),
// s = c t.  d and 2 ga are scaled by a power of two first; square root and
// reciprocal are the hardware approximations refined by Newton steps in fp64.
__device__ __forceinline__ void hestenes_rot(double al, double be, double ga, double& c, double& s) {
    double d = be - al, a2 = 2.0 * ga;
    const int e = ilogb(fmax(fabs(d), fabs(a2)));
    d = ldexp(d, -e);
    a2 = ldexp(a2, -e);
    const double x = fma(d, d, a2 * a2);                     // in [1, 8)
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x, y * y, 1.5);
    y = y * fma(-0.5 * x, y * y, 1.5);
    const double r = x * y;
    const double den = d >= 0.0 ? d + r : d - r;            // |den| >= r >= 1
    double q = __builtin_amdgcn_rcp(den);
    q = q * fma(-den, q, 2.0);
    q = q * fma(-den, q, 2.0);
    const double t = a2 * q;                                 // |t| <= 1
    const double x2 = fma(t, t, 1.0);
    double w = __builtin_amdgcn_rsq(x2);
    w = w * fma(-0.5 * x2, w * w, 1.5);
    w = w * fma(-0.5 * x2, w * w, 1.5);
    c = w;
    s = w * t;
}

// Jacobi layout: G = 8 or 16: one wave, G lanes per pair, RW rows per lane
// (J <= G RW, b <= 128 / G); G = 0: one wave per pair, RW rows per lane (J <= 64 RW).
template <int G, int RW>
__device__ __forceinline__ void block_orth_small_body(const double* __restrict__ Yin, int64_t J, int b,
                                                      double* __restrict__ Qall, int ldq, int k, double drop,
                                                      int* __restrict__ knew, float* __restrict__ Qf,
                                                      int* __restrict__ knew2, const double* __restrict__ y0_ext) {
    __shared__ BlockOrthShared S;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ldy = b | 1;
    const int Ji = (int)J;
    double s = 0.0;
    for (int e = tid; e < Ji * b; e += NT) {
        const double v = Yin[e];
        S.Y[(e / b) * ldy + e % b] = v;
        s += v * v;
    }
    if (tid < 3) S.flag[tid] = 0;
    const double ys = sqrt(blk_sum(s, S.red));     // barrier inside: Y staged
    const double y0 = y0_ext ? y0_ext[0] : ys;
    RT_DENSE_TRACE(1);
    for (int pass = 0; pass < 2 && k > 0; ++pass) {
        // C = Qall[:, :k]^T Y (eight running sums per thread, fixed order)
        for (int e = tid; e < k * b; e += NT) {
            const int a = e / b, j = e - (e / b) * b;
            double c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) c[u] = 0.0;
            int i = 0;
            for (; i + 8 <= Ji; i += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) c[u] = fma(Qall[(int64_t)(i + u) * ldq + a], S.Y[(i + u) * ldy + j], c[u]);
            }
            for (; i < Ji; ++i) c[0] = fma(Qall[(int64_t)i * ldq + a], S.Y[i * ldy + j], c[0]);
            S.C[a][j] = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
        }
        __syncthreads();
        // Y -= Qall[:, :k] C
        for (int e = tid; e < Ji * b; e += NT) {
            const int i = e / b, j = e - (e / b) * b;
            const double* qr = Qall + (int64_t)i * ldq;
            double c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) c[u] = 0.0;
            int a = 0;
            for (; a + 8 <= k; a += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) c[u] = fma(qr[a + u], S.C[a + u][j], c[u]);
            }
            for (; a < k; ++a) c[0] = fma(qr[a], S.C[a][j], c[0]);
            S.Y[i * ldy + j] -= ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
        }
        __syncthreads();
    }
    RT_DENSE_TRACE(2);
    const int m = (b % 2) ? b + 1 : b;
    const int half = m / 2;
    int sweeps = 0;
    if (G > 0) {
        // one wave: pair slot g = lane / G of every step on lanes g G .. g G + G - 1,
        // rows sub + G r (r < RW) of the pair in registers; LDS writes of a step are
        // seen by the next step's reads in program order
        if (wave == 0) {
            const int g = lane / (G > 0 ? G : 1), sub = lane % (G > 0 ? G : 1);
            for (int sweep = 0; sweep < 60 && b > 1; ++sweep) {
                ++sweeps;
                bool any = false;
                for (int step = 0; step < m - 1; ++step) {
                    int p = 0, q = 0;
                    if (g < half) jpair(step, g, m, p, q);
                    const bool ok = g < half && q < b;
                    double yp[RW], yq[RW];
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int r = 0; r < RW; ++r) {
                        const int i = sub + G * r;
                        const bool v = ok && i < Ji;
                        yp[r] = v ? S.Y[i * ldy + p] : 0.0;
                        yq[r] = v ? S.Y[i * ldy + q] : 0.0;
                        al = fma(yp[r], yp[r], al);
                        be = fma(yq[r], yq[r], be);
                        ga = fma(yp[r], yq[r], ga);
                    }
                    al = group_total<G>(al);
                    be = group_total<G>(be);
                    ga = group_total<G>(ga);
                    if (ok && ga != 0.0 && ga * ga > 1e-30 * (al * be)) {
                        double c, sn;
                        hestenes_rot(al, be, ga, c, sn);
#pragma unroll
                        for (int r = 0; r < RW; ++r) {
                            const int i = sub + G * r;
                            if (i < Ji) {
                                S.Y[i * ldy + p] = c * yp[r] - sn * yq[r];
                                S.Y[i * ldy + q] = sn * yp[r] + c * yq[r];
                            }
                        }
                        any = true;
                    }
                }
                if (!__any(any)) break;
            }
        }
        __syncthreads();
    } else {
        // pair t of a step on wave t, rows lane + 64 r (r < RW) in registers; one
        // barrier per step
        for (int sweep = 0; sweep < 60 && b > 1; ++sweep) {
            ++sweeps;
            for (int step = 0; step < m - 1; ++step) {
                int p = 0, q = 0;
                if (wave < half) jpair(step, wave, m, p, q);
                if (wave < half && q < b) {                  // wave-uniform
                    double yp[RW], yq[RW];
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int r = 0; r < RW; ++r) {
                        const int i = lane + 64 * r;
                        yp[r] = i < Ji ? S.Y[i * ldy + p] : 0.0;
                        yq[r] = i < Ji ? S.Y[i * ldy + q] : 0.0;
                        al = fma(yp[r], yp[r], al);
                        be = fma(yq[r], yq[r], be);
                        ga = fma(yp[r], yq[r], ga);
                    }
                    al = wave_total(al);
                    be = wave_total(be);
                    ga = wave_total(ga);
                    if (ga != 0.0 && ga * ga > 1e-30 * (al * be)) {
                        double c, sn;
                        hestenes_rot(al, be, ga, c, sn);
#pragma unroll
                        for (int r = 0; r < RW; ++r) {
                            const int i = lane + 64 * r;
                            if (i < Ji) {
                                S.Y[i * ldy + p] = c * yp[r] - sn * yq[r];
                                S.Y[i * ldy + q] = sn * yp[r] + c * yq[r];
                            }
                        }
                        if (lane == 0) S.flag[sweep % 3] = 1;
                    }
                }
                __syncthreads();
            }
            // flag[s % 3] is set during sweep s and read after its last barrier; the
            // flag of sweep s + 2 is cleared now: its last readers (end of sweep s - 1)
            // are done, and its first writer waits for the barriers of sweep s + 1
            const int rotated = S.flag[sweep % 3];
            if (tid == 0) S.flag[(sweep + 2) % 3] = 0;
            if (!rotated) break;
        }
    }
    RT_DENSE_TRACE(3);
    RT_DENSE_TRACE_VAL(9, sweeps);
    // singular values = column norms
    for (int j = wave; j < b; j += NT / 64) {
        double n2 = 0.0;
        for (int i = lane; i < Ji; i += 64) n2 = fma(S.Y[i * ldy + j], S.Y[i * ldy + j], n2);
        n2 = wave_total(n2);
        if (lane == 0) S.sig[j] = sqrt(n2);
    }
    __syncthreads();
    if (tid == 0) {
        unsigned used = 0u;                                 // bit j: column j placed
        int kept = 0;
        for (int t = 0; t < b; ++t) {
            int best = -1;
            for (int j = 0; j < b; ++j)
                if (!((used >> j) & 1u) && (best < 0 || S.sig[j] > S.sig[best])) best = j;
            used |= 1u << best;
            if (S.sig[best] > drop * y0 && y0 > 0.0) S.perm[kept++] = best;
        }
        S.flag[0] = kept;
    }
    __syncthreads();
    const int kept = S.flag[0];
    // columns k + kept .. k + b - 1 are zero-filled (a projection over all b
    // columns then gives zero rows of B for them)
    for (int e = tid; e < Ji * b; e += NT) {
        const int i = e / b, t = e - (e / b) * b;
        const double v = t < kept ? S.Y[i * ldy + S.perm[t]] / S.sig[S.perm[t]] : 0.0;
        Qall[(int64_t)i * ldq + k + t] = v;
        if (Qf) Qf[(int64_t)i * ldq + k + t] = (float)v;
    }
    if (tid == 0) {
        knew[0] = kept;
        if (knew2) knew2[0] = kept;
    }
    RT_DENSE_TRACE(4);
}

template <int G, int RW>
__global__ __launch_bounds__(NT) void block_orth_small_kernel(const double* __restrict__ Yin, int64_t J, int b,
                                                              double* __restrict__ Qall, int ldq, int k,
                                                              double drop, int* __restrict__ knew,
                                                              float* __restrict__ Qf,
                                                              const double* __restrict__ y0_ext) {
    block_orth_small_body<G, RW>(Yin, J, b, Qall, ldq, k, drop, knew, Qf, nullptr, y0_ext);
}

// Grouped block steps: workgroup i serves request i of the group when its mode
// length falls in (jlo, 64 RW] (one wave per column pair, RW rows per lane).
template <int RW>
__global__ __launch_bounds__(NT) void block_orth_group_kernel(const GHeader* __restrict__ hdr,
                                                              const GBlock* __restrict__ d, int64_t jlo) {
    const int i = blockIdx.x;
    if (i >= hdr->nblock) return;
    const GBlock& q = d[i];
    if (q.J <= jlo || q.J > 64 * RW) return;
    block_orth_small_body<0, RW>(q.Y, q.J, q.b, q.Qall, q.cap, q.kcols, q.drop, q.knew, q.Qallf, &q.rb->knew,
                                 nullptr);
}

struct EigShared {
    Mat A;
    Mat V;
    __attribute__((aligned(16))) double cs[2 * (LMAX / 2 + 1)];
    int pq[LMAX / 2 + 1];
    double red[NT];
    int perm[LMAX];
    double lam[LMAX];
    int k;
};

// Eigen-decomposition of W (ell x ell), eigenvalues in decreasing order, and
// the rank: k = r_fixed, or the smallest k with max(E, 0) + sum_{t >= k}
// max(lambda_t, 0) <= tau2.  Us (ell x ell) = eigenvectors in that order.
__global__ __launch_bounds__(NT) void eig_kernel(const double* __restrict__ W, int ell, int r_fixed,
                                                 const double* __restrict__ E_dev, double tau2,
                                                 double* __restrict__ Us, double* __restrict__ lam_out,
                                                 int* __restrict__ kout, double jtol) {
    __shared__ EigShared S;
    const int tid = threadIdx.x;
    for (int e = tid; e < ell * ell; e += NT) S.A[e / ell][e % ell] = W[e];
    __syncthreads();
    RT_DENSE_TRACE(1);
    jacobi_2p(S.A, ell, S.V, jtol, S.red, S.cs, S.pq);
    RT_DENSE_TRACE(2);
    blk_sort_desc(S.A, ell, S.perm, S.lam);
    RT_DENSE_TRACE(3);
    if (tid == 0) {
        int k;
        if (r_fixed >= 0) {
            k = r_fixed < ell ? r_fixed : ell;
        } else {
            const double E = E_dev ? fmax(E_dev[0], 0.0) : 0.0;
            double tail = 0.0;
            for (int t = ell - 1; t >= 0; --t) tail += fmax(S.lam[t], 0.0);
            k = ell;
            for (int kk = 0; kk <= ell; ++kk) {
                if (E + tail <= tau2) { k = kk; break; }
                if (kk < ell) tail -= fmax(S.lam[kk], 0.0);
            }
        }
        S.k = k;
        kout[0] = k;
    }
    __syncthreads();
    if (lam_out && tid < ell) lam_out[tid] = S.lam[tid];
    for (int e = tid; e < ell * ell; e += NT) {
        const int i = e / ell, j = e % ell;
        Us[e] = S.V[i][S.perm[j]];
    }
}

// Subspace iteration: T = V diag(max(lam, drop lam_max))^-1/2 from the
// eigendecomposition of the Gram W = B B^T, so that T^T B has orthonormal rows
// along the directions above the floor (the eigenvalue form of
// orthonormalisation, Stathopoulos and Wu's SVQB).  Directions below the floor
// are rounding noise; they are scaled by the floor instead of dropped, so that
// they stay noise-sized rather than exactly zero, as in a plain sketch.
__global__ __launch_bounds__(NT) void svqb_kernel(const double* __restrict__ W, int ell, double drop,
                                                  double* __restrict__ T, float* __restrict__ Tf, double jtol) {
    __shared__ EigShared S;
    const int tid = threadIdx.x;
    for (int e = tid; e < ell * ell; e += NT) S.A[e / ell][e % ell] = W[e];
    __syncthreads();
    jacobi_2p(S.A, ell, S.V, jtol, S.red, S.cs, S.pq);
    blk_sort_desc(S.A, ell, S.perm, S.lam);
    const double lmax = S.lam[0];
    for (int e = tid; e < ell * ell; e += NT) {
        const int i = e / ell, j = e % ell;
        const double lam = S.lam[j];
        const double v = lmax > 0.0 ? S.V[i][S.perm[j]] / sqrt(fmax(lam, drop * lmax)) : 0.0;
        T[e] = v;
        if (Tf) Tf[e] = (float)v;
    }
}

// ---- structure-preserving STHOSVD: selection of ell rows of Q (Alg. 6) -----------------
// One workgroup.  First set: the column-pivoted QR order of Q^T, i.e. ell greedy
// steps of Gram-Schmidt on the rows of Q (R, J x ell fp64 scratch, holds the
// residual rows): the unselected row of largest residual norm (lowest index on
// ties) is chosen and projected out of every row.  Then strong-RRQR exchanges
// with k = ell: A = Q Q[sel]^-1 (Gauss-Jordan inverse with partial pivoting); while
// the largest |A[j][i]| over unselected rows j (first in row-major order) exceeds
// eta, sel[i] <- j.  Outputs sel (ell ints), A (J x ell, fp64 in Ad, and in dtype
// at Aout) and the number of exchanges.
struct SelectShared {
    Mat M;                 // Q[sel] being inverted (Gauss-Jordan, left block)
    Mat Inv;               // its inverse (right block)
    double v[LMAX];
    double redv[NT / 64];
    int64_t redi[NT / 64];
    int sel[LMAX];
    int piv;
    int done;
};

// block argmax of (val, idx): largest val, smallest idx on ties; every thread gets it
__device__ __forceinline__ void blk_argmax(double& val, int64_t& idx, double* redv, int64_t* redi) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(val, off, 64);
        const int64_t oi = __shfl_xor(idx, off, 64);
        if (ov > val || (ov == val && oi < idx)) { val = ov; idx = oi; }
    }
    __syncthreads();
    if (lane == 0) { redv[wave] = val; redi[wave] = idx; }
    __syncthreads();
    val = redv[0];
    idx = redi[0];
    for (int w = 1; w < NT / 64; ++w)
        if (redv[w] > val || (redv[w] == val && redi[w] < idx)) { val = redv[w]; idx = redi[w]; }
}

// REG (J <= NT): a thread's single row of R, and later of Q, is kept in registers.
template <bool REG>
__global__ __launch_bounds__(NT) void select_rows_kernel(const double* __restrict__ Q, int64_t J, int ell, double eta,
                                                         int max_swaps, double* __restrict__ R,
                                                         double* __restrict__ Ad, void* __restrict__ Aout,
                                                         int a_is_f64, int* __restrict__ sel_out,
                                                         int* __restrict__ swaps_out) {
    __shared__ SelectShared S;
    const int tid = threadIdx.x;
    double rr[REG ? LMAX : 1];
    if (REG) {
        // greedy pivoted Gram-Schmidt on the rows, row tid in registers
        const bool mine = tid < J;
#pragma unroll
        for (int c = 0; c < (REG ? LMAX : 1); ++c) rr[c] = (mine && c < ell) ? Q[(int64_t)tid * ell + c] : 0.0;
        bool used = !mine;
        for (int k = 0; k < ell; ++k) {
            double n2 = 0.0;
#pragma unroll
            for (int c = 0; c < (REG ? LMAX : 1); ++c) n2 = fma(rr[c], rr[c], n2);
            double best = used ? -1.0 : n2;
            if (!mine) best = -2.0;
            int64_t bi = mine ? tid : INT64_MAX;
            blk_argmax(best, bi, S.redv, S.redi);
            const double rs = best > 0.0 ? 1.0 / sqrt(best) : 0.0;
            if (tid == (int)bi) {
                S.sel[k] = tid;
                used = true;
#pragma unroll
                for (int c = 0; c < (REG ? LMAX : 1); ++c)
                    if (c < ell) S.v[c] = rr[c] * rs;
            }
            __syncthreads();
            double dot = 0.0;
#pragma unroll
            for (int c = 0; c < (REG ? LMAX : 1); ++c)
                if (c < ell) dot = fma(rr[c], S.v[c], dot);
#pragma unroll
            for (int c = 0; c < (REG ? LMAX : 1); ++c)
                if (c < ell) rr[c] = fma(-dot, S.v[c], rr[c]);
            __syncthreads();
        }
    } else {
    for (int64_t e = tid; e < J * ell; e += NT) R[e] = Q[e];
    __syncthreads();
    // greedy pivoted Gram-Schmidt on the rows
    for (int k = 0; k < ell; ++k) {
        double best = -2.0;
        int64_t bi = INT64_MAX;
        for (int64_t i = tid; i < J; i += NT) {
            bool used = false;
            for (int t = 0; t < k; ++t) used = used || (S.sel[t] == (int)i);
            double n2 = 0.0;
            for (int c = 0; c < ell; ++c) n2 = fma(R[i * ell + c], R[i * ell + c], n2);
            const double val = used ? -1.0 : n2;
            if (val > best) { best = val; bi = i; }
        }
        blk_argmax(best, bi, S.redv, S.redi);
        const int p = (int)bi;
        if (tid == 0) S.sel[k] = p;
        if (tid < ell) S.v[tid] = best > 0.0 ? R[(int64_t)p * ell + tid] / sqrt(best) : 0.0;
        __syncthreads();
        for (int64_t i = tid; i < J; i += NT) {
            double dot = 0.0;
            for (int c = 0; c < ell; ++c) dot = fma(R[i * ell + c], S.v[c], dot);
            for (int c = 0; c < ell; ++c) R[i * ell + c] = fma(-dot, S.v[c], R[i * ell + c]);
        }
        __syncthreads();
    }
    }
    // exchanges: the Q row of a REG thread in registers
    if (REG) {
        const bool mine = tid < J;
#pragma unroll
        for (int c = 0; c < (REG ? LMAX : 1); ++c) rr[c] = (mine && c < ell) ? Q[(int64_t)tid * ell + c] : 0.0;
    }
    int swaps = 0;
    for (;;) {
        // Inv = Q[sel]^-1 by Gauss-Jordan with partial pivoting
        for (int e = tid; e < ell * ell; e += NT) {
            const int r = e / ell, c = e % ell;
            S.M[r][c] = Q[(int64_t)S.sel[r] * ell + c];
            S.Inv[r][c] = r == c ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int c = 0; c < ell; ++c) {
            if (tid < 64) {
                double bv = -1.0;
                int br = c;
                for (int r = c + tid; r < ell; r += 64) {
                    const double a = fabs(S.M[r][c]);
                    if (a > bv) { bv = a; br = r; }
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(bv, off, 64);
                    const int orr = __shfl_xor(br, off, 64);
                    if (ov > bv || (ov == bv && orr < br)) { bv = ov; br = orr; }
                }
                if (tid == 0) S.piv = br;
            }
            __syncthreads();
            const int pr = S.piv;
            if (pr != c)
                for (int e = tid; e < 2 * ell; e += NT) {
                    const int col = e % ell;
                    double* a = e < ell ? &S.M[c][col] : &S.Inv[c][col];
                    double* b = e < ell ? &S.M[pr][col] : &S.Inv[pr][col];
                    const double t = *a;
                    *a = *b;
                    *b = t;
                }
            __syncthreads();
            const double d = S.M[c][c];
            __syncthreads();
            for (int e = tid; e < 2 * ell; e += NT) {
                const int col = e % ell;
                if (e < ell) S.M[c][col] /= d;
                else S.Inv[c][col] /= d;
            }
            __syncthreads();
            for (int e = tid; e < ell * 2 * ell; e += NT) {
                const int r = e / (2 * ell), cc = e % (2 * ell);
                if (r != c) {
                    const double f = S.M[r][c];
                    if (cc < ell) { if (cc != c) S.M[r][cc] = fma(-f, S.M[c][cc], S.M[r][cc]); }
                    else S.Inv[r][cc - ell] = fma(-f, S.Inv[c][cc - ell], S.Inv[r][cc - ell]);
                }
            }
            __syncthreads();
            for (int r = tid; r < ell; r += NT)
                if (r != c) S.M[r][c] = 0.0;
            __syncthreads();
        }
        // A = Q Inv, and the largest |A| over unselected rows
        double best = -1.0;
        int64_t bi = INT64_MAX;
        if (REG) {
            if (tid < J) {
                const int64_t i = tid;
                bool used = false;
                for (int t = 0; t < ell; ++t) used = used || (S.sel[t] == (int)i);
                for (int c = 0; c < ell; ++c) {
                    double a = 0.0;
#pragma unroll
                    for (int t = 0; t < (REG ? LMAX : 1); ++t)
                        if (t < ell) a = fma(rr[t], S.Inv[t][c], a);
                    Ad[i * ell + c] = a;
                    if (!used && fabs(a) > best) { best = fabs(a); bi = i * ell + c; }
                }
            }
        } else {
            for (int64_t i = tid; i < J; i += NT) {
                bool used = false;
                for (int t = 0; t < ell; ++t) used = used || (S.sel[t] == (int)i);
                for (int c = 0; c < ell; ++c) {
                    double a = 0.0;
                    for (int t = 0; t < ell; ++t) a = fma(Q[i * ell + t], S.Inv[t][c], a);
                    Ad[i * ell + c] = a;
                    if (!used && fabs(a) > best) { best = fabs(a); bi = i * ell + c; }
                }
            }
        }
        blk_argmax(best, bi, S.redv, S.redi);
        if (!(best > eta) || swaps >= max_swaps) break;
        if (tid == 0) S.sel[bi % ell] = (int)(bi / ell);
        ++swaps;
        __syncthreads();
    }
    __syncthreads();
    for (int64_t e = tid; e < J * ell; e += NT) {
        const double a = Ad[e];
        if (a_is_f64) ((double*)Aout)[e] = a;
        else ((float*)Aout)[e] = (float)a;
    }
    if (tid < ell) sel_out[tid] = S.sel[tid];
    if (tid == 0) swaps_out[0] = swaps;
}

// A = Q Us[:, :k] for rows 64 b .. 64 b + 63: lane l of every wave owns row
// 64 b + l (its row of Q in registers) and wave w the columns j = w, w + 4, ...
// (Us transposed in LDS, read with broadcast 16-byte loads); part[b] = per
// column the (|a|, a, row) of the entry of largest magnitude of these rows
// (lowest row on ties).  A is stored before the sign fix.
template <int NR>
__global__ __launch_bounds__(256) void factor_rows_kernel(const double* __restrict__ Q, int64_t ldq, int64_t J,
                                                          int ell, const double* __restrict__ Us,
                                                          const int* __restrict__ kdev, void* __restrict__ Aout,
                                                          int a_is_f64, double* __restrict__ part) {
    __shared__ __align__(16) double ust[NR][NR + 2];     // ust[j][t] = Us[t][j]
    __shared__ double qs[64][NR + 1];
    const int k = kdev[0];
    if (k <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < NR * NR; e += 256) ust[e / NR][e % NR] = 0.0;
    __syncthreads();
    batched_copy<8>(ell * k, tid, 256, [&](int e) { return Us[(e / k) * ell + e % k]; },
                    [&](int e, double v) { ust[e % k][e / k] = v; });
    const int64_t row0 = (int64_t)blockIdx.x * 64;
    const int rows = (int)(J - row0 < 64 ? J - row0 : 64);
    batched_copy<8>(rows * ell, tid, 256, [&](int e) { return Q[(row0 + e / ell) * ldq + e % ell]; },
                    [&](int e, double v) { qs[e / ell][e % ell] = v; });
    __syncthreads();
    const bool valid = lane < rows;
    const int64_t i = row0 + lane;
    double q[NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) q[t] = (valid && t < ell) ? qs[lane][t] : 0.0;
    constexpr int NJ = (NR + 3) / 4;
    double a[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = wave + 4 * jj;
        a[jj] = 0.0;
        if (j < k) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int t = 0; t < NR; t += 2) {
                const double2 u = *reinterpret_cast<const double2*>(&ust[j][t]);
                s0 = fma(q[t], u.x, s0);
                s1 = fma(q[t + 1], u.y, s1);
            }
            a[jj] = s0 + s1;
        }
    }
    double* A64 = (double*)Aout;
    float* A32 = (float*)Aout;
    __syncthreads();                         // every lane is done reading qs
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = wave + 4 * jj;
        if (j < k) {
            qs[lane][j] = a[jj];
            if (valid && Aout) {
                if (a_is_f64) A64[i * k + j] = a[jj];
                else A32[i * k + j] = (float)a[jj];
            }
        }
    }
    __syncthreads();
    if (tid < k) {
        double b = -1.0, v = 0.0;
        int64_t ix = INT64_MAX;
        for (int r = 0; r < rows; ++r) {
            const double x = qs[r][tid];
            if (fabs(x) > b) { b = fabs(x); v = x; ix = row0 + r; }
        }
        double* pb = part + (int64_t)blockIdx.x * 3 * LMAX;
        pb[tid] = b;
        pb[LMAX + tid] = v;
        pb[2 * LMAX + tid] = (double)ix;
    }
}

// Signs from the nwg partial maxima (fixed order, lowest row on ties); every
// workgroup scales its slice of A, workgroup 0 writes U = Us[:, :k] diag(sgn)
// (ell x k) and its float copy.
__global__ __launch_bounds__(256) void sign_kernel(const double* __restrict__ part, int nwg,
                                                   const int* __restrict__ kdev, int64_t J,
                                                   const double* __restrict__ Us, int ell, void* __restrict__ Aout,
                                                   int a_is_f64, double* __restrict__ U, float* __restrict__ Uf) {
    __shared__ double sg[LMAX];
    const int k = kdev[0];
    if (k <= 0) return;
    const int tid = threadIdx.x;
    if (tid < k) {
        double b = -1.0, v = 0.0, ix = 1e300;
        for (int w = 0; w < nwg; ++w) {
            const double* pb = part + (int64_t)w * 3 * LMAX;
            const double ob = pb[tid], ov = pb[LMAX + tid], oi = pb[2 * LMAX + tid];
            if (ob > b || (ob == b && oi < ix)) { b = ob; v = ov; ix = oi; }
        }
        sg[tid] = (v < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    if (Aout) {
        const int64_t n = J * k;
        const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
        const int64_t e0 = (int64_t)blockIdx.x * chunk;
        const int64_t e1 = e0 + chunk < n ? e0 + chunk : n;
        if (a_is_f64) {
            double* A = (double*)Aout;
            for (int64_t e = e0 + tid; e < e1; e += 256) A[e] *= sg[e % k];
        } else {
            float* A = (float*)Aout;
            for (int64_t e = e0 + tid; e < e1; e += 256) A[e] *= (float)sg[e % k];
        }
    }
    if (blockIdx.x == 0) {
        for (int e = tid; e < ell * k; e += 256) {
            const int i = e / k, j = e % k;
            const double u = Us[i * ell + j] * sg[j];
            U[e] = u;
            if (Uf) Uf[e] = (float)u;
        }
    }
}

template <int NR>
hipError_t truncate_multi(const double* W, int ell, const double* Q, int64_t ldq, int64_t J, int r_fixed,
                          const double* E_dev, double tau2, double* U, float* Uf, void* A, Dt da, double* lam,
                          int* kout, double jtol, double* scratch, hipStream_t stream) {
    double* Us = scratch;
    const int nwg = (int)((J + 63) / 64);
    double* part = Us + (int64_t)ell * ell;
    const int64_t nsign = (J * ell + 4095) / 4096;
    hipLaunchKernelGGL(eig_kernel, dim3(1), dim3(NT), 0, stream, W, ell, r_fixed, E_dev, tau2, Us, lam, kout, jtol);
    hipLaunchKernelGGL(factor_rows_kernel<NR>, dim3(nwg), dim3(256), 0, stream, Q, ldq, J, ell, (const double*)Us,
                       (const int*)kout, A, da == Dt::F64 ? 1 : 0, part);
    hipLaunchKernelGGL(sign_kernel, dim3((unsigned)(nsign < 1 ? 1 : nsign)), dim3(256), 0, stream,
                       (const double*)part, nwg, (const int*)kout, J, (const double*)Us, ell, A,
                       da == Dt::F64 ? 1 : 0, U, Uf);
    return hipGetLastError();
}

// ---- grouped truncation (serving) ----------------------------------------------------------
// Workgroup i truncates request i of the group: the Gram partials summed in a
// fixed order, the parallel Jacobi eigensolver (float data: off-diagonal sum of
// squares down to 1e-14 ||W||^2), eigenvalues sorted in decreasing order, the
// rank k = the smallest with max(E, 0) + sum_{t >= k} lambda_t <= tau2 (the
// truncation of the adaptive range finder's QB), A = Qall U_k row chunk by row
// chunk (lane = row, wave w the columns w, w + 8, ...), each column flipped so
// that its entry of largest magnitude (lowest row on ties) is positive, and
// U_k with the same flips as the float operand of the core update.
struct GTruncShared {
    Mat A;
    Mat V;
    __attribute__((aligned(16))) double cs[2 * (LMAX / 2 + 1)];
    int pq[LMAX / 2 + 1];
    double red[NT];
    int perm[LMAX];
    double lam[LMAX];
    __attribute__((aligned(16))) double ust[LMAX][LMAX + 2];
    __attribute__((aligned(16))) double qs[64][LMAX + 2];
    double sg[LMAX];
    int wrow[NT / 64][LMAX];
    int k;
};

__global__ __launch_bounds__(NT) void trunc_group_kernel(const GHeader* __restrict__ hdr,
                                                         const GTrunc* __restrict__ d) {
    const int i = blockIdx.x;
    if (i >= hdr->ntrunc) return;
    __shared__ GTruncShared S;
    const GTrunc& q = d[i];
    const int n = q.kcols;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < n * n; e += NT) {
        double sum = 0.0;
        for (int c = 0; c < q.nchunk; ++c) sum += q.gpart[(int64_t)c * n * n + e];
        S.A[e / n][e % n] = sum;
    }
    __syncthreads();
    jacobi_2p(S.A, n, S.V, 1e-14, S.red, S.cs, S.pq);
    blk_sort_desc(S.A, n, S.perm, S.lam);
    if (tid == 0) {
        const double E = fmax(q.E, 0.0);
        double tail = 0.0;
        for (int t = n - 1; t >= 0; --t) tail += fmax(S.lam[t], 0.0);
        int k = n;
        for (int kk = 0; kk <= n; ++kk) {
            if (E + tail <= q.tau2) { k = kk; break; }
            if (kk < n) tail -= fmax(S.lam[kk], 0.0);
        }
        S.k = k;
        q.kout[0] = k;
        q.rb->kfinal = k;
    }
    __syncthreads();
    const int k = S.k;
    for (int e = tid; e < LMAX * LMAX; e += NT) {
        const int j = e / LMAX, t = e % LMAX;
        S.ust[j][t] = (j < k && t < n) ? S.V[t][S.perm[j]] : 0.0;
    }
    __syncthreads();
    if (k <= 0) return;
    constexpr int NJ = LMAX / 8;
    double bmax[NJ];
    int brow[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) { bmax[jj] = -1.0; brow[jj] = 0x7fffffff; }
    for (int64_t r0 = 0; r0 < q.J; r0 += 64) {
        const int rows = (int)(q.J - r0 < 64 ? q.J - r0 : 64);
        batched_copy<8>(64 * LMAX, tid, NT,
                        [&](int e) { const int r = e / LMAX, c = e % LMAX;
                                     return (r < rows && c < n) ? q.Qall[(r0 + r) * q.cap + c] : 0.0; },
                        [&](int e, double v) { S.qs[e / LMAX][e % LMAX] = v; });
        __syncthreads();
        // a_j = sum_t Q[row][t] U[t][j] in two running sums (even and odd t),
        // the row's entries streamed from LDS once for all of the wave's columns
        double s0[NJ], s1[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) { s0[jj] = 0.0; s1[jj] = 0.0; }
        for (int t = 0; t < n; t += 2) {
            const double2 v = *reinterpret_cast<const double2*>(&S.qs[lane][t]);
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const double2 u2 = *reinterpret_cast<const double2*>(&S.ust[wave + 8 * jj][t]);
                s0[jj] = fma(v.x, u2.x, s0[jj]);
                s1[jj] = fma(v.y, u2.y, s1[jj]);
            }
        }
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int j = wave + 8 * jj;
            if (j < k) {
                const double a = s0[jj] + s1[jj];
                if (lane < rows) {
                    q.A[(r0 + lane) * k + j] = (float)a;
                    const double x = fabs(a);
                    const int row = (int)r0 + lane;
                    if (x > bmax[jj] || (x == bmax[jj] && row < brow[jj])) {
                        bmax[jj] = x;
                        brow[jj] = row;
                    }
                }
            }
        }
        __syncthreads();
    }
    // sign of each column from its entry of largest magnitude (lowest row on ties)
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        double x = bmax[jj];
        int row = brow[jj];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ox = __shfl_xor(x, off, 64);
            const int orow = __shfl_xor(row, off, 64);
            if (ox > x || (ox == x && orow < row)) { x = ox; row = orow; }
        }
        const int j = wave + 8 * jj;
        if (lane == 0 && j < k) S.wrow[0][j] = row;
    }
    __syncthreads();
    if (tid < k) {
        // the same two running sums as above for the column's largest entry
        const int64_t row = S.wrow[0][tid];
        double s0 = 0.0, s1 = 0.0;
        for (int t = 0; t < n; t += 2) {
            const double q0 = q.Qall[row * q.cap + t];
            const double q1 = t + 1 < n ? q.Qall[row * q.cap + t + 1] : 0.0;
            s0 = fma(q0, S.ust[tid][t], s0);
            s1 = fma(q1, S.ust[tid][t + 1], s1);
        }
        S.sg[tid] = (s0 + s1) < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();                       // the unsigned A is written and visible to the workgroup
    for (int64_t e = tid; e < q.J * k; e += NT) q.A[e] *= (float)S.sg[e % k];
    for (int e = tid; e < n * k; e += NT) {       // U_k as the core update's Q (ld = kcols)
        const int t = e / k, j = e % k;
        q.Uf[t * n + j] = (float)(S.ust[j][t] * S.sg[j]);
    }
}

// ---- CholeskyQR2 over many workgroups ---------------------------------------------------
// The common case of orth(): the Gram of the J x ell sketch is formed by
// ceil(J / OG_ROWS) workgroups (partial Grams summed in a fixed order), the
// Cholesky factor and its acceptance test by one workgroup, and the triangular
// solve Y R^-1 row by row by ceil(J / 64) workgroups; twice.  A sketch that
// fails either acceptance test is left untouched and the single-workgroup
// kernel above (shifted CholeskyQR3, then Householder) runs on it.

constexpr int OG_ROWS = 32;   // rows per partial Gram

// Quad-wide sum (lanes 4 q .. 4 q + 3) of a double through DPP quad permutes.
__device__ __forceinline__ double quad_sum(double v, int G) {
    if (G >= 2) {
        const unsigned long long u = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(u & 0xffffffffull), 0xb1, 0xf, 0xf, false);  // [1,0,3,2]
        const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0xb1, 0xf, 0xf, false);
        v += __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    }
    if (G >= 4) {
        const unsigned long long u = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(u & 0xffffffffull), 0x4e, 0xf, 0xf, false);  // [2,3,0,1]
        const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x4e, 0xf, 0xf, false);
        v += __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    }
    return v;
}

// part[b] = Y[rows of b]^T Y[rows of b] (ell x ell) for OG_ROWS rows staged in
// LDS; each thread owns a 4 x 4 tile of the upper triangle and every G-th row
// (G <= 4 threads of a tile in one quad, summed with DPP).  With stats,
// stats[2 b] = sum of squares of the finite entries and stats[2 b + 1] = count
// of the others.
__global__ __launch_bounds__(256) void gram_rows_kernel(const double* __restrict__ Y, int64_t J, int ell,
                                                        const int* __restrict__ gate, double* __restrict__ part,
                                                        double* __restrict__ stats) {
    if (gate && gate[0] != 0) return;
    __shared__ __align__(16) double ys[OG_ROWS][LMAX + 4];
    __shared__ double red[8];
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * OG_ROWS;
    const int rows = (int)(J - row0 < OG_ROWS ? J - row0 : OG_ROWS);
    const int nt = (ell + 3) / 4;
    double fro = 0.0, bad = 0.0;
    for (int e = tid; e < OG_ROWS * 4 * nt; e += 256) {
        const int r = e / (4 * nt), c = e - r * (4 * nt);
        double y = 0.0;
        if (r < rows && c < ell) {
            y = Y[(row0 + r) * ell + c];
            if (isfinite(y)) fro += y * y;
            else bad += 1.0;
        }
        ys[r][c] = y;
    }
    __syncthreads();
    if (stats) {
        fro = wave_sum(fro);
        bad = wave_sum(bad);
        if ((tid & 63) == 0) { red[tid >> 6] = fro; red[4 + (tid >> 6)] = bad; }
    }
    const int npt = nt * (nt + 1) / 2;
    int G = 4;
    while (G > 1 && G * npt > 256) G >>= 1;
    const int pr = tid / G, g = tid % G;
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    int ti = 0, tj = 0;
    if (pr < npt) {
        int rem = pr;
        while (rem >= nt - ti) { rem -= nt - ti; ++ti; }
        tj = ti + rem;
        for (int r = g; r < OG_ROWS; r += G) {
            const double2 x0 = *reinterpret_cast<const double2*>(&ys[r][4 * ti]);
            const double2 x1 = *reinterpret_cast<const double2*>(&ys[r][4 * ti + 2]);
            const double2 y0 = *reinterpret_cast<const double2*>(&ys[r][4 * tj]);
            const double2 y1 = *reinterpret_cast<const double2*>(&ys[r][4 * tj + 2]);
            const double x[4] = {x0.x, x0.y, x1.x, x1.y}, y[4] = {y0.x, y0.y, y1.x, y1.y};
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(x[u], y[v], acc[u][v]);
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = quad_sum(acc[u][v], G);
    double* out = part + (int64_t)blockIdx.x * ell * ell;
    if (pr < npt && g == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 4 * ti + u, c = 4 * tj + v;
                if (r < ell && c < ell) { out[r * ell + c] = acc[u][v]; out[c * ell + r] = acc[u][v]; }
            }
    }
    if (stats) {
        __syncthreads();
        if (tid == 0) {
            stats[2 * blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
            stats[2 * blockIdx.x + 1] = (red[4] + red[5]) + (red[6] + red[7]);
        }
    }
}

// Sums the nparts partial Grams (fixed order), factors W = L L^T and tests the
// pivots: accepted when every pivot ratio pivot_k / W_kk is >= min_ratio (and,
// with stats, the sketch is finite and non-zero).  On acceptance writes
// Linv = L^-1 (lower, ell x ell, row-major), so that Y R^-1 = Y Linv^T, and
// gate[0] = 0; otherwise gate[0] = 1.  With skip_if_gated, an earlier rejection
// stands and nothing is done.  The factorisation and the inverse are computed
// by wave 0 with row i of W (then column i of Linv) in the registers of lane i
// and the current column (row) broadcast through LDS; LDS accesses of one wave
// complete in order, so no barrier is needed between steps.
template <int NR>
__global__ __launch_bounds__(256) void chol_gate_kernel(const double* __restrict__ part, int nparts, int ell,
                                                        const double* __restrict__ stats, double min_ratio,
                                                        double* __restrict__ Linv, double* __restrict__ unused,
                                                        int* __restrict__ gate, int skip_if_gated,
                                                        uint32_t* __restrict__ status) {
    (void)unused;
    if (skip_if_gated && gate[0] != 0) return;
    RT_DENSE_TRACE(1);
    __shared__ double W[NR][NR + 1];
    __shared__ __align__(16) double Lb[NR][NR + 2];
    __shared__ __align__(16) double colb[NR];
    __shared__ double d0[NR], idg[NR];
    __shared__ int okflag;
    const int tid = threadIdx.x;
    // lower triangle of the summed Gram, the nparts loads of an entry in flight together
    const int ntri = ell * (ell + 1) / 2;
    constexpr int EPT = (NR * (NR + 1) / 2 + 255) / 256;    // triangle entries per thread
    int eoff[EPT], ei[EPT], ej[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + 256 * u;
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= e) ++i;
        while (i * (i + 1) / 2 > e) --i;
        ei[u] = e < ntri ? i : -1;
        ej[u] = e - i * (i + 1) / 2;
        eoff[u] = e < ntri ? i * ell + ej[u] : 0;
    }
    // the partial sums of all of a thread's entries, 8 parts at a time, in flight together
    double acc[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) acc[u] = 0.0;
    for (int b0 = 0; b0 < nparts; b0 += 8) {
        double v[EPT][8];
#pragma unroll
        for (int u = 0; u < EPT; ++u)
#pragma unroll
            for (int q = 0; q < 8; ++q)
                v[u][q] = (b0 + q < nparts) ? part[(int64_t)(b0 + q) * ell * ell + eoff[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < EPT; ++u)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[u] += v[u][q];
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u)
        if (ei[u] >= 0) W[ei[u]][ej[u]] = acc[u];
    if (tid < 64) {
        // finiteness and norm of the sketch from the per-part statistics (wave 0)
        double fro = 0.0, bad = 0.0;
        if (stats)
            for (int b = tid; b < nparts; b += 64) { fro += stats[2 * b]; bad += stats[2 * b + 1]; }
        fro = wave_sum(fro);
        bad = wave_sum(bad);
        if (tid == 0) okflag = (!stats || (bad == 0.0 && fro > 0.0)) ? 1 : 0;
    }
    __syncthreads();
    RT_DENSE_TRACE(2);
    if (tid >= 64) return;
    const int lane = tid;
    if (lane < ell) d0[lane] = W[lane][lane];
    double w[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) w[j] = (lane < ell && j <= lane && j < ell) ? W[lane][j] : 0.0;
    bool ok = okflag != 0;
    double mr = 1.0;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        if (k < ell) {
            const double piv = readlane64(w[k], k);
            const double dk = d0[k];
            const bool bad = !(piv > 0.0) || !isfinite(piv) || !(dk > 0.0);
            ok = ok && !bad;
            const double pv = bad ? 1.0 : piv;
            mr = fmin(mr, bad ? 0.0 : pv / dk);
            // 1/sqrt(pv): hardware estimate refined by two Newton steps (relative
            // error ~1e-16), d = pv / sqrt(pv)
            double rs = __builtin_amdgcn_rsq(pv);
            rs = rs * fma(-0.5 * pv, rs * rs, 1.5);
            rs = rs * fma(-0.5 * pv, rs * rs, 1.5);
            const double d = pv * rs;
            const double l = (lane == k) ? d : w[k] * rs;
            if (lane >= k) w[k] = l;
            if (lane < NR) colb[lane] = (lane > k && lane < ell) ? l : 0.0;
            double cb[NR];
#pragma unroll
            for (int j = 0; j < NR; j += 2) {
                if (j + 1 > k) {
                    const double2 c = *reinterpret_cast<const double2*>(&colb[j]);
                    cb[j] = c.x; cb[j + 1] = c.y;
                }
            }
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if (j > k) w[j] = fma(-l, cb[j], w[j]);
        }
    }
    ok = ok && mr >= min_ratio;
    RT_DENSE_TRACE(3);
    if (!ok) {
        if (lane == 0) { gate[0] = 1; if (status) status[0] = 0u; }
        return;
    }
    // L (row lane) to LDS, then column lane of Linv: x_i = (delta_i,lane - sum_{k<i} L[i][k] x_k) / L[i][i]
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (lane < NR) Lb[lane][j] = (lane < ell && j <= lane) ? w[j] : 0.0;
    double dl = 1.0;
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (j == lane) dl = w[j];
    if (lane < ell) idg[lane] = 1.0 / dl;
    double x[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i < ell) {
            double s0 = (i == lane) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
            for (int k2 = 0; k2 < NR; k2 += 2) {
                if (k2 < i) {
                    const double2 l2 = *reinterpret_cast<const double2*>(&Lb[i][k2]);
                    s0 = fma(-l2.x, x[k2], s0);
                    if (k2 + 1 < i) s1 = fma(-l2.y, x[k2 + 1], s1);
                }
            }
            x[i] = (s0 + s1) * idg[i];
        } else {
            x[i] = 0.0;
        }
    }
    RT_DENSE_TRACE(4);
    // Linv[i][lane] = x_i (zero above the diagonal)
    if (lane < ell) {
#pragma unroll
        for (int i = 0; i < NR; ++i)
            if (i < ell) Linv[(int64_t)i * ell + lane] = (i >= lane) ? x[i] : 0.0;
    }
    if (lane == 0) { gate[0] = 0; if (status) status[0] = 0u; }
}

// Yout = Yin R^-1 = Yin Linv^T when gate[0] == 0 (z_j = sum_{k<=j} y_k Linv[j][k]),
// rows 64 b .. 64 b + 63: lane l of every wave owns a row (in registers) and
// wave w the columns j = w, w + 4, ... (Linv in LDS, broadcast 16-byte loads);
// also the float copy Qf when given.
template <int NR>
__global__ __launch_bounds__(256) void trsm_rows_kernel(const double* __restrict__ Yin, double* __restrict__ Yout,
                                                        float* __restrict__ Qf, int64_t J, int ell,
                                                        const double* __restrict__ Linv,
                                                        const double* __restrict__ unused,
                                                        const int* __restrict__ gate) {
    (void)unused;
    if (gate[0] != 0) return;
    __shared__ __align__(16) double Ls[NR][NR + 2];
    __shared__ double ys[64][NR + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < NR * (NR + 2); e += 256) (&Ls[0][0])[e] = 0.0;
    __syncthreads();
    batched_copy<8>(ell * ell, tid, 256, [&](int e) { return Linv[e]; },
                    [&](int e, double v) { Ls[e / ell][e % ell] = v; });
    const int64_t row0 = (int64_t)blockIdx.x * 64;
    const int rows = (int)(J - row0 < 64 ? J - row0 : 64);
    const double* src = Yin + row0 * ell;
    batched_copy<8>(rows * ell, tid, 256, [&](int e) { return src[e]; },
                    [&](int e, double v) { ys[e / ell][e % ell] = v; });
    __syncthreads();
    double y[NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) y[t] = (t < ell && lane < rows) ? ys[lane][t] : 0.0;
    constexpr int NJ = (NR + 3) / 4;
    double z[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = wave + 4 * jj;
        double s0 = 0.0, s1 = 0.0;
        if (j < ell) {
#pragma unroll
            for (int t = 0; t < NR; t += 2) {
                if (t <= 4 * jj + 3) {                        // t <= j for every wave
                    const double2 l2 = *reinterpret_cast<const double2*>(&Ls[j][t]);
                    s0 = fma(y[t], l2.x, s0);
                    s1 = fma(y[t + 1], l2.y, s1);
                }
            }
        }
        z[jj] = s0 + s1;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = wave + 4 * jj;
        if (j < ell) ys[lane][j] = z[jj];
    }
    __syncthreads();
    double* dst = Yout + row0 * ell;
    float* dstf = Qf ? Qf + row0 * ell : nullptr;
    for (int e = tid; e < rows * ell; e += 256) {
        const double v = ys[e / ell][e % ell];
        dst[e] = v;
        if (dstf) dstf[e] = (float)v;
    }
}

template <int NR>
hipError_t orth_multi(double* Y, int64_t J, int ell, float* Qf, double accept_ratio, uint32_t* status,
                      double* scratch, hipStream_t stream) {
    const int nb = (int)((J + OG_ROWS - 1) / OG_ROWS);
    const int nr = (int)((J + 63) / 64);
    double* T1 = scratch;                         // Q of the first pass (aliases the fallback's V)
    double* part = scratch + 2 * J * (int64_t)ell;
    double* stats = part + (int64_t)nb * ell * ell;
    double* L = stats + 2 * nb;
    double* invd = L + (int64_t)ell * ell;
    int* gate = reinterpret_cast<int*>(invd + LMAX);
    // pass 1 on the sketch
    hipLaunchKernelGGL(gram_rows_kernel, dim3(nb), dim3(256), 0, stream, (const double*)Y, J, ell,
                       (const int*)nullptr, part, stats);
    hipLaunchKernelGGL(chol_gate_kernel<NR>, dim3(1), dim3(256), 0, stream, (const double*)part, nb, ell,
                       (const double*)stats, accept_ratio, L, invd, gate, 0, status);
    hipLaunchKernelGGL(trsm_rows_kernel<NR>, dim3(nr), dim3(256), 0, stream, (const double*)Y, T1, (float*)nullptr, J,
                       ell, (const double*)L, (const double*)invd, (const int*)gate);
    // pass 2 on its result (Y is overwritten only if both passes are accepted)
    hipLaunchKernelGGL(gram_rows_kernel, dim3(nb), dim3(256), 0, stream, (const double*)T1, J, ell,
                       (const int*)gate, part, (double*)nullptr);
    hipLaunchKernelGGL(chol_gate_kernel<NR>, dim3(1), dim3(256), 0, stream, (const double*)part, nb, ell,
                       (const double*)nullptr, 0.5, L, invd, gate, 1, (uint32_t*)nullptr);
    hipLaunchKernelGGL(trsm_rows_kernel<NR>, dim3(nr), dim3(256), 0, stream, (const double*)T1, Y, Qf, J, ell,
                       (const double*)L, (const double*)invd, (const int*)gate);
    // fallback on the untouched sketch
    hipLaunchKernelGGL(orth_kernel<NR>, dim3(1), dim3(NT), 0, stream, Y, J, ell, Qf, scratch, accept_ratio, status,
                       (const int*)gate);
    return hipGetLastError();
}


}  // namespace

hipError_t launch_orth(double* Y, int64_t J, int ell, float* Qf, double accept_ratio, uint32_t* status,
                       double* scratch, hipStream_t stream) {
    if (ell <= 8) return orth_multi<8>(Y, J, ell, Qf, accept_ratio, status, scratch, stream);
    if (ell <= 16) return orth_multi<16>(Y, J, ell, Qf, accept_ratio, status, scratch, stream);
    if (ell <= 24) return orth_multi<24>(Y, J, ell, Qf, accept_ratio, status, scratch, stream);
    if (ell <= 32) return orth_multi<32>(Y, J, ell, Qf, accept_ratio, status, scratch, stream);
    if (ell <= 40) return orth_multi<40>(Y, J, ell, Qf, accept_ratio, status, scratch, stream);
    if (ell <= 48) return orth_multi<48>(Y, J, ell, Qf, accept_ratio, status, scratch, stream);
    if (ell <= 56) return orth_multi<56>(Y, J, ell, Qf, accept_ratio, status, scratch, stream);
    return orth_multi<64>(Y, J, ell, Qf, accept_ratio, status, scratch, stream);
}

size_t orth_scratch(int64_t J, int ell) {
    const int64_t nb = (J + OG_ROWS - 1) / OG_ROWS;
    return (size_t)(2 * J * ell + nb * ell * ell + 2 * nb + (int64_t)ell * ell + LMAX + 8);
}

hipError_t launch_truncate(const double* W, int ell, const double* Q, int64_t ldq, int64_t J, int r_fixed,
                           const double* E_dev, double tau2, double* U, float* Uf, void* A, Dt da, double* lam,
                           int* kout, double jtol, double* scratch, hipStream_t stream) {
#define RT_TRUNC(NRV) \
    return truncate_multi<NRV>(W, ell, Q, ldq, J, r_fixed, E_dev, tau2, U, Uf, A, da, lam, kout, jtol, scratch, stream)
    if (ell <= 8) RT_TRUNC(8);
    if (ell <= 16) RT_TRUNC(16);
    if (ell <= 24) RT_TRUNC(24);
    if (ell <= 32) RT_TRUNC(32);
    if (ell <= 40) RT_TRUNC(40);
    if (ell <= 48) RT_TRUNC(48);
    if (ell <= 56) RT_TRUNC(56);
    RT_TRUNC(64);
#undef RT_TRUNC
}

size_t truncate_scratch(int64_t J, int ell) {
    return (size_t)((int64_t)ell * ell + (J + 63) / 64 * 3 * LMAX + 8);
}

hipError_t launch_block_orth(double* Y, int64_t J, int b, double* Qall, int ldq, int k, double drop, int* knew,
                             float* Qf, double* scratch, hipStream_t stream, const double* y0_ext) {
    if (b <= BO_MAXB && J * (int64_t)(b | 1) <= BO_MAXE && k <= LMAX && J <= 1024) {
#define RT_BO(GV, RWV)                                                                                          \
    hipLaunchKernelGGL((block_orth_small_kernel<GV, RWV>), dim3(1), dim3(NT), 0, stream, (const double*)Y, J, b, \
                       Qall, ldq, k, drop, knew, Qf, y0_ext)
        const int G = b <= 8 ? 16 : 8;
        if (G == 16 && J <= 16) RT_BO(16, 1);
        else if (G == 16 && J <= 32) RT_BO(16, 2);
        else if (G == 16 && J <= 64) RT_BO(16, 4);
        else if (G == 16 && J <= 128) RT_BO(16, 8);
        else if (G == 8 && J <= 8) RT_BO(8, 1);
        else if (G == 8 && J <= 16) RT_BO(8, 2);
        else if (G == 8 && J <= 32) RT_BO(8, 4);
        else if (G == 8 && J <= 64) RT_BO(8, 8);
        else if (J <= 128) RT_BO(0, 2);
        else if (J <= 256) RT_BO(0, 4);
        else if (J <= 512) RT_BO(0, 8);
        else RT_BO(0, 16);
#undef RT_BO
        return hipGetLastError();
    }
    hipLaunchKernelGGL(block_orth_kernel, dim3(1), dim3(NT), 0, stream, Y, J, b, Qall, ldq, k, drop,
                       scratch, knew, Qf, y0_ext);
    return hipGetLastError();
}

hipError_t launch_select_rows(const double* Q, int64_t J, int ell, double eta, int max_swaps, double* scratch,
                              void* Aout, Dt da, int* sel, int* swaps, hipStream_t stream) {
    if (ell < 1 || ell > LMAX || J < ell) return hipErrorInvalidValue;
    double* R = scratch;
    double* Ad = scratch + J * ell;
    if (J <= NT)
        hipLaunchKernelGGL(select_rows_kernel<true>, dim3(1), dim3(NT), 0, stream, Q, J, ell, eta, max_swaps, R, Ad,
                           Aout, da == Dt::F64 ? 1 : 0, sel, swaps);
    else if (J <= select_grid_rows())
        return launch_select_rows_grid(Q, J, ell, eta, max_swaps, scratch, Aout, da, sel, swaps, stream);
    else
        hipLaunchKernelGGL(select_rows_kernel<false>, dim3(1), dim3(NT), 0, stream, Q, J, ell, eta, max_swaps, R, Ad,
                           Aout, da == Dt::F64 ? 1 : 0, sel, swaps);
    return hipGetLastError();
}

hipError_t launch_svqb(const double* W, int ell, double drop, double* T, float* Tf, double jtol, hipStream_t stream) {
    hipLaunchKernelGGL(svqb_kernel, dim3(1), dim3(NT), 0, stream, W, ell, drop, T, Tf, jtol);
    return hipGetLastError();
}

int64_t group_block_maxj(int b) {
    // one wave per column pair, 16 rows per lane, Y staged with row stride b | 1
    int64_t jmax = 64 * 16;
    const int64_t e = BO_MAXE / (b | 1);
    return b <= BO_MAXB ? (e < jmax ? e : jmax) : 0;
}

hipError_t launch_group_dense(const GHeader* hdr, const GBlock* blk, const GTrunc* tr, int maxreq, hipStream_t stream,
                              int stage) {
    if (stage == 0) {
        // block steps: modes of at most 256 rows with 4 rows per lane, longer ones with 16
        hipLaunchKernelGGL(block_orth_group_kernel<4>, dim3(maxreq), dim3(NT), 0, stream, hdr, blk, (int64_t)0);
        hipLaunchKernelGGL(block_orth_group_kernel<16>, dim3(maxreq), dim3(NT), 0, stream, hdr, blk, (int64_t)256);
    } else {
        hipLaunchKernelGGL(trunc_group_kernel, dim3(maxreq), dim3(NT), 0, stream, hdr, tr);
    }
    return hipGetLastError();
}

hipError_t dense_init() { return hipSuccess; }

}  // namespace rt
