// Fixed-rank steps for sketch widths RT_LMAX < ell <= RT_LMAX_FIXED (Alg. 1
// inside Alg. 2 and Alg. 3, §2.4 and §3.1), where the single-wave and
// register-resident dense kernels of the narrow path do not fit:
//   * orth      - CholeskyQR2 (fp64 Gram, Cholesky and triangular inverse in
//                 LDS by one workgroup, Y Linv^T by rows) with an acceptance
//                 test on the pivots, falling back to Householder QR by one
//                 workgroup (reflectors applied column by column in global
//                 memory; always ell orthonormal columns, a numerically
//                 rank-deficient sketch leaves zero-weight padding directions);
//   * gram      - W = B_(n) B_(n)^T in fp64 for the (L, ell, R) projection,
//                 per-workgroup partials of 8 x 8 blocks from LDS tiles;
//   * eig       - eigenvectors of the fp64 Gram by one-sided (Hestenes) Jacobi
//                 on the columns of W + delta I in LDS (delta = ell u ||W||_F
//                 keeps every column away from zero and leaves the
//                 eigenvectors unchanged): the rotated columns are orthogonal,
//                 their norms are the eigenvalues plus delta and the
//                 normalised columns the eigenvectors, so no separate
//                 eigenvector matrix is accumulated;
//   * factor    - A_n = Q U[:, :r] with each column flipped so that its entry
//                 of largest magnitude (lowest row on ties) is positive, and the
//                 same flips on U for the core update.
#include <math.h>

#include "rt_kernels.hpp"

namespace rt {

namespace {

constexpr int WMAX = RT_LMAX_FIXED;   // widest sketch
constexpr int WT = 1024;              // threads of the single-workgroup kernels
constexpr int WNG = WT / WMAX;        // row groups of the Householder column sweeps

__device__ __forceinline__ double wave_sum_w(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum over the workgroup of WT threads, every thread gets the (same) result
__device__ double wg_sum(double v, double* red) {
    const int tid = threadIdx.x;
    v = wave_sum_w(v);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < WT / 64; ++w) r += red[w];
    __syncthreads();
    return r;
}

// dst[j * ldd + off + c] = src[j * w + c]
__global__ __launch_bounds__(256) void wide_copy_cols_kernel(const double* __restrict__ src, int64_t J, int w,
                                                             double* __restrict__ dst, int ldd, int off) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= J * w) return;
    const int64_t j = e / w;
    const int c = (int)(e - j * w);
    dst[j * ldd + off + c] = src[e];
}

// Householder QR of Y (J x n row-major, n <= WMAX, J >= n) in place: Y becomes
// the explicit thin Q.  V (J x n) holds the reflectors.  Thread (rg, jj) owns
// column jj of the trailing matrix and every WNG-th row from rg.  Non-finite
// entries are counted and replaced by zero.  status: RT_FLAG_NONFINITE, and
// RT_FLAG_PADDED when a diagonal entry of R is below 1e-12 of the largest;
// run as the fallback of CholeskyQR2 (gate != NULL) it does nothing when that
// was accepted and adds RT_FLAG_FALLBACK otherwise.
__global__ __launch_bounds__(WT) void wide_orth_kernel(double* __restrict__ Y, int64_t J, int n,
                                                       double* __restrict__ V, float* __restrict__ Qf,
                                                       uint32_t* __restrict__ status, const int* __restrict__ gate) {
    if (gate && gate[0] == 0) return;            // CholeskyQR2 was accepted
    __shared__ double red[WT / 64];
    __shared__ double tau[WMAX], v0[WMAX], rdiag[WMAX];
    __shared__ double wbuf[(WNG + 1) * WMAX];
    const int tid = threadIdx.x;
    const int rg = tid / WMAX, jj = tid % WMAX;
    const int64_t tot = J * (int64_t)n;
    double bad = 0.0;
    for (int64_t e = tid; e < tot; e += WT) {
        const double y = Y[e];
        if (!isfinite(y)) { bad += 1.0; Y[e] = 0.0; }
    }
    bad = wg_sum(bad, red);
    // the reflectors, column by column: H_k = I - tau v v^T with v = V[k:, k]
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int64_t i = k + tid; i < J; i += WT) { const double x = Y[i * n + k]; s += x * x; }
        s = wg_sum(s, red);
        if (tid == 0) {
            const double x0 = Y[(int64_t)k * n + k];
            const double alpha = sqrt(s);
            if (alpha == 0.0) {
                tau[k] = 0.0; v0[k] = 0.0; rdiag[k] = 0.0;
            } else {
                const double beta = x0 >= 0.0 ? -alpha : alpha;
                const double vk = x0 - beta;
                const double vtv = s - x0 * x0 + vk * vk;
                tau[k] = vtv > 0.0 ? 2.0 / vtv : 0.0;
                v0[k] = vk;
                rdiag[k] = beta;
            }
        }
        __syncthreads();
        for (int64_t i = k + tid; i < J; i += WT) V[i * n + k] = i == k ? v0[k] : Y[i * n + k];
        __syncthreads();
        const double tk = tau[k];
        if (tk != 0.0) {                       // uniform (shared memory)
            double w = 0.0;
            if (jj > k && jj < n) {
#pragma unroll 4
                for (int64_t i = k + rg; i < J; i += WNG) w += V[i * n + k] * Y[i * n + jj];
            }
            wbuf[rg * WMAX + jj] = w;
            __syncthreads();
            if (rg == 0) {
                double t = 0.0;
                for (int g = 0; g < WNG; ++g) t += wbuf[g * WMAX + jj];
                wbuf[WNG * WMAX + jj] = t * tk;
            }
            __syncthreads();
            if (jj > k && jj < n) {
                const double f = wbuf[WNG * WMAX + jj];
#pragma unroll 4
                for (int64_t i = k + rg; i < J; i += WNG) Y[i * n + jj] -= f * V[i * n + k];
            }
            __syncthreads();
        }
    }
    // Q = H_0 H_1 ... H_{n-1} [I; 0], the reflectors applied from the last
    for (int64_t e = tid; e < tot; e += WT) {
        const int64_t i = e / n;
        const int j = (int)(e - i * n);
        Y[e] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;               // uniform
        double w = 0.0;
        if (jj >= k && jj < n) {
#pragma unroll 4
            for (int64_t i = k + rg; i < J; i += WNG) w += V[i * n + k] * Y[i * n + jj];
        }
        wbuf[rg * WMAX + jj] = w;
        __syncthreads();
        if (rg == 0) {
            double t = 0.0;
            for (int g = 0; g < WNG; ++g) t += wbuf[g * WMAX + jj];
            wbuf[WNG * WMAX + jj] = t * tk;
        }
        __syncthreads();
        if (jj >= k && jj < n) {
            const double f = wbuf[WNG * WMAX + jj];
#pragma unroll 4
            for (int64_t i = k + rg; i < J; i += WNG) Y[i * n + jj] -= f * V[i * n + k];
        }
        __syncthreads();
    }
    if (Qf)
        for (int64_t e = tid; e < tot; e += WT) Qf[e] = (float)Y[e];
    if (tid == 0 && status) {
        double mx = 0.0;
        for (int k = 0; k < n; ++k) mx = fmax(mx, fabs(rdiag[k]));
        uint32_t st = (bad != 0.0 ? RT_FLAG_NONFINITE : 0u) | (gate ? RT_FLAG_FALLBACK : 0u);
        for (int k = 0; k < n; ++k)
            if (!(fabs(rdiag[k]) > 1e-12 * mx)) st |= RT_FLAG_PADDED;
        status[0] |= st;
    }
}

// Block Gram-Schmidt of an adaptive block against earlier basis columns:
// y0 = ||Y||_F, then twice C = Q^T Y (ka x b), Y -= Q C, for Y (J x b) and
// Q (J x ka, row stride ldq), ka, b <= RT_LMAX; one workgroup.
__global__ __launch_bounds__(WT) void wide_cgs_kernel(double* __restrict__ Y, int64_t J, int b,
                                                      const double* __restrict__ Q, int ldq, int ka,
                                                      double* __restrict__ y0) {
    __shared__ double C[RT_LMAX][RT_LMAX + 1];
    __shared__ double red[WT / 64];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int64_t e = tid; e < J * b; e += WT) s = fma(Y[e], Y[e], s);
    s = wg_sum(s, red);
    if (tid == 0) y0[0] = sqrt(s);
    for (int pass = 0; pass < 2; ++pass) {
        // one wave per entry of C, its lanes across the rows
        const int wave = tid >> 6, lane = tid & 63;
        for (int e = wave; e < ka * b; e += WT / 64) {
            const int a = e / b, c = e - (e / b) * b;
            double t = 0.0;
            for (int64_t i = lane; i < J; i += 64) t = fma(Q[i * ldq + a], Y[i * b + c], t);
            t = wave_sum_w(t);
            if (lane == 0) C[a][c] = t;
        }
        __syncthreads();
        for (int64_t e = tid; e < J * b; e += WT) {
            const int64_t i = e / b;
            const int c = (int)(e - i * b);
            double v = Y[e];
            for (int a = 0; a < ka; ++a) v = fma(-Q[i * ldq + a], C[a][c], v);
            Y[e] = v;
        }
        __syncthreads();
    }
}

// CholeskyQR step on the fp64 Gram W = Y^T Y (n x n): Cholesky W = L L^T in
// LDS (right-looking, one column per step), accepted when every pivot ratio
// pivot_k / W_kk is at least min_ratio (kappa(Y) ~ 1 / sqrt(min_ratio)); then
// L^-1 in place (columns from the last, each the product of the inverted
// trailing block with the column, scaled by -1 / L_jj) to Linv (lower, row
// major).  gate[0] = 0 on acceptance, 1 otherwise; with skip_if_gated an
// earlier rejection stands.
struct WideCholShared {
    double A[WMAX][WMAX + 1];
    double d0[WMAX];
    double col[WMAX];
    int ok;
};

constexpr int WCT = WT;    // threads of the Cholesky kernel

__global__ __launch_bounds__(WCT) void wide_chol_kernel(const double* __restrict__ W, int n, double min_ratio,
                                                        double* __restrict__ Linv, int* __restrict__ gate,
                                                        int skip_if_gated) {
    if (skip_if_gated && gate[0] != 0) return;
    __shared__ WideCholShared S;
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += WCT) S.A[e / n][e % n] = W[e];
    if (tid == 0) S.ok = 1;
    __syncthreads();
    if (tid < n) S.d0[tid] = S.A[tid][tid];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double piv = S.A[k][k];
        const double dk = S.d0[k];
        if (!(piv > 0.0) || !isfinite(piv) || !(dk > 0.0) || !(piv >= min_ratio * dk)) {   // uniform
            if (tid == 0) gate[0] = 1;
            return;
        }
        const double lkk = sqrt(piv);
        __syncthreads();                              // every thread has read the pivot
        if (tid == 0) S.A[k][k] = lkk;
        for (int i = k + 1 + tid; i < n; i += WCT) S.A[i][k] /= lkk;
        __syncthreads();
        // trailing update of the lower triangle: (i, j) with k < j <= i < n
        const int m = n - k - 1;
        for (int e = tid; e < m * m; e += WCT) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j <= i) S.A[i][j] -= S.A[i][k] * S.A[j][k];
        }
        __syncthreads();
    }
    // in-place inverse of the lower triangle
    for (int j = n - 1; j >= 0; --j) {
        if (tid == 0) S.A[j][j] = 1.0 / S.A[j][j];
        if (tid > j && tid < n) S.col[tid] = S.A[tid][j];
        __syncthreads();
        const double ajj = -S.A[j][j];
        if (tid > j && tid < n) {
            double t = 0.0;
            for (int kk = j + 1; kk <= tid; ++kk) t = fma(S.A[tid][kk], S.col[kk], t);
            S.A[tid][j] = t * ajj;
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += WCT) {
        const int i = e / n, j = e % n;
        Linv[e] = j <= i ? S.A[i][j] : 0.0;
    }
    if (tid == 0) gate[0] = 0;
}

// Q = Y R^-1 = Y Linv^T when gate[0] == 0: Q[i][j] = sum_{k <= j} Y[i][k] Linv[j][k];
// also the float copy when Qf != NULL.
__global__ __launch_bounds__(256) void wide_trmm_kernel(const double* __restrict__ Y, int64_t J, int n,
                                                        const double* __restrict__ Linv, double* __restrict__ Q,
                                                        float* __restrict__ Qf, const int* __restrict__ gate) {
    if (gate[0] != 0) return;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= J * n) return;
    const int64_t i = e / n;
    const int j = (int)(e - i * n);
    const double* y = Y + i * n;
    const double* l = Linv + (int64_t)j * n;
    double s0 = 0.0, s1 = 0.0;
    int k = 0;
    for (; k + 1 <= j; k += 2) {
        s0 = fma(y[k], l[k], s0);
        s1 = fma(y[k + 1], l[k + 1], s1);
    }
    if (k <= j) s0 = fma(y[k], l[k], s0);
    const double q = s0 + s1;
    Q[e] = q;
    if (Qf) Qf[e] = (float)q;
}

// Partial Grams of the first n mode rows of the (L, ldb, R) tensor B
// (unfolding columns c = l R + r):
// workgroup w sums the columns [w cpw, (w + 1) cpw) in tiles of WG_TC staged
// in LDS as fp64; thread t owns the 8 x 8 block (rows 8 (t / 16), columns
// 8 (t % 16)) of the n x n result and writes it to part[w].
constexpr int WG_TC = 32;

template <typename T>
__global__ __launch_bounds__(256) void wide_gram_kernel(const T* __restrict__ B, int64_t L, int n, int64_t ldb,
                                                        int64_t R, int64_t cpw, double* __restrict__ part) {
    __shared__ double bs[WMAX][WG_TC + 1];
    __shared__ int64_t coff[WG_TC];
    const int tid = threadIdx.x;
    const int a0 = 8 * (tid >> 4), b0 = 8 * (tid & 15);
    const int64_t K = L * R;
    const int64_t c_begin = (int64_t)blockIdx.x * cpw;
    const int64_t c_end = c_begin + cpw < K ? c_begin + cpw : K;
    double acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
    for (int64_t c0 = c_begin; c0 < c_end; c0 += WG_TC) {
        const int nc = (int)(c_end - c0 < WG_TC ? c_end - c0 : WG_TC);
        if (tid < WG_TC) {
            const int64_t c = c0 + tid;
            const int64_t l = c / R, r = c - (c / R) * R;
            coff[tid] = tid < nc ? l * ldb * R + r : -1;
        }
        __syncthreads();
        for (int e = tid; e < WMAX * WG_TC; e += 256) {
            const int a = e / WG_TC, cc = e - a * WG_TC;
            const int64_t o = coff[cc];
            bs[a][cc] = (a < n && o >= 0) ? (double)B[o + (int64_t)a * R] : 0.0;
        }
        __syncthreads();
        for (int cc = 0; cc < nc; ++cc) {
            double x[8], y[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) { x[i] = bs[a0 + i][cc]; y[i] = bs[b0 + i][cc]; }
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[i][j] = fma(x[i], y[j], acc[i][j]);
        }
        __syncthreads();
    }
    double* pw = part + (int64_t)blockIdx.x * n * n;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (a0 + i < n && b0 + j < n) pw[(a0 + i) * n + b0 + j] = acc[i][j];
}

// Rotation (c, s) that makes columns p, q with Gram [[al, ga], [ga, be]]
// orthogonal under [p q] <- [p q] [c s; -s c]: t = tan of the smaller angle,
// the root of t^2 + 2 zeta t - 1 = 0 with zeta = (be - al) / (2 ga).  t is
// formed in single precision from the block scaled by a power of two (an
// inexact angle only slows the convergence), c = 1 / sqrt(1 + t^2) from the
// single-precision reciprocal square root refined by two Newton steps and
// s = t c, so the rotation is orthogonal to double precision; this keeps the
// fp64 divisions and square roots off the step's critical path.
__device__ __forceinline__ void wrot(double al, double be, double ga, double& c, double& s) {
    const double d = be - al;
    const int e = ilogb(fmax(fmax(fabs(d), fabs(ga)), 1e-300));
    const float df = (float)ldexp(d, -e), gf = (float)ldexp(ga, -e);
    const float r = __builtin_amdgcn_sqrtf(df * df + 4.0f * gf * gf);
    const float den = df >= 0.0f ? df + r : df - r;
    const float tf = 2.0f * gf * __builtin_amdgcn_rcpf(den == 0.0f ? 1.0f : den);
    const double t = (double)tf;
    const double x = fma(t, t, 1.0);
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    y = y * fma(-0.5 * x, y * y, 1.5);
    y = y * fma(-0.5 * x, y * y, 1.5);
    c = y;
    s = t * y;
}

// Round-robin pairing of m (even) indices: in step `step` (0 .. m - 2) pair t
// joins a and b; index m - 1 stays, the others rotate; every index once per step.
__device__ __forceinline__ void wpair(int step, int t, int m, int& p, int& q) {
    int a, b;
    if (t == 0) { a = m - 1; b = step; }
    else {
        a = step + t; if (a >= m - 1) a -= m - 1;
        b = step - t + (m - 1); if (b >= m - 1) b -= m - 1;
    }
    p = a < b ? a : b;
    q = a < b ? b : a;
}

// Eigenvectors and eigenvalues of the symmetric positive semidefinite W (n x n,
// n <= WMAX), decreasing order: U (n x n row-major, column k the k-th
// eigenvector), lam[k].  One-sided Jacobi on the columns of M = W + delta I in
// LDS: in each step of the round-robin order the 16 threads of pair t form the
// 2 x 2 Gram (alpha, beta, gamma) of its columns p, q over their rows
// (butterfly sums, identical in every lane) and rotate the two columns so that
// they become orthogonal; pairs with |gamma| <= tol sqrt(alpha beta) +
// delta (sqrt(alpha) + sqrt(beta)) are left.
// A sweep without rotations ends the iteration.  The column norms are then the
// eigenvalues of W + delta I.
struct WideEigShared {
    double M[WMAX][WMAX + 1];
    double nrm[WMAX];
    double dots[WMAX];
    int perm[WMAX];
    double red[WT / 64];
    int changed;
};

__global__ __launch_bounds__(WT) void wide_eig_kernel(const double* __restrict__ W, int n, double tol, int max_sweeps,
                                                      double* __restrict__ U, double* __restrict__ lam) {
    __shared__ WideEigShared S;
    const int tid = threadIdx.x;
    double f2 = 0.0;
    for (int e = tid; e < n * n; e += WT) f2 += W[e] * W[e];
    f2 = wg_sum(f2, S.red);
    const double delta = (double)n * 0x1p-52 * sqrt(f2);
    // every entry of a rotated column carries an absolute error ~ u ||W||, so
    // the computed inner product of columns p and q is fixed only to about
    // delta (||p|| + ||q||): below that a pair counts as orthogonal (the
    // rotation left out would change the larger column of norm a by about
    // (delta / a)^2 of its norm); directions of columns near the level of
    // delta stay unresolved and are made orthonormal after the iteration
    const int m = n + (n & 1);
    for (int e = tid; e < WMAX * WMAX; e += WT) {
        const int i = e / WMAX, j = e - i * WMAX;
        S.M[i][j] = (i < n && j < n) ? W[i * n + j] + (i == j ? delta : 0.0) : 0.0;
    }
    __syncthreads();
    if (f2 > 0.0 && n > 1) {
        // eight threads per pair (512 threads), each over every eighth row: the
        // step is bound by its LDS traffic, so the pair's rows are read once into
        // registers and rows past n are not touched
        const int t = tid >> 3, sub = tid & 7;
        const int half = m / 2;
        const int nr = (n - sub + 7) / 8;                // rows sub, sub + 8, ... below n
        for (int sweep = 0; sweep < max_sweeps; ++sweep) {
            if (tid == 0) S.changed = 0;
            __syncthreads();
            for (int step = 0; step < m - 1; ++step) {
                if (t < half) {
                    int p, q;
                    wpair(step, t, m, p, q);
                    double av[WMAX / 8], bv[WMAX / 8];
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int u = 0; u < WMAX / 8; ++u) {
                        if (u < nr) {
                            const int i = sub + 8 * u;
                            av[u] = S.M[i][p];
                            bv[u] = S.M[i][q];
                            al = fma(av[u], av[u], al);
                            be = fma(bv[u], bv[u], be);
                            ga = fma(av[u], bv[u], ga);
                        }
                    }
#pragma unroll
                    for (int off = 4; off > 0; off >>= 1) {
                        al += __shfl_xor(al, off, 8);
                        be += __shfl_xor(be, off, 8);
                        ga += __shfl_xor(ga, off, 8);
                    }
                    // (the threshold needs no correctly rounded square roots: the
                    // hardware reciprocal square root estimate serves)
                    const double ra = al > 0.0 ? al * __builtin_amdgcn_rsq(al) : 0.0;
                    const double rb = be > 0.0 ? be * __builtin_amdgcn_rsq(be) : 0.0;
                    if (q < n && al > 0.0 && be > 0.0 && fabs(ga) > tol * ra * rb + delta * (ra + rb)) {
                        double c, s;
                        wrot(al, be, ga, c, s);
#pragma unroll
                        for (int u = 0; u < WMAX / 8; ++u) {
                            if (u < nr) {
                                const int i = sub + 8 * u;
                                S.M[i][p] = c * av[u] - s * bv[u];
                                S.M[i][q] = s * av[u] + c * bv[u];
                            }
                        }
                        if (sub == 0) S.changed = 1;
                    }
                }
                __syncthreads();
            }
            if (S.changed == 0) break;
            __syncthreads();
        }
    }
    // column norms (eight threads per column), the decreasing order (ties by index)
    {
        const int col = tid >> 3, sub = tid & 7;
        double s = 0.0;
        for (int i = sub; i < n; i += 8) s = fma(S.M[i][col], S.M[i][col], s);
#pragma unroll
        for (int off = 4; off > 0; off >>= 1) s += __shfl_xor(s, off, 8);
        if (sub == 0 && col < n) S.nrm[col] = sqrt(s);
    }
    __syncthreads();
    if (tid < n) {
        const double v = S.nrm[tid];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double w = S.nrm[j];
            rank += (w > v || (w == v && j < tid)) ? 1 : 0;
        }
        S.perm[rank] = tid;
    }
    __syncthreads();
    if (f2 == 0.0) {
        for (int e = tid; e < n * n; e += WT) U[e] = (e / n == e % n) ? 1.0 : 0.0;
        if (tid < n) lam[tid] = 0.0;
        return;
    }
    // normalised columns, then Gram-Schmidt (two passes) in the decreasing
    // order: a no-op to rounding for the resolved columns, an orthonormal
    // completion for those left near the level of delta (a column that mostly
    // lies in the span of the earlier ones is replaced by the next unit vector
    // that does not; a unit vector rejected once stays rejected as the span
    // grows, so each is tried at most once)
    for (int e = tid; e < n * n; e += WT) {
        const int i = e / n, c = e - (e / n) * n;
        S.M[i][c] /= S.nrm[c];
    }
    __syncthreads();
    int cand = -1;                                         // last unit vector tried
    for (int k = 1; k < n; ++k) {
        const int c = S.perm[k];
        bool own = true;                                   // the column itself first
        for (;;) {
            for (int pass = 0; pass < 2; ++pass) {
                // dots[j] = u_perm[j] . u_c for j < k: eight threads per j
                {
                    const int j = tid >> 3, sub = tid & 7;
                    double d = 0.0;
                    if (j < k) {
                        const int cj = S.perm[j];
                        for (int i = sub; i < n; i += 8) d = fma(S.M[i][cj], S.M[i][c], d);
                    }
#pragma unroll
                    for (int off = 4; off > 0; off >>= 1) d += __shfl_xor(d, off, 8);
                    if (sub == 0 && j < k) S.dots[j] = d;
                }
                __syncthreads();
                // row i -= sum_j dots[j] u_perm[j][i]: eight threads per row, each
                // over every eighth j, summed by a butterfly
                {
                    const int i = tid >> 3, sub = tid & 7;
                    double v = 0.0;
                    if (i < n)
                        for (int j = sub; j < k; j += 8) v = fma(S.dots[j], S.M[i][S.perm[j]], v);
#pragma unroll
                    for (int off = 4; off > 0; off >>= 1) v += __shfl_xor(v, off, 8);
                    if (sub == 0 && i < n) S.M[i][c] -= v;
                }
                __syncthreads();
            }
            double s2 = 0.0;
            for (int i = tid; i < n; i += WT) s2 = fma(S.M[i][c], S.M[i][c], s2);
            s2 = wg_sum(s2, S.red);
            // (the unit vectors keep n - k >= 1 of their norms squared outside
            // the span of the k earlier columns in all, and the rejected ones
            // less than 1/2, so an untried one keeps more than 1 / (2 n))
            if (s2 >= (own ? 0.25 : 0.5 / n) || cand + 1 >= n) {   // uniform
                const double inv = 1.0 / sqrt(s2);
                if (tid < n) S.M[tid][c] *= inv;
                __syncthreads();
                break;
            }
            own = false;
            ++cand;
            if (tid < n) S.M[tid][c] = tid == cand ? 1.0 : 0.0;
            __syncthreads();
        }
    }
    for (int e = tid; e < n * n; e += WT) {
        const int i = e / n, k = e - (e / n) * n;
        U[e] = S.M[i][S.perm[k]];
    }
    if (tid < n) lam[tid] = fmax(S.nrm[S.perm[tid]] - delta, 0.0);
}

// A64[i][k] = sum_a Q[i][a] U[a][k] (i < J, k < r; Q with row stride ldq)
__global__ __launch_bounds__(256) void wide_qu_kernel(const double* __restrict__ Q, int64_t ldq, int64_t J, int n,
                                                      const double* __restrict__ U, int r, double* __restrict__ A64) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= J * r) return;
    const int64_t i = e / r;
    const int k = (int)(e - i * r);
    const double* q = Q + i * ldq;
    double s0 = 0.0, s1 = 0.0;
    int a = 0;
    for (; a + 1 < n; a += 2) {
        s0 = fma(q[a], U[a * n + k], s0);
        s1 = fma(q[a + 1], U[(a + 1) * n + k], s1);
    }
    if (a < n) s0 = fma(q[a], U[a * n + k], s0);
    A64[e] = s0 + s1;
}

// sgn[k] for column k (one workgroup per column): the sign of the entry of
// largest magnitude, lowest row on ties.
__global__ __launch_bounds__(256) void wide_sign_kernel(const double* __restrict__ A64, int64_t J, int r,
                                                        double* __restrict__ sgn) {
    __shared__ double sb[256], sv[256];
    __shared__ int64_t si[256];
    const int k = blockIdx.x, tid = threadIdx.x;
    double b = -1.0, v = 0.0;
    int64_t ix = INT64_MAX;
    for (int64_t i = tid; i < J; i += 256) {
        const double x = A64[i * r + k];
        if (fabs(x) > b) { b = fabs(x); v = x; ix = i; }
    }
    sb[tid] = b; sv[tid] = v; si[tid] = ix;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            const double ob = sb[tid + h];
            const int64_t oi = si[tid + h];
            if (ob > sb[tid] || (ob == sb[tid] && oi < si[tid])) { sb[tid] = ob; sv[tid] = sv[tid + h]; si[tid] = oi; }
        }
        __syncthreads();
    }
    if (tid == 0) sgn[k] = sv[0] < 0.0 ? -1.0 : 1.0;
}

// A_out[i][k] = sgn[k] A64[i][k] (float or double); Us[a][k] = sgn[k] U[a][k]
// and its float copy (a < n).
__global__ __launch_bounds__(256) void wide_apply_sign_kernel(const double* __restrict__ A64, int64_t J, int r,
                                                              const double* __restrict__ sgn, void* __restrict__ Aout,
                                                              int a_is_f64, const double* __restrict__ U, int n,
                                                              double* __restrict__ Us, float* __restrict__ Usf) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nA = J * r;
    if (e < nA) {
        const double v = A64[e] * sgn[e % r];
        if (a_is_f64) ((double*)Aout)[e] = v;
        else ((float*)Aout)[e] = (float)v;
    }
    if (e < (int64_t)n * r) {
        const int a = (int)(e / r), k = (int)(e % r);
        const double u = U[a * n + k] * sgn[k];
        Us[e] = u;
        if (Usf) Usf[e] = (float)u;
    }
}

}  // namespace

hipError_t launch_wide_copy_cols(const double* src, int64_t J, int w, double* dst, int ldd, int off,
                                 hipStream_t stream) {
    const int64_t n = J * w;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(wide_copy_cols_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, src, J, w, dst,
                       ldd, off);
    return hipGetLastError();
}

hipError_t launch_wide_gram(const void* B, Dt dt, int64_t L, int n, int64_t ldb, int64_t R, double* part, int nwg,
                            hipStream_t stream);

int plan_wide_gram(int64_t K) {
    const int64_t tiles = (K + WG_TC - 1) / WG_TC;
    return (int)(tiles < 256 ? tiles : 256);
}

// scratch: T1 (J n), the Householder reflectors (J n), W and Linv (n n each),
// the Gram partials and their reduction temporaries, the gate word
size_t wide_orth_scratch(int64_t J, int n) {
    const int nwg = plan_wide_gram(J);
    return (size_t)(2 * J * n + 2 * n * n + (int64_t)nwg * n * n + reduce_partials_tmp(nwg, (int64_t)n * n) + 8);
}

// Q = orth(Y) for the J x n sketch (fp64, in place; float copy in Qf):
// CholeskyQR2 (accepted when the first factorisation keeps every pivot ratio
// >= accept_ratio and the second >= 1/2), else Householder QR of the untouched
// sketch; every step is enqueued and the choice is made on the device.
hipError_t launch_wide_orth(double* Y, int64_t J, int n, float* Qf, double accept_ratio, uint32_t* status,
                            double* scratch, hipStream_t stream) {
    if (n < 1 || n > WMAX || J < n) return hipErrorInvalidValue;
    const int nwg = plan_wide_gram(J);
    double* T1 = scratch;
    double* V = T1 + J * (int64_t)n;
    double* Wm = V + J * (int64_t)n;
    double* Li = Wm + (int64_t)n * n;
    double* part = Li + (int64_t)n * n;
    double* rtmp = part + (int64_t)nwg * n * n;
    int* gate = reinterpret_cast<int*>(rtmp + reduce_partials_tmp(nwg, (int64_t)n * n));
    const unsigned gt = (unsigned)((J * n + 255) / 256);
    hipError_t e;
    // pass 1 on the sketch into T1
    if ((e = launch_wide_gram(Y, Dt::F64, J, n, n, 1, part, nwg, stream)) != hipSuccess) return e;
    if ((e = launch_reduce_partials(part, true, nwg, (int64_t)n * n, Wm, stream, rtmp)) != hipSuccess) return e;
    hipLaunchKernelGGL(wide_chol_kernel, dim3(1), dim3(WCT), 0, stream, (const double*)Wm, n, accept_ratio, Li, gate,
                       0);
    hipLaunchKernelGGL(wide_trmm_kernel, dim3(gt), dim3(256), 0, stream, (const double*)Y, J, n, (const double*)Li,
                       T1, (float*)nullptr, (const int*)gate);
    // pass 2 on T1 into Y (Y stays the sketch unless both passes are accepted)
    if ((e = launch_wide_gram(T1, Dt::F64, J, n, n, 1, part, nwg, stream)) != hipSuccess) return e;
    if ((e = launch_reduce_partials(part, true, nwg, (int64_t)n * n, Wm, stream, rtmp)) != hipSuccess) return e;
    hipLaunchKernelGGL(wide_chol_kernel, dim3(1), dim3(WCT), 0, stream, (const double*)Wm, n, 0.5, Li, gate, 1);
    hipLaunchKernelGGL(wide_trmm_kernel, dim3(gt), dim3(256), 0, stream, (const double*)T1, J, n, (const double*)Li,
                       Y, Qf, (const int*)gate);
    // fallback on the untouched sketch
    hipLaunchKernelGGL(wide_orth_kernel, dim3(1), dim3(WT), 0, stream, Y, J, n, V, Qf, status, (const int*)gate);
    return hipGetLastError();
}

hipError_t launch_wide_gram(const void* B, Dt dt, int64_t L, int n, int64_t ldb, int64_t R, double* part, int nwg,
                            hipStream_t stream) {
    if (n < 1 || n > WMAX || ldb < n || nwg < 1) return hipErrorInvalidValue;
    const int64_t K = L * R;
    int64_t cpw = (K + nwg - 1) / nwg;
    cpw = (cpw + WG_TC - 1) / WG_TC * WG_TC;
    if (dt == Dt::F64)
        hipLaunchKernelGGL(wide_gram_kernel<double>, dim3(nwg), dim3(256), 0, stream, (const double*)B, L, n, ldb, R,
                           cpw, part);
    else
        hipLaunchKernelGGL(wide_gram_kernel<float>, dim3(nwg), dim3(256), 0, stream, (const float*)B, L, n, ldb, R,
                           cpw, part);
    return hipGetLastError();
}

hipError_t launch_wide_cgs(double* Y, int64_t J, int b, const double* Q, int ldq, int ka, double* y0,
                           hipStream_t stream) {
    if (b < 1 || b > RT_LMAX || ka < 0 || ka > RT_LMAX || ldq < ka) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wide_cgs_kernel, dim3(1), dim3(WT), 0, stream, Y, J, b, Q, ldq, ka, y0);
    return hipGetLastError();
}

hipError_t launch_wide_eig(const double* W, int n, double tol, double* U, double* lam, hipStream_t stream) {
    if (n < 1 || n > WMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wide_eig_kernel, dim3(1), dim3(WT), 0, stream, W, n, tol, 60, U, lam);
    return hipGetLastError();
}

hipError_t launch_wide_factor(const double* Q, int64_t ldq, int64_t J, int n, const double* U, int r, double* A64,
                              double* sgn, void* Aout, Dt da, double* Us, float* Usf, hipStream_t stream) {
    if (n < 1 || n > WMAX || r < 1 || r > n || ldq < n) return hipErrorInvalidValue;
    const int64_t nA = J * r;
    hipLaunchKernelGGL(wide_qu_kernel, dim3((unsigned)((nA + 255) / 256)), dim3(256), 0, stream, Q, ldq, J, n, U, r,
                       A64);
    hipLaunchKernelGGL(wide_sign_kernel, dim3(r), dim3(256), 0, stream, (const double*)A64, J, r, sgn);
    const int64_t ne = nA > (int64_t)n * r ? nA : (int64_t)n * r;
    hipLaunchKernelGGL(wide_apply_sign_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, stream,
                       (const double*)A64, J, r, (const double*)sgn, Aout, da == Dt::F64 ? 1 : 0, U, n, Us, Usf);
    return hipGetLastError();
}

}  // namespace rt
