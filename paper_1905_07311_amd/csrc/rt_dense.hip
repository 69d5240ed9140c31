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

namespace rt {

namespace {

constexpr int NT = 256;
constexpr int LDW = LMAX + 1;
typedef double Mat[LMAX][LDW];

__device__ double blk_sum(double v, double* red) {
    const int tid = threadIdx.x;
    __syncthreads();
    red[tid] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// W = Y^T Y (n x n) for Y (J x n, row stride ldy) in global memory.
__device__ void blk_gram(const double* Y, int64_t J, int n, int64_t ldy, Mat& W, Mat& stage) {
    const int tid = threadIdx.x;
    const int npairs = n * (n + 1) / 2;
    double acc[9];
    int pa[9], pb[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        acc[m] = 0.0;
        const int t = tid + NT * m;
        int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((a + 1) * (a + 2) / 2 <= t) ++a;
        while (a * (a + 1) / 2 > t) --a;
        pa[m] = a;
        pb[m] = t - a * (a + 1) / 2;
    }
    for (int64_t i0 = 0; i0 < J; i0 += LMAX) {
        const int rows = (int)((J - i0) < LMAX ? (J - i0) : LMAX);
        __syncthreads();
        for (int e = tid; e < rows * n; e += NT) stage[e / n][e % n] = Y[(i0 + e / n) * ldy + e % n];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 9; ++m) {
            if (tid + NT * m < npairs) {
                double s = 0.0;
                for (int r = 0; r < rows; ++r) s += stage[r][pa[m]] * stage[r][pb[m]];
                acc[m] += s;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        if (tid + NT * m < npairs) {
            W[pa[m]][pb[m]] = acc[m];
            W[pb[m]][pa[m]] = acc[m];
        }
    }
    __syncthreads();
}

// In-place Cholesky W = L L^T (lower triangle).  Returns false on a non-positive
// or non-finite pivot; *min_ratio = min_k pivot_k / W_kk(original), the squared
// sine of the angle between column k and the span of the previous columns.
__device__ bool blk_cholesky(Mat& W, int n, double* diag0, double* min_ratio, int* flag) {
    const int tid = threadIdx.x;
    if (tid < n) diag0[tid] = W[tid][tid];
    if (tid == 0) { flag[0] = 0; min_ratio[0] = 1.0; }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (tid == 0) {
            double d = W[k][k];
            if (!(d > 0.0) || !isfinite(d) || !(diag0[k] > 0.0)) {
                flag[0] = 1;
                d = 1.0;
            } else {
                double ratio = d / diag0[k];
                if (ratio < min_ratio[0]) min_ratio[0] = ratio;
            }
            W[k][k] = sqrt(d);
        }
        __syncthreads();
        if (flag[0]) break;
        const double dk = W[k][k];
        for (int i = k + 1 + tid; i < n; i += NT) W[i][k] /= dk;
        __syncthreads();
        const int m = n - k - 1;
        for (int e = tid; e < m * m; e += NT) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j <= i) W[i][j] -= W[i][k] * W[j][k];
        }
        __syncthreads();
    }
    const bool ok = flag[0] == 0;
    __syncthreads();
    return ok;
}

// Rinv = L^{-T} (upper triangular) from the lower Cholesky factor in W.
__device__ void blk_tri_inv(const Mat& W, int n, Mat& Rinv) {
    const int tid = threadIdx.x;
    // Solve L X = I column by column (X lower), then Rinv = X^T.
    if (tid < n) {
        const int j = tid;
        for (int i = 0; i < n; ++i) {
            double s = (i == j) ? 1.0 : 0.0;
            if (i < j) { Rinv[j][i] = 0.0; continue; }
            for (int k = j; k < i; ++k) s -= W[i][k] * Rinv[j][k];
            Rinv[j][i] = s / W[i][i];          // Rinv[j][i] = X[i][j]
        }
    }
    __syncthreads();
}

// Y <- Y * M (J x n times n x n), in place, staging 64-row chunks through LDS.
__device__ void blk_apply_right(double* Y, int64_t J, int n, int64_t ldy, const Mat& M, Mat& stage) {
    const int tid = threadIdx.x;
    for (int64_t i0 = 0; i0 < J; i0 += LMAX) {
        const int rows = (int)((J - i0) < LMAX ? (J - i0) : LMAX);
        __syncthreads();
        for (int e = tid; e < rows * n; e += NT) stage[e / n][e % n] = Y[(i0 + e / n) * ldy + e % n];
        __syncthreads();
        for (int e = tid; e < rows * n; e += NT) {
            const int r = e / n, j = e % n;
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += stage[r][k] * M[k][j];
            Y[(i0 + r) * ldy + j] = s;
        }
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
                for (int64_t i = k + rg; i < J; i += NT / LMAX) w += V[i * n + k] * A[i * lda + j];
            wbuf[rg * LDW + jj] = w;
            __syncthreads();
            if (rg == 0) {
                double t = 0.0;
                for (int g = 0; g < NT / LMAX; ++g) t += wbuf[g * LDW + jj];
                wbuf[4 * LDW + jj] = t * tk;
            }
            __syncthreads();
            if (j > k && j < n) {
                const double f = wbuf[4 * LDW + j];
                for (int64_t i = k + rg; i < J; i += NT / LMAX) A[i * lda + j] -= f * V[i * n + k];
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
            for (int64_t i = k + rg; i < J; i += NT / LMAX) w += V[i * n + k] * A[i * lda + j];
        wbuf[rg * LDW + jj] = w;
        __syncthreads();
        if (rg == 0) {
            double t = 0.0;
            for (int g = 0; g < NT / LMAX; ++g) t += wbuf[g * LDW + jj];
            wbuf[4 * LDW + jj] = t * tk;
        }
        __syncthreads();
        if (j >= k && j < n) {
            const double f = wbuf[4 * LDW + j];
            for (int64_t i = k + rg; i < J; i += NT / LMAX) A[i * lda + j] -= f * V[i * n + k];
        }
        __syncthreads();
    }
}

// Parallel cyclic Jacobi on the symmetric n x n matrix A (LDS): on exit the
// diagonal of A holds the eigenvalues and the columns of V the eigenvectors.
__device__ void blk_jacobi_eig(Mat& A, int n, Mat& V, double* cs, int* pairs, double* red) {
    const int tid = threadIdx.x;
    const int m = (n % 2) ? n + 1 : n;    // even number of players (a dummy if n is odd)
    const int half = m / 2;
    for (int e = tid; e < n * n; e += NT) V[e / n][e % n] = (e / n == e % n) ? 1.0 : 0.0;
    __syncthreads();
    double tot = 0.0;
    for (int e = tid; e < n * n; e += NT) tot += A[e / n][e % n] * A[e / n][e % n];
    tot = blk_sum(tot, red);
    if (tot == 0.0) return;
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0;
        for (int e = tid; e < n * n; e += NT)
            if (e / n != e % n) off += A[e / n][e % n] * A[e / n][e % n];
        off = blk_sum(off, red);
        if (off <= 1e-30 * tot) break;
        for (int step = 0; step < m - 1; ++step) {
            if (tid < half) {
                int a, b;
                if (tid == 0) { a = m - 1; b = step; }
                else { a = (step + tid) % (m - 1); b = (step - tid + (m - 1)) % (m - 1); }
                int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[p][q];
                    const double app = A[p][p], aqq = A[q][q];
                    if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq))) {
                        const double theta = (aqq - app) / (2.0 * apq);
                        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                pairs[2 * tid] = p; pairs[2 * tid + 1] = q;
                cs[2 * tid] = c; cs[2 * tid + 1] = s;
            }
            __syncthreads();
            // A <- R^T A R on every 2x2 block (row pair bi, column pair bj), in place.
            // When n is odd one pair holds the dummy index n: its real member is
            // rotated by nobody (identity) but its entries still take the rotation
            // of the other pair of the block.
            for (int e = tid; e < half * half; e += NT) {
                const int bi = e / half, bj = e % half;
                const int p = pairs[2 * bi], q = pairs[2 * bi + 1];
                const int pp = pairs[2 * bj], qq = pairs[2 * bj + 1];
                const double ci = cs[2 * bi], si = cs[2 * bi + 1];
                const double cj = cs[2 * bj], sj = cs[2 * bj + 1];
                const bool rq = q < n, cq = qq < n;
                const double a = A[p][pp];
                const double b = cq ? A[p][qq] : 0.0;
                const double c = rq ? A[q][pp] : 0.0;
                const double d = (rq && cq) ? A[q][qq] : 0.0;
                // left: rows (p, q) <- R_i^T: [ci -si; si ci]  (identity for a dummy pair)
                const double a1 = ci * a - si * c, b1 = ci * b - si * d;
                const double c1 = si * a + ci * c, d1 = si * b + ci * d;
                // right: cols (pp, qq) <- * R_j: [cj sj; -sj cj]
                A[p][pp] = a1 * cj - b1 * sj;
                if (cq) A[p][qq] = a1 * sj + b1 * cj;
                if (rq) A[q][pp] = c1 * cj - d1 * sj;
                if (rq && cq) A[q][qq] = c1 * sj + d1 * cj;
            }
            // V <- V R
            for (int e = tid; e < n * half; e += NT) {
                const int r = e / half, bj = e % half;
                const int p = pairs[2 * bj], q = pairs[2 * bj + 1];
                if (q >= n) continue;
                const double c = cs[2 * bj], s = cs[2 * bj + 1];
                const double vp = V[r][p], vq = V[r][q];
                V[r][p] = c * vp - s * vq;
                V[r][q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    __syncthreads();
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
    double wbuf[5 * LDW];
    double diag0[LMAX];
    double tau[LMAX];
    double v0[LMAX];
    double rdiag[LMAX];
    double cs[LMAX + 2];
    double lam[LMAX];
    double minr[1];
    int pairs[LMAX + 2];
    int perm[LMAX];
    int flag[4];
};

__global__ __launch_bounds__(NT) void orth_kernel(double* __restrict__ Y, int64_t J, int ell, float* __restrict__ Qf,
                                                  double* __restrict__ V, double accept_ratio,
                                                  uint32_t* __restrict__ status) {
    __shared__ DenseShared S;
    const int tid = threadIdx.x;
    uint32_t st = 0;
    if (tid == 0) S.flag[1] = 0;
    // keep a copy of Y in V's second half? The CholeskyQR passes work in place; the
    // fallback restarts from the copy held in V[J*ell ...].
    double* Ycopy = V + J * (int64_t)ell;
    double nonfinite = 0.0;
    for (int64_t e = tid; e < J * ell; e += NT) {
        const double y = Y[e];
        Ycopy[e] = y;
        if (!isfinite(y)) nonfinite += 1.0;
    }
    nonfinite = blk_sum(nonfinite, S.red);
    bool ok = nonfinite == 0.0;
    if (!ok) st |= 4u;
    double ratio1 = 0.0, ratio2 = 0.0;
    if (ok) {
        blk_gram(Y, J, ell, ell, S.W, S.stage);
        ok = blk_cholesky(S.W, ell, S.diag0, S.minr, S.flag);
        ratio1 = S.minr[0];
        __syncthreads();
        if (ok && ratio1 >= accept_ratio) {
            blk_tri_inv(S.W, ell, S.M2);
            blk_apply_right(Y, J, ell, ell, S.M2, S.stage);
            blk_gram(Y, J, ell, ell, S.W, S.stage);
            ok = blk_cholesky(S.W, ell, S.diag0, S.minr, S.flag);
            ratio2 = S.minr[0];
            __syncthreads();
            if (ok && ratio2 >= 0.5) {
                blk_tri_inv(S.W, ell, S.M2);
                blk_apply_right(Y, J, ell, ell, S.M2, S.stage);
            } else {
                ok = false;
            }
        } else {
            ok = false;
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
    (void)ratio2;
}

// Truncation: eigen-decomposition of the Gram W (ell x ell) of B, rank choice,
// U = leading eigenvectors, A = Q U with sign fix (largest |.| entry positive).
__global__ __launch_bounds__(NT) void truncate_kernel(const double* __restrict__ W, int ell,
                                                      const double* __restrict__ Q, int64_t ldq, int64_t J,
                                                      int r_fixed,
                                                      const double* __restrict__ E_dev, double tau2,
                                                      double* __restrict__ U, float* __restrict__ Uf,
                                                      void* __restrict__ Aout, int a_is_f64,
                                                      double* __restrict__ lam_out, int* __restrict__ kout) {
    __shared__ DenseShared S;
    const int tid = threadIdx.x;
    for (int e = tid; e < ell * ell; e += NT) S.W[e / ell][e % ell] = W[e];
    __syncthreads();
    blk_jacobi_eig(S.W, ell, S.M2, S.cs, S.pairs, S.red);
    blk_sort_desc(S.W, ell, S.perm, S.lam);
    if (tid == 0) {
        int k;
        if (r_fixed >= 0) {
            k = r_fixed < ell ? r_fixed : ell;
        } else {
            const double E = E_dev ? fmax(E_dev[0], 0.0) : 0.0;
            // tail[k] = sum_{t >= k} max(lam_t, 0)
            double tail = 0.0;
            k = ell;
            // smallest k with E + tail[k] <= tau2: scan from the end
            double tails[LMAX + 1];
            tails[ell] = 0.0;
            for (int t = ell - 1; t >= 0; --t) { tail += fmax(S.lam[t], 0.0); tails[t] = tail; }
            for (int kk = 0; kk <= ell; ++kk)
                if (E + tails[kk] <= tau2) { k = kk; break; }
        }
        S.flag[2] = k;
    }
    __syncthreads();
    const int k = S.flag[2];
    if (lam_out && tid < ell) lam_out[tid] = S.lam[tid];
    if (kout && tid == 0) kout[0] = k;
    // U columns = eigenvectors in sorted order: stage as S.W (ell x k)
    for (int e = tid; e < ell * k; e += NT) {
        const int i = e / k, j = e % k;
        S.W[i][j] = S.M2[i][S.perm[j]];
    }
    __syncthreads();
    // sign fix: column j of A = Q U[:, j]; find the entry of largest magnitude
    for (int j = 0; j < k; ++j) {
        double best = -1.0;
        int64_t bi = 0;
        double bval = 0.0;
        for (int64_t i = tid; i < J; i += NT) {
            double a = 0.0;
            for (int t = 0; t < ell; ++t) a += Q[i * ldq + t] * S.W[t][j];
            if (fabs(a) > best) { best = fabs(a); bi = i; bval = a; }
        }
        // block argmax (ties -> lowest index)
        S.red[tid] = best;
        S.stage[tid / LMAX][tid % LMAX] = bval;
        __syncthreads();
        if (tid == 0) {
            double b = -1.0, v = 0.0;
            for (int t = 0; t < NT; ++t) {
                if (S.red[t] > b) { b = S.red[t]; v = S.stage[t / LMAX][t % LMAX]; }
            }
            S.cs[0] = (v < 0.0) ? -1.0 : 1.0;
        }
        __syncthreads();
        const double sgn = S.cs[0];
        __syncthreads();
        if (tid < ell) S.W[tid][j] *= sgn;
        __syncthreads();
        (void)bi;
    }
    for (int e = tid; e < ell * k; e += NT) {
        const int i = e / k, j = e % k;
        U[i * k + j] = S.W[i][j];
        if (Uf) Uf[i * k + j] = (float)S.W[i][j];
    }
    if (Aout) {
        for (int64_t e = tid; e < J * k; e += NT) {
            const int64_t i = e / k;
            const int j = (int)(e % k);
            double a = 0.0;
            for (int t = 0; t < ell; ++t) a += Q[i * ldq + t] * S.W[t][j];
            if (a_is_f64) ((double*)Aout)[e] = a;
            else ((float*)Aout)[e] = (float)a;
        }
    }
}

// One adaptive block: Y (J x b) <- (I - Q Q^T) Y twice, then the kept left singular
// vectors of Y are appended to Qall (ld = ldq) at column k.
__global__ __launch_bounds__(NT) void block_orth_kernel(double* __restrict__ Y, int64_t J, int b,
                                                        double* __restrict__ Qall, int ldq, int k, double drop,
                                                        double* __restrict__ V, int* __restrict__ knew) {
    __shared__ DenseShared S;
    const int tid = threadIdx.x;
    // y0 = ||Y||_F before the projections
    double s = 0.0;
    for (int64_t e = tid; e < J * b; e += NT) s += Y[e] * Y[e];
    const double y0 = sqrt(blk_sum(s, S.red));
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
    // new basis columns: Qy * Vr[:, perm[t]]  (Qy in Y, J x b)
    for (int64_t e = tid; e < J * kept; e += NT) {
        const int64_t i = e / kept;
        const int t = (int)(e % kept);
        const int j = S.perm[t];
        double c = 0.0;
        for (int a = 0; a < b; ++a) c += Y[i * b + a] * S.W[a][j];
        Qall[i * ldq + k + t] = c;
    }
    if (tid == 0) knew[0] = kept;
}


}  // namespace

hipError_t launch_orth(double* Y, int64_t J, int ell, float* Qf, double accept_ratio, uint32_t* status,
                       double* scratch, hipStream_t stream) {
    hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(NT), 0, stream, Y, J, ell, Qf, scratch, accept_ratio,
                       status);
    return hipGetLastError();
}

hipError_t launch_truncate(const double* W, int ell, const double* Q, int64_t ldq, int64_t J, int r_fixed,
                           const double* E_dev, double tau2, double* U, float* Uf, void* A, Dt da, double* lam,
                           int* kout, hipStream_t stream) {
    hipLaunchKernelGGL(truncate_kernel, dim3(1), dim3(NT), 0, stream, W, ell, Q, ldq, J, r_fixed, E_dev,
                       tau2,
                       U, Uf, A, da == Dt::F64 ? 1 : 0, lam, kout);
    return hipGetLastError();
}

hipError_t launch_block_orth(double* Y, int64_t J, int b, double* Qall, int ldq, int k, double drop, int* knew,
                             double* scratch, hipStream_t stream) {
    hipLaunchKernelGGL(block_orth_kernel, dim3(1), dim3(NT), 0, stream, Y, J, b, Qall, ldq, k, drop,
                       scratch, knew);
    return hipGetLastError();
}

hipError_t dense_init() { return hipSuccess; }

}  // namespace rt
