// Row selection of SP-STHOSVD (Alg. 6, §5) for tall bases: ell rows of the
// orthonormal Q (J x ell) chosen by the column-pivoted QR order of Q^T followed
// by strong rank-revealing exchanges with parameter eta (the same reading and
// the same arithmetic as the single-workgroup kernel used for J <= 512):
//   * greedy: ell steps; the unselected row of largest residual norm (lowest
//     index on ties) is chosen and projected out of every row;
//   * exchanges: A = Q Q[sel]^-1; while the largest |A[j][i]| over unselected
//     rows j (first in row-major order) exceeds eta, sel[i] <- j.
// One cooperative grid of ceil(J / 256) workgroups: thread t of workgroup w owns
// row 256 w + t in registers.  Every step ends in one grid-wide barrier: each
// workgroup publishes its best candidate (value, index and, in the greedy
// phase, the candidate's residual row) into a slot of `cand`, and after the
// barrier every workgroup takes the same winner from the slots.  Slots
// alternate between two banks by round, so a workgroup still reading round s
// never sees round s + 1's writes.  The small inverse Q[sel]^-1 is formed by
// every workgroup in LDS (identical inputs and code, identical results).
#include <hip/hip_cooperative_groups.h>
#include <stdint.h>

#include "rt_kernels.hpp"

namespace rt {

namespace {

namespace cg = cooperative_groups;

constexpr int SG_T = 256;            // threads (rows) per workgroup
constexpr int SG_LD = LMAX + 1;

struct SelectGridShared {
    double M[LMAX][SG_LD];           // Q[sel] being inverted
    double Inv[LMAX][SG_LD];         // its inverse
    double v[LMAX];
    double redv[SG_T / 64];
    int64_t redi[SG_T / 64];
    int sel[LMAX];
    int piv;
};

// workgroup argmax of (val, idx): largest val, smallest idx on ties; every thread gets it
__device__ __forceinline__ void wg_argmax(double& val, int64_t& idx, double* redv, int64_t* redi) {
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
    for (int w = 1; w < SG_T / 64; ++w)
        if (redv[w] > val || (redv[w] == val && redi[w] < idx)) { val = redv[w]; idx = redi[w]; }
    __syncthreads();
}

// The winner of a round over the G slots of bank `bank`: every thread gets it.
__device__ __forceinline__ void grid_winner(const double* cand, int bank, int G, int stride, double& val, int64_t& idx,
                                            double* redv, int64_t* redi) {
    val = -3.0;
    idx = INT64_MAX;
    for (int w = threadIdx.x; w < G; w += SG_T) {
        const double* sl = cand + ((int64_t)bank * G + w) * stride;
        const double v = sl[0];
        const int64_t i = __double_as_longlong(sl[1]);
        if (v > val || (v == val && i < idx)) { val = v; idx = i; }
    }
    wg_argmax(val, idx, redv, redi);
}

// Inv = Q[sel]^-1 by Gauss-Jordan elimination with partial pivoting (largest
// |pivot|, lowest row on ties), in LDS.
__device__ void select_inverse(const double* __restrict__ Q, int ell, SelectGridShared& S) {
    const int tid = threadIdx.x;
    for (int e = tid; e < ell * ell; e += SG_T) {
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
            for (int e = tid; e < 2 * ell; e += SG_T) {
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
        for (int e = tid; e < 2 * ell; e += SG_T) {
            const int col = e % ell;
            if (e < ell) S.M[c][col] /= d;
            else S.Inv[c][col] /= d;
        }
        __syncthreads();
        for (int e = tid; e < ell * 2 * ell; e += SG_T) {
            const int r = e / (2 * ell), cc = e % (2 * ell);
            if (r != c) {
                const double f = S.M[r][c];
                if (cc < ell) { if (cc != c) S.M[r][cc] = fma(-f, S.M[c][cc], S.M[r][cc]); }
                else S.Inv[r][cc - ell] = fma(-f, S.Inv[c][cc - ell], S.Inv[r][cc - ell]);
            }
        }
        __syncthreads();
        for (int r = tid; r < ell; r += SG_T)
            if (r != c) S.M[r][c] = 0.0;
        __syncthreads();
    }
}

__global__ __launch_bounds__(SG_T) void select_rows_grid_kernel(const double* __restrict__ Q, int64_t J, int ell,
                                                                double eta, int max_swaps, double* __restrict__ cand,
                                                                double* __restrict__ Ad, void* __restrict__ Aout,
                                                                int a_is_f64, int* __restrict__ sel_out,
                                                                int* __restrict__ swaps_out) {
    cg::grid_group grid = cg::this_grid();
    __shared__ SelectGridShared S;
    const int tid = threadIdx.x;
    const int G = gridDim.x;
    const int stride = ell + 2;                  // slot: value, index bits, residual row
    const int64_t i = (int64_t)blockIdx.x * SG_T + tid;
    const bool mine = i < J;
    int round = 0;
    double rr[LMAX];
#pragma unroll
    for (int c = 0; c < LMAX; ++c) rr[c] = (mine && c < ell) ? Q[i * ell + c] : 0.0;
    bool used = !mine;
    // greedy pivoted Gram-Schmidt on the rows
    for (int k = 0; k < ell; ++k, ++round) {
        double n2 = 0.0;
#pragma unroll
        for (int c = 0; c < LMAX; ++c) n2 = fma(rr[c], rr[c], n2);
        double best = used ? -1.0 : n2;
        if (!mine) best = -2.0;
        int64_t bi = mine ? i : INT64_MAX;
        wg_argmax(best, bi, S.redv, S.redi);
        double* slot = cand + ((int64_t)(round & 1) * G + blockIdx.x) * stride;
        if (i == bi) {
            slot[0] = best;
            slot[1] = __longlong_as_double(bi);
#pragma unroll
            for (int c = 0; c < LMAX; ++c)
                if (c < ell) slot[2 + c] = rr[c];
        }
        grid.sync();
        double gb;
        int64_t gi;
        grid_winner(cand, round & 1, G, stride, gb, gi, S.redv, S.redi);
        const double rs = gb > 0.0 ? 1.0 / sqrt(gb) : 0.0;
        const double* win = cand + ((int64_t)(round & 1) * G + gi / SG_T) * stride;
        if (tid < ell) S.v[tid] = win[2 + tid] * rs;
        if (tid == 0) S.sel[k] = (int)gi;
        if (i == gi) used = true;
        __syncthreads();
        double dot = 0.0;
#pragma unroll
        for (int c = 0; c < LMAX; ++c)
            if (c < ell) dot = fma(rr[c], S.v[c], dot);
#pragma unroll
        for (int c = 0; c < LMAX; ++c)
            if (c < ell) rr[c] = fma(-dot, S.v[c], rr[c]);
        __syncthreads();
    }
    // exchanges, the thread's row of Q in registers
#pragma unroll
    for (int c = 0; c < LMAX; ++c) rr[c] = (mine && c < ell) ? Q[i * ell + c] : 0.0;
    int swaps = 0;
    for (;; ++round) {
        select_inverse(Q, ell, S);
        double best = -1.0;
        int64_t bi = INT64_MAX;
        if (mine) {
            bool sel_row = false;
            for (int t = 0; t < ell; ++t) sel_row = sel_row || (S.sel[t] == (int)i);
            for (int c = 0; c < ell; ++c) {
                double a = 0.0;
#pragma unroll
                for (int t = 0; t < LMAX; ++t)
                    if (t < ell) a = fma(rr[t], S.Inv[t][c], a);
                Ad[i * ell + c] = a;
                if (!sel_row && fabs(a) > best) { best = fabs(a); bi = i * ell + c; }
            }
        }
        wg_argmax(best, bi, S.redv, S.redi);
        if (tid == 0) {
            double* slot = cand + ((int64_t)(round & 1) * G + blockIdx.x) * stride;
            slot[0] = best;
            slot[1] = __longlong_as_double(bi);
        }
        grid.sync();
        double gb;
        int64_t gi;
        grid_winner(cand, round & 1, G, stride, gb, gi, S.redv, S.redi);
        if (!(gb > eta) || swaps >= max_swaps) break;          // the same decision in every workgroup
        if (tid == 0) S.sel[gi % ell] = (int)(gi / ell);
        ++swaps;
        __syncthreads();
    }
    if (mine)
        for (int c = 0; c < ell; ++c) {
            const double a = Ad[i * ell + c];
            if (a_is_f64) ((double*)Aout)[i * ell + c] = a;
            else ((float*)Aout)[i * ell + c] = (float)a;
        }
    if (blockIdx.x == 0) {
        if (tid < ell) sel_out[tid] = S.sel[tid];
        if (tid == 0) swaps_out[0] = swaps;
    }
}

}  // namespace

int64_t select_grid_rows() { return (int64_t)SG_T * 256; }

hipError_t launch_select_rows_grid(const double* Q, int64_t J, int ell, double eta, int max_swaps, double* scratch,
                                   void* Aout, Dt da, int* sel, int* swaps, hipStream_t stream) {
    if (ell < 1 || ell > LMAX || J < ell || J > select_grid_rows()) return hipErrorInvalidValue;
    if (2 * ((J + SG_T - 1) / SG_T) * (ell + 2) > J * ell) return hipErrorInvalidValue;   // candidate banks fit
    // scratch: 2 J ell doubles; the candidate banks (2 G (ell + 2) doubles, at most
    // J ell for J > 512) first, A (J x ell) after them
    double* cand = scratch;
    double* Ad = scratch + J * ell;
    int a_is_f64 = da == Dt::F64 ? 1 : 0;
    const unsigned G = (unsigned)((J + SG_T - 1) / SG_T);
    void* args[] = {(void*)&Q, (void*)&J, (void*)&ell, (void*)&eta, (void*)&max_swaps, (void*)&cand, (void*)&Ad,
                    (void*)&Aout, (void*)&a_is_f64, (void*)&sel, (void*)&swaps};
    return hipLaunchCooperativeKernel((const void*)select_rows_grid_kernel, dim3(G), dim3(SG_T), args, 0, stream);
}

}  // namespace rt
