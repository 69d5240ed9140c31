// Mode-n expansion of a Tucker core, the step of reconstruction X_hat =
// G x_1 A_1 ... x_d A_d (§2.1, the Tucker format): on the (L, r, R) view of the
// current tensor and a factor A (I x r, row-major),
//     out[l, i, q] = sum_k A[i, k] G[l, k, q]     (out viewed as (L, I, R)).
// The output is much larger than its inputs (I >> r), so the kernels are laid
// out for the output stream: lanes own consecutive output entries (coalesced
// 4- or 8-byte stores), the operand that varies along the lanes sits in
// registers, and the other one is read from LDS as a broadcast.
//   * R == 1 (the last mode): out (L x I) = G (L x r) A^T: lane i holds A[i, :]
//     in registers, a block of G rows is staged in LDS.
//   * R >= 64: lane q holds G[l, :, q] in registers, a block of A rows is staged
//     in LDS.
//   * 1 < R < 64: lanes own consecutive entries of one l's I x R output slab,
//     both operands staged in LDS.
// Each output is a dot product of length r summed in order k = 0, 1, ...
#include "rt_kernels.hpp"

namespace rt {

namespace {

constexpr int EX_T = 256;     // threads per workgroup
constexpr int EX_LB = 32;     // G rows (R == 1) or A rows (R > 1) staged per workgroup

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

// 1 < R < 64: for a fixed l the output is one contiguous I x R slab; lane t of
// the workgroup's 256 consecutive slab entries computes entry (i, q) =
// (t / R, t % R) from G[l, :, q] and A[i, :], both staged in LDS.
// grid: x = (l, block of EX_T slab entries) flattened
template <typename T, int RK>
__global__ __launch_bounds__(EX_T) void expand_slab_kernel(const T* __restrict__ G, int64_t L, int r, int64_t R,
                                                           const T* __restrict__ A, int64_t I, T* __restrict__ out) {
    constexpr int AROWS = EX_T / 2 + 2;                  // R >= 2: at most EX_T / R + 2 rows of A
    __shared__ T gs[RK][64];
    __shared__ T as[AROWS][RK + 1];
    const int64_t slab = I * R;
    const int64_t nb = (slab + EX_T - 1) / EX_T;
    const int64_t l = blockIdx.x / nb;
    const int64_t t0 = (blockIdx.x - l * nb) * EX_T;
    const int64_t ilo = t0 / R;
    const int64_t t1 = t0 + EX_T < slab ? t0 + EX_T : slab;
    const int nrow = (int)((t1 - 1) / R - ilo + 1);
    for (int e = threadIdx.x; e < RK * 64; e += EX_T) {
        const int k = e / 64, q = e % 64;
        gs[k][q] = (k < r && q < R) ? G[(l * r + k) * R + q] : T(0);
    }
    for (int e = threadIdx.x; e < nrow * RK; e += EX_T) {
        const int ii = e / RK, k = e % RK;
        as[ii][k] = k < r ? A[(ilo + ii) * r + k] : T(0);
    }
    __syncthreads();
    const int64_t t = t0 + threadIdx.x;
    if (t >= slab) return;
    const int ii = (int)(t / R - ilo);
    const int q = (int)(t % R);
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < RK; ++k) acc += as[ii][k] * gs[k][q];
    out[l * slab + t] = acc;
}

template <typename T, int RK>
hipError_t expand_rk(Shape3 s, const T* G, const T* A, int64_t I, T* out, hipStream_t st) {
    const int r = (int)s.J;
    if (s.R > 1 && s.R < 64) {
        const dim3 grid((unsigned)(((I * s.R + EX_T - 1) / EX_T) * s.L));
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
    if (s.R == 1) return (s.L + EX_LB - 1) / EX_LB < 0x7fffffffLL && (I + EX_T - 1) / EX_T < 65536;
    if (s.R < 64) return ((I * s.R + EX_T - 1) / EX_T) * s.L < 0x7fffffffLL;
    return ((s.R + EX_T - 1) / EX_T) * s.L < 0x7fffffffLL && (I + EX_LB - 1) / EX_LB < 65536;
}

hipError_t launch_expand(Dt dt, const void* G, Shape3 s, const void* A, int64_t I, void* out, hipStream_t stream) {
    if (!expand_ok(s, I)) return hipErrorInvalidValue;
    if (dt == Dt::F64) return expand_t<double>(s, (const double*)G, (const double*)A, I, (double*)out, stream);
    return expand_t<float>(s, (const float*)G, (const float*)A, I, (float*)out, stream);
}

}  // namespace rt
