// Sparse (COO) steps of SP-STHOSVD (Alg. 6, §5): the sketch Y = G_(n) Omega of
// a coordinate-stored core, the restriction G_(n) <- P^T G_(n) to the selected
// mode-n slices (the next core stays sparse and holds entries of X only), and
// the final scatter of the small core into dense storage.
//
// Storage: entry e has coordinates idx[m * ldi + e] (int32, one array per mode,
// so the lanes of a wave read consecutive words) and value vals[e].  The entry
// count of an intermediate core lives on the device (written by the compaction)
// and is read by the next kernels, so a whole decomposition runs without a host
// round trip; grids are sized by the input's count, an upper bound.
//
// The sketch scatters v * Omega[c, k] into Y (fp64) with hardware atomic adds:
// the order of the additions into one Y entry is not fixed, so the sparse sketch
// is reproducible to fp64 rounding, not bitwise.  Every other step here is
// order-preserving and exact (copies and index arithmetic); the dense core is
// formed by atomic adds onto zeros, exact when the coordinates are distinct
// (repeated coordinates are summed, as in the sketch).
//
// Every kernel checks each entry's coordinates against the dims and skips an
// entry with one out of range; coo_check_kernel reports such entries.
#include "rt_kernels.hpp"
#include "rt_philox.hpp"

namespace rt {

namespace {

constexpr int CO_CHUNK = 1024;   // entries per compaction workgroup (256 threads x 4)

__device__ __forceinline__ bool coo_valid(const int32_t* __restrict__ idx, int64_t ldi, int64_t e, const CooDims& cd) {
    bool ok = true;
    for (int m = 0; m < cd.d; ++m) {
        const int32_t v = idx[m * ldi + e];
        ok = ok && v >= 0 && (int64_t)v < cd.dims[m];
    }
    return ok;
}

__global__ __launch_bounds__(256) void coo_check_kernel(const int32_t* __restrict__ idx, int64_t ldi, int64_t nnz,
                                                        CooDims cd, uint32_t* __restrict__ status, uint32_t bit) {
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256)
        bad = bad || !coo_valid(idx, ldi, e, cd);
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(status, bit);
}

template <typename T>
__global__ __launch_bounds__(256) void coo_sketch_kernel(const int32_t* __restrict__ idx, int64_t ldi,
                                                         const T* __restrict__ vals, const int64_t* __restrict__ nnz_dev,
                                                         int64_t bound, CooDims cd, int mode, int ell, int64_t col0,
                                                         uint64_t seed, double* __restrict__ Y) {
    const int64_t nnz = nnz_dev ? *nnz_dev : bound;
    const int64_t q_first = col0 / 4;
    const int64_t q_last = (col0 + ell - 1) / 4;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256) {
        if (!coo_valid(idx, ldi, e, cd)) continue;
        // column of the mode-n unfolding: row-major index over the other modes
        int64_t c = 0;
        for (int m = 0; m < cd.d; ++m)
            if (m != mode) c = c * cd.dims[m] + idx[m * ldi + e];
        const int64_t i = idx[mode * ldi + e];
        const double v = (double)vals[e];
        double* yrow = Y + i * ell;
        for (int64_t q = q_first; q <= q_last; ++q) {
            T z[4];
            OmegaGen<T>::gen4(seed, (uint32_t)mode, (uint64_t)c, (uint32_t)q, z);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t k = 4 * q + t - col0;
                if (k >= 0 && k < ell) unsafeAtomicAdd(yrow + k, v * (double)z[t]);
            }
        }
    }
}

__global__ void coo_inverse_kernel(const int* __restrict__ sel, int ell, int32_t* __restrict__ inv) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < ell) inv[sel[j]] = j;
}

// Kept flags of entries [b CO_CHUNK, (b + 1) CO_CHUNK): thread t owns the four
// consecutive entries b CO_CHUNK + 4 t + u.
__device__ __forceinline__ int coo_flags(const int32_t* __restrict__ idx, int64_t ldi, int64_t nnz, const CooDims& cd,
                                         int mode, const int32_t* __restrict__ inv, int64_t b, int32_t pos[4]) {
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t e = b * CO_CHUNK + 4 * threadIdx.x + u;
        pos[u] = e < nnz && coo_valid(idx, ldi, e, cd) ? inv[idx[mode * ldi + e]] : -1;
        cnt += pos[u] >= 0;
    }
    return cnt;
}

// Exclusive prefix over the 256 threads of a workgroup; returns the prefix of
// this thread, *total the sum.
__device__ __forceinline__ int block_exclusive(int v, int* sh, int* total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = 1; s < 256; s <<= 1) {
        const int a = t >= s ? sh[t - s] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    const int incl = sh[t];
    *total = sh[255];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void coo_count_kernel(const int32_t* __restrict__ idx, int64_t ldi,
                                                        const int64_t* __restrict__ nnz_dev, int64_t bound, CooDims cd,
                                                        int mode, const int32_t* __restrict__ inv,
                                                        int64_t* __restrict__ cnt) {
    __shared__ int sh[256];
    const int64_t nnz = nnz_dev ? *nnz_dev : bound;
    const int64_t b = blockIdx.x;
    int32_t pos[4];
    const int c = coo_flags(idx, ldi, nnz, cd, mode, inv, b, pos);
    int total = 0;
    (void)block_exclusive(c, sh, &total);
    if (threadIdx.x == 0) cnt[b] = total;
}

// One workgroup: off[b] = sum of cnt[0 .. b), *nnz_out = sum of all.
__global__ __launch_bounds__(256) void coo_scan_kernel(const int64_t* __restrict__ cnt, int64_t nb,
                                                       int64_t* __restrict__ off, int64_t* __restrict__ nnz_out) {
    __shared__ int64_t sh[256];
    const int t = threadIdx.x;
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t v = b0 + t < nb ? cnt[b0 + t] : 0;
        sh[t] = v;
        __syncthreads();
        for (int s = 1; s < 256; s <<= 1) {
            const int64_t a = t >= s ? sh[t - s] : 0;
            __syncthreads();
            sh[t] += a;
            __syncthreads();
        }
        if (b0 + t < nb) off[b0 + t] = carry + sh[t] - v;
        carry += sh[255];
        __syncthreads();
    }
    if (t == 0) *nnz_out = carry;
}

// Order-preserving compaction of the kept entries; the mode-n coordinate
// becomes the entry's position in the selection.
template <typename T>
__global__ __launch_bounds__(256) void coo_scatter_kernel(const int32_t* __restrict__ idx, int64_t ldi,
                                                          const T* __restrict__ vals, const int64_t* __restrict__ nnz_dev,
                                                          int64_t bound, CooDims cd, int mode,
                                                          const int32_t* __restrict__ inv,
                                                          const int64_t* __restrict__ off, int32_t* __restrict__ idx_out,
                                                          int64_t ldo, T* __restrict__ vals_out) {
    __shared__ int sh[256];
    const int64_t nnz = nnz_dev ? *nnz_dev : bound;
    const int64_t b = blockIdx.x;
    int32_t pos[4];
    const int c = coo_flags(idx, ldi, nnz, cd, mode, inv, b, pos);
    int total = 0;
    int64_t o = off[b] + block_exclusive(c, sh, &total);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (pos[u] < 0) continue;
        const int64_t e = b * CO_CHUNK + 4 * threadIdx.x + u;
        for (int m = 0; m < cd.d; ++m) idx_out[m * ldo + o] = m == mode ? pos[u] : idx[m * ldi + e];
        vals_out[o] = vals[e];
        ++o;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void coo_densify_kernel(const int32_t* __restrict__ idx, int64_t ldi,
                                                          const T* __restrict__ vals, const int64_t* __restrict__ nnz_dev,
                                                          int64_t bound, CooDims cd, T* __restrict__ out) {
    const int64_t nnz = nnz_dev ? *nnz_dev : bound;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256) {
        if (!coo_valid(idx, ldi, e, cd)) continue;
        int64_t lin = 0;
        for (int m = 0; m < cd.d; ++m) lin = lin * cd.dims[m] + idx[m * ldi + e];
        unsafeAtomicAdd(out + lin, vals[e]);
    }
}

// ---- binned sketch: the entries grouped by blocks of 2^shift rows first ----------------
// Device-scope atomic adds resolve beyond the per-XCD L2, so scattering every
// v * Omega[c, k] into Y directly runs at the atomic rate.  For a large core the
// entries are first grouped by row block (a counting sort without stable
// order: per-chunk histograms in LDS, one scan, LDS cursors), then each piece of
// a block's entries is accumulated into an LDS copy of the block's rows and
// added to Y once.
constexpr int BN_CH = 65536;     // entries per counting workgroup
constexpr int BN_MAXB = 2048;    // row blocks
constexpr int BN_PS = 8192;      // entries per accumulation piece
constexpr int BN_LDSY = 4096;    // doubles of an LDS row block (rows x ell)

__device__ __forceinline__ int64_t coo_column(const int32_t* __restrict__ idx, int64_t ldi, int64_t e,
                                              const CooDims& cd, int mode) {
    int64_t c = 0;
    for (int m = 0; m < cd.d; ++m)
        if (m != mode) c = c * cd.dims[m] + idx[m * ldi + e];
    return c;
}

__global__ __launch_bounds__(256) void coo_bin_count_kernel(const int32_t* __restrict__ idx, int64_t nnz, CooDims cd,
                                                            int mode, int shift, int nbk, int32_t* __restrict__ hist) {
    __shared__ int h[BN_MAXB];
    for (int b = threadIdx.x; b < nbk; b += 256) h[b] = 0;
    __syncthreads();
    const int64_t e0 = (int64_t)blockIdx.x * BN_CH;
    const int64_t e1 = e0 + BN_CH < nnz ? e0 + BN_CH : nnz;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256)
        if (coo_valid(idx, nnz, e, cd)) atomicAdd(&h[idx[mode * nnz + e] >> shift], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < nbk; b += 256) hist[(int64_t)blockIdx.x * nbk + b] = h[b];
}

// One workgroup: bucket totals, their exclusive scan (bstart[0 .. nbk]), the
// pieces per bucket and their scan (pstart[0 .. nbk]), and every chunk's
// starting offset in every bucket (off[chunk][b]).
__global__ __launch_bounds__(256) void coo_bin_scan_kernel(const int32_t* __restrict__ hist, int64_t nch, int nbk,
                                                           int64_t* __restrict__ bstart, int64_t* __restrict__ pstart,
                                                           int64_t* __restrict__ off) {
    __shared__ int64_t tot[BN_MAXB];
    __shared__ int64_t sb[256], sp[256];
    const int t = threadIdx.x;
    for (int b = t; b < nbk; b += 256) {
        int64_t s = 0;
        for (int64_t c = 0; c < nch; ++c) s += hist[c * nbk + b];
        tot[b] = s;
    }
    __syncthreads();
    // each thread scans eight consecutive buckets; the 256 partial sums are scanned in LDS
    constexpr int PER = BN_MAXB / 256;
    int64_t vb = 0, vp = 0;
    for (int u = 0; u < PER; ++u) {
        const int b = t * PER + u;
        if (b < nbk) { vb += tot[b]; vp += (tot[b] + BN_PS - 1) / BN_PS; }
    }
    sb[t] = vb;
    sp[t] = vp;
    __syncthreads();
    for (int s2 = 1; s2 < 256; s2 <<= 1) {
        const int64_t ab = t >= s2 ? sb[t - s2] : 0, ap = t >= s2 ? sp[t - s2] : 0;
        __syncthreads();
        sb[t] += ab;
        sp[t] += ap;
        __syncthreads();
    }
    int64_t rb = sb[t] - vb, rp = sp[t] - vp;
    for (int u = 0; u < PER; ++u) {
        const int b = t * PER + u;
        if (b < nbk) {
            bstart[b] = rb;
            pstart[b] = rp;
            rb += tot[b];
            rp += (tot[b] + BN_PS - 1) / BN_PS;
        }
    }
    if (t == 255) { bstart[nbk] = sb[255]; pstart[nbk] = sp[255]; }
    __syncthreads();
    for (int b = t; b < nbk; b += 256) {
        int64_t run = 0;
        for (int u = 0; u < b; ++u) run += tot[u];
        for (int64_t c = 0; c < nch; ++c) {
            off[c * nbk + b] = run;
            run += hist[c * nbk + b];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void coo_bin_scatter_kernel(const int32_t* __restrict__ idx,
                                                              const T* __restrict__ vals, int64_t nnz, CooDims cd,
                                                              int mode, int shift, int nbk,
                                                              const int64_t* __restrict__ off,
                                                              int64_t* __restrict__ keys, double* __restrict__ rv) {
    __shared__ unsigned long long cur[BN_MAXB];
    for (int b = threadIdx.x; b < nbk; b += 256) cur[b] = (unsigned long long)off[(int64_t)blockIdx.x * nbk + b];
    __syncthreads();
    const int64_t e0 = (int64_t)blockIdx.x * BN_CH;
    const int64_t e1 = e0 + BN_CH < nnz ? e0 + BN_CH : nnz;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        if (!coo_valid(idx, nnz, e, cd)) continue;
        const int32_t row = idx[mode * nnz + e];
        const int64_t pos = (int64_t)atomicAdd(&cur[row >> shift], 1ull);
        keys[pos] = (coo_column(idx, nnz, e, cd, mode) << shift) | (row & ((1 << shift) - 1));
        rv[pos] = (double)vals[e];
    }
}

// Pieces p = blockIdx.x, blockIdx.x + gridDim.x, ... of pstart[nbk]; piece j of
// bucket b covers its entries [bstart[b] + j BN_PS, ...).
template <typename TO>
__global__ __launch_bounds__(256) void coo_bin_sketch_kernel(const int64_t* __restrict__ keys,
                                                             const double* __restrict__ rv,
                                                             const int64_t* __restrict__ bstart,
                                                             const int64_t* __restrict__ pstart, int nbk, int shift,
                                                             int64_t J, int ell, int64_t col0, uint64_t seed,
                                                             uint32_t mode, double* __restrict__ Y) {
    __shared__ double yb[BN_LDSY];
    const int br = 1 << shift;
    const int64_t P = pstart[nbk];
    const int64_t q_first = col0 / 4;
    const int64_t q_last = (col0 + ell - 1) / 4;
    for (int64_t p = blockIdx.x; p < P; p += gridDim.x) {
        int lo = 0, hi = nbk - 1;
        while (lo < hi) {                          // last bucket with pstart <= p
            const int mid = (lo + hi + 1) >> 1;
            if (pstart[mid] <= p) lo = mid;
            else hi = mid - 1;
        }
        const int b = lo;
        const int64_t r0 = bstart[b] + (p - pstart[b]) * BN_PS;
        const int64_t r1 = r0 + BN_PS < bstart[b + 1] ? r0 + BN_PS : bstart[b + 1];
        for (int e = threadIdx.x; e < br * ell; e += 256) yb[e] = 0.0;
        __syncthreads();
        for (int64_t e = r0 + threadIdx.x; e < r1; e += 256) {
            const int64_t key = keys[e];
            const double v = rv[e];
            const int r = (int)(key & (br - 1));
            const int64_t c = key >> shift;
            double* yr = yb + r * ell;
            for (int64_t q = q_first; q <= q_last; ++q) {
                TO z[4];
                OmegaGen<TO>::gen4(seed, mode, (uint64_t)c, (uint32_t)q, z);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int64_t k = 4 * q + t - col0;
                    if (k >= 0 && k < ell)
                        __hip_atomic_fetch_add(yr + k, v * (double)z[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < br * ell; e += 256) {
            const int64_t row = (int64_t)b * br + e / ell;
            const double val = yb[e];
            if (row < J && val != 0.0) unsafeAtomicAdd(Y + row * ell + e % ell, val);
        }
        __syncthreads();
    }
}

unsigned stride_grid(int64_t bound) {
    const int64_t g = (bound + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

int64_t coo_chunks(int64_t bound) { return bound > 0 ? (bound + CO_CHUNK - 1) / CO_CHUNK : 0; }

hipError_t launch_coo_sketch(const int32_t* idx, int64_t ldi, const void* vals, Dt dt, const int64_t* nnz_dev,
                             int64_t bound, const CooDims& cd, int mode, int ell, int64_t col0, uint64_t seed,
                             double* Y, hipStream_t stream) {
    if (bound <= 0) return hipSuccess;
    if (dt == Dt::F64)
        hipLaunchKernelGGL(coo_sketch_kernel<double>, dim3(stride_grid(bound)), dim3(256), 0, stream, idx, ldi,
                           (const double*)vals, nnz_dev, bound, cd, mode, ell, col0, seed, Y);
    else
        hipLaunchKernelGGL(coo_sketch_kernel<float>, dim3(stride_grid(bound)), dim3(256), 0, stream, idx, ldi,
                           (const float*)vals, nnz_dev, bound, cd, mode, ell, col0, seed, Y);
    return hipGetLastError();
}

hipError_t launch_coo_check(const int32_t* idx, int64_t ldi, int64_t nnz, const CooDims& cd, uint32_t* status,
                            uint32_t bit, hipStream_t stream) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(coo_check_kernel, dim3(stride_grid(nnz)), dim3(256), 0, stream, idx, ldi, nnz, cd, status, bit);
    return hipGetLastError();
}

BinPlan plan_coo_bins(int64_t J, int ell, int64_t nnz) {
    BinPlan p{};
    int shift = 0;
    while (((J + (1LL << shift) - 1) >> shift) > BN_MAXB) ++shift;
    p.shift = shift;
    p.nbk = (int)((J + (1LL << shift) - 1) >> shift);
    p.nch = (nnz + BN_CH - 1) / BN_CH;
    p.ok = nnz > 0 && (1LL << shift) * ell <= BN_LDSY && shift < 20;
    return p;
}

hipError_t launch_coo_sketch_binned(const BinPlan& bp, const int32_t* idx, const void* vals, Dt dt, int64_t nnz,
                                    const CooDims& cd, int mode, int ell, int64_t col0, uint64_t seed, double* Y,
                                    int32_t* hist, int64_t* off, int64_t* bstart, int64_t* pstart, int64_t* keys,
                                    double* rv, hipStream_t stream) {
    if (!bp.ok || ell < 1 || ell > LMAX) return hipErrorInvalidValue;
    const unsigned nch = (unsigned)bp.nch;
    hipLaunchKernelGGL(coo_bin_count_kernel, dim3(nch), dim3(256), 0, stream, idx, nnz, cd, mode, bp.shift, bp.nbk,
                       hist);
    hipLaunchKernelGGL(coo_bin_scan_kernel, dim3(1), dim3(256), 0, stream, (const int32_t*)hist, bp.nch, bp.nbk,
                       bstart, pstart, off);
    if (dt == Dt::F64)
        hipLaunchKernelGGL(coo_bin_scatter_kernel<double>, dim3(nch), dim3(256), 0, stream, idx, (const double*)vals,
                           nnz, cd, mode, bp.shift, bp.nbk, (const int64_t*)off, keys, rv);
    else
        hipLaunchKernelGGL(coo_bin_scatter_kernel<float>, dim3(nch), dim3(256), 0, stream, idx, (const float*)vals,
                           nnz, cd, mode, bp.shift, bp.nbk, (const int64_t*)off, keys, rv);
    // pieces: at most nnz / BN_PS + nbk
    int64_t maxp = nnz / BN_PS + bp.nbk;
    const unsigned g = (unsigned)(maxp < 2048 ? maxp : 2048);
    if (dt == Dt::F64)
        hipLaunchKernelGGL(coo_bin_sketch_kernel<double>, dim3(g), dim3(256), 0, stream, (const int64_t*)keys,
                           (const double*)rv, (const int64_t*)bstart, (const int64_t*)pstart, bp.nbk, bp.shift,
                           cd.dims[mode], ell, col0, seed, (uint32_t)mode, Y);
    else
        hipLaunchKernelGGL(coo_bin_sketch_kernel<float>, dim3(g), dim3(256), 0, stream, (const int64_t*)keys,
                           (const double*)rv, (const int64_t*)bstart, (const int64_t*)pstart, bp.nbk, bp.shift,
                           cd.dims[mode], ell, col0, seed, (uint32_t)mode, Y);
    return hipGetLastError();
}

hipError_t launch_coo_restrict(const int32_t* idx, int64_t ldi, const void* vals, Dt dt, const int64_t* nnz_dev,
                               int64_t bound, const CooDims& cd, int mode, const int* sel, int ell, int32_t* inv,
                               int64_t* cnt, int64_t* off, int32_t* idx_out, int64_t ldo, void* vals_out,
                               int64_t* nnz_out, hipStream_t stream) {
    hipError_t err = hipMemsetAsync(inv, 0xff, (size_t)cd.dims[mode] * sizeof(int32_t), stream);   // -1: not selected
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(coo_inverse_kernel, dim3((ell + 255) / 256), dim3(256), 0, stream, sel, ell, inv);
    const int64_t nb = coo_chunks(bound);
    if (nb > 0)
        hipLaunchKernelGGL(coo_count_kernel, dim3((unsigned)nb), dim3(256), 0, stream, idx, ldi, nnz_dev, bound, cd,
                           mode, (const int32_t*)inv, cnt);
    hipLaunchKernelGGL(coo_scan_kernel, dim3(1), dim3(256), 0, stream, (const int64_t*)cnt, nb, off, nnz_out);
    if (nb > 0) {
        if (dt == Dt::F64)
            hipLaunchKernelGGL(coo_scatter_kernel<double>, dim3((unsigned)nb), dim3(256), 0, stream, idx, ldi,
                               (const double*)vals, nnz_dev, bound, cd, mode, (const int32_t*)inv,
                               (const int64_t*)off, idx_out, ldo, (double*)vals_out);
        else
            hipLaunchKernelGGL(coo_scatter_kernel<float>, dim3((unsigned)nb), dim3(256), 0, stream, idx, ldi,
                               (const float*)vals, nnz_dev, bound, cd, mode, (const int32_t*)inv,
                               (const int64_t*)off, idx_out, ldo, (float*)vals_out);
    }
    return hipGetLastError();
}

hipError_t launch_coo_densify(const int32_t* idx, int64_t ldi, const void* vals, Dt dt, const int64_t* nnz_dev,
                              int64_t bound, const CooDims& cd, void* out, hipStream_t stream) {
    if (bound <= 0) return hipSuccess;
    if (dt == Dt::F64)
        hipLaunchKernelGGL(coo_densify_kernel<double>, dim3(stride_grid(bound)), dim3(256), 0, stream, idx, ldi,
                           (const double*)vals, nnz_dev, bound, cd, (double*)out);
    else
        hipLaunchKernelGGL(coo_densify_kernel<float>, dim3(stride_grid(bound)), dim3(256), 0, stream, idx, ldi,
                           (const float*)vals, nnz_dev, bound, cd, (float*)out);
    return hipGetLastError();
}

}  // namespace rt
