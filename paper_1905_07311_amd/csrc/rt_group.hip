// Grouped execution of the adaptive R-STHOSVD steps (Alg. 5, §4) for many
// requests at once: the tensor-side kernels (sums of the sketch partials, the
// projections B = Q^T G_(n) and U_k^T B, the fp64 Gram of B, the per-request
// norms) and the fixed launch sequence of one iteration of the serving
// executor.  Every kernel takes its work from the descriptor arrays of
// rt_kernels.hpp; a request's work is split by its own shape only and every sum
// runs in a fixed order, so a request's result does not depend on the group.
#include "rt_kernels.hpp"

namespace rt {
namespace {

constexpr int GP_CT = 256;     // unfolding columns per projection work item
constexpr int GP_CH = 8;       // output rows per projection work item
constexpr int GG_TC = 64;      // columns per staged Gram tile

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Y = sum of the sketch partials (fixed order) and, for a first block, ||G||^2
// from the sketch's per-workgroup partials; one workgroup per request.
__global__ __launch_bounds__(256) void block_reduce_group_kernel(const GHeader* __restrict__ hdr,
                                                                 const GBlock* __restrict__ d) {
    const int i = blockIdx.x;
    if (i >= hdr->nblock) return;
    const GBlock& q = d[i];
    const int64_t n = q.J * q.b;
    for (int64_t e = threadIdx.x; e < n; e += 256) {
        double s = 0.0;
        for (int p = 0; p < q.nsplit; ++p) s += (double)q.partial[(int64_t)p * n + e];
        q.Y[e] = s;
    }
    if (q.nrm_partial) {
        __shared__ double red[256];
        double s = 0.0;
        const int np = q.nsplit * q.nrowtile;
        for (int p = threadIdx.x; p < np; p += 256) s += q.nrm_partial[p];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int k = 128; k > 0; k >>= 1) {
            if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) q.rb->xnorm2 = red[0];
    }
}

// out rows koff + 8 ch .. of (L, ldo, R) = Q^T G over the first J mode rows;
// one thread per unfolding column c = l R + r (contiguous r: coalesced loads and
// stores), Q's chunk staged in LDS, float32 fmas over the rows in order.
constexpr int GP_QMAX = 1024;  // staged Q rows per pass (x 8 floats)

__device__ void proj_item(const GProj& q, int ct, int ch, double* red) {
    __shared__ float qs[GP_QMAX][GP_CH];
    const int ell = q.ell_dev ? *q.ell_dev : q.ellmax;
    const int j0 = ch * GP_CH;
    const int tid = threadIdx.x;
    if (j0 >= ell) {
        if (tid == 0) q.nrm_partial[(int64_t)ch * q.nct + ct] = 0.0;
        return;
    }
    const int64_t ldo = q.ldo > 0 ? q.ldo : ell;
    const int64_t K = q.L * q.R;
    const int64_t c = (int64_t)ct * GP_CT + tid;
    const bool valid = c < K;
    const int64_t l = valid ? c / q.R : 0, r = valid ? c - l * q.R : 0;
    float acc[GP_CH];
#pragma unroll
    for (int t = 0; t < GP_CH; ++t) acc[t] = 0.f;
    for (int64_t i0 = 0; i0 < q.J; i0 += GP_QMAX) {
        const int rows = (int)(q.J - i0 < GP_QMAX ? q.J - i0 : GP_QMAX);
        __syncthreads();
        for (int e = tid; e < rows * GP_CH; e += 256) {
            const int ii = e / GP_CH, t = e % GP_CH;
            qs[ii][t] = (j0 + t < ell) ? q.Q[(i0 + ii) * q.ldq + j0 + t] : 0.f;
        }
        __syncthreads();
        if (valid) {
            const float* g = q.G + (l * q.ldj + i0) * q.R + r;
            for (int ii = 0; ii < rows; ++ii) {
                const float x = g[(int64_t)ii * q.R];
#pragma unroll
                for (int t = 0; t < GP_CH; ++t) acc[t] = fmaf(qs[ii][t], x, acc[t]);
            }
        }
    }
    double s2 = 0.0;
    if (valid) {
        float* o = q.out + (l * ldo + q.koff + j0) * q.R + r;
#pragma unroll
        for (int t = 0; t < GP_CH; ++t) {
            if (j0 + t < ell) {
                o[(int64_t)t * q.R] = acc[t];
                s2 += (double)acc[t] * (double)acc[t];
            }
        }
    }
    red[tid] = s2;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    if (tid == 0) q.nrm_partial[(int64_t)ch * q.nct + ct] = red[0];
}

__global__ __launch_bounds__(256) void proj_group_kernel(const GHeader* __restrict__ hdr,
                                                         const GProj* __restrict__ d, int which) {
    __shared__ double red[256];
    const int n = which == 0 ? hdr->nbproj : hdr->ncproj;
    const int64_t total = which == 0 ? hdr->bproj_items : hdr->cproj_items;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].wi0 <= w) lo = mid;
            else hi = mid - 1;
        }
        const GProj& q = d[lo];
        const int64_t local = w - q.wi0;
        proj_item(q, (int)(local % q.nct), (int)(local / q.nct), red);
        __syncthreads();
    }
}

// *rb_norm = the projection's sum of squares (its item partials in order)
__global__ __launch_bounds__(256) void proj_norm_group_kernel(const GHeader* __restrict__ hdr,
                                                              const GProj* __restrict__ d, int which) {
    const int i = blockIdx.x;
    if (i >= (which == 0 ? hdr->nbproj : hdr->ncproj)) return;
    const GProj& q = d[i];
    __shared__ double red[256];
    double s = 0.0;
    const int np = q.nct * q.nch;
    for (int p = threadIdx.x; p < np; p += 256) s += q.nrm_partial[p];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *q.rb_norm = red[0];
}

// fp64 Gram partial of B rows 0 .. n over the columns of chunk `ch`:
// gpart[ch][u][v] = sum_c B[u][c] B[v][c] (float products exact in fp64);
// threads own (u, v) pairs u <= v, columns staged GG_TC at a time.
__device__ void gram_item(const GTrunc& q, int ch) {
    __shared__ double bs[LMAX][GG_TC + 1];
    const int n = q.kcols;
    const int tid = threadIdx.x;
    const int64_t K = q.L * q.R;
    const int64_t per = (K + q.nchunk - 1) / q.nchunk;
    const int64_t c0 = (int64_t)ch * per;
    const int64_t c1 = c0 + per < K ? c0 + per : K;
    const int npairs = n * (n + 1) / 2;
    constexpr int PMAX = (LMAX * (LMAX + 1) / 2 + 255) / 256;
    int pu[PMAX], pv[PMAX];
    double acc[PMAX];
#pragma unroll
    for (int m = 0; m < PMAX; ++m) {
        const int p = tid + 256 * m;
        int u = 0, v = 0;
        if (p < npairs) {
            // pair p of the upper triangle, row by row
            int rem = p;
            while (rem >= n - u) { rem -= n - u; ++u; }
            v = u + rem;
        }
        pu[m] = p < npairs ? u : -1;
        pv[m] = v;
        acc[m] = 0.0;
    }
    for (int64_t t0 = c0; t0 < c1; t0 += GG_TC) {
        const int cols = (int)(c1 - t0 < GG_TC ? c1 - t0 : GG_TC);
        __syncthreads();
        for (int e = tid; e < n * GG_TC; e += 256) {
            const int u = e / GG_TC, cc = e % GG_TC;
            double x = 0.0;
            if (cc < cols) {
                const int64_t c = t0 + cc, l = c / q.R, r = c - l * q.R;
                x = (double)q.B[(l * q.ldk + u) * q.R + r];
            }
            bs[u][cc] = x;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PMAX; ++m) {
            if (pu[m] >= 0) {
                const double* bu = bs[pu[m]];
                const double* bv = bs[pv[m]];
                double s = acc[m];
                for (int cc = 0; cc < cols; ++cc) s = fma(bu[cc], bv[cc], s);
                acc[m] = s;
            }
        }
    }
    double* out = q.gpart + (int64_t)ch * n * n;
#pragma unroll
    for (int m = 0; m < PMAX; ++m) {
        if (pu[m] >= 0) {
            out[pu[m] * n + pv[m]] = acc[m];
            out[pv[m] * n + pu[m]] = acc[m];
        }
    }
}

__global__ __launch_bounds__(256) void gram_group_kernel(const GHeader* __restrict__ hdr,
                                                         const GTrunc* __restrict__ d) {
    const int n = hdr->ntrunc;
    const int64_t total = hdr->gram_items;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].wi0 <= w) lo = mid;
            else hi = mid - 1;
        }
        gram_item(d[lo], (int)(w - d[lo].wi0));
        __syncthreads();
    }
}

}  // namespace

int group_gram_chunks(int64_t K) {
    const int64_t c = (K + 2047) / 2048;
    return (int)(c < 1 ? 1 : (c > 32 ? 32 : c));
}

size_t group_desc_bytes(int maxreq) {
    return align256(sizeof(GHeader)) + align256(sizeof(GBlock) * maxreq) + 2 * align256(sizeof(GProj) * maxreq) +
           align256(sizeof(GTrunc) * maxreq);
}

hipError_t launch_group_tensor(const GHeader* hdr, const GBlock* blk, const GProj* bproj, const GTrunc* tr,
                               const GProj* cproj, int maxreq, hipStream_t stream, int stage) {
    switch (stage) {
        case 0:
            hipLaunchKernelGGL(block_reduce_group_kernel, dim3(maxreq), dim3(256), 0, stream, hdr, blk);
            break;
        case 1:
            hipLaunchKernelGGL(proj_group_kernel, dim3(1024), dim3(256), 0, stream, hdr, bproj, 0);
            hipLaunchKernelGGL(proj_norm_group_kernel, dim3(maxreq), dim3(256), 0, stream, hdr, bproj, 0);
            break;
        case 2:
            hipLaunchKernelGGL(gram_group_kernel, dim3(1024), dim3(256), 0, stream, hdr, tr);
            break;
        default:
            hipLaunchKernelGGL(proj_group_kernel, dim3(1024), dim3(256), 0, stream, hdr, cproj, 1);
            hipLaunchKernelGGL(proj_norm_group_kernel, dim3(maxreq), dim3(256), 0, stream, hdr, cproj, 1);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_group_iteration(const void* desc_dev, int maxreq, hipStream_t stream) {
    const char* p = (const char*)desc_dev;
    const GHeader* hdr = (const GHeader*)p;
    p += align256(sizeof(GHeader));
    const GBlock* blk = (const GBlock*)p;
    p += align256(sizeof(GBlock) * maxreq);
    const GProj* bproj = (const GProj*)p;
    p += align256(sizeof(GProj) * maxreq);
    const GTrunc* tr = (const GTrunc*)p;
    p += align256(sizeof(GTrunc) * maxreq);
    const GProj* cproj = (const GProj*)p;
    hipError_t e;
    // block steps: sketch, its sums, the orthonormalisation, the projection
    if ((e = launch_group_sketch(hdr, blk, stream)) != hipSuccess) return e;
    if ((e = launch_group_tensor(hdr, blk, bproj, tr, cproj, maxreq, stream, 0)) != hipSuccess) return e;
    if ((e = launch_group_dense(hdr, blk, tr, maxreq, stream, 0)) != hipSuccess) return e;
    if ((e = launch_group_tensor(hdr, blk, bproj, tr, cproj, maxreq, stream, 1)) != hipSuccess) return e;
    // truncations: Gram, eigensolver and factor, core update
    if ((e = launch_group_tensor(hdr, blk, bproj, tr, cproj, maxreq, stream, 2)) != hipSuccess) return e;
    if ((e = launch_group_dense(hdr, blk, tr, maxreq, stream, 1)) != hipSuccess) return e;
    return launch_group_tensor(hdr, blk, bproj, tr, cproj, maxreq, stream, 3);
}

}  // namespace rt
