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
// gpart[ch][u][v] = sum_c B[u][c] B[v][c] (float products exact in fp64).
// Thread (tile p, group g) owns the 4 x 4 tile p of the upper triangle and the
// staged columns g, g + G, ... of every 64-column tile (8 LDS reads per 16
// fmas); the G partial tiles of a tile are then added in group order.
__device__ void gram_item(const GTrunc& q, int ch) {
    __shared__ double bs[LMAX][GG_TC + 1];
    __shared__ double red[256 * 16];
    const int n = q.kcols;
    const int tid = threadIdx.x;
    const int64_t K = q.L * q.R;
    const int64_t per = (K + q.nchunk - 1) / q.nchunk;
    const int64_t c0 = (int64_t)ch * per;
    const int64_t c1 = c0 + per < K ? c0 + per : K;
    const int nt4 = (n + 3) / 4;
    const int npt = nt4 * (nt4 + 1) / 2;
    const int G = 256 / npt;                 // >= 1 (npt <= 136)
    const int pr = tid / G, g = tid - pr * G;
    const bool own = pr < npt;
    int ti = 0, tj = 0;
    {
        int rem = own ? pr : 0;
        while (rem >= nt4 - ti) { rem -= nt4 - ti; ++ti; }
        tj = ti + rem;
    }
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    for (int64_t t0 = c0; t0 < c1; t0 += GG_TC) {
        const int cols = (int)(c1 - t0 < GG_TC ? c1 - t0 : GG_TC);
        __syncthreads();
        for (int e = tid; e < LMAX * GG_TC; e += 256) {
            const int u = e / GG_TC, cc = e % GG_TC;
            double x = 0.0;
            if (cc < cols && u < n) {
                const int64_t c = t0 + cc, l = c / q.R, r = c - l * q.R;
                x = (double)q.B[(l * q.ldk + u) * q.R + r];
            }
            bs[u][cc] = x;
        }
        __syncthreads();
        if (own) {
            for (int cc = g; cc < cols; cc += G) {
                double xa[4], xb[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) { xa[x] = bs[4 * ti + x][cc]; xb[x] = bs[4 * tj + x][cc]; }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = fma(xa[x], xb[y], acc[x][y]);
            }
        }
    }
    __syncthreads();
    if (own) {
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) red[(g * npt + pr) * 16 + 4 * x + y] = acc[x][y];
    }
    __syncthreads();
    double* out = q.gpart + (int64_t)ch * n * n;
    for (int e = tid; e < npt * 16; e += 256) {
        const int p = e / 16, xy = e % 16, x = xy / 4, y = xy % 4;
        double sum = 0.0;
        for (int gg = 0; gg < G; ++gg) sum += red[(gg * npt + p) * 16 + xy];
        int rem = p, a = 0;
        while (rem >= nt4 - a) { rem -= nt4 - a; ++a; }
        const int u = 4 * a + x, v = 4 * (a + rem) + y;
        if (u < n && v < n) {
            out[u * n + v] = sum;
            out[v * n + u] = sum;
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

hipError_t launch_group_iteration(const void* desc_dev, int maxreq, int block, hipStream_t stream) {
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
    if ((e = launch_group_sketch(hdr, blk, block, stream)) != hipSuccess) return e;
    if ((e = launch_group_tensor(hdr, blk, bproj, tr, cproj, maxreq, stream, 0)) != hipSuccess) return e;
    if ((e = launch_group_dense(hdr, blk, tr, maxreq, stream, 0)) != hipSuccess) return e;
    if ((e = launch_group_tensor(hdr, blk, bproj, tr, cproj, maxreq, stream, 1)) != hipSuccess) return e;
    // truncations: Gram, eigensolver and factor, core update
    if ((e = launch_group_tensor(hdr, blk, bproj, tr, cproj, maxreq, stream, 2)) != hipSuccess) return e;
    if ((e = launch_group_dense(hdr, blk, tr, maxreq, stream, 1)) != hipSuccess) return e;
    return launch_group_tensor(hdr, blk, bproj, tr, cproj, maxreq, stream, 3);
}

}  // namespace rt
