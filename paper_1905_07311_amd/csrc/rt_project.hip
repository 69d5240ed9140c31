// Mode-n projection B = G x_n Q^T (§2.4 Alg. 1 step 3, B = Q^T X on the unfolding;
// the core update of Alg. 3 G_(n) <- U^T G_(n) is the same contraction), on the
// strided (L, J, R) view: B[l, k, r] = sum_i Q[i, k] G[l, i, r].  The output keeps
// the row-major layout with mode n resized to ell, so no transpose is needed
// before the next mode.  Optionally fused: the fp64 Gram B_(n) B_(n)^T of the
// workgroup's columns (input of the truncation SVD) and sum B^2 (fp64, the
// adaptive error indicator update).
//
// Plus the small helpers: Frobenius norms with fp64 accumulation, dtype casts,
// and the explicit Omega / raw Philox words used by the tests.
#include "rt_kernels.hpp"
#include "rt_philox.hpp"

namespace rt {

namespace {

constexpr int PJ_NC = 64;    // unfolding columns per tile
constexpr int PJ_JT = 32;    // contraction rows per stage
constexpr int PJ_NACC = LMAX / 4;

template <typename TX, typename TQ, typename TA>
__global__ __launch_bounds__(256) void project_generic_kernel(
    const TX* __restrict__ G, int64_t L, int64_t J, int64_t ldj, int64_t R, const TQ* __restrict__ Q, int64_t ldq,
    int ell, TX* __restrict__ B, int64_t ldk, int64_t koff, double* __restrict__ gram_partial,
    double* __restrict__ nrm2_partial) {
    __shared__ TA gs[PJ_JT][PJ_NC + 1];
    __shared__ TA qs[PJ_JT][LMAX + 4];
    __shared__ double bs[LMAX][PJ_NC + 1];
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int cl = tid % PJ_NC;
    const int kg = tid / PJ_NC;
    const int64_t K = L * R;
    const int64_t ntiles = (K + PJ_NC - 1) / PJ_NC;
    const bool want_gram = gram_partial != nullptr;
    const int npairs = ell * (ell + 1) / 2;
    double gacc[9];
    int pa[9], pb[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        gacc[m] = 0.0;
        const int t = tid + 256 * m;
        int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((a + 1) * (a + 2) / 2 <= t) ++a;
        while (a * (a + 1) / 2 > t) --a;
        pa[m] = a;
        pb[m] = t - a * (a + 1) / 2;
    }
    double nrm = 0.0;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t cbase = tile * PJ_NC;
        TA acc[PJ_NACC];
#pragma unroll
        for (int j = 0; j < PJ_NACC; ++j) acc[j] = TA(0);
        for (int64_t i0 = 0; i0 < J; i0 += PJ_JT) {
            __syncthreads();
            for (int e = tid; e < PJ_JT * PJ_NC; e += 256) {
                int ii, cc;
                if (R == 1) { ii = e % PJ_JT; cc = e / PJ_JT; }
                else        { cc = e % PJ_NC; ii = e / PJ_NC; }
                const int64_t c = cbase + cc, i = i0 + ii;
                TA v = TA(0);
                if (c < K && i < J) {
                    const int64_t l = c / R, r = c - l * R;
                    v = (TA)G[(l * ldj + i) * R + r];
                }
                gs[ii][cc] = v;
            }
            for (int e = tid; e < PJ_JT * ell; e += 256) {
                const int ii = e / ell, k = e % ell;
                const int64_t i = i0 + ii;
                qs[ii][k] = (i < J) ? (TA)Q[i * ldq + k] : TA(0);
            }
            __syncthreads();
            const int rows = (int)((J - i0) < PJ_JT ? (J - i0) : PJ_JT);
            for (int ii = 0; ii < rows; ++ii) {
                const TA g = gs[ii][cl];
#pragma unroll
                for (int j = 0; j < PJ_NACC; ++j) {
                    const int k = kg + 4 * j;
                    if (k < ell) acc[j] += qs[ii][k] * g;
                }
            }
        }
        const int64_t c = cbase + cl;
        const bool cvalid = c < K;
        int64_t l = 0, r = 0;
        if (cvalid) { l = c / R; r = c - l * R; }
#pragma unroll
        for (int j = 0; j < PJ_NACC; ++j) {
            const int k = kg + 4 * j;
            if (k < ell) {
                const double v = cvalid ? (double)acc[j] : 0.0;
                if (cvalid) B[(l * ldk + koff + k) * R + r] = (TX)acc[j];
                nrm += v * v;
                if (want_gram) bs[k][cl] = v;
            }
        }
        if (want_gram) {
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 9; ++m) {
                if (tid + 256 * m < npairs) {
                    double s = 0.0;
                    for (int q = 0; q < PJ_NC; ++q) s += bs[pa[m]][q] * bs[pb[m]][q];
                    gacc[m] += s;
                }
            }
        }
    }
    if (want_gram) {
        double* gp = gram_partial + (int64_t)blockIdx.x * ell * ell;
#pragma unroll
        for (int m = 0; m < 9; ++m) {
            if (tid + 256 * m < npairs) {
                gp[pa[m] * ell + pb[m]] = gacc[m];
                gp[pb[m] * ell + pa[m]] = gacc[m];
            }
        }
    }
    if (nrm2_partial) {
        __syncthreads();
        red[tid] = nrm;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        if (tid == 0) nrm2_partial[blockIdx.x] = red[0];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void norm2_kernel(const T* __restrict__ X, int64_t n, double* __restrict__ partial) {
    __shared__ double red[256];
    // 16-byte loads, four in flight per thread, over the 16-byte-aligned body;
    // the scalar head and tail go to the first threads of workgroup 0
    constexpr int V = 16 / sizeof(T);
    typedef T tv __attribute__((ext_vector_type(V)));
    const int64_t head = (int64_t)(((16 - ((uintptr_t)X & 15)) & 15) / sizeof(T));
    const int64_t h = head < n ? head : n;
    const int64_t nv = (n - h) / V;
    const tv* Xv = reinterpret_cast<const tv*>(X + h);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; e + 3 * stride < nv; e += 4 * stride) {
        const tv a = Xv[e], b = Xv[e + stride], c = Xv[e + 2 * stride], d = Xv[e + 3 * stride];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            s0 = fma((double)a[u], (double)a[u], s0);
            s1 = fma((double)b[u], (double)b[u], s1);
            s2 = fma((double)c[u], (double)c[u], s2);
            s3 = fma((double)d[u], (double)d[u], s3);
        }
    }
    for (; e < nv; e += stride) {
        const tv a = Xv[e];
#pragma unroll
        for (int u = 0; u < V; ++u) s0 = fma((double)a[u], (double)a[u], s0);
    }
    double s = (s0 + s1) + (s2 + s3);
    if (blockIdx.x == 0) {
        const int64_t t0 = h + nv * V;
        if ((int64_t)threadIdx.x < h) { const double v = (double)X[threadIdx.x]; s = fma(v, v, s); }
        if (t0 + (int64_t)threadIdx.x < n) { const double v = (double)X[t0 + threadIdx.x]; s = fma(v, v, s); }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

template <typename T>
__global__ __launch_bounds__(256) void cast_kernel(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = (T)src[e];
}

template <typename T>
__global__ __launch_bounds__(256) void omega_kernel(uint64_t seed, uint32_t mode, int64_t c0, int64_t nrows,
                                                    int64_t col0, int ncols, T* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nrows * ncols) return;
    const int64_t i = e / ncols;
    const int j = (int)(e % ncols);
    const int64_t k = col0 + j;
    T z[4];
    OmegaGen<T>::gen4(seed, mode, (uint64_t)(c0 + i), (uint32_t)(k / 4), z);
    out[e] = z[k % 4];
}

__global__ __launch_bounds__(256) void philox_words_kernel(uint64_t seed, uint32_t mode, int64_t c0, int64_t n,
                                                           uint32_t q, uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    PhiloxOut w = omega_words(seed, mode, (uint64_t)(c0 + i), q);
    out[4 * i + 0] = w.w0;
    out[4 * i + 1] = w.w1;
    out[4 * i + 2] = w.w2;
    out[4 * i + 3] = w.w3;
}

}  // namespace

ProjectPlan plan_project(Dt dx, Dt dq, Shape3 s, int ell, const void* G, const void* B, int64_t koff) {
    ProjectPlan p{};
    if (dx == Dt::F32 && dq == Dt::F32 && project_mfma_ok(s, ell, G, B, koff)) {
        p.kind = 1;
        plan_project_mfma(p, s, ell);
        p.ntiles = 0;
        return p;
    }
    if (dx == Dt::F32 && dq == Dt::F32 && s.R == 1 && ell <= LMAX) {
        p.kind = 2;
        plan_project_r1_mfma(p, s, ell);
        p.ntiles = 0;
        return p;
    }
    const int64_t K = s.L * s.R;
    p.ntiles = (K + PJ_NC - 1) / PJ_NC;
    p.nwg = (int)(p.ntiles < 1024 ? p.ntiles : 1024);
    if (p.nwg < 1) p.nwg = 1;
    p.kind = 0;
    return p;
}

hipError_t launch_project(const ProjectPlan& p, Dt dx, Dt dq, const void* G, Shape3 s, int64_t ldj, const void* Q,
                          int64_t ldq, int ell, void* B, int64_t ldk, int64_t koff, double* gram_partial,
                          double* nrm2_partial, hipStream_t stream) {
    if (p.kind == 1 || p.kind == 2) {
        if (gram_partial) return hipErrorInvalidValue;   // the MFMA variants have no fused Gram
        if (p.kind == 2)
            return launch_project_r1_mfma(p, (const float*)G, s, ldj, (const float*)Q, ldq, ell, (float*)B, ldk,
                                          koff, nrm2_partial, stream);
        return launch_project_mfma(p, (const float*)G, s, ldj, (const float*)Q, ldq, ell, (float*)B, ldk, koff,
                                   nrm2_partial, stream);
    }
    dim3 grid(p.nwg);
    if (dx == Dt::F64) {
        if (dq != Dt::F64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((project_generic_kernel<double, double, double>), grid, dim3(256), 0, stream,
                           (const double*)G, s.L, s.J, ldj, s.R, (const double*)Q, ldq, ell, (double*)B, ldk, koff,
                           gram_partial, nrm2_partial);
    } else if (dq == Dt::F64) {
        hipLaunchKernelGGL((project_generic_kernel<float, double, double>), grid, dim3(256), 0, stream,
                           (const float*)G, s.L, s.J, ldj, s.R, (const double*)Q, ldq, ell, (float*)B, ldk, koff,
                           gram_partial, nrm2_partial);
    } else {
        hipLaunchKernelGGL((project_generic_kernel<float, float, float>), grid, dim3(256), 0, stream,
                           (const float*)G, s.L, s.J, ldj, s.R, (const float*)Q, ldq, ell, (float*)B, ldk, koff,
                           gram_partial, nrm2_partial);
    }
    return hipGetLastError();
}

// fp64 Gram of the first k mode rows of a (L, ldk, R) tensor: per-workgroup
// partials W_wg[a][b] = sum over the workgroup's columns c of B[l, a, r] B[l, b, r].
// Tiles of 64 columns are staged in LDS as doubles (bs[c][a]); every thread owns
// an 8 x 8 block of the upper triangle of W and every G-th column of a tile, and
// the G partial blocks are added through LDS at the end (16 entries per round).
constexpr int G3_NC = 64;
constexpr int G3_LD = LMAX + 4;

template <typename T, bool WIDE>
__device__ __forceinline__ void gram3_body(const T* __restrict__ B, int64_t L, int64_t ldk, int64_t R, int k,
                                           double* __restrict__ partial, double* bs) {
    const int tid = threadIdx.x;
    const int64_t K = L * R;
    const int64_t ntiles = (K + G3_NC - 1) / G3_NC;
    const int nt = (k + 7) / 8, kpad = 8 * nt;
    const int npt = nt * (nt + 1) / 2;
    int G = 64;
    while (G > 1 && G * npt > 256) G >>= 1;
    const int pr = tid / G, g = tid % G;
    int ti = 0, tj = 0;
    if (pr < npt) {
        int rem = pr;
        while (rem >= nt - ti) { rem -= nt - ti; ++ti; }
        tj = ti + rem;
    }
    double acc[8][8];
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) acc[x][y] = 0.0;
    // staging of a tile: each thread loads up to G3_PER elements into registers
    // (the next tile's loads are issued before the current tile is used); the
    // loads are unconditional (offset clamped into B, out-of-range values
    // replaced by zero) so that they all stay in flight together
    constexpr int G3_PER = (G3_NC * (LMAX + 8) + 255) / 256;
    const int nst = G3_NC * kpad;
    const int64_t maxoff = L * ldk * R - 1;
    int e_aa[G3_PER], e_cc[G3_PER];
#pragma unroll
    for (int u = 0; u < G3_PER; ++u) {
        const int e = u * 256 + tid;
        if (R == 1) { e_aa[u] = e % kpad; e_cc[u] = e / kpad; }
        else        { e_cc[u] = e % G3_NC; e_aa[u] = e / G3_NC; }
    }
    double pre[G3_PER];
    auto load_tile = [&](int64_t tile) {
        const int64_t cbase = tile * G3_NC;
        // column c = l R + r: one division per tile, then at most one wrap (WIDE,
        // R >= G3_NC) or a 32-bit division per element
        const int64_t l0 = cbase / R, r0 = cbase - l0 * R;
        float raw[G3_PER];
#pragma unroll
        for (int u = 0; u < G3_PER; ++u) {
            const int aa = e_aa[u], cc = e_cc[u];
            int64_t l = l0, r = r0 + cc;
            if (WIDE) {
                const bool w = r >= R;
                r = w ? r - R : r;
                l = w ? l + 1 : l;
            } else {
                const uint32_t q = (uint32_t)r / (uint32_t)R;
                l += q;
                r -= (int64_t)q * R;
            }
            int64_t off = (l * ldk + aa) * R + r;
            off = off < maxoff ? off : maxoff;
            raw[u] = (float)B[off];
        }
#pragma unroll
        for (int u = 0; u < G3_PER; ++u) {
            const bool ok = u * 256 + tid < nst && e_aa[u] < k && cbase + e_cc[u] < K;
            pre[u] = ok ? (double)raw[u] : 0.0;
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int u = 0; u < G3_PER; ++u)
            if (u * 256 + tid < nst) bs[e_cc[u] * G3_LD + e_aa[u]] = pre[u];
    };
    if ((int64_t)blockIdx.x < ntiles) load_tile(blockIdx.x);
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        __syncthreads();
        store_tile();
        __syncthreads();
        if (tile + gridDim.x < ntiles) load_tile(tile + gridDim.x);
        if (pr < npt) {
            for (int c = g; c < G3_NC; c += G) {
                const double* row = bs + c * G3_LD;
                double x[8], y[8];
#pragma unroll
                for (int q = 0; q < 8; q += 2) {
                    const double2 vx = *reinterpret_cast<const double2*>(row + 8 * ti + q);
                    const double2 vy = *reinterpret_cast<const double2*>(row + 8 * tj + q);
                    x[q] = vx.x; x[q + 1] = vx.y; y[q] = vy.x; y[q + 1] = vy.y;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int w = 0; w < 8; ++w) acc[u][w] = fma(x[u], y[w], acc[u][w]);
            }
        }
    }
    __syncthreads();
    double* gp = partial + (int64_t)blockIdx.x * k * k;
#pragma unroll
    for (int round = 0; round < 4; ++round) {
#pragma unroll
        for (int v = 0; v < 16; ++v) bs[tid * 16 + v] = acc[2 * round + v / 8][v % 8];
        __syncthreads();
        for (int t = tid; t < npt * 16; t += 256) {
            const int tile = t / 16, v = t % 16;
            double s0 = 0.0, s1 = 0.0;
            for (int gg = 0; gg < G; gg += 2) {
                s0 += bs[(tile * G + gg) * 16 + v];
                if (gg + 1 < G) s1 += bs[(tile * G + gg + 1) * 16 + v];
            }
            int ti2 = 0, rem = tile;
            while (rem >= nt - ti2) { rem -= nt - ti2; ++ti2; }
            const int tj2 = ti2 + rem;
            const int r = 8 * ti2 + 2 * round + v / 8, c = 8 * tj2 + v % 8;
            if (r < k && c < k) { gp[r * k + c] = s0 + s1; gp[c * k + r] = s0 + s1; }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(256) void gram3_kernel(const T* __restrict__ B, int64_t L, int64_t ldk, int64_t R,
                                                    int k, double* __restrict__ partial) {
    __shared__ __align__(16) double bs[G3_NC * G3_LD];
    if (R >= G3_NC) gram3_body<T, true>(B, L, ldk, R, k, partial, bs);
    else gram3_body<T, false>(B, L, ldk, R, k, partial, bs);
}

// fp64 Gram of the first k <= 64 mode rows of a float (L, ldk, R) tensor with
// R % 4 == 0 on the fp64 matrix cores: W = sum over unfolding columns c of
// b_c b_c^T, b_c = B[l, 0:k, r], c = l R + r.  Rows are taken in blocks of 16;
// v_mfma_f64_16x16x4f64 forms D += A_i A_j^T for every block pair i <= j, lane
// 16 q + s supplying row s of its block at column q of the four (both operands
// have this layout, since the second factor is a transposed row block), and
// lane 16 q + s of the result holding D[4 v + q][s] in component v.  A lane
// loads the four consecutive columns 4 q .. 4 q + 3 of a 16-column chunk as one
// float4 (one l-slab, since R % 4 == 0) and feeds component u to the u-th MFMA
// of the chunk: each MFMA then sums over columns {u, 4 + u, 8 + u, 12 + u},
// the same set for both operands.  Float products are exact in fp64 and the
// sums are fp64.  A wave takes a contiguous run of chunks; the four waves of a
// workgroup add their blocks in a fixed order into partial[wg] (k x k).
typedef double gd4 __attribute__((ext_vector_type(4)));
typedef float gf4 __attribute__((ext_vector_type(4)));

template <int NB>
static __global__ __launch_bounds__(256) void gram_mfma_kernel(const float* __restrict__ B, int64_t L, int64_t ldk,
                                                        int64_t R, int k, int64_t chunks_per_wave,
                                                        double* __restrict__ partial) {
    constexpr int NP = NB * (NB + 1) / 2;
    __shared__ double red[3][NP * 256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4, srow = lane & 15;
    const int64_t K = L * R;
    const int64_t nchunks = (K + 15) / 16;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
    const int64_t c_begin = gw * chunks_per_wave;
    const int64_t c_end = c_begin + chunks_per_wave < nchunks ? c_begin + chunks_per_wave : nchunks;
    gd4 acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = gd4{0.0, 0.0, 0.0, 0.0};
    bool rowok[NB];
    int64_t rowoff[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int a = 16 * b + srow;
        rowok[b] = a < k;
        rowoff[b] = (int64_t)(a < k ? a : 0) * R;
    }
    const int64_t maxoff = L * ldk * R - 4;
    // (l, r) of this lane's first column, advanced by 16 columns per chunk
    int64_t cl = 0, cr = 0;
    if (c_begin < c_end) {
        const int64_t c0 = 16 * c_begin + 4 * q;
        cl = c0 / R;
        cr = c0 - cl * R;
    }
    auto load = [&](int64_t chunk, gf4 (&v)[NB]) {
        const bool colok = 16 * chunk + 4 * q < K;
        const int64_t base = cl * ldk * R + cr;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            int64_t off = base + rowoff[b];
            off = off < maxoff ? off : maxoff;
            const gf4 x = *reinterpret_cast<const gf4*>(B + off);
            v[b] = (rowok[b] && colok) ? x : gf4{0.f, 0.f, 0.f, 0.f};
        }
        cr += 16;
        while (cr >= R) { cr -= R; ++cl; }
    };
    gf4 cur[NB], nxt[NB];
    if (c_begin < c_end) load(c_begin, cur);
    for (int64_t ch = c_begin; ch < c_end; ++ch) {
        if (ch + 1 < c_end) load(ch + 1, nxt);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double x[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) x[b] = (double)cur[b][u];
            int p = 0;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int bj = bi; bj < NB; ++bj) {
                    acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[bi], x[bj], acc[p], 0, 0, 0);
                    ++p;
                }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) cur[b] = nxt[b];
    }
    // waves 1..3 hand their blocks to wave 0, which adds them in wave order
    if (wave > 0) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[wave - 1][p * 256 + v * 64 + lane] = acc[p][v];
    }
    __syncthreads();
    if (wave == 0) {
        double* gp = partial + (int64_t)blockIdx.x * k * k;
        int p = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = bi; bj < NB; ++bj) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double sum = ((acc[p][v] + red[0][p * 256 + v * 64 + lane]) + red[1][p * 256 + v * 64 + lane]) +
                                       red[2][p * 256 + v * 64 + lane];
                    const int i = 16 * bi + 4 * v + q, j = 16 * bj + srow;
                    if (i < k && j < k) {
                        gp[i * k + j] = sum;
                        if (bi != bj) gp[j * k + i] = sum;
                    }
                }
                ++p;
            }
    }
}

int plan_gram3(int64_t L, int64_t R) {
    const int64_t nt = (L * R + G3_NC - 1) / G3_NC;
    return (int)(nt < 512 ? (nt < 1 ? 1 : nt) : 512);
}

hipError_t launch_gram3(const void* B, Dt dt, int64_t L, int64_t ldk, int64_t R, int k, double* partial, int nwg,
                        hipStream_t stream) {
    if (dt == Dt::F32 && R % 4 == 0 && k <= 64 && ((uintptr_t)B & 15) == 0) {
        const int64_t nchunks = (L * R + 15) / 16;
        const int64_t waves = 4 * (int64_t)nwg;
        const int64_t cpw = (nchunks + waves - 1) / waves;
#define RT_GM(NBV)                                                                                                \
    hipLaunchKernelGGL(gram_mfma_kernel<NBV>, dim3(nwg), dim3(256), 0, stream, (const float*)B, L, ldk, R, k, cpw, \
                       partial)
        if (k <= 16) RT_GM(1);
        else if (k <= 32) RT_GM(2);
        else if (k <= 48) RT_GM(3);
        else RT_GM(4);
#undef RT_GM
        return hipGetLastError();
    }
    if (dt == Dt::F64)
        hipLaunchKernelGGL(gram3_kernel<double>, dim3(nwg), dim3(256), 0, stream, (const double*)B, L, ldk, R, k,
                           partial);
    else
        hipLaunchKernelGGL(gram3_kernel<float>, dim3(nwg), dim3(256), 0, stream, (const float*)B, L, ldk, R, k,
                           partial);
    return hipGetLastError();
}

int plan_norm(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return (int)g;
}

template <typename T>
__global__ __launch_bounds__(256) void finish_kernel(const T* __restrict__ core, T* __restrict__ out, int64_t n,
                                                     int copy, const double* __restrict__ partial, int npart,
                                                     const double* __restrict__ nx2,
                                                     const uint32_t* __restrict__ status, FinishScalars* hs) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    if (partial) {
        for (int e = tid; e < npart; e += 256) s += partial[e];
    } else {
        for (int64_t e = tid; e < n; e += 256) {
            const T v = core[e];
            if (copy) out[e] = v;
            s = fma((double)v, (double)v, s);
        }
    }
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid < RT_MAXD) hs->status[tid] = status[tid];
    if (tid == 0) {
        hs->nx2 = nx2[0];
        hs->ng2 = red[0];
    }
    __threadfence_system();
}

hipError_t launch_finish(const void* core, void* out, Dt dt, int64_t n, bool copy, const double* partial, int npart,
                         const double* nx2, const uint32_t* status, FinishScalars* hs, hipStream_t stream) {
    if (!partial && n > FINISH_DIRECT_MAX) return hipErrorInvalidValue;
    if (dt == Dt::F64)
        hipLaunchKernelGGL(finish_kernel<double>, dim3(1), dim3(256), 0, stream, (const double*)core, (double*)out, n,
                           copy ? 1 : 0, partial, npart, nx2, status, hs);
    else
        hipLaunchKernelGGL(finish_kernel<float>, dim3(1), dim3(256), 0, stream, (const float*)core, (float*)out, n,
                           copy ? 1 : 0, partial, npart, nx2, status, hs);
    return hipGetLastError();
}

hipError_t launch_norm2(const void* X, Dt dt, int64_t n, double* partial, int nwg, hipStream_t stream) {
    if (dt == Dt::F64)
        hipLaunchKernelGGL(norm2_kernel<double>, dim3(nwg), dim3(256), 0, stream, (const double*)X, n, partial);
    else
        hipLaunchKernelGGL(norm2_kernel<float>, dim3(nwg), dim3(256), 0, stream, (const float*)X, n, partial);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ A, int64_t rows, int64_t cols,
                                                        T* __restrict__ AT) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows * cols; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / cols, k = e - (e / cols) * cols;
        AT[k * rows + i] = A[e];
    }
}

hipError_t launch_transpose(const void* A, int64_t rows, int64_t cols, void* AT, Dt dt, hipStream_t stream) {
    const int64_t n = rows * cols;
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (dt == Dt::F64)
        hipLaunchKernelGGL(transpose_kernel<double>, dim3((unsigned)g), dim3(256), 0, stream, (const double*)A, rows,
                           cols, (double*)AT);
    else
        hipLaunchKernelGGL(transpose_kernel<float>, dim3((unsigned)g), dim3(256), 0, stream, (const float*)A, rows,
                           cols, (float*)AT);
    return hipGetLastError();
}

// out[(l ell + k) R + r] = G[(l J + sel[k]) R + r]: one output row of R elements per
// (l, k), rows strided over the grid
template <typename T>
__global__ __launch_bounds__(256) void gather_mode_kernel(const T* __restrict__ G, int64_t L, int64_t J, int64_t R,
                                                          const int* __restrict__ sel, int ell, T* __restrict__ out) {
    const int64_t rows = L * ell;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int64_t l = row / ell;
        const int k = (int)(row - l * ell);
        const T* src = G + (l * J + sel[k]) * R;
        T* dst = out + row * R;
        for (int64_t r = threadIdx.x; r < R; r += 256) dst[r] = src[r];
    }
}

hipError_t launch_gather_mode(const void* G, Dt dt, Shape3 s, const int* sel, int ell, void* out,
                              hipStream_t stream) {
    const int64_t rows = s.L * ell;
    if (rows <= 0 || s.R <= 0) return hipSuccess;
    const unsigned g = (unsigned)(rows < 8192 ? rows : 8192);
    if (dt == Dt::F64)
        hipLaunchKernelGGL(gather_mode_kernel<double>, dim3(g), dim3(256), 0, stream, (const double*)G, s.L, s.J,
                           s.R, sel, ell, (double*)out);
    else
        hipLaunchKernelGGL(gather_mode_kernel<float>, dim3(g), dim3(256), 0, stream, (const float*)G, s.L, s.J, s.R,
                           sel, ell, (float*)out);
    return hipGetLastError();
}

hipError_t launch_cast_from_f64(const double* src, void* dst, Dt dt, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (dt == Dt::F64)
        hipLaunchKernelGGL(cast_kernel<double>, dim3((unsigned)g), dim3(256), 0, stream, src, (double*)dst, n);
    else
        hipLaunchKernelGGL(cast_kernel<float>, dim3((unsigned)g), dim3(256), 0, stream, src, (float*)dst, n);
    return hipGetLastError();
}

hipError_t launch_omega(uint64_t seed, uint32_t mode, int64_t c0, int64_t nrows, int64_t col0, int ncols, void* out,
                        Dt dt, hipStream_t stream) {
    const int64_t n = nrows * ncols;
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256));
    if (dt == Dt::F64)
        hipLaunchKernelGGL(omega_kernel<double>, grid, dim3(256), 0, stream, seed, mode, c0, nrows, col0, ncols,
                           (double*)out);
    else
        hipLaunchKernelGGL(omega_kernel<float>, grid, dim3(256), 0, stream, seed, mode, c0, nrows, col0, ncols,
                           (float*)out);
    return hipGetLastError();
}

hipError_t launch_philox_words(uint64_t seed, uint32_t mode, int64_t c0, int64_t n, uint32_t q, uint32_t* out,
                               hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_words_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, seed, mode, c0,
                       n, q, out);
    return hipGetLastError();
}

}  // namespace rt
