// Mode-n sketch Y = X_(n) Omega (§2.4 Alg. 1 step 1; Alg. 2 and Alg. 3 RandSVD
// call), formed on the strided (L, J, R) view of a row-major tensor, so no
// unfolding is ever materialised, with Omega generated on the fly.
//
// Generic LDS-staged kernel (any dtype, any stride class): a workgroup owns a
// tile of 64 rows of Y and a contiguous run of 64-column tiles of the
// unfolding.  Per tile it stages X[rows, cols] through LDS with loads that are
// contiguous in memory for the tensor's stride class (along c when R > 1, along
// the rows when R == 1) and generates the 64 x ell slab of Omega once into LDS;
// each wave then accumulates every fourth group of four adjacent columns for all
// 64 rows.  The next tile's loads are issued before the current one is consumed.
#include <mutex>
#include <vector>

#include "rt_kernels.hpp"
#include "rt_philox.hpp"

namespace rt {

namespace {

constexpr int SK_MT = 64;     // rows per tile
constexpr int SK_KC = 64;     // unfolding columns per tile
constexpr int SK_NACC = LMAX / 4;

// EXPL: Omega is not generated but read from Om, an (L, ell, R) row-major tensor
// with Omega[l R + r][k] = Om[(l ell + k) R + r] (the subspace-iteration product
// Y = X_(n) Z with Z = Om_(n)^T); seed, mode and col0 are unused.
// The work of one workgroup (split `split`, row tile `rowtile` of nsplit
// splits), shared by the per-request kernel below and the grouped one.
template <typename TX, typename TA, bool EXPL, int NACC = SK_NACC>
__device__ __forceinline__ void sketch_generic_tile(
    const TX* __restrict__ X, int64_t L, int64_t J, int64_t R, int ell, int64_t col0,
    uint64_t seed, uint32_t mode, int64_t tiles_per_split, TA* __restrict__ partial,
    double* __restrict__ nrm2_partial, const TX* __restrict__ Om, int64_t split, int64_t rowtile, int64_t nsplit) {
    __shared__ TA xs[SK_KC][SK_MT + 1];
    __shared__ TA om[SK_KC][LMAX + 4];
    __shared__ double red[256];

    const int tid = threadIdx.x;
    const int row = tid % SK_MT;
    const int kg = tid / SK_MT;            // wave index: column groups kg, kg + 4, ...
    const int64_t K = L * R;
    const int64_t ntiles = (K + SK_KC - 1) / SK_KC;
    const int64_t row0 = rowtile * SK_MT;
    const int64_t t_begin = split * tiles_per_split;
    const int64_t t_end = t_begin + tiles_per_split < ntiles ? t_begin + tiles_per_split : ntiles;
    const int64_t q_first = col0 / 4;
    const int64_t q_last = (col0 + ell - 1) / 4;
    const int nq = (int)(q_last - q_first + 1);
    static_assert(NACC % 4 == 0, "accumulators come in groups of four columns");
    constexpr int NG = NACC / 4;           // groups of four adjacent columns per thread
    constexpr int NLD = SK_MT * SK_KC / 256;

    // Staging map: element m of this thread is X tile entry (rl, cl) with
    // cl = tid % 64, rl = tid / 64 + 4 m (R > 1: runs along c are contiguous)
    // or rl = tid % 64, cl = tid / 64 + 4 m (R == 1: runs along the rows are).
    // Its address is base + m * step, so a tile costs one division per thread.
    TX xr[NLD];
    auto load_tile = [&](int64_t t) {
        const int64_t cbase = t * SK_KC;
        int64_t base, step, c0;
        int64_t i0;
        if (R == 1) {
            c0 = cbase + kg;
            i0 = row0 + row;
            base = c0 * J + i0;
            step = 4 * J;
        } else {
            c0 = cbase + row;
            i0 = row0 + kg;
            const int64_t l = c0 / R;
            base = (l * J + i0) * R + (c0 - l * R);
            step = 4 * R;
        }
#pragma unroll
        for (int m = 0; m < NLD; ++m) {
            const int64_t c = R == 1 ? c0 + 4 * m : c0;
            const int64_t i = R == 1 ? i0 : i0 + 4 * m;
            xr[m] = (c < K && i < J) ? X[base + m * step] : TX(0);
        }
    };

    TA acc[NACC];
#pragma unroll
    for (int j = 0; j < NACC; ++j) acc[j] = TA(0);
    double nrm = 0.0;

    if (t_begin < t_end) load_tile(t_begin);
    for (int64_t t = t_begin; t < t_end; ++t) {
        const int64_t cbase = t * SK_KC;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < NLD; ++m) {
            const TA v = (TA)xr[m];
            if (nrm2_partial) nrm += (double)v * (double)v;
            if (R == 1) xs[kg + 4 * m][row] = v;
            else        xs[row][kg + 4 * m] = v;
        }
        // generate (or, EXPL, load) the Omega slab for these 64 unfolding columns
        if (EXPL) {
            for (int e = tid; e < SK_KC * ell; e += 256) {
                const int cl = e % SK_KC, k = e / SK_KC;
                const int64_t c = cbase + cl;
                TA v = TA(0);
                if (c < K) {
                    const int64_t l = c / R;
                    v = (TA)Om[(l * ell + k) * R + (c - l * R)];
                }
                om[cl][k] = v;
            }
        }
        for (int e = tid; !EXPL && e < SK_KC * nq; e += 256) {
            const int cl = e % SK_KC;
            const int qi = e / SK_KC;
            const int64_t q = q_first + qi;
            TA z[4];
            OmegaGen<TA>::gen4(seed, mode, (uint64_t)(cbase + cl), (uint32_t)q, z);
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                const int64_t k = 4 * q + tt - col0;
                if (k >= 0 && k < ell) om[cl][k] = z[tt];
            }
        }
        // the next tile's loads are in flight while this one is consumed
        if (t + 1 < t_end) load_tile(t + 1);
        __syncthreads();
        const int cmax = (int)((K - cbase) < SK_KC ? (K - cbase) : SK_KC);
        for (int cl = 0; cl < cmax; ++cl) {
            const TA x = xs[cl][row];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int k0 = 4 * (kg + 4 * g);
                if (k0 < ell) {
                    const TA* o = &om[cl][k0];
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[4 * g + u] += x * o[u];
                }
            }
        }
    }
    const int64_t i = row0 + row;
    if (i < J) {
        TA* dst = partial + (split * J + i) * ell;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 4 * (kg + 4 * g) + u;
                if (k < ell) dst[k] = acc[4 * g + u];
            }
        }
    }
    if (nrm2_partial) {
        red[tid] = nrm;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        if (tid == 0) nrm2_partial[rowtile * nsplit + split] = red[0];
    }
}

template <typename TX, typename TA, bool EXPL = false>
__global__ __launch_bounds__(256) void sketch_generic_kernel(
    const TX* __restrict__ X, int64_t L, int64_t J, int64_t R, int ell, int64_t col0,
    uint64_t seed, uint32_t mode, int64_t tiles_per_split, TA* __restrict__ partial,
    double* __restrict__ nrm2_partial, const TX* __restrict__ Om = nullptr) {
    sketch_generic_tile<TX, TA, EXPL>(X, L, J, R, ell, col0, seed, mode, tiles_per_split, partial, nrm2_partial, Om,
                                      blockIdx.x, blockIdx.y, gridDim.x);
}

// Grouped block sketches: work item w of the group belongs to the request whose
// [wi0, wi0 + nsplit nrowtile) holds it (wi0 ascending); the workgroups of the
// fixed grid take items w = blockIdx.x, blockIdx.x + gridDim.x, ...  NACC
// accumulators per thread cover blocks of up to 4 NACC columns (the same sums,
// in the same order, as the per-request kernel).
template <int NACC>
__global__ __launch_bounds__(256) void sketch_group_kernel(const GHeader* __restrict__ hdr,
                                                           const GBlock* __restrict__ d) {
    const int n = hdr->nblock;
    const int64_t total = hdr->sketch_items;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {                      // last request with wi0 <= w
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].wi0 <= w) lo = mid;
            else hi = mid - 1;
        }
        const GBlock& q = d[lo];
        const int64_t local = w - q.wi0;
        sketch_generic_tile<float, float, false, NACC>(q.G, q.L, q.J, q.R, q.b, q.col0, q.seed, q.mode, q.tiles_per_split,
                                                 q.partial, q.nrm_partial, nullptr, local % q.nsplit,
                                                 local / q.nsplit, q.nsplit);
        __syncthreads();
    }
}

// out[chunk][e] = sum of in[p][e] over p in [chunk * pc, min(nparts, (chunk+1) * pc)),
// summed in fp64 in a fixed order (eight independent running sums combined
// pairwise), so the result does not depend on the launch shape.
constexpr int RP_PC = 32;

template <typename T>
__global__ __launch_bounds__(256) void reduce_partials_kernel(const T* __restrict__ in, int64_t nparts, int64_t pc,
                                                              int64_t n, int64_t cols, int64_t ldin,
                                                              double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.y * pc;
    const int64_t p1 = p0 + pc < nparts ? p0 + pc : nparts;
    if (e >= n) return;
    const int64_t src = ldin == cols ? e : (e / cols) * ldin + e % cols;
    const int64_t ps = ldin == cols ? n : n / cols * ldin;   // elements per part
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.0;
    int64_t p = p0;
    for (; p + 8 <= p1; p += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = in[(p + u) * ps + src];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += (double)v[u];
    }
    for (; p < p1; ++p) a[0] += (double)in[p * ps + src];
    out[(int64_t)blockIdx.y * n + e] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

__global__ __launch_bounds__(256) void sum_scalar_kernel(const double* __restrict__ in, int64_t n,
                                                         double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += in[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

bool sketch_mfma_ok(Shape3 s, int ell, int64_t col0, const void* X) {
    if (ell > 64) return false;
    if (((uintptr_t)X & 15) != 0) return false;
    if ((col0 + ell - 1) / 4 - col0 / 4 + 1 > 16) return false;   // Omega blocks per tile row: 2 per thread
    if (s.R % 4 == 0) return true;
    if (s.R == 1 && s.J % 4 == 0) return true;
    return false;
}

namespace {
// Row configuration (RB row blocks of 64 per wave, RW row blocks per
// workgroup) for a mode of length J, and the compiled column quads for ell.
// (Measured on 512 x 262144 float32 unfoldings: two 128-row waves per
// 256-row block with four resident workgroups per CU beat one 256-row wave
// per block, whose accumulators leave room for one wave per SIMD only.)
void sketch_rows_config(int64_t J, int& rb, int& rw) {
    if (J <= 64) { rb = 1; rw = 1; }
    else if (J <= 128) { rb = 2; rw = 1; }
    else { rb = 2; rw = 2; }
}
int sketch_nq_bucket(int nq) {
    if (nq <= 10) return nq;
    if (nq <= 12) return 12;
    if (nq <= 14) return 14;
    return 16;
}
// workgroups to aim for: enough to fill every CU with a few resident groups
int64_t sketch_target_wg(const SketchPlan&) { return 1024; }
}  // namespace

namespace {

// The split of the unfolding's columns: `target` workgroups over nrowtile row tiles.
void split_columns(SketchPlan& p, int64_t ntl, int64_t target) {
    int64_t want = target / p.nrowtile;
    if (want < 1) want = 1;
    if (want > ntl) want = ntl;
    p.tiles_per_split = (ntl + want - 1) / want;
    p.nsplit = (int)((ntl + p.tiles_per_split - 1) / p.tiles_per_split);
    if (p.nsplit < 1) p.nsplit = 1;
    p.nwg = p.nsplit * p.nrowtile;
}

void plan_mfma(SketchPlan& p, Shape3 s, int ell, int rb, int rw, int wgs) {
    p.kind = 1;
    if ((rb == 1 && rw == 1) || (rb == 2 && rw == 1) || (rb == 2 && rw == 2)) { p.rb = rb; p.rw = rw; }
    else sketch_rows_config(s.J, p.rb, p.rw);
    p.nq = sketch_nq_bucket((ell + 3) / 4);
    p.ldp = 4 * p.nq;
    const int64_t mt = 64 * p.rb * p.rw;
    p.nrowtile = (int)((s.J + mt - 1) / mt);
    split_columns(p, (s.L * s.R + 31) / 32, wgs > 0 ? wgs : sketch_target_wg(p));
    p.partial_elems = (size_t)p.nsplit * (size_t)s.J * (size_t)p.ldp;
}

void plan_generic(SketchPlan& p, Shape3 s, int ell, int wgs) {
    p.kind = 0;
    p.rb = p.rw = p.nq = 0;
    p.ldp = ell;
    p.nrowtile = (int)((s.J + SK_MT - 1) / SK_MT);
    split_columns(p, (s.L * s.R + SK_KC - 1) / SK_KC, wgs > 0 ? wgs : 2048);
    p.partial_elems = (size_t)p.nsplit * (size_t)s.J * (size_t)ell;
}

std::mutex g_tune_mu;
std::vector<rt_tune_entry> g_tune;

bool find_entry(Dt dt, int prec, Shape3 s, int ell, rt_tune_entry& out) {
    const int64_t K = s.L * s.R;
    const int sc = stride_class(s);
    const rt_dtype dtype = dt == Dt::F64 ? RT_F64 : RT_F32;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const rt_tune_entry& e : g_tune)
        if (e.op == RT_TUNE_SKETCH && e.dtype == dtype && (int)e.prec == prec && e.stride == sc && s.J >= e.j_lo &&
            s.J <= e.j_hi && K >= e.k_lo && K <= e.k_hi && ell >= e.ell_lo && ell <= e.ell_hi) {
            out = e;
            return true;
        }
    return false;
}

// The plan of a table entry, when its variant serves the shape at (at least) the
// requested precision.
bool plan_from_entry(const rt_tune_entry& e, Dt dt, int prec, Shape3 s, int ell, int64_t col0, const void* X,
                     SketchPlan& p) {
    const bool f32 = dt == Dt::F32;
    switch (e.kind) {
        case 3:   // float32-accurate sketch from bfloat16 pieces
            if (!(f32 && prec == 1 && sketch_x6_ok(s, ell, col0, X))) return false;
            plan_sketch_x6(p, s, ell, false, e.rb, e.wgs);
            return true;
        case 4:   // the bfloat16 sketch
            if (!(f32 && prec == 2 && sketch_x6_ok(s, ell, col0, X))) return false;
            plan_sketch_x6(p, s, ell, true, e.rb, e.wgs);
            return true;
        case 1:
            if (!(f32 && prec != 0 && sketch_mfma_ok(s, ell, col0, X))) return false;
            plan_mfma(p, s, ell, e.rb, e.rw, e.wgs);
            return true;
        case 0:
            plan_generic(p, s, ell, e.wgs);
            return true;
        default:
            return false;
    }
}

}  // namespace

int stride_class(Shape3 s) { return s.L == 1 ? RT_STRIDE_FIRST : (s.R == 1 ? RT_STRIDE_LAST : RT_STRIDE_INNER); }

rt_status tuning_set(const rt_tune_entry* entries, int32_t n) {
    std::vector<rt_tune_entry> t;
    if (n > 0) t.assign(entries, entries + n);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.swap(t);
    return RT_OK;
}

SketchPlan plan_sketch_info(Dt dt, int prec, Shape3 s, int ell, int64_t col0, const void* X, bool split3,
                            bool* from_table) {
    SketchPlan p{};
    if (from_table) *from_table = false;
    // a table entry (for the ordinary sketch with generated Omega)
    rt_tune_entry e;
    if (split3 && find_entry(dt, prec, s, ell, e) && plan_from_entry(e, dt, prec, s, ell, col0, X, p)) {
        if (from_table) *from_table = true;
        return p;
    }
    // built-in rules
    if (dt == Dt::F32 && (prec == 1 || prec == 2) && split3 && sketch_x6_ok(s, ell, col0, X)) {
        plan_sketch_x6(p, s, ell, prec == 2);
        return p;
    }
    // the bfloat16 sketch exists on the 16x16x32 kernel only; other modes take
    // the float32 sketch (at least as accurate)
    if (dt == Dt::F32 && prec != 0 && sketch_mfma_ok(s, ell, col0, X)) {
        plan_mfma(p, s, ell, 0, 0, 0);
        return p;
    }
    plan_generic(p, s, ell, 0);
    return p;
}

SketchPlan plan_sketch(Dt dt, int prec, Shape3 s, int ell, int64_t col0, const void* X, bool split3) {
    return plan_sketch_info(dt, prec, s, ell, col0, X, split3, nullptr);
}

hipError_t launch_sketch(const SketchPlan& p, Dt dt, int prec, const void* X, Shape3 s, int ell,
                         int64_t col0, uint64_t seed, uint32_t mode, void* partial,
                         double* nrm2_partial, hipStream_t stream) {
    if (p.kind == 3 || p.kind == 4)
        return launch_sketch_f32_x6(p, (const float*)X, s, ell, col0, seed, mode, (float*)partial, nrm2_partial,
                                    stream);
    (void)prec;
    if (p.kind == 1) {
        if (s.R % 4 == 0)
            return launch_sketch_f32_rows(p, (const float*)X, s, ell, col0, seed, mode, (float*)partial, nrm2_partial,
                                          stream);
        return launch_sketch_f32_cols(p, (const float*)X, s, ell, col0, seed, mode, (float*)partial, nrm2_partial,
                                      stream);
    }
    dim3 grid(p.nsplit, p.nrowtile);
    if (dt == Dt::F64)
        hipLaunchKernelGGL((sketch_generic_kernel<double, double>), grid, dim3(256), 0, stream, (const double*)X, s.L,
                           s.J, s.R, ell, col0, seed, mode, p.tiles_per_split, (double*)partial, nrm2_partial);
    else
        hipLaunchKernelGGL((sketch_generic_kernel<float, float>), grid, dim3(256), 0, stream, (const float*)X, s.L,
                           s.J, s.R, ell, col0, seed, mode, p.tiles_per_split, (float*)partial, nrm2_partial);
    return hipGetLastError();
}

hipError_t launch_sketch_explicit(const SketchPlan& p, Dt dt, const void* X, Shape3 s, int ell, const void* Om,
                                  void* partial, hipStream_t stream) {
    if (p.kind == 1) {
        if (s.R % 4 != 0 || ((uintptr_t)Om & 15) != 0) return hipErrorInvalidValue;
        return launch_sketch_f32_rows_explicit(p, (const float*)X, s, ell, (const float*)Om, (float*)partial, stream);
    }
    if (p.kind != 0) return hipErrorInvalidValue;
    dim3 grid(p.nsplit, p.nrowtile);
    if (dt == Dt::F64)
        hipLaunchKernelGGL((sketch_generic_kernel<double, double, true>), grid, dim3(256), 0, stream,
                           (const double*)X, s.L, s.J, s.R, ell, (int64_t)0, (uint64_t)0, 0u, p.tiles_per_split,
                           (double*)partial, (double*)nullptr, (const double*)Om);
    else
        hipLaunchKernelGGL((sketch_generic_kernel<float, float, true>), grid, dim3(256), 0, stream,
                           (const float*)X, s.L, s.J, s.R, ell, (int64_t)0, (uint64_t)0, 0u, p.tiles_per_split,
                           (float*)partial, (double*)nullptr, (const float*)Om);
    return hipGetLastError();
}

hipError_t launch_reduce_rows(const void* in, bool in_is_f64, int64_t nparts, int64_t rows, int64_t cols,
                              int64_t ldin, double* out, hipStream_t stream, double* tmp) {
    const int64_t n = rows * cols;
    if (n <= 0) return hipSuccess;
    const unsigned ex = (unsigned)((n + 255) / 256);
    const int64_t nchunk = (nparts + RP_PC - 1) / RP_PC;
    if (nchunk <= 1) {
        // one pass over all parts (fixed order)
        if (in_is_f64)
            hipLaunchKernelGGL(reduce_partials_kernel<double>, dim3(ex, 1), dim3(256), 0, stream, (const double*)in,
                               nparts, nparts, n, cols, ldin, out);
        else
            hipLaunchKernelGGL(reduce_partials_kernel<float>, dim3(ex, 1), dim3(256), 0, stream, (const float*)in,
                               nparts, nparts, n, cols, ldin, out);
        return hipGetLastError();
    }
    if (tmp == nullptr) return hipErrorInvalidValue;
    // two passes: chunks of RP_PC parts, then all nchunk chunk sums in one run
    if (in_is_f64)
        hipLaunchKernelGGL(reduce_partials_kernel<double>, dim3(ex, (unsigned)nchunk), dim3(256), 0, stream,
                           (const double*)in, nparts, (int64_t)RP_PC, n, cols, ldin, tmp);
    else
        hipLaunchKernelGGL(reduce_partials_kernel<float>, dim3(ex, (unsigned)nchunk), dim3(256), 0, stream,
                           (const float*)in, nparts, (int64_t)RP_PC, n, cols, ldin, tmp);
    hipLaunchKernelGGL(reduce_partials_kernel<double>, dim3(ex, 1), dim3(256), 0, stream, (const double*)tmp, nchunk,
                       nchunk, n, n, n, out);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const void* in, bool in_is_f64, int64_t nparts, int64_t n,
                                  double* out, hipStream_t stream, double* tmp) {
    return launch_reduce_rows(in, in_is_f64, nparts, 1, n, n, out, stream, tmp);
}

void group_sketch_plan(int64_t L, int64_t J, int64_t R, int b, int& nsplit, int& nrowtile, int64_t& tps) {
    // the generic kernel's plan for a request of its own (depends on the shape only)
    const int64_t K = L * R;
    const int64_t ntiles = (K + SK_KC - 1) / SK_KC;
    nrowtile = (int)((J + SK_MT - 1) / SK_MT);
    int64_t want = 128 / nrowtile;
    if (want < 1) want = 1;
    if (want > ntiles) want = ntiles;
    tps = (ntiles + want - 1) / want;
    nsplit = (int)((ntiles + tps - 1) / tps);
    if (nsplit < 1) nsplit = 1;
    (void)b;
}

hipError_t launch_group_sketch(const GHeader* hdr, const GBlock* d, int block, hipStream_t stream) {
    (void)block;   // blocks of at most 16 columns: one group of four columns per wave
    hipLaunchKernelGGL(sketch_group_kernel<4>, dim3(1024), dim3(256), 0, stream, hdr, d);
    return hipGetLastError();
}

hipError_t launch_sum_scalar(const double* in, int64_t n, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(sum_scalar_kernel, dim3(1), dim3(256), 0, stream, in, n, out);
    return hipGetLastError();
}

}  // namespace rt
