// C ABI of librtucker.so (include/rtucker.h): argument validation, the
// per-context workspace, and the host drivers that sequence the device kernels
// of R-HOSVD (Alg. 2), R-STHOSVD (Alg. 3) and adaptive R-STHOSVD (Alg. 5).
#include "rtucker.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rt_kernels.hpp"

using rt::Dt;
using rt::Shape3;

namespace {

thread_local std::string g_err;

rt_status fail(rt_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define RT_HIP(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(RT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
    } while (0)

#define RT_TRY(expr)                    \
    do {                                \
        rt_status s_ = (expr);          \
        if (s_ != RT_OK) return s_;     \
    } while (0)

size_t dsize(rt_dtype t) { return t == RT_F64 ? 8 : 4; }
Dt dt_of(rt_dtype t) { return t == RT_F64 ? Dt::F64 : Dt::F32; }

}  // namespace

namespace rt {
// error message of the calling thread, for the other translation units of the library
rt_status set_error(rt_status s, const char* msg) { return fail(s, msg); }
}  // namespace rt

struct rt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    rt_alloc_fn alloc = nullptr;
    rt_free_fn free_fn = nullptr;
    void* user = nullptr;
    // workspace: chunks kept across calls, bump-allocated within a call
    struct Chunk { char* p; size_t size; size_t used; };
    std::vector<Chunk> chunks;
    double* host = nullptr;       // pinned scratch for small read-backs
    double* host_dev = nullptr;   // the same block as the device addresses it
    // Results of asynchronous calls: each takes a slot of scalars in the pinned
    // block (after the first 4 KiB of read-back scratch), written by the call's
    // last kernel and copied into the caller's rt_tucker by rt_sync.
    static constexpr int NSLOT = 255;
    static constexpr size_t SLOT_OFFSET = 4096;
    static constexpr size_t SLOT_BYTES = 64;
    struct Pending { rt_tucker* out; bool oblique; };
    std::vector<Pending> pending;
    rt_tucker discard{};          // stands in for a pending result released before rt_sync
    rt::FinishScalars* slot_host(size_t i) const {
        return (rt::FinishScalars*)((char*)host + SLOT_OFFSET + i * SLOT_BYTES);
    }
    rt::FinishScalars* slot_dev(size_t i) const {
        return (rt::FinishScalars*)((char*)host_dev + SLOT_OFFSET + i * SLOT_BYTES);
    }
    std::vector<void*> outputs;   // outputs handed to the caller (for release)
    // optional per-launch timing log (HIP events on the context's stream)
    struct Timed { int kind; hipEvent_t a, b; double bytes, flops; int64_t rows, cols; int ell; int variant; };
    uint32_t timing = 0;          // bit k: record launches of kind k
    std::vector<Timed> tlog;
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    hipEvent_t next_event() {
        if (evused < evpool.size()) return evpool[evused++];
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        evpool.push_back(e);
        ++evused;
        return e;
    }
    // streams (default priority) and events for work forked off `stream` and
    // joined back into it within one call
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> sync_ev;
    hipStream_t side_stream(size_t i) {
        while (side.size() <= i) {
            hipStream_t s = nullptr;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
            side.push_back(s);
        }
        return side[i];
    }
    hipEvent_t sync_event(size_t i) {
        while (sync_ev.size() <= i) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
            sync_ev.push_back(e);
        }
        return sync_ev[i];
    }
    int64_t cur_J = 0;            // rows of the basis Q of the mode being truncated
    double* last_nrm2 = nullptr;  // optional: receives ||core||^2 of the truncation's core update

    void* raw_alloc(size_t bytes) {
        if (bytes == 0) bytes = 256;
        if (alloc) return alloc(bytes, user);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        return p;
    }
    void raw_free(void* p) {
        if (!p) return;
        if (free_fn) free_fn(p, user);
        else (void)hipFree(p);
    }
    void reset_ws() { for (auto& c : chunks) c.used = 0; }
    void* ws(size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto& c : chunks) {
            if (c.size - c.used >= bytes) {
                void* p = c.p + c.used;
                c.used += bytes;
                return p;
            }
        }
        size_t sz = std::max(bytes, size_t(64) << 20);
        char* p = (char*)raw_alloc(sz);
        if (!p) return nullptr;
        chunks.push_back({p, sz, bytes});
        return p;
    }
};

namespace rt {
hipStream_t ctx_stream(const rt_ctx* c) { return c->stream; }
int ctx_device(const rt_ctx* c) { return c->device; }
}  // namespace rt

namespace {

// Records HIP events around one kernel launch when the context's timing log is on.
struct TimeScope {
    rt_ctx* c;
    rt_ctx::Timed t{};
    bool on;
    TimeScope(rt_ctx* ctx, int kind, double bytes, double flops, int64_t rows, int64_t cols, int ell)
        : c(ctx), on(((ctx->timing >> kind) & 1u) != 0) {
        if (!on) return;
        t = rt_ctx::Timed{kind, c->next_event(), c->next_event(), bytes, flops, rows, cols, ell, 0};
        if (!t.a || !t.b) { on = false; return; }
        (void)hipEventRecord(t.a, c->stream);
    }
    ~TimeScope() {
        if (!on) return;
        (void)hipEventRecord(t.b, c->stream);
        c->tlog.push_back(t);
    }
};

struct Call {
    rt_ctx* c;
    explicit Call(rt_ctx* ctx) : c(ctx) { c->reset_ws(); }
    template <typename T> T* ws(size_t n) { return (T*)c->ws(n * sizeof(T)); }
};

Shape3 shape3(const std::vector<int64_t>& dims, int n) {
    Shape3 s{1, dims[n], 1};
    for (int i = 0; i < n; ++i) s.L *= dims[i];
    for (int i = n + 1; i < (int)dims.size(); ++i) s.R *= dims[i];
    return s;
}

rt_status check_tensor(const rt_tensor* X) {
    if (!X) return fail(RT_EINVAL, "X is NULL");
    if (X->ndim < 2 || X->ndim > RT_MAXD) return fail(RT_EINVAL, "ndim must be in [2, RT_MAXD]");
    if (X->dtype != RT_F32 && X->dtype != RT_F64) return fail(RT_EINVAL, "dtype must be RT_F32 or RT_F64");
    if (!X->data) return fail(RT_EINVAL, "X->data is NULL");
    for (int i = 0; i < X->ndim; ++i)
        if (X->dims[i] < 1) return fail(RT_EINVAL, "every dim must be >= 1");
    return RT_OK;
}

rt_status check_prec(const rt_tensor* X, rt_precision prec) {
    if (prec == RT_PREC_F64 && X->dtype != RT_F64) return fail(RT_EINVAL, "RT_PREC_F64 needs an RT_F64 tensor");
    if (prec != RT_PREC_F64 && X->dtype != RT_F32) return fail(RT_EINVAL, "RT_PREC_F32/BF16 need an RT_F32 tensor");
    if (prec != RT_PREC_F64 && prec != RT_PREC_F32 && prec != RT_PREC_BF16_SKETCH)
        return fail(RT_EINVAL, "unknown precision");
    return RT_OK;
}

rt_status make_order(const rt_tensor* X, const int32_t* order, std::vector<int>& out) {
    const int d = X->ndim;
    out.resize(d);
    if (order) {
        std::vector<int> seen(d, 0);
        for (int i = 0; i < d; ++i) {
            if (order[i] < 0 || order[i] >= d || seen[order[i]]) return fail(RT_EINVAL, "order is not a permutation");
            seen[order[i]] = 1;
            out[i] = order[i];
        }
    } else {
        for (int i = 0; i < d; ++i) out[i] = i;
        std::stable_sort(out.begin(), out.end(), [&](int a, int b) { return X->dims[a] > X->dims[b]; });
    }
    return RT_OK;
}

rt_status check_ranks(const rt_tensor* X, const int32_t* ranks, int p, int cap = RT_LMAX) {
    if (!ranks) return fail(RT_EINVAL, "ranks is NULL");
    if (p < 0) return fail(RT_EINVAL, "oversampling p must be >= 0");
    int64_t total = 1;
    for (int i = 0; i < X->ndim; ++i) total *= X->dims[i];
    for (int j = 0; j < X->ndim; ++j) {
        if (ranks[j] == RT_KEEP) continue;
        if (ranks[j] < 1) return fail(RT_EINVAL, "ranks must be >= 1 or RT_KEEP");
        const int64_t ell = (int64_t)ranks[j] + p;
        if (ell > std::min<int64_t>(X->dims[j], total / X->dims[j]))
            return fail(RT_EINVAL, "r_j + p exceeds min(I_j, prod_{i!=j} I_i) for mode " + std::to_string(j));
        if (ell > cap)
            return fail(RT_EINVAL, std::string("r_j + p exceeds ") + (cap == RT_LMAX ? "RT_LMAX" : "RT_LMAX_FIXED") +
                                       " for mode " + std::to_string(j));
    }
    return RT_OK;
}

// the wide path (r_j + p > RT_LMAX) has no subspace iteration
rt_status check_wide_power(const rt_tensor* X, const int32_t* ranks, const rt_opts* opts) {
    if (opts->power_iters == 0) return RT_OK;
    for (int j = 0; j < X->ndim; ++j)
        if (ranks[j] != RT_KEEP && ranks[j] + opts->oversample > RT_LMAX)
            return fail(RT_EINVAL, "power_iters > 0 needs r_j + p <= RT_LMAX");
    return RT_OK;
}

rt_status check_coo(const rt_coo* X) {
    if (!X) return fail(RT_EINVAL, "X is NULL");
    if (X->ndim < 2 || X->ndim > RT_MAXD) return fail(RT_EINVAL, "ndim must be in [2, RT_MAXD]");
    if (X->dtype != RT_F32 && X->dtype != RT_F64) return fail(RT_EINVAL, "dtype must be RT_F32 or RT_F64");
    if (X->nnz < 0) return fail(RT_EINVAL, "nnz must be >= 0");
    if (X->nnz > 0 && (!X->idx || !X->vals)) return fail(RT_EINVAL, "idx or vals is NULL");
    if (X->nnz > ((int64_t)1 << 40)) return fail(RT_EINVAL, "nnz too large");
    for (int i = 0; i < X->ndim; ++i)
        if (X->dims[i] < 1 || X->dims[i] > INT32_MAX) return fail(RT_EINVAL, "every dim must be in [1, 2^31 - 1]");
    return RT_OK;
}

// The dense header of a COO tensor (dims, dtype) for the shape and rank checks.
rt_tensor coo_header(const rt_coo* X) {
    rt_tensor t{};
    t.ndim = X->ndim;
    for (int i = 0; i < X->ndim; ++i) t.dims[i] = X->dims[i];
    t.dtype = X->dtype;
    t.data = X->vals ? X->vals : (const void*)X;
    return t;
}

// Sketch of a COO core whose entry count the host knows (the input): large
// inputs take the row-binned kernels (LDS accumulation, one add per block row
// into Y), the others the direct scatter.
rt_status coo_sketch_input(Call& k, const int32_t* idx, const void* vals, Dt dt, int64_t nnz,
                           const rt::CooDims& cd, int mode, int ell, int64_t col0, uint64_t seed, double* Y) {
    hipStream_t st = k.c->stream;
    int64_t K = 1;
    for (int m = 0; m < cd.d; ++m)
        if (m != mode) K *= cd.dims[m];
    const rt::BinPlan bp = rt::plan_coo_bins(cd.dims[mode], ell, nnz);
    if (nnz >= (int64_t(1) << 18) && bp.ok && K < (int64_t(1) << (62 - bp.shift))) {
        int32_t* hist = k.ws<int32_t>((size_t)bp.nch * bp.nbk);
        int64_t* off = k.ws<int64_t>((size_t)bp.nch * bp.nbk);
        int64_t* bstart = k.ws<int64_t>((size_t)bp.nbk + 1);
        int64_t* pstart = k.ws<int64_t>((size_t)bp.nbk + 1);
        int64_t* keys = k.ws<int64_t>((size_t)nnz);
        double* rv = k.ws<double>((size_t)nnz);
        if (!hist || !off || !bstart || !pstart || !keys || !rv) return fail(RT_ENOMEM, "workspace allocation failed");
        RT_HIP(rt::launch_coo_sketch_binned(bp, idx, vals, dt, nnz, cd, mode, ell, col0, seed, Y, hist, off, bstart,
                                            pstart, keys, rv, st));
        return RT_OK;
    }
    RT_HIP(rt::launch_coo_sketch(idx, nnz, vals, dt, nullptr, nnz, cd, mode, ell, col0, seed, Y, st));
    return RT_OK;
}

rt::CooDims coo_dims(const std::vector<int64_t>& dims) {
    rt::CooDims cd{};
    cd.d = (int32_t)dims.size();
    for (size_t i = 0; i < dims.size(); ++i) cd.dims[i] = dims[i];
    return cd;
}

}  // namespace

namespace rt {
// Arguments of the sketch entry points (rt_sketch and its allocation-free variant).
rt_status check_sketch_args(const rt_ctx* ctx, const rt_tensor* X, int32_t mode, int32_t ell, int64_t col0,
                            rt_precision prec, const double* Y) {
    if (!ctx || !Y) return fail(RT_EINVAL, "NULL argument");
    RT_TRY(check_tensor(X));
    RT_TRY(check_prec(X, prec));
    if (mode < 0 || mode >= X->ndim) return fail(RT_EINVAL, "mode out of range");
    if (ell < 1 || ell > RT_LMAX) return fail(RT_EINVAL, "ell must be in [1, RT_LMAX]");
    if (col0 < 0) return fail(RT_EINVAL, "col0 must be >= 0");
    return RT_OK;
}
}  // namespace rt

namespace {

// ---- building blocks ----------------------------------------------------------------

// Y (J x ell, fp64) = G_(n) Omega[:, col0 : col0 + ell]; optional ||G||^2 into nrm2 (device).
rt_status do_sketch(Call& k, Dt dt, int prec, const void* G, Shape3 s, int ell, int64_t col0, uint64_t seed,
                    int mode, double* Y, double* nrm2) {
    rt::SketchPlan plan = rt::plan_sketch(dt, prec, s, ell, col0, G);
    const bool f64acc = dt == Dt::F64;
    void* partial = k.c->ws(plan.partial_elems * (f64acc ? 8 : 4));
    double* np = nrm2 ? k.ws<double>(plan.nwg) : nullptr;
    if (!partial || (nrm2 && !np)) return fail(RT_ENOMEM, "workspace allocation failed");
    {
        const double n = (double)s.L * s.J * s.R;
        TimeScope ts(k.c, 0, n * (dt == Dt::F64 ? 8 : 4), 2.0 * ell * n, s.J, s.L * s.R, ell);
        ts.t.variant = plan.kind;
        RT_HIP(rt::launch_sketch(plan, dt, prec, G, s, ell, col0, seed, (uint32_t)mode, partial, np, k.c->stream));
    }
    double* rtmp = k.ws<double>(rt::reduce_partials_tmp(plan.nsplit, s.J * ell) + 1);
    if (!rtmp) return fail(RT_ENOMEM, "workspace allocation failed");
    {
        TimeScope ts(k.c, 5, (double)plan.partial_elems * (f64acc ? 8 : 4), 0.0, s.J, plan.nsplit, ell);
        RT_HIP(rt::launch_reduce_rows(partial, f64acc, plan.nsplit, s.J, ell, plan.ldp, Y, k.c->stream, rtmp));
    }
    if (nrm2) RT_HIP(rt::launch_sum_scalar(np, plan.nwg, nrm2, k.c->stream));
    return RT_OK;
}

// Y = G_(n) Z, Z[l R + r][k] = Om[(l ell + k) R + r] (Om: (L, ell, R) in dtype dt)
rt_status do_sketch_explicit(Call& k, Dt dt, const void* G, Shape3 s, int ell, const void* Om, double* Y) {
    const bool mfma = dt == Dt::F32 && s.R % 4 == 0 && ((uintptr_t)Om & 15) == 0;
    rt::SketchPlan plan = rt::plan_sketch(dt, mfma ? 1 : 0, s, ell, 0, G, false);
    if (plan.kind == 1 && s.R % 4 != 0) plan = rt::plan_sketch(dt, 0, s, ell, 0, G);
    const bool f64acc = dt == Dt::F64;
    void* partial = k.c->ws(plan.partial_elems * (f64acc ? 8 : 4));
    double* rtmp = k.ws<double>(rt::reduce_partials_tmp(plan.nsplit, s.J * ell) + 1);
    if (!partial || !rtmp) return fail(RT_ENOMEM, "workspace allocation failed");
    {
        const double n = (double)s.L * s.J * s.R;
        TimeScope ts(k.c, 0, n * (dt == Dt::F64 ? 8 : 4) * (1.0 + (double)ell / s.J), 2.0 * ell * n, s.J, s.L * s.R,
                     ell);
        ts.t.variant = plan.kind;
        RT_HIP(rt::launch_sketch_explicit(plan, dt, G, s, ell, Om, partial, k.c->stream));
    }
    RT_HIP(rt::launch_reduce_rows(partial, f64acc, plan.nsplit, s.J, ell, plan.ldp, Y, k.c->stream, rtmp));
    return RT_OK;
}

rt_status do_norm2(Call& k, const void* X, Dt dt, int64_t n, double* out) {
    int nwg = rt::plan_norm(n);
    double* part = k.ws<double>(nwg);
    if (!part) return fail(RT_ENOMEM, "workspace allocation failed");
    RT_HIP(rt::launch_norm2(X, dt, n, part, nwg, k.c->stream));
    RT_HIP(rt::launch_sum_scalar(part, nwg, out, k.c->stream));
    return RT_OK;
}

// B = G x_n Q^T with the fp64 Gram of B reduced into W (ell x ell) when W != NULL.
rt_status do_project(Call& k, Dt dx, Dt dq, const void* G, Shape3 s, int64_t ldj, const void* Q, int64_t ldq,
                     int ell, void* B, int64_t ldk, int64_t koff, double* W, double* nrm2) {
    rt::ProjectPlan plan = rt::plan_project(dx, dq, s, ell, G, B, koff);
    const bool fused_gram = W && plan.kind == 0;
    const bool split = plan.nsplit > 1;
    const int nred = split ? rt::plan_project_reduce(s.L * (int64_t)ell * s.R) : 0;
    const int nnrm = split ? nred : plan.nwg;
    double* gp = fused_gram ? k.ws<double>((size_t)plan.nwg * ell * ell) : nullptr;
    double* np = nrm2 ? k.ws<double>(nnrm) : nullptr;
    float* part = split ? k.ws<float>(plan.partial_elems) : nullptr;
    if ((fused_gram && !gp) || (nrm2 && !np) || (split && !part)) return fail(RT_ENOMEM, "workspace allocation failed");
    {
        const double n = (double)s.L * s.J * s.R, es = dx == Dt::F64 ? 8 : 4;
        TimeScope ts(k.c, 1, n * es + (double)s.L * ell * s.R * es, 2.0 * ell * n, s.J, s.L * s.R, ell);
        if (split) {
            // contraction split: float partials, then their fixed-order sum into B
            RT_HIP(rt::launch_project(plan, dx, dq, G, s, ldj, Q, ldq, ell, part, ell, 0, nullptr, nullptr,
                                      k.c->stream));
            RT_HIP(rt::launch_project_reduce(part, plan.nsplit, s, ell, (float*)B, ldk, koff, np, nred, k.c->stream));
        } else {
            RT_HIP(rt::launch_project(plan, dx, dq, G, s, ldj, Q, ldq, ell, B, ldk, koff, gp, np, k.c->stream));
        }
    }
    if (fused_gram) {
        double* rtmp = k.ws<double>(rt::reduce_partials_tmp(plan.nwg, (int64_t)ell * ell) + 1);
        if (!rtmp) return fail(RT_ENOMEM, "workspace allocation failed");
        RT_HIP(rt::launch_reduce_partials(gp, true, plan.nwg, (int64_t)ell * ell, W, k.c->stream, rtmp));
    }
    if (W && !fused_gram) {
        // fp64 Gram of the freshly written B rows koff .. koff + ell
        const int nwg = rt::plan_gram3(s.L, s.R);
        double* g3 = k.ws<double>((size_t)nwg * ell * ell);
        if (!g3) return fail(RT_ENOMEM, "workspace allocation failed");
        const size_t es = dx == Dt::F64 ? 8 : 4;
        const char* Bk = (const char*)B + (size_t)koff * s.R * es;
        {
            TimeScope ts(k.c, 4, (double)s.L * ell * s.R * es, 2.0 * ell * ell * (double)s.L * s.R, ell, s.L * s.R, ell);
            RT_HIP(rt::launch_gram3(Bk, dx, s.L, ldk, s.R, ell, g3, nwg, k.c->stream));
        }
        double* rtmp = k.ws<double>(rt::reduce_partials_tmp(nwg, (int64_t)ell * ell) + 1);
        if (!rtmp) return fail(RT_ENOMEM, "workspace allocation failed");
        RT_HIP(rt::launch_reduce_partials(g3, true, nwg, (int64_t)ell * ell, W, k.c->stream, rtmp));
    }
    if (nrm2) RT_HIP(rt::launch_sum_scalar(np, nnrm, nrm2, k.c->stream));
    return RT_OK;
}

double orth_accept_ratio() { return 1e-15; }

// Truncation of a QB factorisation (Alg. 1 steps 4-6).  B is (L, ldb-strided mode
// of kb rows, R) with its fp64 Gram W; Q (J x kb, fp64, leading dimension ldq).
// Fixed rank: r_fixed >= 0.  Adaptive: r_fixed < 0 and the rank is the smallest
// k with max(E, 0) + tail <= tau2 (E on the device).
// Writes A_out (J x k, dtype dt), the new core (L, k, R) and returns k.
// refine: eigenvectors of a Gram are accurate only to about u ||B||^2 / gap; for the
// fp64 path the basis is refined by rotating B into the first eigenbasis
// (C = U1^T B) and taking the eigenvectors of C C^T, whose entries carry relative
// accuracy, before the final choice.
rt_status do_truncate(Call& k, Dt dt, const void* B, Shape3 sb, int64_t ldb, const double* W, const double* Q,
                      int64_t ldq, int r_fixed, const double* Edev, double tau2, bool refine, void* A_out,
                      void** core_out, int* k_host) {
    hipStream_t st = k.c->stream;
    const int kb = (int)sb.J;
    double* lam = k.ws<double>(kb);
    int* kdev = k.ws<int>(1);
    double* U = k.ws<double>((size_t)kb * kb);
    float* Uf = k.ws<float>((size_t)kb * kb);
    double* tscr = k.ws<double>(rt::truncate_scratch(k.c->cur_J, kb));
    if (!lam || !kdev || !U || !Uf || !tscr) return fail(RT_ENOMEM, "workspace allocation failed");
    const void* Bcur = B;
    int64_t ldcur = ldb;
    const double* Wcur = W;
    const double* Qcur = Q;
    int64_t ldqcur = ldq;
    const int64_t Jq = k.c->cur_J;
    if (refine) {
        double* Q1 = k.ws<double>((size_t)Jq * kb);
        void* C = k.c->ws((size_t)sb.L * kb * sb.R * (dt == Dt::F64 ? 8 : 4));
        double* W2 = k.ws<double>((size_t)kb * kb);
        if (!Q1 || !C || !W2) return fail(RT_ENOMEM, "workspace allocation failed");
        RT_HIP(rt::launch_truncate(Wcur, kb, Qcur, ldqcur, Jq, kb, nullptr, 0.0, U, Uf, Q1, Dt::F64, lam, kdev,
                                   1e-20, tscr, st));
        RT_TRY(do_project(k, dt, Dt::F64, Bcur, sb, ldcur, U, kb, kb, C, kb, 0, W2, nullptr));
        Bcur = C;
        ldcur = kb;
        Wcur = W2;
        Qcur = Q1;
        ldqcur = kb;
        U = k.ws<double>((size_t)kb * kb);
        if (!U) return fail(RT_ENOMEM, "workspace allocation failed");
    }
    {
        // Jacobi stops at an off-diagonal sum of squares of jtol ||W||_F^2.  For
        // float data W is the Gram of a float32 B, whose entries already carry a
        // relative rounding of 2^-24: W and its eigenvectors are fixed only to
        // about 1e-7 ||W||, so the sweeps stop there (jtol = 1e-14); fp64 data
        // sweeps to 1e-15 ||W||.
        TimeScope ts(k.c, 3, 0.0, 0.0, Jq, kb, kb);
        RT_HIP(rt::launch_truncate(Wcur, kb, Qcur, ldqcur, Jq, r_fixed, Edev, tau2, U, Uf, A_out, dt, lam, kdev,
                                   dt == Dt::F64 ? 1e-30 : 1e-14, tscr, st));
    }
    int kk = r_fixed;
    if (r_fixed < 0) {
        RT_HIP(hipMemcpyAsync(k.c->host + 8, kdev, sizeof(int), hipMemcpyDeviceToHost, st));
        RT_HIP(hipStreamSynchronize(st));
        std::memcpy(&kk, k.c->host + 8, sizeof(int));
    }
    if (k_host) *k_host = kk;
    if (core_out && kk > 0) {
        const size_t es = dt == Dt::F64 ? 8 : 4;
        if (!*core_out) *core_out = k.c->ws((size_t)sb.L * kk * sb.R * es);
        if (!*core_out) return fail(RT_ENOMEM, "workspace allocation failed");
        const bool f64q = dt == Dt::F64 || refine;
        RT_TRY(do_project(k, dt, f64q ? Dt::F64 : Dt::F32, Bcur, sb, ldcur, f64q ? (const void*)U : (const void*)Uf,
                          kk, kk, *core_out, kk, 0, nullptr, k.c->last_nrm2));
    }
    return RT_OK;
}

// One fixed-rank RandSVD step (Alg. 1) on the mode-n unfolding of G:
// A_out (J x r, dtype dt) and, if core_out != NULL, the truncated core (L, r, R).
rt_status fixed_mode(Call& k, Dt dt, int prec, const void* G, Shape3 s, int mode, int ell, int r, uint64_t seed,
                     int power_iters, void* A_out, void* core_out, double* nrm2_dev, uint32_t* status_dev) {
    hipStream_t st = k.c->stream;
    const int64_t J = s.J;
    double* Y = k.ws<double>((size_t)J * ell);
    double* scratch = k.ws<double>(rt::orth_scratch(J, ell));
    float* Qf = dt == Dt::F32 ? k.ws<float>((size_t)J * ell) : nullptr;
    if (!Y || !scratch || (dt == Dt::F32 && !Qf)) return fail(RT_ENOMEM, "workspace allocation failed");
    RT_TRY(do_sketch(k, dt, prec, G, s, ell, 0, seed, mode, Y, nrm2_dev));                      // Alg. 1 step 1
    {
        TimeScope ts(k.c, 2, 0.0, 0.0, J, ell, ell);
        RT_HIP(rt::launch_orth(Y, J, ell, Qf, orth_accept_ratio(), status_dev, scratch, st));    // step 2
    }
    void* B = k.c->ws((size_t)s.L * ell * s.R * (dt == Dt::F64 ? 8 : 4));
    double* W = k.ws<double>((size_t)ell * ell);
    if (!B || !W) return fail(RT_ENOMEM, "workspace allocation failed");
    const void* Qp = dt == Dt::F64 ? (const void*)Y : (const void*)Qf;
    if (power_iters > 0) {
        // subspace iteration, power_iters times: Z = G_(n)^T Q (stored as B = G x_n Q^T),
        // Z <- orth(Z) by the eigendecomposition of its fp64 Gram (rows of T^T B
        // orthonormal above a floor of the largest eigenvalue), then Y = G_(n) Z and
        // Q = orth(Y)
        void* B2 = k.c->ws((size_t)s.L * ell * s.R * (dt == Dt::F64 ? 8 : 4));
        double* T = k.ws<double>((size_t)ell * ell);
        float* Tf = k.ws<float>((size_t)ell * ell);
        const int nwg = rt::plan_gram3(s.L, s.R);
        double* gp = k.ws<double>((size_t)nwg * ell * ell);
        double* rtmp = k.ws<double>(rt::reduce_partials_tmp(nwg, (int64_t)ell * ell) + 1);
        if (!B2 || !T || !Tf || !gp || !rtmp) return fail(RT_ENOMEM, "workspace allocation failed");
        const Shape3 sb{s.L, ell, s.R};
        const double drop = dt == Dt::F64 ? 1e-26 : 1e-12;     // eigenvalue floor, relative to the largest
        for (int it = 0; it < power_iters; ++it) {
            RT_TRY(do_project(k, dt, dt, G, s, s.J, Qp, ell, ell, B, ell, 0, nullptr, nullptr));
            RT_HIP(rt::launch_gram3(B, dt, s.L, ell, s.R, ell, gp, nwg, st));
            RT_HIP(rt::launch_reduce_partials(gp, true, nwg, (int64_t)ell * ell, W, st, rtmp));
            // Jacobi tolerance as for the truncation: float data fixes W only to ~2^-24 ||W||
            RT_HIP(rt::launch_svqb(W, ell, drop, T, Tf, dt == Dt::F64 ? 1e-30 : 1e-14, st));
            RT_TRY(do_project(k, dt, dt, B, sb, ell, dt == Dt::F64 ? (const void*)T : (const void*)Tf, ell, ell, B2,
                              ell, 0, nullptr, nullptr));
            RT_TRY(do_sketch_explicit(k, dt, G, s, ell, B2, Y));
            TimeScope ts(k.c, 2, 0.0, 0.0, J, ell, ell);
            RT_HIP(rt::launch_orth(Y, J, ell, Qf, orth_accept_ratio(), status_dev, scratch, st));
        }
    }
    RT_TRY(do_project(k, dt, dt, G, s, s.J, Qp, ell, ell, B, ell, 0, W, nullptr));               // step 3
    k.c->cur_J = J;
    k.c->last_nrm2 = nullptr;
    void* core = core_out;
    return do_truncate(k, dt, B, Shape3{s.L, ell, s.R}, ell, W, Y, ell, r, nullptr, 0.0, dt == Dt::F64, A_out,
                       core_out ? &core : nullptr, nullptr);                                      // steps 4-6
}

// B = G x_n Q^T for ncols columns of Q (J x ldq) of any count, in column blocks
// of at most RT_LMAX written at their offset in B (L, ldk, R).
rt_status project_cols(Call& k, Dt dx, Dt dq, const void* G, Shape3 s, int64_t ldj, const void* Q, int64_t ldq,
                       int ncols, void* B, int64_t ldk) {
    const size_t esq = dq == Dt::F64 ? 8 : 4;
    for (int c0 = 0; c0 < ncols; c0 += RT_LMAX) {
        const int w = std::min(RT_LMAX, ncols - c0);
        RT_TRY(do_project(k, dx, dq, G, s, ldj, (const char*)Q + (size_t)c0 * esq, ldq, w, B, ldk, c0, nullptr,
                          nullptr));
    }
    return RT_OK;
}

// One fixed-rank RandSVD step (Alg. 1) for RT_LMAX < ell <= RT_LMAX_FIXED: the
// sketch in column blocks of at most RT_LMAX (the same Omega columns as one wide
// sketch) gathered into Y (J x ell, fp64), Q by CholeskyQR2 with a Householder
// fallback, B = G x_n Q^T in
// column blocks, the fp64 Gram of B, its eigenvectors by one-sided Jacobi, A_n
// = Q U_r with the sign rule, and the core U_r^T B.
rt_status fixed_mode_wide(Call& k, Dt dt, int prec, const void* G, Shape3 s, int mode, int ell, int r,
                          uint64_t seed, void* A_out, void* core_out, double* nrm2_dev, uint32_t* status_dev) {
    hipStream_t st = k.c->stream;
    const int64_t J = s.J;
    const size_t es = dt == Dt::F64 ? 8 : 4;
    double* Y = k.ws<double>((size_t)J * ell);
    double* Yb = k.ws<double>((size_t)J * RT_LMAX);
    double* V = k.ws<double>(rt::wide_orth_scratch(J, ell));
    float* Qf = dt == Dt::F32 ? k.ws<float>((size_t)J * ell) : nullptr;
    if (!Y || !Yb || !V || (dt == Dt::F32 && !Qf)) return fail(RT_ENOMEM, "workspace allocation failed");
    for (int c0 = 0; c0 < ell; c0 += RT_LMAX) {                                             // step 1
        const int w = std::min(RT_LMAX, ell - c0);
        RT_TRY(do_sketch(k, dt, prec, G, s, w, c0, seed, mode, Yb, c0 == 0 ? nrm2_dev : nullptr));
        RT_HIP(rt::launch_wide_copy_cols(Yb, J, w, Y, ell, c0, st));
    }
    {
        TimeScope ts(k.c, 2, 0.0, 0.0, J, ell, ell);
        RT_HIP(rt::launch_wide_orth(Y, J, ell, Qf, orth_accept_ratio(), status_dev, V, st));  // step 2
    }
    void* B = k.c->ws((size_t)s.L * ell * s.R * es);
    if (!B) return fail(RT_ENOMEM, "workspace allocation failed");
    const void* Qp = dt == Dt::F64 ? (const void*)Y : (const void*)Qf;
    RT_TRY(project_cols(k, dt, dt, G, s, s.J, Qp, ell, ell, B, ell));                        // step 3
    const int nwg = rt::plan_wide_gram(s.L * s.R);
    double* gp = k.ws<double>((size_t)nwg * ell * ell);
    double* Wm = k.ws<double>((size_t)ell * ell);
    double* rtmp = k.ws<double>(rt::reduce_partials_tmp(nwg, (int64_t)ell * ell) + 1);
    double* U = k.ws<double>((size_t)ell * ell);
    double* lam = k.ws<double>(ell);
    double* A64 = k.ws<double>((size_t)J * r);
    double* sgn = k.ws<double>(r);
    double* Us = k.ws<double>((size_t)ell * r);
    float* Usf = k.ws<float>((size_t)ell * r);
    if (!gp || !Wm || !rtmp || !U || !lam || !A64 || !sgn || !Us || !Usf)
        return fail(RT_ENOMEM, "workspace allocation failed");
    {
        TimeScope ts(k.c, 4, (double)s.L * ell * s.R * es, 2.0 * ell * ell * (double)s.L * s.R, ell, s.L * s.R, ell);
        RT_HIP(rt::launch_wide_gram(B, dt, s.L, ell, ell, s.R, gp, nwg, st));
        RT_HIP(rt::launch_reduce_partials(gp, true, nwg, (int64_t)ell * ell, Wm, st, rtmp));
    }
    {
        // rotations stop at columns orthogonal to ell u (fp64 data) or 1e-9 (the
        // Gram of float data is fixed only to ~2^-24 of its norm)
        TimeScope ts(k.c, 3, 0.0, 0.0, J, ell, ell);
        RT_HIP(rt::launch_wide_eig(Wm, ell, dt == Dt::F64 ? ell * 0x1p-52 : 1e-9, U, lam, st));   // steps 4-5
        RT_HIP(rt::launch_wide_factor(Y, ell, J, ell, U, r, A64, sgn, A_out, dt, Us, Usf, st));
    }
    if (core_out)                                                                             // step 6
        RT_TRY(project_cols(k, dt, dt == Dt::F64 ? Dt::F64 : Dt::F32, B, Shape3{s.L, ell, s.R}, ell,
                            dt == Dt::F64 ? (const void*)Us : (const void*)Usf, r, r, core_out, r));
    return RT_OK;
}

// Adaptive post-truncation of a QB with RT_LMAX < kb <= RT_LMAX_FIXED basis
// columns: B is (L, kb, R) stored with mode length ldb, Q (J x kb, row stride
// ldq).  The eigenvalues of B's fp64 Gram come back to the host, where the rank
// is the smallest k with max(E, 0) + sum_{t >= k} lambda_t <= tau2; then A (J x
// k, written with leading dimension k), the core U_k^T B into *core_out and its
// squared norm into core_nrm2 (device) when those are given.
rt_status truncate_wide(Call& k, Dt dt, const void* B, Shape3 sb, int64_t ldb, const double* Q, int64_t J,
                        int64_t ldq, double E, double tau2, void* A_out, void** core_out, double* core_nrm2,
                        int* k_host) {
    hipStream_t st = k.c->stream;
    const int kb = (int)sb.J;
    const size_t es = dt == Dt::F64 ? 8 : 4;
    const int nwg = rt::plan_wide_gram(sb.L * sb.R);
    double* gp = k.ws<double>((size_t)nwg * kb * kb);
    double* Wm = k.ws<double>((size_t)kb * kb);
    double* rtmp = k.ws<double>(rt::reduce_partials_tmp(nwg, (int64_t)kb * kb) + 1);
    double* U = k.ws<double>((size_t)kb * kb);
    double* lam = k.ws<double>(kb);
    double* A64 = k.ws<double>((size_t)J * kb);
    double* sgn = k.ws<double>(kb);
    double* Us = k.ws<double>((size_t)kb * kb);
    float* Usf = k.ws<float>((size_t)kb * kb);
    if (!gp || !Wm || !rtmp || !U || !lam || !A64 || !sgn || !Us || !Usf)
        return fail(RT_ENOMEM, "workspace allocation failed");
    RT_HIP(rt::launch_wide_gram(B, dt, sb.L, kb, ldb, sb.R, gp, nwg, st));
    RT_HIP(rt::launch_reduce_partials(gp, true, nwg, (int64_t)kb * kb, Wm, st, rtmp));
    {
        TimeScope ts(k.c, 3, 0.0, 0.0, J, kb, kb);
        RT_HIP(rt::launch_wide_eig(Wm, kb, dt == Dt::F64 ? kb * 0x1p-52 : 1e-9, U, lam, st));
    }
    std::vector<double> lh(kb);
    RT_HIP(hipMemcpyAsync(lh.data(), lam, sizeof(double) * kb, hipMemcpyDeviceToHost, st));
    RT_HIP(hipStreamSynchronize(st));
    double tail = 0.0;
    int kk = kb;
    const double e0 = std::max(E, 0.0);
    for (int t = kb - 1; t >= 0; --t) {                  // tail = sum_{t' >= t} max(lambda_t', 0)
        const double lt = std::max(lh[t], 0.0);          // a Gram's eigenvalue is >= 0 up to rounding
        if (e0 + tail + lt > tau2) break;
        tail += lt;
        kk = t;
    }
    if (e0 > tau2) kk = kb;                              // a capped mode keeps every column
    *k_host = kk;
    if (kk == 0) return RT_OK;
    RT_HIP(rt::launch_wide_factor(Q, ldq, J, kb, U, kk, A64, sgn, A_out, dt, Us, Usf, st));
    if (core_out) {
        if (!*core_out) *core_out = k.c->ws((size_t)sb.L * kk * sb.R * es);
        if (!*core_out) return fail(RT_ENOMEM, "workspace allocation failed");
        RT_TRY(project_cols(k, dt, dt == Dt::F64 ? Dt::F64 : Dt::F32, B, sb, ldb,
                            dt == Dt::F64 ? (const void*)Us : (const void*)Usf, kk, kk, *core_out, kk));
        if (core_nrm2) RT_TRY(do_norm2(k, *core_out, dt, sb.L * kk * sb.R, core_nrm2));
    }
    return RT_OK;
}

void init_out(rt_tucker* out, const rt_tensor* X) {
    std::memset(out, 0, sizeof(*out));
    out->ndim = X->ndim;
    out->dtype = X->dtype;
    for (int i = 0; i < X->ndim; ++i) {
        out->dims[i] = X->dims[i];
        out->ranks[i] = (int32_t)X->dims[i];
    }
}

void release_partial(rt_ctx* ctx, rt_tucker* out) {
    if (!out) return;
    ctx->raw_free(out->core);
    out->core = nullptr;
    for (int i = 0; i < RT_MAXD; ++i) {
        ctx->raw_free(out->factors[i]);
        out->factors[i] = nullptr;
    }
}

// Scalars of a finished result from its slot: norms, error estimate, flags.
rt_status fill_result(rt_tucker* out, const rt::FinishScalars* h, bool oblique) {
    out->norm_x = std::sqrt(std::max(h->nx2, 0.0));
    out->core_norm = std::sqrt(std::max(h->ng2, 0.0));
    out->rel_err_est = out->norm_x > 0 ? std::sqrt(std::max(0.0, h->nx2 - h->ng2)) / out->norm_x : 0.0;
    if (oblique) out->rel_err_est = -1.0;   // no identity: the projections are oblique
    uint32_t fl = 0;
    bool nonfinite = false;
    for (int i = 0; i < RT_MAXD; ++i) {
        fl |= h->status[i] & (RT_FLAG_PADDED | RT_FLAG_FALLBACK | RT_FLAG_BADCOORD);
        if (h->status[i] & RT_FLAG_NONFINITE) nonfinite = true;
    }
    if (fl & RT_FLAG_BADCOORD) {
        out->flags = fl | (nonfinite ? RT_FLAG_NONFINITE : 0u);
        return RT_EINVAL;
    }
    if (nonfinite || !std::isfinite(h->nx2)) {
        out->flags = fl | RT_FLAG_NONFINITE;
        return RT_ENONFINITE;
    }
    out->flags = fl;
    return RT_OK;
}

const char* deferred_message(rt_status s) {
    return s == RT_EINVAL ? "sparse input has a coordinate out of range (those entries were ignored)"
                          : "input holds NaN or Inf";
}

// Waits for the stream and fills every pending result; returns the first
// deferred error (RT_ENONFINITE) or RT_OK.  `mine`, when set, receives the
// status of that result alone.
rt_status drain_pending(rt_ctx* c, const rt_tucker* self = nullptr, rt_status* mine = nullptr) {
    RT_HIP(hipStreamSynchronize(c->stream));
    rt_status first = RT_OK;
    for (size_t i = 0; i < c->pending.size(); ++i) {
        const rt_status s = fill_result(c->pending[i].out, c->slot_host(i), c->pending[i].oblique);
        if (mine && c->pending[i].out == self) *mine = s;
        if (s != RT_OK && first == RT_OK) first = s;
    }
    c->pending.clear();
    if (first != RT_OK) fail(first, deferred_message(first));
    return first;
}

// Last step of a decomposition: the core copied into its output buffer, its
// squared norm and the device status words written into a slot of the pinned
// block.  defer: the call returns at once and rt_sync fills the scalars of
// *out; otherwise they are filled here (after waiting for the stream).
rt_status finish(Call& k, rt_tucker* out, const void* core_dev, const std::vector<int64_t>& cdims, Dt dt,
                 double* nx2_dev, uint32_t* status_dev, bool defer, bool oblique = false) {
    int64_t n = 1;
    for (auto v : cdims) n *= v;
    const size_t bytes = (size_t)n * (dt == Dt::F64 ? 8 : 4);
    out->core = k.c->raw_alloc(bytes);
    if (!out->core) return fail(RT_ENOMEM, "core allocation failed");
    if (k.c->pending.size() >= (size_t)rt_ctx::NSLOT) RT_TRY(drain_pending(k.c) == RT_EHIP ? RT_EHIP : RT_OK);
    const size_t slot = k.c->pending.size();
    // one launch copies the core, sums its squares and writes the scalars into
    // the slot; a large core is copied and its partial sums taken first
    rt::FinishScalars* hd = k.c->slot_dev(slot);
    if (n <= rt::FINISH_DIRECT_MAX) {
        RT_HIP(rt::launch_finish(core_dev, out->core, dt, n, true, nullptr, 0, nx2_dev, status_dev, hd,
                                 k.c->stream));
    } else {
        RT_HIP(hipMemcpyAsync(out->core, core_dev, bytes, hipMemcpyDeviceToDevice, k.c->stream));
        const int nwg = rt::plan_norm(n);
        double* part = k.ws<double>(nwg);
        if (!part) return fail(RT_ENOMEM, "workspace allocation failed");
        RT_HIP(rt::launch_norm2(out->core, dt, n, part, nwg, k.c->stream));
        RT_HIP(rt::launch_finish(nullptr, nullptr, dt, 0, false, part, nwg, nx2_dev, status_dev, hd, k.c->stream));
    }
    k.c->pending.push_back({out, oblique});
    if (defer) {
        const double nan = std::nan("");
        out->norm_x = out->core_norm = out->rel_err_est = nan;
        return RT_OK;
    }
    rt_status mine = RT_OK;
    const rt_status all = drain_pending(k.c, out, &mine);
    if (all == RT_EHIP) return all;
    if (mine != RT_OK) return fail(mine, deferred_message(mine));
    return RT_OK;
}

}  // namespace

extern "C" {

const char* rt_version(void) { return "rtucker 0.1 (gfx950)"; }

const char* rt_last_error(void) { return g_err.c_str(); }

rt_status rt_create(rt_ctx** ctx, int device, void* stream, rt_alloc_fn alloc, rt_free_fn free_fn, void* user) {
    if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
    *ctx = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(RT_EINVAL, "alloc and free must both be set or NULL");
    RT_HIP(hipSetDevice(device));
    RT_HIP(rt::dense_init());
    RT_HIP(rt::noalloc_init(device));
    rt_ctx* c = new rt_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    if (hipHostMalloc((void**)&c->host, rt_ctx::SLOT_OFFSET + rt_ctx::NSLOT * rt_ctx::SLOT_BYTES,
                      hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(RT_ENOMEM, "pinned host allocation failed");
    }
    if (hipHostGetDevicePointer((void**)&c->host_dev, c->host, 0) != hipSuccess || !c->host_dev) {
        (void)hipHostFree(c->host);
        delete c;
        return fail(RT_EHIP, "pinned host block is not mapped for the device");
    }
    *ctx = c;
    return RT_OK;
}

rt_status rt_set_stream(rt_ctx* ctx, void* stream) {
    if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
    ctx->stream = (hipStream_t)stream;
    return RT_OK;
}

rt_status rt_destroy(rt_ctx* ctx) {
    if (!ctx) return RT_OK;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& c : ctx->chunks) ctx->raw_free(c.p);
    ctx->chunks.clear();
    for (auto e : ctx->evpool) (void)hipEventDestroy(e);
    ctx->evpool.clear();
    for (auto sd : ctx->side) {
        (void)hipStreamSynchronize(sd);
        (void)hipStreamDestroy(sd);
    }
    ctx->side.clear();
    for (auto e : ctx->sync_ev) (void)hipEventDestroy(e);
    ctx->sync_ev.clear();
    if (ctx->host) (void)hipHostFree(ctx->host);
    delete ctx;
    return RT_OK;
}

rt_status rt_timing(rt_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
    RT_HIP(hipStreamSynchronize(ctx->stream));
    ctx->timing = (uint32_t)enable & 0x1fu;
    ctx->tlog.clear();
    ctx->evused = 0;
    return RT_OK;
}

rt_status rt_timing_count(rt_ctx* ctx, int64_t* n) {
    if (!ctx || !n) return fail(RT_EINVAL, "NULL argument");
    *n = (int64_t)ctx->tlog.size();
    return RT_OK;
}

rt_status rt_timing_variant(rt_ctx* ctx, int64_t i, int32_t* variant) {
    if (!ctx || !variant) return fail(RT_EINVAL, "NULL argument");
    if (i < 0 || i >= (int64_t)ctx->tlog.size()) return fail(RT_EINVAL, "entry index out of range");
    *variant = ctx->tlog[(size_t)i].variant;
    return RT_OK;
}

rt_status rt_timing_entry(rt_ctx* ctx, int64_t i, int32_t* kind, double* ms, double* bytes, double* flops,
                          int64_t* rows, int64_t* cols, int32_t* ell) {
    if (!ctx || !kind || !ms || !bytes || !flops || !rows || !cols || !ell) return fail(RT_EINVAL, "NULL argument");
    if (i < 0 || i >= (int64_t)ctx->tlog.size()) return fail(RT_EINVAL, "entry index out of range");
    RT_HIP(hipStreamSynchronize(ctx->stream));
    const auto& t = ctx->tlog[(size_t)i];
    float f = 0.0f;
    RT_HIP(hipEventElapsedTime(&f, t.a, t.b));
    *kind = t.kind;
    *ms = f;
    *bytes = t.bytes;
    *flops = t.flops;
    *rows = t.rows;
    *cols = t.cols;
    *ell = t.ell;
    return RT_OK;
}

rt_status rt_sync(rt_ctx* ctx) {
    if (!ctx) return fail(RT_EINVAL, "ctx is NULL");
    return drain_pending(ctx);
}

rt_status rt_tucker_release(rt_ctx* ctx, rt_tucker* t) {
    if (!ctx || !t) return fail(RT_EINVAL, "NULL argument");
    (void)hipStreamSynchronize(ctx->stream);
    // a result released before rt_sync: its scalars are not filled later
    for (auto& p : ctx->pending)
        if (p.out == t) p.out = &ctx->discard;
    release_partial(ctx, t);
    return RT_OK;
}

rt_status rt_rsthosvd(rt_ctx* ctx, const rt_tensor* X, const int32_t* ranks, const rt_opts* opts, rt_tucker* out) {
    if (!ctx || !opts || !out) return fail(RT_EINVAL, "NULL argument");
    RT_TRY(check_tensor(X));
    RT_TRY(check_prec(X, opts->prec));
    if (opts->power_iters < 0 || opts->power_iters > RT_MAX_POWER_ITERS)
        return fail(RT_EINVAL, "power_iters must be in [0, RT_MAX_POWER_ITERS]");
    RT_TRY(check_ranks(X, ranks, opts->oversample, RT_LMAX_FIXED));
    RT_TRY(check_wide_power(X, ranks, opts));
    std::vector<int> order;
    RT_TRY(make_order(X, opts->order, order));
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    const Dt dt = dt_of(X->dtype);
    const int prec = (int)opts->prec;
    const size_t es = dsize(X->dtype);
    init_out(out, X);
    std::vector<int64_t> dims(X->dims, X->dims + X->ndim);
    double* nx2 = k.ws<double>(1);
    uint32_t* status = k.ws<uint32_t>(RT_MAXD);
    if (!nx2 || !status) return fail(RT_ENOMEM, "workspace allocation failed");
    RT_HIP(hipMemsetAsync(status, 0, sizeof(uint32_t) * RT_MAXD, ctx->stream));
    const void* cur = X->data;
    bool have_norm = false;
    for (int n : order) {
        if (ranks[n] == RT_KEEP) continue;
        const int r = ranks[n];
        const int ell = r + opts->oversample;
        Shape3 s = shape3(dims, n);
        out->factors[n] = ctx->raw_alloc((size_t)s.J * r * es);
        void* core = k.c->ws((size_t)s.L * r * s.R * es);
        if (!out->factors[n] || !core) {
            release_partial(ctx, out);
            return fail(RT_ENOMEM, "allocation failed");
        }
        rt_status rs = ell > RT_LMAX
                           ? fixed_mode_wide(k, dt, prec, cur, s, n, ell, r, opts->seed, out->factors[n], core,
                                             have_norm ? nullptr : nx2, status + n)
                           : fixed_mode(k, dt, prec, cur, s, n, ell, r, opts->seed, opts->power_iters,
                                        out->factors[n], core, have_norm ? nullptr : nx2, status + n);
        if (rs != RT_OK) { release_partial(ctx, out); return rs; }
        have_norm = true;
        out->ranks[n] = r;
        dims[n] = r;
        cur = core;
    }
    if (!have_norm) {
        int64_t n = 1;
        for (auto v : dims) n *= v;
        rt_status rs = do_norm2(k, X->data, dt, n, nx2);
        if (rs != RT_OK) { release_partial(ctx, out); return rs; }
    }
    rt_status rs = finish(k, out, cur, dims, dt, nx2, status, true);
    if (rs != RT_OK && rs != RT_ENONFINITE) release_partial(ctx, out);
    return rs;
}

rt_status rt_sp_sthosvd(rt_ctx* ctx, const rt_tensor* X, const int32_t* ranks, const rt_opts* opts, rt_tucker* out) {
    if (!ctx || !opts || !out) return fail(RT_EINVAL, "NULL argument");
    RT_TRY(check_tensor(X));
    RT_TRY(check_prec(X, opts->prec));
    if (opts->power_iters != 0) return fail(RT_EINVAL, "power_iters must be 0 for rt_sp_sthosvd");
    RT_TRY(check_ranks(X, ranks, opts->oversample));
    std::vector<int> order;
    RT_TRY(make_order(X, opts->order, order));
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    hipStream_t st = ctx->stream;
    const Dt dt = dt_of(X->dtype);
    const int prec = (int)opts->prec;
    const size_t es = dsize(X->dtype);
    init_out(out, X);
    std::vector<int64_t> dims(X->dims, X->dims + X->ndim);
    double* nx2 = k.ws<double>(1);
    uint32_t* status = k.ws<uint32_t>(RT_MAXD);
    int* sel = k.ws<int>(RT_LMAX);
    int* swaps = k.ws<int>(1);
    if (!nx2 || !status || !sel || !swaps) return fail(RT_ENOMEM, "workspace allocation failed");
    RT_HIP(hipMemsetAsync(status, 0, sizeof(uint32_t) * RT_MAXD, st));
    const void* cur = X->data;
    bool have_norm = false;
    for (int n : order) {
        if (ranks[n] == RT_KEEP) continue;
        const int ell = ranks[n] + opts->oversample;
        const Shape3 s = shape3(dims, n);
        const int64_t J = s.J;
        double* Y = k.ws<double>((size_t)J * ell);
        double* oscr = k.ws<double>(rt::orth_scratch(J, ell));
        double* sscr = k.ws<double>((size_t)2 * J * ell);
        out->factors[n] = ctx->raw_alloc((size_t)J * ell * es);
        void* core = k.c->ws((size_t)s.L * ell * s.R * es);
        if (!Y || !oscr || !sscr || !out->factors[n] || !core) {
            release_partial(ctx, out);
            return fail(RT_ENOMEM, "allocation failed");
        }
        // Alg. 6: Y = G_(n) Omega, Q = orth(Y), selection P, A = Q (P^T Q)^-1, G <- P^T G
        rt_status rs = do_sketch(k, dt, prec, cur, s, ell, 0, opts->seed, n, Y, have_norm ? nullptr : nx2);
        if (rs != RT_OK) { release_partial(ctx, out); return rs; }
        {
            TimeScope ts(k.c, 2, 0.0, 0.0, J, ell, ell);
            RT_HIP(rt::launch_orth(Y, J, ell, nullptr, orth_accept_ratio(), status + n, oscr, st));
            RT_HIP(rt::launch_select_rows(Y, J, ell, 2.0, 1000, sscr, out->factors[n], dt, sel, swaps, st));
        }
        RT_HIP(rt::launch_gather_mode(cur, dt, s, sel, ell, core, st));
        have_norm = true;
        out->ranks[n] = ell;
        dims[n] = ell;
        cur = core;
    }
    if (!have_norm) {
        int64_t n = 1;
        for (auto v : dims) n *= v;
        rt_status rs = do_norm2(k, X->data, dt, n, nx2);
        if (rs != RT_OK) { release_partial(ctx, out); return rs; }
    }
    rt_status rs = finish(k, out, cur, dims, dt, nx2, status, true, true);
    if (rs != RT_OK && rs != RT_ENONFINITE) release_partial(ctx, out);
    return rs;
}

rt_status rt_sp_sthosvd_coo(rt_ctx* ctx, const rt_coo* X, const int32_t* ranks, const rt_opts* opts,
                            rt_tucker* out) {
    if (!ctx || !opts || !out) return fail(RT_EINVAL, "NULL argument");
    RT_TRY(check_coo(X));
    const rt_tensor T = coo_header(X);
    RT_TRY(check_prec(&T, opts->prec));
    if (opts->prec == RT_PREC_BF16_SKETCH) return fail(RT_EINVAL, "sparse tensors take RT_PREC_F32 or RT_PREC_F64");
    if (opts->power_iters != 0) return fail(RT_EINVAL, "power_iters must be 0 for rt_sp_sthosvd_coo");
    RT_TRY(check_ranks(&T, ranks, opts->oversample));
    std::vector<int> order;
    RT_TRY(make_order(&T, opts->order, order));
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    hipStream_t st = ctx->stream;
    const Dt dt = dt_of(X->dtype);
    const size_t es = dsize(X->dtype);
    const int d = X->ndim;
    const int64_t bound = X->nnz;
    init_out(out, &T);
    std::vector<int64_t> dims(X->dims, X->dims + d);
    double* nx2 = k.ws<double>(1);
    uint32_t* status = k.ws<uint32_t>(RT_MAXD);
    int* sel = k.ws<int>(RT_LMAX);
    int* swaps = k.ws<int>(1);
    int64_t* cnt_dev = k.ws<int64_t>(2);
    // two coordinate buffers (capacity: the input's entry count) alternate as
    // the intermediate cores
    const int64_t cap = std::max<int64_t>(bound, 1);
    int32_t* cidx[2] = {k.ws<int32_t>((size_t)d * cap), k.ws<int32_t>((size_t)d * cap)};
    void* cval[2] = {k.c->ws((size_t)cap * es), k.c->ws((size_t)cap * es)};
    const int64_t nb = rt::coo_chunks(bound);
    int64_t* cnt = k.ws<int64_t>(std::max<int64_t>(nb, 1));
    int64_t* off = k.ws<int64_t>(std::max<int64_t>(nb, 1));
    if (!nx2 || !status || !sel || !swaps || !cnt_dev || !cidx[0] || !cidx[1] || !cval[0] || !cval[1] || !cnt ||
        !off)
        return fail(RT_ENOMEM, "workspace allocation failed");
    RT_HIP(hipMemsetAsync(status, 0, sizeof(uint32_t) * RT_MAXD, st));
    const rt::CooDims xdims = coo_dims(dims);
    if (bound > 0) RT_TRY(do_norm2(k, X->vals, dt, bound, nx2));
    else RT_HIP(hipMemsetAsync(nx2, 0, sizeof(double), st));
    const int32_t* cur_idx = X->idx;
    int64_t cur_ld = bound;
    const void* cur_val = X->vals;
    const int64_t* cur_nnz = nullptr;   // the input's count is `bound` itself
    int pp = 0;
    for (int n : order) {
        if (ranks[n] == RT_KEEP) continue;
        const int ell = ranks[n] + opts->oversample;
        const int64_t J = dims[n];
        double* Y = k.ws<double>((size_t)J * ell);
        double* oscr = k.ws<double>(rt::orth_scratch(J, ell));
        double* sscr = k.ws<double>((size_t)2 * J * ell);
        int32_t* inv = k.ws<int32_t>((size_t)J);
        out->factors[n] = ctx->raw_alloc((size_t)J * ell * es);
        if (!Y || !oscr || !sscr || !inv || !out->factors[n]) {
            release_partial(ctx, out);
            return fail(RT_ENOMEM, "allocation failed");
        }
        // Alg. 6: Y = G_(n) Omega, Q = orth(Y), selection P, A = Q (P^T Q)^-1, G <- P^T G
        RT_HIP(hipMemsetAsync(Y, 0, (size_t)J * ell * sizeof(double), st));
        {
            TimeScope ts(k.c, 0, (double)bound * (d * 4.0 + es), 2.0 * ell * bound, J, bound, ell);
            ts.t.variant = RT_SKETCH_COO;
            if (cur_nnz)
                RT_HIP(rt::launch_coo_sketch(cur_idx, cur_ld, cur_val, dt, cur_nnz, bound, coo_dims(dims), n, ell, 0,
                                             opts->seed, Y, st));
            else
                RT_TRY(coo_sketch_input(k, cur_idx, cur_val, dt, bound, coo_dims(dims), n, ell, 0, opts->seed, Y));
        }
        {
            TimeScope ts(k.c, 2, 0.0, 0.0, J, ell, ell);
            RT_HIP(rt::launch_orth(Y, J, ell, nullptr, orth_accept_ratio(), status + n, oscr, st));
            RT_HIP(rt::launch_select_rows(Y, J, ell, 2.0, 1000, sscr, out->factors[n], dt, sel, swaps, st));
        }
        RT_HIP(rt::launch_coo_restrict(cur_idx, cur_ld, cur_val, dt, cur_nnz, bound, coo_dims(dims), n, sel, ell, inv,
                                       cnt, off, cidx[pp], cap, cval[pp], cnt_dev + pp, st));
        cur_idx = cidx[pp];
        cur_ld = cap;
        cur_val = cval[pp];
        cur_nnz = cnt_dev + pp;
        pp ^= 1;
        out->ranks[n] = ell;
        dims[n] = ell;
    }
    // entries with a coordinate out of range (skipped by every kernel) are
    // reported through the status words (after orth has written its own)
    RT_HIP(rt::launch_coo_check(X->idx, bound, bound, xdims, status, RT_FLAG_BADCOORD, st));
    int64_t ncore = 1;
    for (auto v : dims) ncore *= v;
    void* core = k.c->ws((size_t)ncore * es);
    if (!core) {
        release_partial(ctx, out);
        return fail(RT_ENOMEM, "allocation failed");
    }
    RT_HIP(hipMemsetAsync(core, 0, (size_t)ncore * es, st));
    RT_HIP(rt::launch_coo_densify(cur_idx, cur_ld, cur_val, dt, cur_nnz, bound, coo_dims(dims), core, st));
    rt_status rs = finish(k, out, core, dims, dt, nx2, status, true, true);
    if (rs != RT_OK && rs != RT_ENONFINITE && rs != RT_EINVAL) release_partial(ctx, out);
    return rs;
}

rt_status rt_rhosvd(rt_ctx* ctx, const rt_tensor* X, const int32_t* ranks, const rt_opts* opts, rt_tucker* out) {
    if (!ctx || !opts || !out) return fail(RT_EINVAL, "NULL argument");
    RT_TRY(check_tensor(X));
    RT_TRY(check_prec(X, opts->prec));
    if (opts->power_iters < 0 || opts->power_iters > RT_MAX_POWER_ITERS)
        return fail(RT_EINVAL, "power_iters must be in [0, RT_MAX_POWER_ITERS]");
    RT_TRY(check_ranks(X, ranks, opts->oversample, RT_LMAX_FIXED));
    RT_TRY(check_wide_power(X, ranks, opts));
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    const Dt dt = dt_of(X->dtype);
    const int prec = (int)opts->prec;
    const size_t es = dsize(X->dtype);
    const int d = X->ndim;
    init_out(out, X);
    std::vector<int64_t> xdims(X->dims, X->dims + d);
    double* nx2 = k.ws<double>(1);
    uint32_t* status = k.ws<uint32_t>(RT_MAXD);
    if (!nx2 || !status) return fail(RT_ENOMEM, "workspace allocation failed");
    RT_HIP(hipMemsetAsync(status, 0, sizeof(uint32_t) * RT_MAXD, ctx->stream));
    int first = -1;
    void* core0 = nullptr;
    // Alg. 2's modes are independent: each runs on a stream of its own, forked
    // from the context's stream and joined back into it before the core, so the
    // single-workgroup steps of one mode overlap the sweeps over X of another.
    // Every mode's workspace is its own (the arena is bump-allocated within a
    // call); the host enqueues the modes one after another.
    hipStream_t main_st = ctx->stream;
    hipEvent_t fork = ctx->sync_event(0);
    if (!fork) return fail(RT_EHIP, "event creation failed");
    RT_HIP(hipEventRecord(fork, main_st));
    int nside = 0;
    for (int j = 0; j < d; ++j) {                          // Alg. 2: every mode from X itself
        if (ranks[j] == RT_KEEP) continue;
        const int r = ranks[j];
        const int ell = r + opts->oversample;
        Shape3 s = shape3(xdims, j);
        out->factors[j] = ctx->raw_alloc((size_t)s.J * r * es);
        void* core = nullptr;
        if (first < 0) core = k.c->ws((size_t)s.L * r * s.R * es);
        if (!out->factors[j] || (first < 0 && !core)) {
            release_partial(ctx, out);
            return fail(RT_ENOMEM, "allocation failed");
        }
        hipStream_t sj = ctx->side_stream((size_t)nside);
        hipEvent_t done = ctx->sync_event((size_t)nside + 1);
        if (!sj || !done) { release_partial(ctx, out); return fail(RT_EHIP, "stream creation failed"); }
        RT_HIP(hipStreamWaitEvent(sj, fork, 0));
        ctx->stream = sj;
        rt_status rs = ell > RT_LMAX
                           ? fixed_mode_wide(k, dt, prec, X->data, s, j, ell, r, opts->seed, out->factors[j], core,
                                             first < 0 ? nx2 : nullptr, status + j)
                           : fixed_mode(k, dt, prec, X->data, s, j, ell, r, opts->seed, opts->power_iters,
                                        out->factors[j], core, first < 0 ? nx2 : nullptr, status + j);
        ctx->stream = main_st;
        RT_HIP(hipEventRecord(done, sj));
        RT_HIP(hipStreamWaitEvent(main_st, done, 0));
        ++nside;
        if (rs != RT_OK) {
            (void)hipStreamSynchronize(main_st);
            release_partial(ctx, out);
            return rs;
        }
        if (first < 0) { first = j; core0 = core; }
        out->ranks[j] = r;
    }
    std::vector<int64_t> dims = xdims;
    const void* cur = X->data;
    if (first >= 0) {
        // G = X x_1 A_1^T ... x_d A_d^T, starting from the truncated B of the first mode
        dims[first] = ranks[first];
        cur = core0;
        for (int j = 0; j < d; ++j) {
            if (j == first || ranks[j] == RT_KEEP) continue;
            Shape3 s = shape3(dims, j);
            const int r = ranks[j];
            void* nc = k.c->ws((size_t)s.L * r * s.R * es);
            if (!nc) { release_partial(ctx, out); return fail(RT_ENOMEM, "allocation failed"); }
            rt_status rs = project_cols(k, dt, dt, cur, s, s.J, out->factors[j], r, r, nc, r);
            if (rs != RT_OK) { release_partial(ctx, out); return rs; }
            dims[j] = r;
            cur = nc;
        }
    } else {
        int64_t n = 1;
        for (auto v : dims) n *= v;
        rt_status rs = do_norm2(k, X->data, dt, n, nx2);
        if (rs != RT_OK) { release_partial(ctx, out); return rs; }
    }
    rt_status rs = finish(k, out, cur, dims, dt, nx2, status, true);
    if (rs != RT_OK && rs != RT_ENONFINITE) release_partial(ctx, out);
    return rs;
}

// Adaptive R-STHOSVD (Alg. 5, sequential: every mode works on the core left by
// the previous one) or adaptive R-HOSVD (Alg. 4: every mode works on X, the
// core is X x_j A_j^T at the end).
static rt_status adaptive_impl(rt_ctx* ctx, const rt_tensor* X, double eps, const double* eps_per_mode,
                               int32_t block, const int32_t* max_rank, const rt_opts* opts, rt_tucker* out,
                               bool sequential) {
    if (!ctx || !opts || !out) return fail(RT_EINVAL, "NULL argument");
    RT_TRY(check_tensor(X));
    RT_TRY(check_prec(X, opts->prec));
    if (opts->power_iters != 0) return fail(RT_EINVAL, "power_iters must be 0 for the adaptive call");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(RT_EINVAL, "eps must be finite and >= 0");
    if (block < 1 || block > RT_LMAX) return fail(RT_EINVAL, "block must be in [1, RT_LMAX]");
    const int d = X->ndim;
    std::vector<double> epsn(d, eps / std::sqrt((double)d));
    if (eps_per_mode) {
        double s2 = 0.0;
        for (int j = 0; j < d; ++j) {
            if (!(eps_per_mode[j] >= 0.0)) return fail(RT_EINVAL, "eps_per_mode entries must be >= 0");
            epsn[j] = eps_per_mode[j];
            s2 += epsn[j] * epsn[j];
        }
        if (std::fabs(s2 - eps * eps) > 1e-12 * std::max(eps * eps, 1e-300))
            return fail(RT_EINVAL, "sum of eps_per_mode^2 must equal eps^2");
    }
    std::vector<int> order;
    RT_TRY(make_order(X, opts->order, order));
    if (max_rank)
        for (int j = 0; j < d; ++j)
            if (max_rank[j] < 1) return fail(RT_EINVAL, "max_rank entries must be >= 1");
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    hipStream_t st = ctx->stream;
    const Dt dt = dt_of(X->dtype);
    const int prec = (int)opts->prec;
    const size_t es = dsize(X->dtype);
    const double drop = X->dtype == RT_F64 ? 1e-10 : 1e-5;
    // With the bfloat16 sketch (two pieces per operand, relative rounding near
    // 2^-15) a block's directions below ~1e-5 of its norm are sketch noise: such
    // blocks use a drop threshold above that level, and once a bfloat16 block
    // resolves no new direction the mode continues with float32 sketches, so the
    // tolerance is still met.
    const double drop_bf16 = 1e-4;
    init_out(out, X);
    std::vector<int64_t> dims(X->dims, X->dims + d);
    double* nx2 = k.ws<double>(1);
    double* tmp = k.ws<double>(4);
    uint32_t* status = k.ws<uint32_t>(RT_MAXD);
    if (!nx2 || !tmp || !status) return fail(RT_ENOMEM, "workspace allocation failed");
    RT_HIP(hipMemsetAsync(status, 0, sizeof(uint32_t) * RT_MAXD, st));
    double* h = ctx->host;
    // per-block results read by the host: the device writes them into the
    // pinned block through its mapped address (no copy launches per block)
    int* kmap = reinterpret_cast<int*>(ctx->host_dev + 1);
    double* bmap = ctx->host_dev + 2;
    // ||X||^2 is summed by the first sketch (which reads every entry of X) and read
    // back with that block's results; no separate pass over X
    bool have_norm = false;
    double normx2 = 0.0, normx = 0.0;
    const void* cur = X->data;
    double cur_norm2 = 0.0;
    bool capped = false;
    for (int n : order) {
        if (epsn[n] == 0.0) continue;
        double tau2 = (epsn[n] * normx) * (epsn[n] * normx);
        Shape3 s = shape3(dims, n);
        const int64_t J = s.J, K = s.L * s.R;
        int cap = (int)std::min<int64_t>(std::min<int64_t>(J, K), RT_LMAX_FIXED);
        if (max_rank) cap = std::min(cap, (int)max_rank[n]);
        double* Qall = k.ws<double>((size_t)J * cap);
        // float copy of the basis: float32 data is projected on MFMA with a float Q
        // (||B_i||^2 is still summed in fp64)
        float* Qallf = dt == Dt::F32 ? k.ws<float>((size_t)J * cap) : nullptr;
        void* Bbuf = k.c->ws((size_t)s.L * cap * s.R * es);
        double* Y = k.ws<double>((size_t)J * block);
        double* scratch = k.ws<double>((size_t)2 * J * block);
        double* W = k.ws<double>((size_t)cap * cap);
        double* Edev = k.ws<double>(1);
        double* y0dev = k.ws<double>(1);
        if (!Qall || !Bbuf || !Y || !scratch || !W || !Edev || !y0dev || (dt == Dt::F32 && !Qallf)) {
            release_partial(ctx, out);
            return fail(RT_ENOMEM, "workspace allocation failed");
        }
        double E = cur_norm2;
        int kcols = 0, blk = 0;
        bool stop_cap = false;
        int prec_cur = prec;
        for (int attempt = 0; attempt < 2; ++attempt) {
            E = cur_norm2;
            kcols = 0;
            blk = 0;
            stop_cap = false;
            prec_cur = attempt == 0 ? prec : (int)RT_PREC_F32;
            while (!have_norm || E > tau2) {                    // AdaptRangeFinder block loop
                if (kcols >= cap) { stop_cap = true; break; }
                const int bi = std::min(block, cap - kcols);
                rt_status rs = do_sketch(k, dt, prec_cur, cur, s, bi, (int64_t)blk * block, opts->seed, n, Y,
                                         have_norm ? nullptr : nx2);
                if (rs != RT_OK) { release_partial(ctx, out); return rs; }
                {
                    TimeScope ts(k.c, 2, 8.0 * J * (bi + 2.0 * kcols), 8.0 * J * bi * kcols, J, kcols, bi);
                    const double dr = prec_cur == RT_PREC_BF16_SKETCH ? drop_bf16 : drop;
                    if (kcols + bi <= RT_LMAX) {
                        RT_HIP(rt::launch_block_orth(Y, J, bi, Qall, cap, kcols, dr, kmap, Qallf, scratch, st));
                    } else {
                        // a basis beyond RT_LMAX columns: Gram-Schmidt (twice) against its
                        // first ka columns, then the block step against the last kb with
                        // the drop rule on the block's norm before any projection
                        const int kb = RT_LMAX - bi, ka = kcols - kb;
                        RT_HIP(rt::launch_wide_cgs(Y, J, bi, Qall, cap, ka, y0dev, st));
                        RT_HIP(rt::launch_block_orth(Y, J, bi, Qall + ka, cap, kb, dr, kmap,
                                                     Qallf ? Qallf + ka : nullptr, scratch, st, y0dev));
                    }
                }
                // B_i over all bi columns (the dropped ones are zero); kn and ||B_i||^2
                // are written by the kernels straight into the mapped host block
                rs = Qallf ? do_project(k, dt, Dt::F32, cur, s, s.J, Qallf + kcols, cap, bi, Bbuf, cap, kcols, nullptr, bmap)
                           : do_project(k, dt, Dt::F64, cur, s, s.J, Qall + kcols, cap, bi, Bbuf, cap, kcols, nullptr, bmap);
                if (rs != RT_OK) { release_partial(ctx, out); return rs; }
                if (!have_norm) RT_HIP(hipMemcpyAsync(h, nx2, sizeof(double), hipMemcpyDeviceToHost, st));
                RT_HIP(hipStreamSynchronize(st));
                if (!have_norm) {
                    // the loop test for the first block, now that ||X|| is known
                    normx2 = h[0];
                    if (!std::isfinite(normx2)) {
                        release_partial(ctx, out);
                        return fail(RT_ENONFINITE, "input holds NaN or Inf");
                    }
                    normx = std::sqrt(normx2);
                    have_norm = true;
                    cur_norm2 = normx2;
                    E = normx2;
                    tau2 = (epsn[n] * normx) * (epsn[n] * normx);
                    if (!(E > tau2)) break;                      // no block: this one is discarded
                }
                int kn = 0;
                std::memcpy(&kn, h + 1, sizeof(int));
                ++blk;
                if (kn <= 0 && prec_cur == RT_PREC_BF16_SKETCH) {   // bfloat16 resolves nothing more
                    prec_cur = RT_PREC_F32;
                    continue;
                }
                if (kn <= 0) break;                              // range exhausted
                E -= h[2];                                       // E <- E - ||B_i||^2
                kcols += kn;
            }
            // A mode whose columns all went into a basis carrying the bfloat16
            // sketch's ~1e-3 subspace error (rank cap = K) may stop above the
            // tolerance: it is redone with float32 sketches.
            if (!(stop_cap && E > tau2 && prec == RT_PREC_BF16_SKETCH)) break;
        }
        if (stop_cap && E > tau2) capped = true;
        // SVD post-truncation: smallest k with max(E,0) + tail <= tau2
        h[3] = E;
        RT_HIP(hipMemcpyAsync(Edev, h + 3, sizeof(double), hipMemcpyHostToDevice, st));
        int kfinal = 0;
        void* A = k.c->ws((size_t)J * std::max(kcols, 1) * es);
        void* core = nullptr;
        if (!A) { release_partial(ctx, out); return fail(RT_ENOMEM, "workspace allocation failed"); }
        if (kcols > RT_LMAX) {
            rt_status rs = truncate_wide(k, dt, Bbuf, Shape3{s.L, kcols, s.R}, cap, Qall, J, cap, E, tau2, A,
                                         sequential ? &core : nullptr, sequential ? tmp : nullptr, &kfinal);
            if (rs != RT_OK) { release_partial(ctx, out); return rs; }
        } else if (kcols > 0) {
            int nwg = rt::plan_gram3(s.L, s.R);
            double* gp = k.ws<double>((size_t)nwg * kcols * kcols);
            if (!gp) { release_partial(ctx, out); return fail(RT_ENOMEM, "workspace allocation failed"); }
            RT_HIP(rt::launch_gram3(Bbuf, dt, s.L, cap, s.R, kcols, gp, nwg, st));
            double* rtmp = k.ws<double>(rt::reduce_partials_tmp(nwg, (int64_t)kcols * kcols) + 1);
            if (!rtmp) { release_partial(ctx, out); return fail(RT_ENOMEM, "workspace allocation failed"); }
            RT_HIP(rt::launch_reduce_partials(gp, true, nwg, (int64_t)kcols * kcols, W, st, rtmp));
            k.c->cur_J = J;
            k.c->last_nrm2 = sequential ? tmp : nullptr;
            rt_status rs = do_truncate(k, dt, Bbuf, Shape3{s.L, kcols, s.R}, cap, W, Qall, cap, -1, Edev, tau2,
                                       dt == Dt::F64, A, sequential ? &core : nullptr, &kfinal);
            k.c->last_nrm2 = nullptr;
            if (rs != RT_OK) { release_partial(ctx, out); return rs; }
        }
        out->factors[n] = ctx->raw_alloc((size_t)J * std::max(kfinal, 1) * es);
        if (sequential && !core) core = k.c->ws((size_t)s.L * std::max(kfinal, 1) * s.R * es);
        if (!out->factors[n] || (sequential && !core)) {
            release_partial(ctx, out);
            return fail(RT_ENOMEM, "allocation failed");
        }
        if (kfinal > 0) {
            // A was written with leading dimension kfinal by the truncation kernel
            RT_HIP(hipMemcpyAsync(out->factors[n], A, (size_t)J * kfinal * es, hipMemcpyDeviceToDevice, st));
        }
        out->ranks[n] = kfinal;
        if (sequential) {
            if (kfinal > 0) {
                RT_HIP(hipMemcpyAsync(h + 2, tmp, sizeof(double), hipMemcpyDeviceToHost, st));
                RT_HIP(hipStreamSynchronize(st));
                cur_norm2 = h[2];
            } else {
                cur_norm2 = 0.0;
            }
            dims[n] = kfinal;
            cur = core;
        }
    }
    if (!sequential) {
        // Alg. 4: G = X x_1 A_1^T ... x_d A_d^T over the compressed modes
        for (int j = 0; j < d; ++j) {
            if (epsn[j] == 0.0) continue;
            const int r = out->ranks[j];
            const Shape3 s = shape3(dims, j);
            void* nc = k.c->ws((size_t)s.L * std::max(r, 1) * s.R * es);
            if (!nc) { release_partial(ctx, out); return fail(RT_ENOMEM, "workspace allocation failed"); }
            if (r > 0) {
                rt_status rs = project_cols(k, dt, dt, cur, s, s.J, out->factors[j], r, r, nc, r);
                if (rs != RT_OK) { release_partial(ctx, out); return rs; }
            }
            dims[j] = r;
            cur = nc;
        }
    }
    if (!have_norm) {                                    // every mode kept whole (eps 0)
        int64_t ntot = 1;
        for (int j = 0; j < d; ++j) ntot *= X->dims[j];
        RT_TRY(do_norm2(k, X->data, dt, ntot, nx2));
    }
    rt_status rs = finish(k, out, cur, dims, dt, nx2, status, false);
    if (rs != RT_OK && rs != RT_ENONFINITE) { release_partial(ctx, out); return rs; }
    if (rs == RT_OK && capped) return fail(RT_ECAP, "a mode reached its rank cap before the tolerance");
    return rs;
}

rt_status rt_rsthosvd_adaptive(rt_ctx* ctx, const rt_tensor* X, double eps, const double* eps_per_mode, int32_t block,
                               const int32_t* max_rank, const rt_opts* opts, rt_tucker* out) {
    return adaptive_impl(ctx, X, eps, eps_per_mode, block, max_rank, opts, out, true);
}

rt_status rt_rhosvd_adaptive(rt_ctx* ctx, const rt_tensor* X, double eps, const double* eps_per_mode, int32_t block,
                             const int32_t* max_rank, const rt_opts* opts, rt_tucker* out) {
    return adaptive_impl(ctx, X, eps, eps_per_mode, block, max_rank, opts, out, false);
}

// ---- Tucker reconstruction ------------------------------------------------------------------

rt_status rt_reconstruct(rt_ctx* ctx, const rt_tucker* t, void* out) {
    if (!ctx || !t || !out) return fail(RT_EINVAL, "NULL argument");
    const int d = t->ndim;
    if (d < 2 || d > RT_MAXD) return fail(RT_EINVAL, "ndim must be in [2, RT_MAXD]");
    if (t->dtype != RT_F32 && t->dtype != RT_F64) return fail(RT_EINVAL, "unknown dtype");
    int64_t ncore = 1, nout = 1;
    for (int j = 0; j < d; ++j) {
        if (t->dims[j] < 1) return fail(RT_EINVAL, "dims must be >= 1");
        if (t->ranks[j] < 0 || t->ranks[j] > t->dims[j]) return fail(RT_EINVAL, "ranks must be in [0, dims]");
        if (!t->factors[j] && t->ranks[j] != t->dims[j] && t->ranks[j] != 0)
            return fail(RT_EINVAL, "a mode without a factor must keep its dimension");
        ncore *= t->ranks[j];
        nout *= t->dims[j];
    }
    if (ncore > 0 && !t->core) return fail(RT_EINVAL, "NULL core");
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    hipStream_t st = ctx->stream;
    const Dt dt = dt_of(t->dtype);
    const size_t es = dsize(t->dtype);
    if (ncore == 0) {
        RT_HIP(hipMemsetAsync(out, 0, (size_t)nout * es, st));
        return RT_OK;
    }
    int last = -1;
    for (int j = 0; j < d; ++j)
        if (t->factors[j]) last = j;
    if (last < 0) {
        RT_HIP(hipMemcpyAsync(out, t->core, (size_t)nout * es, hipMemcpyDeviceToDevice, st));
        return RT_OK;
    }
    // G x_j A_j one mode at a time: out[l, i, r] = sum_k A_j[i, k] G[l, k, r], by the
    // expansion kernels (the output streamed once); shapes beyond their grid
    // limits take the projection kernels with Q = A_j^T (r_j x I_j), in column
    // blocks of at most RT_LMAX written at their offset
    std::vector<int64_t> cur_dims(t->ranks, t->ranks + d);
    const void* cur = t->core;
    for (int j = 0; j < d; ++j) {
        if (!t->factors[j]) continue;
        const int64_t I = t->dims[j];
        const int r = t->ranks[j];
        const Shape3 s = shape3(cur_dims, j);
        void* dst = j == last ? out : k.c->ws((size_t)s.L * I * s.R * es);
        if (!dst) return fail(RT_ENOMEM, "workspace allocation failed");
        if (rt::expand_ok(s, I)) {
            RT_HIP(rt::launch_expand(dt, cur, s, t->factors[j], I, dst, st));
            cur_dims[j] = I;
            cur = dst;
            continue;
        }
        void* AT = k.c->ws((size_t)r * I * es);
        if (!AT) return fail(RT_ENOMEM, "workspace allocation failed");
        RT_HIP(rt::launch_transpose(t->factors[j], I, r, AT, dt, st));
        for (int64_t i0 = 0; i0 < I; i0 += RT_LMAX) {
            const int e = (int)std::min<int64_t>(RT_LMAX, I - i0);
            RT_TRY(do_project(k, dt, dt, cur, s, s.J, (const char*)AT + (size_t)i0 * es, I, e, dst, I, i0, nullptr,
                              nullptr));
        }
        cur_dims[j] = I;
        cur = dst;
    }
    return RT_OK;
}

// ---- step entry points -------------------------------------------------------------------

rt_status rt_sketch(rt_ctx* ctx, const rt_tensor* X, int32_t mode, int32_t ell, int64_t col0, uint64_t seed,
                    rt_precision prec, double* Y, double* nrm2) {
    RT_TRY(rt::check_sketch_args(ctx, X, mode, ell, col0, prec, Y));
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    std::vector<int64_t> dims(X->dims, X->dims + X->ndim);
    RT_TRY(do_sketch(k, dt_of(X->dtype), (int)prec, X->data, shape3(dims, mode), ell, col0, seed, mode, Y, nrm2));
    RT_HIP(hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

rt_status rt_sketch_coo(rt_ctx* ctx, const rt_coo* X, int32_t mode, int32_t ell, int64_t col0, uint64_t seed,
                        double* Y, double* nrm2) {
    if (!ctx || !Y) return fail(RT_EINVAL, "NULL argument");
    RT_TRY(check_coo(X));
    if (mode < 0 || mode >= X->ndim) return fail(RT_EINVAL, "mode out of range");
    if (ell < 1 || ell > RT_LMAX) return fail(RT_EINVAL, "ell must be in [1, RT_LMAX]");
    if (col0 < 0) return fail(RT_EINVAL, "col0 must be >= 0");
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    hipStream_t st = ctx->stream;
    const Dt dt = dt_of(X->dtype);
    std::vector<int64_t> dims(X->dims, X->dims + X->ndim);
    uint32_t* status = k.ws<uint32_t>(1);
    if (!status) return fail(RT_ENOMEM, "workspace allocation failed");
    RT_HIP(hipMemsetAsync(status, 0, sizeof(uint32_t), st));
    RT_HIP(rt::launch_coo_check(X->idx, X->nnz, X->nnz, coo_dims(dims), status, 1u, st));
    RT_HIP(hipMemsetAsync(Y, 0, (size_t)dims[mode] * ell * sizeof(double), st));
    {
        TimeScope ts(k.c, 0, (double)X->nnz * (X->ndim * 4.0 + dsize(X->dtype)), 2.0 * ell * X->nnz, dims[mode],
                     X->nnz, ell);
        ts.t.variant = RT_SKETCH_COO;
        RT_TRY(coo_sketch_input(k, X->idx, X->vals, dt, X->nnz, coo_dims(dims), mode, ell, col0, seed, Y));
    }
    if (nrm2) {
        if (X->nnz > 0) RT_TRY(do_norm2(k, X->vals, dt, X->nnz, nrm2));
        else RT_HIP(hipMemsetAsync(nrm2, 0, sizeof(double), st));
    }
    uint32_t* h = (uint32_t*)ctx->host;
    RT_HIP(hipMemcpyAsync(h, status, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    RT_HIP(hipStreamSynchronize(st));
    if (h[0]) return fail(RT_EINVAL, "sparse input has a coordinate out of range (those entries were skipped)");
    return RT_OK;
}

rt_status rt_tuning_set(const rt_tune_entry* entries, int32_t n) {
    if (n < 0 || (n > 0 && !entries)) return fail(RT_EINVAL, "entries is NULL or n < 0");
    for (int32_t i = 0; i < n; ++i) {
        const rt_tune_entry& e = entries[i];
        if (e.op != RT_TUNE_SKETCH || (e.dtype != RT_F32 && e.dtype != RT_F64) || e.prec < RT_PREC_F64 ||
            e.prec > RT_PREC_BF16_SKETCH || e.stride < RT_STRIDE_FIRST || e.stride > RT_STRIDE_LAST ||
            e.j_lo > e.j_hi || e.k_lo > e.k_hi || e.ell_lo > e.ell_hi || e.wgs < 0 || e.wgs > (1 << 20) ||
            (e.kind != RT_SKETCH_GENERIC && e.kind != RT_SKETCH_MFMA_F32 && e.kind != RT_SKETCH_SPLIT_BF16 &&
             e.kind != RT_SKETCH_BF16X3))
            return fail(RT_EINVAL, "tile table entry " + std::to_string(i) + " is malformed");
    }
    return rt::tuning_set(entries, n);
}

rt_status rt_tuning_plan(rt_dtype dtype, rt_precision prec, const int64_t* dims, int32_t ndim, int32_t mode,
                         int32_t ell, rt_tune_entry* out, int32_t* from_table) {
    if (!dims || !out) return fail(RT_EINVAL, "NULL argument");
    if (ndim < 2 || ndim > RT_MAXD || mode < 0 || mode >= ndim) return fail(RT_EINVAL, "bad ndim or mode");
    if (ell < 1 || ell > RT_LMAX) return fail(RT_EINVAL, "ell must be in [1, RT_LMAX]");
    if (dtype != RT_F32 && dtype != RT_F64) return fail(RT_EINVAL, "dtype must be RT_F32 or RT_F64");
    std::vector<int64_t> d(dims, dims + ndim);
    for (auto v : d)
        if (v < 1) return fail(RT_EINVAL, "every dim must be >= 1");
    const Shape3 s = shape3(d, mode);
    bool tab = false;
    alignas(256) static const double aligned_probe[2] = {0.0, 0.0};   // stands for aligned data
    const rt::SketchPlan p = rt::plan_sketch_info(dt_of(dtype), (int)prec, s, ell, 0, aligned_probe, true, &tab);
    std::memset(out, 0, sizeof(*out));
    out->op = RT_TUNE_SKETCH;
    out->dtype = dtype;
    out->prec = prec;
    out->stride = rt::stride_class(s);
    out->j_lo = out->j_hi = s.J;
    out->k_lo = out->k_hi = s.L * s.R;
    out->ell_lo = out->ell_hi = ell;
    out->kind = p.kind;
    out->rb = p.rb;
    out->rw = p.rw;
    out->wgs = p.nwg;
    if (from_table) *from_table = tab ? 1 : 0;
    return RT_OK;
}

rt_status rt_orth(rt_ctx* ctx, double* Y, int64_t rows, int32_t ell, uint32_t* flags) {
    if (!ctx || !Y) return fail(RT_EINVAL, "NULL argument");
    if (ell < 1 || ell > RT_LMAX || rows < ell) return fail(RT_EINVAL, "need 1 <= ell <= min(rows, RT_LMAX)");
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    double* scratch = k.ws<double>(rt::orth_scratch(rows, ell));
    uint32_t* st = k.ws<uint32_t>(1);
    if (!scratch || !st) return fail(RT_ENOMEM, "workspace allocation failed");
    RT_HIP(rt::launch_orth(Y, rows, ell, nullptr, orth_accept_ratio(), st, scratch, ctx->stream));
    uint32_t* h = (uint32_t*)ctx->host;
    RT_HIP(hipMemcpyAsync(h, st, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    RT_HIP(hipStreamSynchronize(ctx->stream));
    if (flags) *flags = h[0] & 3u;
    if (h[0] & 4u) return fail(RT_ENONFINITE, "Y holds NaN or Inf");
    return RT_OK;
}

rt_status rt_project(rt_ctx* ctx, const rt_tensor* X, int32_t mode, const void* Q, rt_dtype qtype, int32_t ell,
                     void* B, double* gram) {
    if (!ctx || !Q || !B) return fail(RT_EINVAL, "NULL argument");
    RT_TRY(check_tensor(X));
    if (mode < 0 || mode >= X->ndim) return fail(RT_EINVAL, "mode out of range");
    if (ell < 1 || ell > RT_LMAX) return fail(RT_EINVAL, "ell must be in [1, RT_LMAX]");
    if (X->dtype == RT_F64 && qtype != RT_F64) return fail(RT_EINVAL, "an RT_F64 tensor needs an RT_F64 Q");
    RT_HIP(hipSetDevice(ctx->device));
    Call k(ctx);
    std::vector<int64_t> dims(X->dims, X->dims + X->ndim);
    Shape3 s = shape3(dims, mode);
    RT_TRY(do_project(k, dt_of(X->dtype), dt_of(qtype), X->data, s, s.J, Q, ell, ell, B, ell, 0, gram, nullptr));
    RT_HIP(hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

rt_status rt_omega(rt_ctx* ctx, uint64_t seed, int32_t mode, int64_t c0, int64_t nrows, int64_t col0, int32_t ncols,
                   rt_dtype dtype, void* out) {
    if (!ctx || !out) return fail(RT_EINVAL, "NULL argument");
    if (c0 < 0 || nrows < 0 || col0 < 0 || ncols < 0 || mode < 0) return fail(RT_EINVAL, "negative argument");
    RT_HIP(hipSetDevice(ctx->device));
    RT_HIP(rt::launch_omega(seed, (uint32_t)mode, c0, nrows, col0, ncols, out, dt_of(dtype), ctx->stream));
    RT_HIP(hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

rt_status rt_philox_words(rt_ctx* ctx, uint64_t seed, int32_t mode, int64_t c0, int64_t n, uint32_t q, uint32_t* out) {
    if (!ctx || !out) return fail(RT_EINVAL, "NULL argument");
    if (c0 < 0 || n < 0 || mode < 0) return fail(RT_EINVAL, "negative argument");
    RT_HIP(hipSetDevice(ctx->device));
    RT_HIP(rt::launch_philox_words(seed, (uint32_t)mode, c0, n, q, out, ctx->stream));
    RT_HIP(hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

}  // extern "C"
