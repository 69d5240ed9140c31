// Serving: a request loop that admits float32 tensors of uneven shapes by
// device-memory footprint and keeps many of them in flight, running adaptive
// R-STHOSVD (Alg. 5, §4) with a common tolerance.
//
// Grouped mode (the default): one executor thread drives all admitted requests
// through the method in lock-step iterations.  Each request is a small state
// machine (mode, block loop or truncation, error indicator E, tolerance);
// every iteration the executor writes one descriptor per request into a pinned
// buffer and replays one captured HIP graph: the descriptor copy, then grouped
// launches of the block sketch, its sums, the block orthonormalisation and the
// projection for the requests in a block loop, and of the Gram, the
// eigensolver with rank choice and factor, and the core update for the
// requests whose mode stopped growing (rt_group.hip, the grouped kernels of
// rt_sketch.hip and rt_dense.hip).  The scalars each request needs (kept
// columns, ||B_i||^2, ||X||^2, chosen rank, ||G'||^2) come back through mapped
// pinned slots; after one wait the host applies the same decisions as the
// single-request driver (rtucker.cpp, adaptive_impl) and admits new requests.
// Device memory comes from an arena pool; a request is admitted when its exact
// footprint fits the budget.
//
// Slots mode: each slot thread takes whole requests and runs them through
// rt_rsthosvd_adaptive on a stream of its own (the pipelines overlap on the
// device).  Its blocks are reused rather than freed, because freeing device
// memory synchronises the whole device and would stall the other slots.
//
// Results are copied to host memory owned by the server until the caller
// releases them.
#include <hip/hip_runtime.h>

#include <chrono>
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rt_kernels.hpp"
#include "rtucker.h"

namespace {

using Clock = std::chrono::steady_clock;

// Device blocks of one slot, kept for reuse until the server is destroyed.
struct BlockCache {
    std::multimap<size_t, void*> free_blocks;
    std::unordered_map<void*, size_t> sizes;

    static size_t round_up(size_t b) {
        if (b <= (size_t(1) << 20)) {
            size_t r = 4096;
            while (r < b) r <<= 1;
            return r;
        }
        const size_t mb = size_t(1) << 20;
        return (b + mb - 1) / mb * mb;
    }
    void* get(size_t bytes) {
        const size_t sz = round_up(bytes ? bytes : 1);
        auto it = free_blocks.lower_bound(sz);
        if (it != free_blocks.end() && it->first <= 2 * sz) {
            void* p = it->second;
            free_blocks.erase(it);
            return p;
        }
        void* p = nullptr;
        if (hipMalloc(&p, sz) != hipSuccess) return nullptr;
        sizes[p] = sz;
        return p;
    }
    void put(void* p) {
        auto it = sizes.find(p);
        if (it != sizes.end()) free_blocks.emplace(it->second, p);
    }
    void clear() {
        for (auto& kv : sizes) (void)hipFree(kv.first);
        sizes.clear();
        free_blocks.clear();
    }
};

void* cache_alloc(size_t bytes, void* user) { return static_cast<BlockCache*>(user)->get(bytes); }
void cache_free(void* p, void* user) { static_cast<BlockCache*>(user)->put(p); }

struct Request {
    uint64_t id = 0;
    bool decompress = false;         // rt_server_submit_reconstruct
    rt_tucker_host T{};              // its input
    float* out = nullptr;            // and output (host)
    rt_tensor X{};
    uint64_t seed = 0;
    size_t footprint = 0;
    Clock::time_point t_submit, t_admit, t_done;
    bool done = false;
    rt_result res{};
    std::string err;
    std::vector<float> core;
    std::vector<std::vector<float>> factors;
};

int64_t numel(const rt_tensor& X) {
    int64_t n = 1;
    for (int i = 0; i < X.ndim; ++i) n *= X.dims[i];
    return n;
}

}  // namespace

struct rt_server {
    int device = 0;
    rt_server_opts opts{};
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_done;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, Request*> reqs;
    uint64_t next_id = 1;
    size_t in_use = 0;
    int in_flight = 0;
    bool stopping = false;
    std::vector<std::thread> threads;
    std::vector<std::string> slot_errors;
    rt_server_stats stats{};

    bool admissible(const Request* r) const { return in_flight == 0 || in_use + r->footprint <= budget; }
    void slot_main(int slot);
    void run(Request* r, rt_ctx* ctx, hipStream_t st, BlockCache& cache, float*& dX, size_t& dX_cap,
             float*& stage, size_t& stage_cap);
    void run_decompress(Request* r, rt_ctx* ctx, hipStream_t st, BlockCache& cache);
    void complete(Request* r);
    void exec_main();
};

// Marks a request done (results in its host vectors) and wakes its waiters.
void rt_server::complete(Request* r) {
    {
        std::lock_guard<std::mutex> lk(mu);
        in_use -= r->footprint;
        --in_flight;
        r->t_done = Clock::now();
        r->res.queue_s = std::chrono::duration<double>(r->t_admit - r->t_submit).count();
        r->res.latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        r->res.core = r->core.empty() ? nullptr : r->core.data();
        for (int i = 0; i < RT_MAXD; ++i)
            r->res.factors[i] = (i < (int)r->factors.size() && !r->factors[i].empty()) ? r->factors[i].data() : nullptr;
        r->done = true;
        ++stats.completed;
    }
    cv_done.notify_all();
    cv_work.notify_all();
}

// A decompression on the context's stream: the core and factors up, rt_reconstruct,
// X_hat down into the caller's buffer (device buffers from the block cache).
void rt_server::run_decompress(Request* r, rt_ctx* ctx, hipStream_t st, BlockCache& cache) {
    const rt_tucker_host& T = r->T;
    rt_result& res = r->res;
    res.ndim = T.ndim;
    int64_t ncore = 1, nout = 1;
    for (int i = 0; i < T.ndim; ++i) {
        res.dims[i] = T.dims[i];
        res.ranks[i] = T.ranks[i];
        ncore *= T.ranks[i];
        nout *= T.dims[i];
    }
    std::vector<void*> bufs;
    bool nomem = false;
    auto get = [&](int64_t n) -> float* {
        void* p = cache.get((size_t)std::max<int64_t>(n, 1) * sizeof(float));
        if (p) bufs.push_back(p);
        else nomem = true;
        return static_cast<float*>(p);
    };
    rt_tucker d{};
    d.ndim = T.ndim;
    d.dtype = RT_F32;
    bool ok = true;
    float* dc = get(ncore);
    float* dout = get(nout);
    ok = dc && dout;
    if (ok && ncore > 0) ok = hipMemcpyAsync(dc, T.core, (size_t)ncore * 4, hipMemcpyHostToDevice, st) == hipSuccess;
    d.core = dc;
    for (int i = 0; i < T.ndim && ok; ++i) {
        d.dims[i] = T.dims[i];
        d.ranks[i] = T.ranks[i];
        if (T.factors[i]) {
            float* f = get(T.dims[i] * (int64_t)T.ranks[i]);
            ok = f && hipMemcpyAsync(f, T.factors[i], (size_t)T.dims[i] * T.ranks[i] * 4, hipMemcpyHostToDevice,
                                     st) == hipSuccess;
            d.factors[i] = f;
        }
    }
    if (!ok) {
        res.status = nomem ? RT_ENOMEM : RT_EHIP;
        r->err = "device buffers or copies for the decompression failed";
    } else {
        const rt_status s = rt_reconstruct(ctx, &d, dout);
        if (s != RT_OK) {
            res.status = s;
            r->err = rt_last_error();
        } else if (hipMemcpyAsync(r->out, dout, (size_t)nout * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                   hipStreamSynchronize(st) != hipSuccess) {
            res.status = RT_EHIP;
            r->err = "device to host copy failed";
        } else {
            res.status = RT_OK;
        }
    }
    (void)hipStreamSynchronize(st);
    for (void* p : bufs) cache.put(p);
}

void rt_server::run(Request* r, rt_ctx* ctx, hipStream_t st, BlockCache& cache, float*& dX, size_t& dX_cap,
                    float*& stage, size_t& stage_cap) {
    if (r->decompress) {
        run_decompress(r, ctx, st, cache);
        return;
    }
    const int64_t n = numel(r->X);
    rt_result& res = r->res;
    res.ndim = r->X.ndim;
    for (int i = 0; i < r->X.ndim; ++i) res.dims[i] = r->X.dims[i];
    if ((size_t)n > dX_cap) {
        if (dX) cache.put(dX);
        dX = static_cast<float*>(cache.get((size_t)n * sizeof(float)));
        dX_cap = dX ? (size_t)n : 0;
        if (!dX) { res.status = RT_ENOMEM; r->err = "device allocation failed"; return; }
    }
    if (hipMemcpyAsync(dX, r->X.data, (size_t)n * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess) {
        res.status = RT_EHIP; r->err = "host to device copy failed"; return;
    }
    rt_tensor Xd = r->X;
    Xd.data = dX;
    rt_opts o{};
    o.oversample = 0;
    o.seed = r->seed;
    o.order = nullptr;
    o.prec = opts.prec;
    rt_tucker out{};
    rt_status s = rt_rsthosvd_adaptive(ctx, &Xd, opts.eps, nullptr, opts.block, nullptr, &o, &out);
    res.status = s;
    if (s != RT_OK && s != RT_ECAP) { r->err = rt_last_error(); return; }
    // results to host: core, then the factors, through one page-locked staging buffer
    int64_t ncore = 1;
    for (int i = 0; i < out.ndim; ++i) ncore *= out.ranks[i];
    std::vector<int64_t> nf(out.ndim, 0);
    int64_t total = ncore;
    for (int i = 0; i < out.ndim; ++i) {
        nf[i] = out.factors[i] ? out.dims[i] * (int64_t)out.ranks[i] : 0;
        total += nf[i];
    }
    if ((size_t)total > stage_cap) {
        if (stage) (void)hipHostFree(stage);
        stage = nullptr;
        stage_cap = 0;
        if (hipHostMalloc((void**)&stage, (size_t)total * sizeof(float), hipHostMallocDefault) != hipSuccess) {
            res.status = RT_ENOMEM; r->err = "page-locked host allocation failed";
            rt_tucker_release(ctx, &out);
            return;
        }
        stage_cap = (size_t)total;
    }
    bool ok = hipMemcpyAsync(stage, out.core, (size_t)ncore * sizeof(float), hipMemcpyDeviceToHost, st) == hipSuccess;
    int64_t off = ncore;
    for (int i = 0; i < out.ndim; ++i) {
        if (nf[i] > 0)
            ok = ok && hipMemcpyAsync(stage + off, out.factors[i], (size_t)nf[i] * sizeof(float),
                                      hipMemcpyDeviceToHost, st) == hipSuccess;
        off += nf[i];
    }
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        res.status = RT_EHIP; r->err = "device to host copy failed";
        rt_tucker_release(ctx, &out);
        return;
    }
    r->core.assign(stage, stage + ncore);
    r->factors.assign(out.ndim, std::vector<float>());
    off = ncore;
    for (int i = 0; i < out.ndim; ++i) {
        r->factors[i].assign(stage + off, stage + off + nf[i]);
        off += nf[i];
    }
    for (int i = 0; i < out.ndim; ++i) res.ranks[i] = out.ranks[i];
    res.norm_x = out.norm_x;
    res.core_norm = out.core_norm;
    res.rel_err_est = out.rel_err_est;
    res.flags = out.flags;
    rt_tucker_release(ctx, &out);
}

void rt_server::slot_main(int slot) {
    BlockCache cache;
    hipStream_t st = nullptr;
    rt_ctx* ctx = nullptr;
    // a slot that cannot be set up still drains its share of the queue, failing each request
    const bool ready = hipSetDevice(device) == hipSuccess &&
                       hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
                       rt_create(&ctx, device, st, cache_alloc, cache_free, &cache) == RT_OK;
    if (!ready) {
        std::lock_guard<std::mutex> lk(mu);
        slot_errors[slot] = "slot set-up failed";
    }
    float* dX = nullptr;
    size_t dX_cap = 0;
    float* stage = nullptr;
    size_t stage_cap = 0;
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return (!queue.empty() && admissible(queue.front())) || (stopping && queue.empty()); });
            if (queue.empty()) break;
            r = queue.front();
            queue.pop_front();
            in_use += r->footprint;
            ++in_flight;
            r->t_admit = Clock::now();
            if (!queue.empty()) cv_work.notify_one();
        }
        if (ready) {
            run(r, ctx, st, cache, dX, dX_cap, stage, stage_cap);
        } else {
            r->res.status = RT_EHIP;
            r->err = "slot set-up failed";
        }
        complete(r);
    }
    if (st) (void)hipStreamSynchronize(st);
    if (dX) cache.put(dX);
    if (ctx) rt_destroy(ctx);
    if (stage) (void)hipHostFree(stage);
    cache.clear();
    if (st) (void)hipStreamDestroy(st);
}

// ---- grouped mode ------------------------------------------------------------------------
namespace {

constexpr size_t MIB = size_t(1) << 20;
size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// Device memory of the grouped executor: chunks of at least 256 MiB, request
// arenas placed first-fit in their free segments and merged back when freed.
struct ArenaPool {
    struct Chunk { char* base; size_t size; std::map<size_t, size_t> free; };
    std::vector<Chunk> chunks;
    size_t reserved = 0;
    void* get(size_t bytes, size_t limit) {
        bytes = (bytes + MIB - 1) / MIB * MIB;
        for (auto& c : chunks)
            for (auto it = c.free.begin(); it != c.free.end(); ++it)
                if (it->second >= bytes) {
                    const size_t off = it->first, sz = it->second;
                    c.free.erase(it);
                    if (sz > bytes) c.free[off + bytes] = sz - bytes;
                    return c.base + off;
                }
        const size_t csz = std::max(bytes, size_t(256) * MIB);
        if (reserved + csz > limit && !chunks.empty()) return nullptr;
        void* p = nullptr;
        if (hipMalloc(&p, csz) != hipSuccess) return nullptr;
        Chunk c{(char*)p, csz, {}};
        if (csz > bytes) c.free[bytes] = csz - bytes;
        chunks.push_back(c);
        reserved += csz;
        return p;
    }
    void put(void* p, size_t bytes) {
        bytes = (bytes + MIB - 1) / MIB * MIB;
        for (auto& c : chunks) {
            if ((char*)p < c.base || (char*)p >= c.base + c.size) continue;
            size_t off = (char*)p - c.base, sz = bytes;
            auto nx = c.free.lower_bound(off);
            if (nx != c.free.end() && off + sz == nx->first) { sz += nx->second; nx = c.free.erase(nx); }
            if (nx != c.free.begin()) {
                auto pv = std::prev(nx);
                if (pv->first + pv->second == off) { off = pv->first; sz += pv->second; c.free.erase(pv); }
            }
            c.free[off] = sz;
            return;
        }
    }
    void clear() {
        for (auto& c : chunks) (void)hipFree(c.base);
        chunks.clear();
        reserved = 0;
    }
};

// Per-request state of the grouped executor.
struct GState {
    Request* r = nullptr;
    int slot = -1;
    char* arena = nullptr;
    size_t bytes = 0;
    int d = 0;
    int64_t dims[RT_MAXD] = {}, cdims[RT_MAXD] = {};
    int order[RT_MAXD] = {};
    int mi = 0;
    const float* cur = nullptr;
    float* core[2] = {nullptr, nullptr};
    int pp = 0;
    float* fac[RT_MAXD] = {};
    int ranks[RT_MAXD] = {};
    char* scratch = nullptr;
    float* B = nullptr;
    // the mode being processed
    int n = -1;
    int64_t L = 0, J = 0, R = 0;
    int cap = 0, nsplit = 0, nrowtile = 0, nchunk = 0;
    int64_t tps = 0;
    int kcols = 0, blk = 0, bi = 0;
    double E = 0.0, tau2 = 0.0, nx2 = 0.0, cur_norm2 = 0.0;
    bool have_norm = false, capped = false;
    bool rerun = false;       // needs more than RT_LMAX basis columns: redone alone
    enum Phase { BLOCK, TRUNC, DONE } phase = BLOCK;
    hipEvent_t ev = nullptr;  // completion of the input copy, then of the result copy
    int cs = 0;               // copy stream of both copies (stream order keeps them apart)
    int64_t ncore = 0;        // result: core entries (staged first, then the factors)
    // scratch views of the mode
    float* partial = nullptr;
    double* nrm_partial = nullptr;
    double* Y = nullptr;
    double* Qall = nullptr;
    float* Qallf = nullptr;
    double* bnrm = nullptr;
    double* gpart = nullptr;
    float* Uf = nullptr;
    int* ints = nullptr;
    double* cnrm = nullptr;
};

// Sizes of one mode's scratch (bytes) for current dims `cd`; optionally lays
// the views out from `base`.
size_t mode_scratch(GState* s, const int64_t* cd, int d, int n, int block, char* base) {
    int64_t L = 1, R = 1;
    for (int i = 0; i < n; ++i) L *= cd[i];
    for (int i = n + 1; i < d; ++i) R *= cd[i];
    const int64_t J = cd[n], K = L * R;
    const int cap = (int)std::min<int64_t>(std::min<int64_t>(J, K), RT_LMAX);
    int nsplit = 1, nrowtile = 1;
    int64_t tps = 1;
    rt::group_sketch_plan(L, J, R, block, nsplit, nrowtile, tps);
    const int64_t nct = (K + 255) / 256;
    const int nchunk = rt::group_gram_chunks(K);
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += al256(bytes); return base ? base + o : nullptr; };
    char* partial = take((size_t)nsplit * J * block * 4);
    char* nrm = take((size_t)nsplit * nrowtile * 8);
    char* Y = take((size_t)J * block * 8);
    char* Qall = take((size_t)J * cap * 8);
    char* Qallf = take((size_t)J * cap * 4);
    char* bnrm = take((size_t)nct * ((block + 7) / 8) * 8);
    char* gpart = take((size_t)nchunk * cap * cap * 8);
    char* Uf = take((size_t)cap * cap * 4);
    char* ints = take(64);
    char* cnrm = take((size_t)nct * ((cap + 7) / 8) * 8);
    if (base && s) {
        s->L = L; s->J = J; s->R = R; s->cap = cap;
        s->nsplit = nsplit; s->nrowtile = nrowtile; s->tps = tps; s->nchunk = nchunk;
        s->partial = (float*)partial; s->nrm_partial = (double*)nrm; s->Y = (double*)Y;
        s->Qall = (double*)Qall; s->Qallf = (float*)Qallf; s->bnrm = (double*)bnrm;
        s->gpart = (double*)gpart; s->Uf = (float*)Uf; s->ints = (int*)ints; s->cnrm = (double*)cnrm;
    }
    return off;
}

// Footprint of a request (bytes) and whether the grouped kernels serve it: the
// input, the largest mode scratch, B and two cores at the largest (L, cap, R),
// and the factors, with every rank bounded by its cap.
bool group_footprint(const rt_tensor& X, int block, size_t& bytes, size_t& scratch, size_t& big) {
    const int d = X.ndim;
    int64_t cd[RT_MAXD];
    int order[RT_MAXD];
    for (int i = 0; i < d; ++i) { cd[i] = X.dims[i]; order[i] = i; }
    std::stable_sort(order, order + d, [&](int a, int b) { return X.dims[a] > X.dims[b]; });
    int64_t N = 1;
    for (int i = 0; i < d; ++i) N *= cd[i];
    bool ok = block <= 16;
    scratch = 0;
    big = 0;
    size_t fac = 0;
    for (int m = 0; m < d; ++m) {
        const int n = order[m];
        int64_t L = 1, R = 1;
        for (int i = 0; i < n; ++i) L *= cd[i];
        for (int i = n + 1; i < d; ++i) R *= cd[i];
        const int64_t J = cd[n];
        const int cap = (int)std::min<int64_t>(std::min<int64_t>(J, L * R), RT_LMAX);
        if (J > rt::group_block_maxj(block)) ok = false;
        scratch = std::max(scratch, mode_scratch(nullptr, cd, d, n, block, nullptr));
        big = std::max(big, al256((size_t)L * cap * R * 4));
        fac += al256((size_t)J * std::max(cap, 1) * 4);
        cd[n] = cap;
    }
    bytes = al256((size_t)N * 4) + scratch + 3 * big + fac;
    return ok;
}

}  // namespace

void rt_server::exec_main() {
    const int maxreq = opts.max_inflight;
    const int block = opts.block;
    hipStream_t st = nullptr;
    char* desc_host = nullptr;
    char* desc_dev = nullptr;
    rt::GRead* rb_host = nullptr;
    rt::GRead* rb_dev = nullptr;
    float* stage = nullptr;
    size_t stage_cap = 0;
    const size_t dbytes = rt::group_desc_bytes(maxreq);
    // a request the grouped kernels do not serve runs alone on a context of its own
    BlockCache cache;
    rt_ctx* ctx = nullptr;
    float* dX = nullptr;
    size_t dX_cap = 0;
    hipStream_t cst[2] = {nullptr, nullptr};   // copy streams (inputs in, results out)
    int ccur = 0;
    std::vector<hipEvent_t> evpool;
    std::vector<float*> sstage(maxreq, nullptr);   // pinned result staging per slot
    std::vector<size_t> scap(maxreq, 0);
    bool ready = hipSetDevice(device) == hipSuccess &&
                 hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
                 hipStreamCreateWithFlags(&cst[0], hipStreamNonBlocking) == hipSuccess &&
                 hipStreamCreateWithFlags(&cst[1], hipStreamNonBlocking) == hipSuccess &&
                 hipHostMalloc((void**)&desc_host, dbytes, hipHostMallocDefault) == hipSuccess &&
                 hipMalloc((void**)&desc_dev, dbytes) == hipSuccess &&
                 hipHostMalloc((void**)&rb_host, sizeof(rt::GRead) * maxreq, hipHostMallocMapped) == hipSuccess &&
                 hipHostGetDevicePointer((void**)&rb_dev, rb_host, 0) == hipSuccess &&
                 rt_create(&ctx, device, st, cache_alloc, cache_free, &cache) == RT_OK;
    if (ready) std::memset(desc_host, 0, dbytes);
    ArenaPool pool;
    std::vector<GState*> active;
    std::vector<GState*> pending, draining;   // input copy issued / result copy issued
    auto get_event = [&]() -> hipEvent_t {
        if (!evpool.empty()) { hipEvent_t e = evpool.back(); evpool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    };
    std::vector<int> free_slots;
    for (int i = maxreq - 1; i >= 0; --i) free_slots.push_back(i);
    hipGraphExec_t gexec = nullptr;
    bool graph_ok = true;
    const char* dp = desc_host;
    rt::GHeader* hdr = (rt::GHeader*)dp;
    dp += al256(sizeof(rt::GHeader));
    rt::GBlock* gblk = (rt::GBlock*)dp;
    dp += al256(sizeof(rt::GBlock) * maxreq);
    rt::GProj* gbproj = (rt::GProj*)dp;
    dp += al256(sizeof(rt::GProj) * maxreq);
    rt::GTrunc* gtr = (rt::GTrunc*)dp;
    dp += al256(sizeof(rt::GTrunc) * maxreq);
    rt::GProj* gcproj = (rt::GProj*)dp;

    auto fail = [&](GState* g, rt_status stt, const char* msg) {
        g->r->res.status = stt;
        g->r->err = msg;
        g->phase = GState::DONE;
    };
    // the next mode of a request (or done); modes whose core has no entries, or
    // whose core is already within the tolerance, take rank 0 without work
    auto next_mode = [&](GState* g) {
        for (;;) {
            if (g->mi >= g->d) { g->phase = GState::DONE; return; }
            const int n = g->order[g->mi];
            int64_t N = 1;
            for (int i = 0; i < g->d; ++i) N *= g->cdims[i];
            if (N == 0 || (g->have_norm && !(g->cur_norm2 > g->tau2))) {
                g->ranks[n] = 0;
                g->cdims[n] = 0;
                g->cur_norm2 = 0.0;
                ++g->mi;
                continue;
            }
            g->n = n;
            mode_scratch(g, g->cdims, g->d, n, block, g->scratch);
            g->kcols = 0;
            g->blk = 0;
            g->E = g->cur_norm2;
            g->phase = GState::BLOCK;
            return;
        }
    };
    auto end_blocks = [&](GState* g) {
        if (g->kcols > 0) { g->phase = GState::TRUNC; return; }
        g->ranks[g->n] = 0;
        g->cdims[g->n] = 0;
        g->cur_norm2 = 0.0;
        ++g->mi;
        next_mode(g);
    };
    auto admit = [&](Request* r) -> bool {      // false: wait for memory
        size_t bytes = 0, scratch = 0, big = 0;
        group_footprint(r->X, block, bytes, scratch, big);
        GState* g = new GState();
        g->arena = (char*)pool.get(bytes, budget);
        if (!g->arena) { delete g; return false; }
        g->r = r;
        g->bytes = bytes;
        g->slot = free_slots.back();
        free_slots.pop_back();
        g->d = r->X.ndim;
        for (int i = 0; i < g->d; ++i) { g->dims[i] = g->cdims[i] = r->X.dims[i]; g->order[i] = i; }
        std::stable_sort(g->order, g->order + g->d, [&](int a, int b) { return g->dims[a] > g->dims[b]; });
        int64_t N = 1;
        for (int i = 0; i < g->d; ++i) N *= g->dims[i];
        char* p = g->arena;
        float* X = (float*)p;
        p += al256((size_t)N * 4);
        g->scratch = p;
        p += scratch;
        g->B = (float*)p;
        p += big;
        g->core[0] = (float*)p;
        p += big;
        g->core[1] = (float*)p;
        p += big;
        int64_t cd[RT_MAXD];
        for (int i = 0; i < g->d; ++i) cd[i] = g->dims[i];
        for (int m = 0; m < g->d; ++m) {
            const int n = g->order[m];
            int64_t K = 1;
            for (int i = 0; i < g->d; ++i) if (i != n) K *= cd[i];
            const int cap = (int)std::min<int64_t>(std::min<int64_t>(cd[n], K), RT_LMAX);
            g->fac[n] = (float*)p;
            p += al256((size_t)cd[n] * std::max(cap, 1) * 4);
            cd[n] = cap;
        }
        r->res.ndim = g->d;
        for (int i = 0; i < g->d; ++i) r->res.dims[i] = g->dims[i];
        r->res.status = RT_OK;
        // the input crosses on a copy stream while the current iteration computes;
        // the request joins the iteration after (or at once when none is running)
        g->cs = ccur;
        hipStream_t cs = cst[ccur];
        ccur ^= 1;
        g->ev = get_event();
        if (!g->ev || hipMemcpyAsync(X, r->X.data, (size_t)N * 4, hipMemcpyHostToDevice, cs) != hipSuccess ||
            hipEventRecord(g->ev, cs) != hipSuccess)
            fail(g, RT_EHIP, "host to device copy failed");
        g->cur = X;
        g->mi = 0;
        if (g->phase != GState::DONE) next_mode(g);
        pending.push_back(g);
        return true;
    };
    // results: core and factors copied into the slot's pinned staging on a copy
    // stream; the request completes once that copy is done (complete_drain)
    auto start_drain = [&](GState* g) {
        Request* r = g->r;
        if (r->res.status == RT_OK || r->res.status == RT_ECAP) {
            int64_t ncore = 1;
            for (int i = 0; i < g->d; ++i) ncore *= g->cdims[i];
            g->ncore = ncore;
            int64_t total = ncore;
            for (int i = 0; i < g->d; ++i) total += g->dims[i] * g->ranks[i];
            bool ok = true;
            float*& stg = sstage[g->slot];
            if ((size_t)total > scap[g->slot]) {
                if (stg) (void)hipHostFree(stg);
                stg = nullptr;
                scap[g->slot] = 0;
                ok = hipHostMalloc((void**)&stg, (size_t)std::max<int64_t>(total, 1) * 4, hipHostMallocDefault) ==
                     hipSuccess;
                if (ok) scap[g->slot] = (size_t)std::max<int64_t>(total, 1);
            }
            // the iteration that produced the result has been waited for, and the
            // request's own input copy went down the same copy stream before
            hipStream_t cs = cst[g->cs];
            if (!g->ev) g->ev = get_event();
            ok = ok && g->ev;
            if (ok && ncore > 0)
                ok = hipMemcpyAsync(stg, g->cur, (size_t)ncore * 4, hipMemcpyDeviceToHost, cs) == hipSuccess;
            int64_t off = ncore;
            for (int i = 0; i < g->d && ok; ++i) {
                const int64_t nf = g->dims[i] * g->ranks[i];
                if (nf > 0)
                    ok = hipMemcpyAsync(stg + off, g->fac[i], (size_t)nf * 4, hipMemcpyDeviceToHost, cs) == hipSuccess;
                off += nf;
            }
            ok = ok && hipEventRecord(g->ev, cs) == hipSuccess;
            if (!ok) {
                r->res.status = RT_EHIP;
                r->err = "device to host copy failed";
            }
        }
        draining.push_back(g);
    };
    auto complete_drain = [&](GState* g) {
        Request* r = g->r;
        if (r->res.status == RT_OK || r->res.status == RT_ECAP) {
            const float* stg = sstage[g->slot];
            const int64_t ncore = g->ncore;
            r->core.assign(stg, stg + ncore);
            r->factors.assign(g->d, std::vector<float>());
            int64_t off = ncore;
            for (int i = 0; i < g->d; ++i) {
                const int64_t nf = g->dims[i] * g->ranks[i];
                r->factors[i].assign(stg + off, stg + off + nf);
                off += nf;
                r->res.ranks[i] = g->ranks[i];
            }
            r->res.norm_x = std::sqrt(std::max(g->nx2, 0.0));
            r->res.core_norm = std::sqrt(std::max(g->cur_norm2, 0.0));
            r->res.rel_err_est = r->res.norm_x > 0 ? std::sqrt(std::max(0.0, g->nx2 - g->cur_norm2)) / r->res.norm_x
                                                   : 0.0;
            r->res.flags = 0;
            if (g->capped) {
                r->res.status = RT_ECAP;
                r->err = "a mode reached its rank cap before the tolerance";
            }
        }
        if (g->ev) evpool.push_back(g->ev);
        pool.put(g->arena, g->bytes);
        free_slots.push_back(g->slot);
        delete g;
    };
    // completes every drained request whose copy has finished (all of them when wait)
    auto poll_drains = [&](bool wait) {
        for (size_t i = 0; i < draining.size();) {
            GState* g = draining[i];
            const bool done = !g->ev || (wait ? hipEventSynchronize(g->ev) == hipSuccess
                                              : hipEventQuery(g->ev) != hipErrorNotReady);
            if (done) {
                Request* r = g->r;
                const bool rerun = g->rerun;
                draining.erase(draining.begin() + i);
                complete_drain(g);
                if (rerun) {
                    r->err.clear();
                    run(r, ctx, st, cache, dX, dX_cap, stage, stage_cap);
                }
                complete(r);
            } else {
                ++i;
            }
        }
    };

    const double eps_n_base = opts.eps;
    using Sec = std::chrono::duration<double>;
    std::vector<GState*> finished;   // done at the last readback, results not yet copied out
    // admission: arrival order, while a slot is free and the footprint fits;
    // may_wait: block for work when nothing at all is in flight
    auto admit_queue = [&](bool may_wait) {
        for (;;) {
            Request* r = nullptr;
            bool alone = false;
            {
                std::unique_lock<std::mutex> lk(mu);
                if (may_wait && active.empty() && pending.empty() && draining.empty() && finished.empty())
                    cv_work.wait(lk, [&] { return !queue.empty() || stopping; });
                if (queue.empty() || free_slots.empty()) break;
                Request* h = queue.front();
                size_t bytes = 0, scratch = 0, big = 0;
                alone = h->decompress || !group_footprint(h->X, block, bytes, scratch, big);
                const bool busy = !active.empty() || !pending.empty();
                if (!alone && busy && in_use + bytes > budget) break;
                queue.pop_front();
                h->footprint = alone ? 0 : bytes;
                in_use += h->footprint;
                ++in_flight;
                h->t_admit = Clock::now();
                r = h;
            }
            if (!ready) {
                r->res.status = RT_EHIP;
                r->err = "executor set-up failed";
                complete(r);
                continue;
            }
            if (alone) {
                run(r, ctx, st, cache, dX, dX_cap, stage, stage_cap);
                complete(r);
                continue;
            }
            if (!admit(r)) {
                if (!active.empty() || !pending.empty() || !draining.empty()) {
                    // no memory now: back to the head of the queue until requests finish
                    std::lock_guard<std::mutex> lk(mu);
                    in_use -= r->footprint;
                    --in_flight;
                    queue.push_front(r);
                    break;
                }
                r->res.status = RT_ENOMEM;
                r->err = "device allocation failed";
                complete(r);
            }
        }
    };
    // requests whose input copy has landed join the next iteration (no request
    // waits on another's copy); with nothing running, wait for the oldest copy
    auto activate = [&](bool wait) {
        if (wait && active.empty() && !pending.empty() && pending.front()->ev)
            (void)hipEventSynchronize(pending.front()->ev);
        size_t k = 0;
        for (GState* g : pending) {
            if (!g->ev || hipEventQuery(g->ev) != hipErrorNotReady) active.push_back(g);
            else pending[k++] = g;
        }
        pending.resize(k);
    };
    auto drain_finished = [&]() {
        for (GState* g : finished) start_drain(g);
        finished.clear();
        poll_drains(false);
    };
    for (;;) {
        const Clock::time_point t_top = Clock::now();
        activate(false);
        if (active.empty()) {
            // nothing running: copy results out, admit, and start the new requests
            drain_finished();
            admit_queue(true);
            activate(true);
        }
        // requests that finished without device work (rank 0 everywhere, failures)
        for (size_t i = 0; i < active.size();) {
            if (active[i]->phase == GState::DONE) { finished.push_back(active[i]); active.erase(active.begin() + i); }
            else ++i;
        }
        if (active.empty()) {
            if (!finished.empty()) continue;
            if (!draining.empty()) { poll_drains(true); continue; }
            std::lock_guard<std::mutex> lk(mu);
            if (stopping && queue.empty()) break;
            continue;
        }
        // descriptors of this iteration
        std::memset(hdr, 0, sizeof(rt::GHeader));
        int nb = 0, nt = 0;
        int64_t swi = 0, pwi = 0, gwi = 0, cwi = 0;
        for (GState* g : active) {
            const int64_t K = g->L * g->R;
            const int64_t nct = (K + 255) / 256;
            rt::GRead* rb = rb_dev + g->slot;
            if (g->phase == GState::BLOCK) {
                g->bi = std::min(block, g->cap - g->kcols);
                rt::GBlock& b = gblk[nb];
                b.G = g->cur; b.L = g->L; b.J = g->J; b.R = g->R;
                b.col0 = (int64_t)g->blk * block;
                b.seed = g->r->seed;
                b.mode = (uint32_t)g->n;
                b.b = g->bi;
                b.nsplit = g->nsplit; b.nrowtile = g->nrowtile; b.tiles_per_split = g->tps;
                b.wi0 = swi;
                swi += (int64_t)g->nsplit * g->nrowtile;
                b.partial = g->partial;
                b.nrm_partial = g->have_norm ? nullptr : g->nrm_partial;
                b.Y = g->Y; b.Qall = g->Qall; b.Qallf = g->Qallf; b.cap = g->cap; b.kcols = g->kcols;
                b.drop = 1e-5;
                b.knew = g->ints;
                b.rb = rb;
                rt::GProj& q = gbproj[nb];
                q.G = g->cur; q.L = g->L; q.J = g->J; q.R = g->R; q.ldj = g->J;
                q.Q = g->Qallf + g->kcols; q.ldq = g->cap;
                q.ellmax = g->bi; q.ell_dev = nullptr;
                q.out = g->B; q.ldo = g->cap; q.koff = g->kcols;
                q.wi0 = pwi; q.nct = (int)nct; q.nch = (g->bi + 7) / 8;
                pwi += nct * q.nch;
                q.nrm_partial = g->bnrm;
                q.rb_norm = &rb->bnorm2;
                ++nb;
            } else if (g->phase == GState::TRUNC) {
                rt::GTrunc& t = gtr[nt];
                t.B = g->B; t.L = g->L; t.ldk = g->cap; t.R = g->R; t.kcols = g->kcols;
                t.Qall = g->Qall; t.J = g->J; t.cap = g->cap;
                t.E = g->E; t.tau2 = g->tau2;
                t.wi0 = gwi; t.nchunk = g->nchunk;
                gwi += g->nchunk;
                t.gpart = g->gpart; t.A = g->fac[g->n]; t.Uf = g->Uf; t.kout = g->ints + 1; t.rb = rb;
                rt::GProj& q = gcproj[nt];
                q.G = g->B; q.L = g->L; q.J = g->kcols; q.R = g->R; q.ldj = g->cap;
                q.Q = g->Uf; q.ldq = g->kcols;
                q.ellmax = g->kcols; q.ell_dev = g->ints + 1;
                q.out = g->core[g->pp]; q.ldo = 0; q.koff = 0;
                q.wi0 = cwi; q.nct = (int)nct; q.nch = (g->kcols + 7) / 8;
                cwi += nct * q.nch;
                q.nrm_partial = g->cnrm;
                q.rb_norm = &rb->gnorm2;
                ++nt;
            }
        }
        hdr->nblock = nb; hdr->nbproj = nb; hdr->ntrunc = nt; hdr->ncproj = nt;
        hdr->sketch_items = swi; hdr->bproj_items = pwi; hdr->gram_items = gwi; hdr->cproj_items = cwi;
        // one graph: the descriptor copy and the iteration's launches (captured
        // once, replayed every iteration with the pinned buffer's new contents)
        bool launched = false;
        if (graph_ok && !gexec) {
            hipGraph_t graph = nullptr;
            bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                const bool body = hipMemcpyAsync(desc_dev, desc_host, dbytes, hipMemcpyHostToDevice, st) == hipSuccess &&
                                  rt::launch_group_iteration(desc_dev, maxreq, block, st) == hipSuccess;
                ok = hipStreamEndCapture(st, &graph) == hipSuccess && body && graph;
            }
            ok = ok && hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) == hipSuccess;
            if (graph) (void)hipGraphDestroy(graph);
            if (!ok) {
                graph_ok = false;
                gexec = nullptr;
                (void)hipGetLastError();
            }
        }
        if (graph_ok && gexec) launched = hipGraphLaunch(gexec, st) == hipSuccess;
        if (!launched)
            launched = hipMemcpyAsync(desc_dev, desc_host, dbytes, hipMemcpyHostToDevice, st) == hipSuccess &&
                       rt::launch_group_iteration(desc_dev, maxreq, block, st) == hipSuccess;
        const Clock::time_point t_launch = Clock::now();
        // while the iteration runs: results of the last one out, new requests in
        // (their inputs cross on the copy streams and join a later iteration)
        drain_finished();
        admit_queue(false);
        const Clock::time_point t_overlap = Clock::now();
        const bool synced = launched && hipStreamSynchronize(st) == hipSuccess;
        const Clock::time_point t_synced = Clock::now();
        const int64_t nadv = (int64_t)active.size();
        // advance every request from its readback slot
        for (GState* g : active) {
            if (!synced) { fail(g, RT_EHIP, "grouped launch failed"); continue; }
            const rt::GRead& rb = rb_host[g->slot];
            if (g->phase == GState::BLOCK) {
                if (!g->have_norm) {
                    g->nx2 = rb.xnorm2;
                    if (!std::isfinite(g->nx2)) { fail(g, RT_ENONFINITE, "input holds NaN or Inf"); continue; }
                    g->have_norm = true;
                    const double en = eps_n_base / std::sqrt((double)g->d) * std::sqrt(g->nx2);
                    g->tau2 = en * en;
                    g->E = g->nx2;
                    g->cur_norm2 = g->nx2;
                    if (!(g->E > g->tau2)) { end_blocks(g); continue; }   // the block is discarded
                }
                ++g->blk;
                const int kn = rb.knew;
                if (kn <= 0) { end_blocks(g); continue; }                  // range exhausted
                g->E -= rb.bnorm2;
                g->kcols += kn;
                if (!(g->E > g->tau2)) end_blocks(g);
                else if (g->kcols >= g->cap) {
                    if (g->cap == RT_LMAX && g->cap < std::min<int64_t>(g->J, g->L * g->R)) {
                        // the shared kernels stop at RT_LMAX columns, the single-request
                        // path at RT_LMAX_FIXED: the request is redone alone
                        g->rerun = true;
                        fail(g, RT_EINVAL, "redone alone");
                    } else {
                        g->capped = true;
                        end_blocks(g);
                    }
                }
            } else if (g->phase == GState::TRUNC) {
                const int k = rb.kfinal;
                g->ranks[g->n] = k;
                g->cdims[g->n] = k;
                g->cur_norm2 = rb.gnorm2;
                g->cur = g->core[g->pp];
                g->pp ^= 1;
                ++g->mi;
                next_mode(g);
            }
        }
        for (size_t i = 0; i < active.size();) {
            if (active[i]->phase == GState::DONE) { finished.push_back(active[i]); active.erase(active.begin() + i); }
            else ++i;
        }
        {
            const Clock::time_point t_end = Clock::now();
            std::lock_guard<std::mutex> lk(mu);
            ++stats.iterations;
            stats.request_steps += nadv;
            stats.wait_s += Sec(t_synced - t_overlap).count();
            stats.overlap_s += Sec(t_overlap - t_launch).count();
            stats.host_s += Sec(t_launch - t_top).count() + Sec(t_end - t_synced).count();
        }
    }
    poll_drains(true);
    if (st) (void)hipStreamSynchronize(st);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (dX) cache.put(dX);
    if (ctx) rt_destroy(ctx);
    cache.clear();
    pool.clear();
    if (stage) (void)hipHostFree(stage);
    if (desc_host) (void)hipHostFree(desc_host);
    if (desc_dev) (void)hipFree(desc_dev);
    if (rb_host) (void)hipHostFree(rb_host);
    for (float* p : sstage) if (p) (void)hipHostFree(p);
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    for (hipStream_t c : cst) if (c) { (void)hipStreamSynchronize(c); (void)hipStreamDestroy(c); }
    if (st) (void)hipStreamDestroy(st);
}

extern "C" {

rt_status rt_server_create(rt_server** srv, int device, const rt_server_opts* opts) {
    if (!srv || !opts) return rt::set_error(RT_EINVAL, "NULL argument");
    *srv = nullptr;
    if (opts->max_inflight < 1 || opts->max_inflight > 64) return rt::set_error(RT_EINVAL, "max_inflight must be in [1, 64]");
    if (opts->prec != RT_PREC_F32 && opts->prec != RT_PREC_BF16_SKETCH)
        return rt::set_error(RT_EINVAL, "serving precision must be RT_PREC_F32 or RT_PREC_BF16_SKETCH");
    if (!(opts->eps >= 0.0) || !std::isfinite(opts->eps)) return rt::set_error(RT_EINVAL, "eps must be finite and >= 0");
    if (opts->block < 1 || opts->block > RT_LMAX) return rt::set_error(RT_EINVAL, "block must be in [1, RT_LMAX]");
    if (opts->mode != RT_SERVE_GROUPED && opts->mode != RT_SERVE_SLOTS)
        return rt::set_error(RT_EINVAL, "mode must be RT_SERVE_GROUPED or RT_SERVE_SLOTS");
    if (opts->max_queued < 0) return rt::set_error(RT_EINVAL, "max_queued must be >= 0");
    if (opts->mode == RT_SERVE_GROUPED && (opts->prec != RT_PREC_F32 || opts->block > 16))
        return rt::set_error(RT_EINVAL, "grouped serving runs float32 sketches with blocks of at most 16 columns");
    if (hipSetDevice(device) != hipSuccess) return rt::set_error(RT_EHIP, "hipSetDevice failed");
    size_t budget = opts->hbm_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return rt::set_error(RT_EHIP, "hipMemGetInfo failed");
        budget = fr / 4 * 3;
    }
    rt_server* s = new rt_server();
    s->device = device;
    s->opts = *opts;
    s->budget = budget;
    s->slot_errors.assign(opts->max_inflight, std::string());
    if (opts->mode == RT_SERVE_GROUPED)
        s->threads.emplace_back(&rt_server::exec_main, s);
    else
        for (int i = 0; i < opts->max_inflight; ++i) s->threads.emplace_back(&rt_server::slot_main, s, i);
    *srv = s;
    return RT_OK;
}

rt_status rt_server_submit(rt_server* srv, const rt_tensor* X, uint64_t seed, uint64_t* ticket) {
    if (!srv || !X || !ticket || !X->data) return rt::set_error(RT_EINVAL, "NULL argument");
    if (X->ndim < 2 || X->ndim > RT_MAXD) return rt::set_error(RT_EINVAL, "ndim must be in [2, RT_MAXD]");
    if (X->dtype != RT_F32) return rt::set_error(RT_EINVAL, "serving takes float32 tensors");
    for (int i = 0; i < X->ndim; ++i)
        if (X->dims[i] < 1) return rt::set_error(RT_EINVAL, "every dim must be >= 1");
    Request* r = new Request();
    r->X = *X;
    r->seed = seed;
    // input + sketch/projection buffers of the first mode + workspace slack
    r->footprint = (size_t)numel(*X) * sizeof(float) * 3 + (size_t(8) << 20);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stopping) {
            delete r;
            return rt::set_error(RT_EINVAL, "server is stopping");
        }
        if (srv->opts.max_queued > 0 && srv->queue.size() >= (size_t)srv->opts.max_queued) {
            delete r;
            return rt::set_error(RT_EBUSY, "the wait queue is full");
        }
        r->id = srv->next_id++;
        srv->reqs[r->id] = r;
        srv->queue.push_back(r);
        *ticket = r->id;
    }
    srv->cv_work.notify_one();
    return RT_OK;
}

rt_status rt_server_submit_reconstruct(rt_server* srv, const rt_tucker_host* t, float* out, uint64_t* ticket) {
    if (!srv || !t || !out || !ticket) return rt::set_error(RT_EINVAL, "NULL argument");
    if (t->ndim < 2 || t->ndim > RT_MAXD) return rt::set_error(RT_EINVAL, "ndim must be in [2, RT_MAXD]");
    int64_t ncore = 1, nout = 1, nfac = 0;
    for (int i = 0; i < t->ndim; ++i) {
        if (t->dims[i] < 1) return rt::set_error(RT_EINVAL, "every dim must be >= 1");
        if (t->ranks[i] < 0 || t->ranks[i] > t->dims[i]) return rt::set_error(RT_EINVAL, "ranks must be in [0, dims]");
        if (!t->factors[i] && t->ranks[i] != t->dims[i] && t->ranks[i] != 0)
            return rt::set_error(RT_EINVAL, "a mode without a factor must keep its dimension");
        ncore *= t->ranks[i];
        nout *= t->dims[i];
        if (t->factors[i]) nfac += t->dims[i] * (int64_t)t->ranks[i];
    }
    if (ncore > 0 && !t->core) return rt::set_error(RT_EINVAL, "NULL core");
    Request* r = new Request();
    r->decompress = true;
    r->T = *t;
    r->out = out;
    // output, its largest intermediate (at most the output), core and factors
    r->footprint = (size_t)(2 * nout + ncore + nfac) * sizeof(float) + (size_t(8) << 20);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stopping) {
            delete r;
            return rt::set_error(RT_EINVAL, "server is stopping");
        }
        if (srv->opts.max_queued > 0 && srv->queue.size() >= (size_t)srv->opts.max_queued) {
            delete r;
            return rt::set_error(RT_EBUSY, "the wait queue is full");
        }
        r->id = srv->next_id++;
        srv->reqs[r->id] = r;
        srv->queue.push_back(r);
        *ticket = r->id;
    }
    srv->cv_work.notify_one();
    return RT_OK;
}

rt_status rt_server_poll(rt_server* srv, uint64_t ticket, int32_t* done, rt_result* out) {
    if (!srv || !done || !out) return rt::set_error(RT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return rt::set_error(RT_EINVAL, "unknown ticket");
    *done = it->second->done ? 1 : 0;
    if (*done) *out = it->second->res;
    return RT_OK;
}

rt_status rt_server_wait(rt_server* srv, uint64_t ticket, rt_result* out) {
    if (!srv || !out) return rt::set_error(RT_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return rt::set_error(RT_EINVAL, "unknown ticket");
    Request* r = it->second;
    srv->cv_done.wait(lk, [&] { return r->done; });
    *out = r->res;
    if (r->res.status != RT_OK && r->res.status != RT_ECAP) return rt::set_error(r->res.status, r->err.c_str());
    return RT_OK;
}

rt_status rt_server_release(rt_server* srv, uint64_t ticket) {
    if (!srv) return rt::set_error(RT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return rt::set_error(RT_EINVAL, "unknown ticket");
    if (!it->second->done) return rt::set_error(RT_EINVAL, "request has not completed");
    delete it->second;
    srv->reqs.erase(it);
    return RT_OK;
}

rt_status rt_server_cancel(rt_server* srv, uint64_t ticket) {
    if (!srv) return rt::set_error(RT_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end()) return rt::set_error(RT_EINVAL, "unknown ticket");
        Request* r = it->second;
        auto q = std::find(srv->queue.begin(), srv->queue.end(), r);
        if (q == srv->queue.end()) return rt::set_error(RT_EBUSY, "request already admitted");
        srv->queue.erase(q);
        r->t_admit = r->t_done = Clock::now();
        rt_result& res = r->res;
        res.status = RT_ECANCELLED;
        res.ndim = r->decompress ? r->T.ndim : r->X.ndim;
        for (int i = 0; i < res.ndim; ++i) {
            res.dims[i] = r->decompress ? r->T.dims[i] : r->X.dims[i];
            res.ranks[i] = r->decompress ? r->T.ranks[i] : 0;
        }
        res.queue_s = 0.0;
        res.latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        r->err = "request cancelled";
        r->done = true;
    }
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();
    return RT_OK;
}

rt_status rt_server_get_stats(rt_server* srv, rt_server_stats* out) {
    if (!srv || !out) return rt::set_error(RT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    return RT_OK;
}

rt_status rt_server_destroy(rt_server* srv) {
    if (!srv) return RT_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    for (auto& t : srv->threads) t.join();
    for (auto& kv : srv->reqs) delete kv.second;
    delete srv;
    return RT_OK;
}

}  // extern "C"
