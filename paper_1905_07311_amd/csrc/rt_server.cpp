// Serving: a request loop that admits float32 tensors of uneven shapes by
// device-memory footprint and keeps several of them in flight, each on its own
// stream, running adaptive R-STHOSVD (Alg. 5, §4) with a common tolerance.
//
// Requests wait in arrival order.  A slot thread takes the request at the head
// as soon as it is free and the estimated footprint of the admitted requests
// stays within the budget (a request is always admitted when nothing else is
// in flight, so an oversized one cannot block the queue for ever).  Each slot
// owns a stream (default priority, not synchronising with the null stream), a
// library context with its workspace, and a cache of device blocks: blocks are
// reused rather than freed, because freeing device memory synchronises the
// whole device and would stall the other slots.  Results are copied to host
// memory owned by the server until the caller releases them.
#include <hip/hip_runtime.h>

#include <chrono>
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

#include "rtucker.h"

namespace rt {
rt_status set_error(rt_status s, const char* msg);
}

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

    bool admissible(const Request* r) const { return in_flight == 0 || in_use + r->footprint <= budget; }
    void slot_main(int slot);
    void run(Request* r, rt_ctx* ctx, hipStream_t st, BlockCache& cache, float*& dX, size_t& dX_cap,
             float*& stage, size_t& stage_cap);
};

void rt_server::run(Request* r, rt_ctx* ctx, hipStream_t st, BlockCache& cache, float*& dX, size_t& dX_cap,
                    float*& stage, size_t& stage_cap) {
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
        {
            std::lock_guard<std::mutex> lk(mu);
            in_use -= r->footprint;
            --in_flight;
            r->t_done = Clock::now();
            r->res.queue_s = std::chrono::duration<double>(r->t_admit - r->t_submit).count();
            r->res.latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
            r->res.core = r->core.data();
            for (int i = 0; i < RT_MAXD; ++i)
                r->res.factors[i] = (i < (int)r->factors.size() && !r->factors[i].empty()) ? r->factors[i].data()
                                                                                            : nullptr;
            r->done = true;
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
    if (st) (void)hipStreamSynchronize(st);
    if (dX) cache.put(dX);
    if (ctx) rt_destroy(ctx);
    if (stage) (void)hipHostFree(stage);
    cache.clear();
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
