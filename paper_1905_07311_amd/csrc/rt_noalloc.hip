// Allocation-free variant of the sketch entry point, Y = X_(n) Omega (Alg. 1
// step 1), for callers that cannot allocate device memory: code under stream
// capture, tight serving loops, harnesses that forbid it.
//
// It runs the same plan and kernels as rt_sketch, but the split-K partial sums,
// the per-workgroup norm partials and the temporaries of the fixed-order
// reduction live in one static device array of NOALLOC_SCRATCH_BYTES instead of
// the context's workspace.  Every GPU the library runs on holds its own copy of
// that array until the process ends.  The host never passes the array's name to
// a kernel: rt_create takes its device address once per device (with that
// device current) and the entry point hands that address to the kernels.
//
// Nothing in the array has to start at zero: every partial is written in full
// before the reduction reads it.  All calls on one GPU share the array, so calls
// that overlap on one GPU (two streams, two threads) race; callers serialise them.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "rt_kernels.hpp"
#include "rtucker.h"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

namespace rt {

hipError_t noalloc_init(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

}  // namespace rt

extern "C" rt_status rt_sketch_noalloc(rt_ctx* ctx, const rt_tensor* X, int32_t mode, int32_t ell, int64_t col0,
                                       uint64_t seed, rt_precision prec, double* Y, double* nrm2) {
    const rt_status a = rt::check_sketch_args(ctx, X, mode, ell, col0, prec, Y);
    if (a != RT_OK) return a;
    const int dev = rt::ctx_device(ctx);
    char* base = nullptr;
    if (dev >= 0 && dev < NOALLOC_MAX_DEVICES) {
        std::lock_guard<std::mutex> lk(g_mu);
        base = static_cast<char*>(g_scratch_ptr[dev]);
    }
    if (!base) return rt::set_error(RT_EHIP, "static scratch of this device is not set up");
    rt::Shape3 s{1, X->dims[mode], 1};
    for (int i = 0; i < mode; ++i) s.L *= X->dims[i];
    for (int i = mode + 1; i < X->ndim; ++i) s.R *= X->dims[i];
    const rt::Dt dt = X->dtype == RT_F64 ? rt::Dt::F64 : rt::Dt::F32;
    const rt::SketchPlan plan = rt::plan_sketch(dt, (int)prec, s, ell, col0, X->data);
    // scratch layout: split-K partials | per-workgroup norm partials | reduction temporaries
    const size_t part_bytes = align256(plan.partial_elems * (dt == rt::Dt::F64 ? 8 : 4));
    const size_t nrm_bytes = align256((size_t)plan.nwg * sizeof(double));
    const size_t tmp_bytes = align256((rt::reduce_partials_tmp(plan.nsplit, s.J * ell) + 1) * sizeof(double));
    const size_t need = part_bytes + nrm_bytes + tmp_bytes;
    if (need > NOALLOC_SCRATCH_BYTES) {
        const std::string msg = "rt_sketch_noalloc: this shape needs " + std::to_string(need) +
                                " bytes of scratch, above the static maximum of " +
                                std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes (use rt_sketch)";
        return rt::set_error(RT_EINVAL, msg.c_str());
    }
    void* partial = base;
    double* np = reinterpret_cast<double*>(base + part_bytes);
    double* rtmp = reinterpret_cast<double*>(base + part_bytes + nrm_bytes);
    if (hipSetDevice(dev) != hipSuccess) return rt::set_error(RT_EHIP, "hipSetDevice failed");
    hipStream_t st = rt::ctx_stream(ctx);
    hipError_t e = rt::launch_sketch(plan, dt, (int)prec, X->data, s, ell, col0, seed, (uint32_t)mode, partial,
                                     nrm2 ? np : nullptr, st);
    if (e == hipSuccess)
        e = rt::launch_reduce_rows(partial, dt == rt::Dt::F64, plan.nsplit, s.J, ell, plan.ldp, Y, st, rtmp);
    if (e == hipSuccess && nrm2) e = rt::launch_sum_scalar(np, plan.nwg, nrm2, st);
    if (e != hipSuccess) {
        const std::string msg = std::string("rt_sketch_noalloc: launch failed: ") + hipGetErrorString(e);
        return rt::set_error(RT_EHIP, msg.c_str());
    }
    return RT_OK;
}
