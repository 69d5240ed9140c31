// Compile-time dispatch of the MFMA sketch over (RB, RW, NQ).
#pragma once
#include "rt_sketch_mfma.hpp"

namespace rt {
namespace skm {

struct SketchArgs {
    const float* X;
    Shape3 s;
    int ell;
    int64_t col0;
    uint64_t seed;
    uint32_t mode;
    int64_t tiles_per_split;
    float* partial;
    double* nrm2;
    const float* Om;   // explicit Omega (EXPL), else null
};

template <int LOADER, int RB, int RW, int NQ, bool EXPL>
hipError_t go(dim3 grid, const SketchArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL((sketch_f32_kernel<RB, RW, NQ, LOADER, EXPL>), grid, dim3(256), 0, stream, a.X, a.s.L,
                       a.s.J, a.s.R, a.ell, a.col0, a.seed, a.mode, a.tiles_per_split, a.partial, a.nrm2, a.Om);
    return hipGetLastError();
}

template <int LOADER, int RB, int RW, bool EXPL>
hipError_t by_nq(int nq, dim3 grid, const SketchArgs& a, hipStream_t st) {
    switch (nq) {
        case 1: return go<LOADER, RB, RW, 1, EXPL>(grid, a, st);
        case 2: return go<LOADER, RB, RW, 2, EXPL>(grid, a, st);
        case 3: return go<LOADER, RB, RW, 3, EXPL>(grid, a, st);
        case 4: return go<LOADER, RB, RW, 4, EXPL>(grid, a, st);
        case 5: return go<LOADER, RB, RW, 5, EXPL>(grid, a, st);
        case 6: return go<LOADER, RB, RW, 6, EXPL>(grid, a, st);
        case 7: return go<LOADER, RB, RW, 7, EXPL>(grid, a, st);
        case 8: return go<LOADER, RB, RW, 8, EXPL>(grid, a, st);
        case 9: return go<LOADER, RB, RW, 9, EXPL>(grid, a, st);
        case 10: return go<LOADER, RB, RW, 10, EXPL>(grid, a, st);
        case 12: return go<LOADER, RB, RW, 12, EXPL>(grid, a, st);
        case 14: return go<LOADER, RB, RW, 14, EXPL>(grid, a, st);
        case 16: return go<LOADER, RB, RW, 16, EXPL>(grid, a, st);
        default: return hipErrorInvalidValue;
    }
}

template <int LOADER, bool EXPL = false>
hipError_t launch_loader(const SketchPlan& p, const float* X, Shape3 s, int ell, int64_t col0, uint64_t seed,
                         uint32_t mode, float* partial, double* nrm2, hipStream_t stream, const float* Om = nullptr) {
    const SketchArgs a{X, s, ell, col0, seed, mode, p.tiles_per_split, partial, nrm2, Om};
    const dim3 grid(p.nsplit, p.nrowtile);
    if (p.rb == 1 && p.rw == 1) return by_nq<LOADER, 1, 1, EXPL>(p.nq, grid, a, stream);
    if (p.rb == 2 && p.rw == 1) return by_nq<LOADER, 2, 1, EXPL>(p.nq, grid, a, stream);
    if (p.rb == 2 && p.rw == 2) return by_nq<LOADER, 2, 2, EXPL>(p.nq, grid, a, stream);
    return hipErrorInvalidValue;
}

}  // namespace skm
}  // namespace rt
