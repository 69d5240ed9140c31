// Instantiations of the float32 MFMA sketch with an explicit Omega read from an
// (L, ell, R) tensor (subspace iteration), rows loader (R % 4 == 0).
#include "rt_sketch_mfma_launch.hpp"

namespace rt {
hipError_t launch_sketch_f32_rows_explicit(const SketchPlan& p, const float* X, Shape3 s, int ell, const float* Om,
                                           float* partial, hipStream_t stream) {
    return skm::launch_loader<skm::LOAD_ROWS, true>(p, X, s, ell, 0, 0, 0, partial, nullptr, stream, Om);
}
}  // namespace rt
