// Instantiations of the float32 MFMA sketch for the last mode (R == 1), whose
// unfolding columns are contiguous in memory.
#include "rt_sketch_mfma_launch.hpp"

namespace rt {
hipError_t launch_sketch_f32_cols(const SketchPlan& p, const float* X, Shape3 s, int ell, int64_t col0,
                                  uint64_t seed, uint32_t mode, float* partial, double* nrm2, hipStream_t stream) {
    return skm::launch_loader<skm::LOAD_COLS>(p, X, s, ell, col0, seed, mode, partial, nrm2, stream);
}
}  // namespace rt
