// Vector estimation kernels, 4 coordinates: the compile-time shapes p = 1..18 (s >= kVecU) and the
// shape-array evaluator (any p, s < kVecU).
#include "pimc_vector_impl.hpp"

namespace pimc {

hipError_t launch_vector_d4(const VecArgs& A, int p, int U, bool specialized, int grid, hipStream_t st) {
    if (specialized) {
        if (U != kVecU) return hipErrorInvalidValue;
        return vec::launch_spec<4, 1>(A, p, grid, st);
    }
    return vec::launch_rt<4>(A, U, grid, st);
}

int vector_resident_d4(int p, int U, bool specialized, size_t lds, int device) {
    if (specialized) return vec::resident_spec<4, 1>(p, lds, device);
    return vec::resident_rt<4>(U, lds, device);
}

}  // namespace pimc
