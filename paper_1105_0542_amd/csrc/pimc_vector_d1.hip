// Vector estimation kernels, one coordinate (the rotation-invariant potential in one dimension; the
// shape-array evaluator only).
#include "pimc_vector_impl.hpp"

namespace pimc {

hipError_t launch_vector_d1(const VecArgs& A, int p, int U, bool specialized, int grid, hipStream_t st) {
    (void)p;
    if (specialized) return hipErrorInvalidValue;
    return vec::launch_rt<1>(A, U, grid, st);
}

int vector_resident_d1(int p, int U, bool specialized, size_t lds, int device) {
    (void)p;
    (void)specialized;
    return vec::resident_rt<1>(U, lds, device);
}

}  // namespace pimc
