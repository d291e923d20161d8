// Vector estimation kernels of the component evaluator (any polynomial V) for one dimension,
// chosen at build time by PIMC_POLY_DIM (this file is compiled once per dimension, in parallel:
// subtrees of up to kPolyU levels make these the largest kernels of the vector mode).
#include "pimc_vector_impl.hpp"

#ifndef PIMC_POLY_DIM
#error "PIMC_POLY_DIM (the number of coordinates of this translation unit) is not defined"
#endif

namespace pimc {

template <>
hipError_t launch_vector_poly_dim<PIMC_POLY_DIM>(const VecArgs& A, int U, int grid, hipStream_t st) {
    return vec::launch_poly<PIMC_POLY_DIM>(A, U, grid, st);
}

template <>
int vector_poly_resident_dim<PIMC_POLY_DIM>(int U, size_t lds, int device) {
    return vec::resident_poly<PIMC_POLY_DIM>(U, lds, device);
}

}  // namespace pimc
