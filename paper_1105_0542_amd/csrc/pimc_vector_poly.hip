// Vector estimation kernels of the component evaluator (any polynomial V) for one dimension,
// chosen at build time by PIMC_POLY_DIM (this file is compiled once per dimension, in parallel:
// subtrees of up to kPolyU levels make these the largest kernels of the vector mode). With
// PIMC_POLY_DEEP it holds only the deepest subtree of that dimension, when that is kPolySplitU
// levels or more, so that the deepest and the shallower kernels compile in parallel.
#include "pimc_vector_impl.hpp"

#ifndef PIMC_POLY_DIM
#error "PIMC_POLY_DIM (the number of coordinates of this translation unit) is not defined"
#endif
#ifndef PIMC_POLY_DEEP
#define PIMC_POLY_DEEP 0
#endif

namespace pimc {

constexpr int kUDeep = poly_subtree_levels(PIMC_POLY_DIM);
constexpr bool kSplit = kUDeep >= kPolySplitU;

#if PIMC_POLY_DEEP

template <>
hipError_t launch_vector_poly_deep<PIMC_POLY_DIM>(const VecArgs& A, int grid, hipStream_t st) {
    if constexpr (kSplit) {
        const vec::PolyEvalRT<PIMC_POLY_DIM> ev{A.tab, A.shape, A.stride};
        return vec::launch_one<PIMC_POLY_DIM, kUDeep>(A, ev, grid, st);
    } else {
        return hipErrorInvalidValue;
    }
}

template <>
int vector_poly_resident_deep<PIMC_POLY_DIM>(size_t lds, int device) {
    if constexpr (kSplit) return vec::resident_one<PIMC_POLY_DIM, kUDeep, vec::PolyEvalRT<PIMC_POLY_DIM>>(lds, device);
    else return 0;
}

#else

constexpr int kUShallow = kSplit ? kPolySplitU - 1 : kUDeep;

template <>
hipError_t launch_vector_poly_dim<PIMC_POLY_DIM>(const VecArgs& A, int U, int grid, hipStream_t st) {
    if constexpr (kSplit)
        if (U == kUDeep) return launch_vector_poly_deep<PIMC_POLY_DIM>(A, grid, st);
    return vec::launch_poly<PIMC_POLY_DIM, kUShallow>(A, U, grid, st);
}

template <>
int vector_poly_resident_dim<PIMC_POLY_DIM>(int U, size_t lds, int device) {
    if constexpr (kSplit)
        if (U == kUDeep) return vector_poly_resident_deep<PIMC_POLY_DIM>(lds, device);
    return vec::resident_poly<PIMC_POLY_DIM, kUShallow>(U, lds, device);
}

#endif

}  // namespace pimc
