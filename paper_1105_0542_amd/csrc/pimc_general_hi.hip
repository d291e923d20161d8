// Estimation kernels of the general-potential mode for one level p > kGenInlineMaxP, chosen at build
// time by PIMC_GEN_P (this file is compiled once per level): the walker (pimc_walker.hpp) with
// GenSliceEval<p>, whose out-of-line slice functions (one slice, two slices) hold the straight-line
// code generated for p (pimc_general_gen_p<p>.hpp, up to 24,196 monomials at p = 18), subtrees of up
// to three levels.
#include <hip/hip_runtime.h>

#include "pimc_general_device.hpp"
#include "pimc_walker.hpp"

#ifndef PIMC_GEN_P
#error "PIMC_GEN_P (the level p of this translation unit) is not defined"
#endif
#define PIMC_GEN_STR2(x) #x
#define PIMC_GEN_STR(x) PIMC_GEN_STR2(x)
#define PIMC_GEN_HEADER2(p) PIMC_GEN_STR(pimc_general_gen_p##p.hpp)
#define PIMC_GEN_HEADER(p) PIMC_GEN_HEADER2(p)
#include PIMC_GEN_HEADER(PIMC_GEN_P)

namespace pimc {

static_assert(PIMC_GEN_P > kGenInlineMaxP && PIMC_GEN_P <= kGenMaxP, "level of an out-of-line evaluator");
static_assert(gen_subtree_levels(PIMC_GEN_P) == 3, "three-level subtrees above the inline levels");

// U = min(s, 3): subtrees of 1 and 2 levels only for N = 2 and 4
template <>
hipError_t gen_hi_launch<PIMC_GEN_P>(const AmpArgs& A, int U, int grid, hipStream_t st) {
    const GenSliceEval<PIMC_GEN_P> ev{A.tab64, A.gen};
    switch (U) {
        case 1: return launch_one<DefaultShape<1>>(A, ev, grid, st);
        case 2: return launch_one<DefaultShape<2>>(A, ev, grid, st);
        case 3: return launch_one<DefaultShape<3>>(A, ev, grid, st);
        default: return hipErrorInvalidValue;
    }
}

template <>
int gen_hi_resident<PIMC_GEN_P>(int U, size_t lds_bytes, int device) {
    switch (U) {
        case 2: return resident_one<DefaultShape<2>, GenSliceEval<PIMC_GEN_P>>(lds_bytes, device);
        case 3: return resident_one<DefaultShape<3>, GenSliceEval<PIMC_GEN_P>>(lds_bytes, device);
        default: return resident_one<DefaultShape<1>, GenSliceEval<PIMC_GEN_P>>(lds_bytes, device);
    }
}

template <>
int gen_hi_nrec<PIMC_GEN_P>() {
    return GenCompiled<PIMC_GEN_P>::NREC;
}

}  // namespace pimc
