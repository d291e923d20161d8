// Estimation kernels of the general-potential mode: the walker (pimc_walker.hpp) instantiated with
// the evaluators generated for p = 1..kGenMaxP (pimc_general_device.hpp), subtrees of
// U = 1..gen_subtree_levels(p) levels.
#include <hip/hip_runtime.h>

#include "pimc_general_device.hpp"
#include "pimc_walker.hpp"

namespace pimc {

namespace {

template <int P>
hipError_t launch_p(const AmpArgs& A, int p, int U, int grid, hipStream_t st) {
    if constexpr (P <= kGenMaxP) {
        if (p != P) return launch_p<P + 1>(A, p, U, grid, st);
        const GenCompiledEval<P> ev{A.tab64, A.gen};
        switch (U) {
            case 1: return launch_one<DefaultShape<1>>(A, ev, grid, st);
            case 2: if constexpr (gen_subtree_levels(P) >= 2) return launch_one<DefaultShape<2>>(A, ev, grid, st); else break;
            case 3: if constexpr (gen_subtree_levels(P) >= 3) return launch_one<DefaultShape<3>>(A, ev, grid, st); else break;
            case 4: if constexpr (gen_subtree_levels(P) >= 4) return launch_one<DefaultShape<4>>(A, ev, grid, st); else break;
            default: break;
        }
        return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
}

template <int P>
int resident_p(int p, int U, size_t lds, int device) {
    if constexpr (P <= kGenMaxP) {
        if (p != P) return resident_p<P + 1>(p, U, lds, device);
        switch (U) {
            case 2: if constexpr (gen_subtree_levels(P) >= 2) return resident_one<DefaultShape<2>, GenCompiledEval<P>>(lds, device); else break;
            case 3: if constexpr (gen_subtree_levels(P) >= 3) return resident_one<DefaultShape<3>, GenCompiledEval<P>>(lds, device); else break;
            case 4: if constexpr (gen_subtree_levels(P) >= 4) return resident_one<DefaultShape<4>, GenCompiledEval<P>>(lds, device); else break;
            default: break;
        }
        return resident_one<DefaultShape<1>, GenCompiledEval<P>>(lds, device);
    } else {
        return 256;
    }
}

template <int P>
int nrec_p(int p) {
    if constexpr (P <= kGenMaxP) {
        return p == P ? GenCompiled<P>::NREC : nrec_p<P + 1>(p);
    } else {
        return -1;
    }
}

}  // namespace

hipError_t launch_general_compiled(const AmpArgs& A, int p, int U, int grid, hipStream_t st) {
    return launch_p<1>(A, p, U, grid, st);
}

int general_compiled_resident(int p, int U, size_t lds_bytes, int device) { return resident_p<1>(p, U, lds_bytes, device); }

int general_compiled_nrec(int p) { return nrec_p<1>(p); }

}  // namespace pimc
