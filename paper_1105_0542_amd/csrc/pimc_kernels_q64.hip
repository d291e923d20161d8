// Estimation kernels with the compile-time table shapes of level p = 1..kMaxP (the quartic family in FP64),
// subtrees of 4 levels; one translation unit per evaluator family so that they
// compile in parallel.
#include <hip/hip_runtime.h>

#include "pimc_walker.hpp"

namespace pimc {

namespace {

template <int P>
hipError_t launch_p(const AmpArgs& A, int p, int U, int grid, hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p != P) return launch_p<P + 1>(A, p, U, grid, st);
        const QuarticEval64<P> ev{A.tab64};
        switch (U) {
            case 4: return launch_one<DefaultShape<4>>(A, ev, grid, st);
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
}

template <int P>
int resident_p(int p, int U, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p != P) return resident_p<P + 1>(p, U, lds, device);
        return U == 4 ? resident_one<DefaultShape<4>, QuarticEval64<P>>(lds, device) : 0;
    } else {
        return 256;
    }
}

}  // namespace

hipError_t launch_quartic64(const AmpArgs& A, int p, int U, int grid, hipStream_t st) {
    return launch_p<1>(A, p, U, grid, st);
}

int resident_quartic64(int p, int U, size_t lds_bytes, int device) { return resident_p<1>(p, U, lds_bytes, device); }

}  // namespace pimc
