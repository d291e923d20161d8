// Estimation kernels with the compile-time table shapes of level p = 1..kMaxP (the Poeschl-Teller tables); one
// translation unit per evaluator family so that they compile in parallel.
#include <hip/hip_runtime.h>

#include "pimc_walker.hpp"

namespace pimc {

namespace {

template <int P>
hipError_t launch_p(const AmpArgs& A, int p, int grid, hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p != P) return launch_p<P + 1>(A, p, grid, st);
        const TanhEvalP<P> ev{A.tab64, A.alpha};
        return launch_one<DefaultShape<4>>(A, ev, grid, st);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int P>
int resident_p(int p, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p != P) return resident_p<P + 1>(p, lds, device);
        return resident_one<DefaultShape<4>, TanhEvalP<P>>(lds, device);
    } else {
        return 256;
    }
}

}  // namespace

hipError_t launch_tanh_fixed(const AmpArgs& A, int p, int grid, hipStream_t st) { return launch_p<1>(A, p, grid, st); }

int resident_tanh_fixed(int p, size_t lds_bytes, int device) { return resident_p<1>(p, lds_bytes, device); }

}  // namespace pimc
