// Estimation kernels of the general-potential mode: the walker (pimc_walker.hpp) instantiated with
// the evaluators generated for p = 1..kGenInlineMaxP (pimc_general_device.hpp), subtrees of
// U = 1..gen_subtree_levels(p) levels; the levels above are dispatched to their own translation units
// (pimc_general_hi.hip).
#include <hip/hip_runtime.h>

#include "pimc_general_device.hpp"
#include "pimc_walker.hpp"

namespace pimc {

namespace {

template <int P>
hipError_t launch_p(const AmpArgs& A, int p, int U, int grid, hipStream_t st) {
    if constexpr (P <= kGenInlineMaxP) {
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
    if constexpr (P <= kGenInlineMaxP) {
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
    if constexpr (P <= kGenInlineMaxP) {
        return p == P ? GenCompiled<P>::NREC : nrec_p<P + 1>(p);
    } else {
        return -1;
    }
}

}  // namespace

static_assert(kGenInlineMaxP == 10 && kGenMaxP == 18, "the out-of-line levels 11..18 are declared in pimc_internal.hpp");

hipError_t launch_general_compiled(const AmpArgs& A, int p, int U, int grid, hipStream_t st) {
    switch (p) {
        case 11: return gen_hi_launch<11>(A, U, grid, st);
        case 12: return gen_hi_launch<12>(A, U, grid, st);
        case 13: return gen_hi_launch<13>(A, U, grid, st);
        case 14: return gen_hi_launch<14>(A, U, grid, st);
        case 15: return gen_hi_launch<15>(A, U, grid, st);
        case 16: return gen_hi_launch<16>(A, U, grid, st);
        case 17: return gen_hi_launch<17>(A, U, grid, st);
        case 18: return gen_hi_launch<18>(A, U, grid, st);
        default: return launch_p<1>(A, p, U, grid, st);
    }
}

int general_compiled_resident(int p, int U, size_t lds_bytes, int device) {
    switch (p) {
        case 11: return gen_hi_resident<11>(U, lds_bytes, device);
        case 12: return gen_hi_resident<12>(U, lds_bytes, device);
        case 13: return gen_hi_resident<13>(U, lds_bytes, device);
        case 14: return gen_hi_resident<14>(U, lds_bytes, device);
        case 15: return gen_hi_resident<15>(U, lds_bytes, device);
        case 16: return gen_hi_resident<16>(U, lds_bytes, device);
        case 17: return gen_hi_resident<17>(U, lds_bytes, device);
        case 18: return gen_hi_resident<18>(U, lds_bytes, device);
        default: return resident_p<1>(p, U, lds_bytes, device);
    }
}

int general_compiled_nrec(int p) {
    switch (p) {
        case 11: return gen_hi_nrec<11>();
        case 12: return gen_hi_nrec<12>();
        case 13: return gen_hi_nrec<13>();
        case 14: return gen_hi_nrec<14>();
        case 15: return gen_hi_nrec<15>();
        case 16: return gen_hi_nrec<16>();
        case 17: return gen_hi_nrec<17>();
        case 18: return gen_hi_nrec<18>();
        default: return nrec_p<1>(p);
    }
}

}  // namespace pimc
