// Several coordinates (Sec. 2.2): paths in d = D*M dimensions and the level-p effective potential of
// a rotation-invariant V(x) = sum_n a_n (x.x)^n, shared by the host library and the vector kernels.
//
// The contractions W_{m,k} of eq.(EXP) (homogeneous of degree 2k in the deviation) are polynomials in
// the invariants u = x.x, w = x.xbar, z = xbar.xbar; W is even in xbar, so every term is
// u^i (w^2)^j z^(k-j). At level n (eps = T/2^n) the slice action is
//     eps W_p = sum_j (w^2)^j sum_l z^l Q_{j+l,j}(u),   Q_{k,j} = sum_{m>=k} eps^(m-k+1) [W_{m,k}]_j,
// evaluated by Horner in u (each Q), then in z (over l), then in w^2 (over j).
//
// Table layout of one level ("consumption order"): groups (j, l) for j = nj-1 down to 0 and, within
// j, l = nl(j)-1 down to 0; group (j, l) holds Q_{j+l,j} highest power of u first, radial_len(p, j+l, j)
// coefficients. The shape is a bound that depends on p only: the x-degree of W_{m,k} follows the
// degree recursion of the one-dimensional quartic (u-degree 2, the anharmonic oscillator of Sec. 3.3
// and any lower degree), and a term u^i w^(2j) z^(k-j) has x-degree 2i + 2j. The device copy is
// pre-scaled by 4^-(i + 2j + l) so that the kernels use the endpoint sums and differences
// (qa + qb, qb - qa) directly: u' = 4u, w' = 4w, z' = 4z (exact scaling by powers of two).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pimc_device.hpp"
#include "pimc_internal.hpp"

namespace pimc {

constexpr int kVecMaxDim = 4;
constexpr int kVecBlock = 256;          // lanes of a workgroup
#ifndef PIMC_VEC_U
#define PIMC_VEC_U 3
#endif
#ifndef PIMC_VEC_BATCH
#define PIMC_VEC_BATCH 8
#endif
constexpr int kVecU = PIMC_VEC_U;       // bisection levels of a register subtree (s >= kVecU)
constexpr int kVecBatch = PIMC_VEC_BATCH;   // slices evaluated together, coefficient-major
constexpr uint32_t kCoordPairStride = 1u << 20;   // generator-call offset of coordinate c: c * 2^20

// x-degree bound of W_{m,k}, m < P (the one-dimensional quartic degree table, maximized over m).
constexpr int radial_xdeg(int P, int k) {
    int d = -1;
    for (int m = k; m < P; ++m) d = imax(d, kQuarticDegrees.d[m][k]);
    return d;
}
// Coefficients of Q_{k,j}(u) in the layout (0 if the group is empty).
constexpr int radial_len(int P, int k, int j) {
    const int xd = radial_xdeg(P, k);
    if (xd < 0 || k >= P || j > k) return 0;
    const int n = xd / 2 - j + 1;
    return n > 0 ? n : 0;
}
// Number of z-groups l of power j of w^2 (the last non-empty l, plus one).
constexpr int radial_nl(int P, int j) {
    int n = 0;
    for (int l = 0; j + l < P; ++l)
        if (radial_len(P, j + l, j) > 0) n = l + 1;
    return n;
}
constexpr int radial_nj(int P) {
    int n = 0;
    for (int j = 0; j < P; ++j)
        if (radial_nl(P, j) > 0) n = j + 1;
    return n;
}
// Offset of group (j, l) in consumption order.
constexpr int radial_off(int P, int j, int l) {
    int o = 0;
    for (int jj = radial_nj(P) - 1; jj >= 0; --jj)
        for (int ll = radial_nl(P, jj) - 1; ll >= 0; --ll) {
            if (jj == j && ll == l) return o;
            o += radial_len(P, jj + ll, jj);
        }
    return o;
}
constexpr int radial_size(int P) {
    int o = 0;
    for (int j = 0; j < radial_nj(P); ++j)
        for (int l = 0; l < radial_nl(P, j); ++l) o += radial_len(P, j + l, j);
    return o;
}

static_assert(radial_size(18) == 102 && radial_nj(18) == 5, "radial table shape at p = 18");
static_assert(radial_size(10) == 34 && radial_nj(10) == 3, "radial table shape at p = 10");

// Arguments of one vector estimation launch (kernel argument segment: wave-uniform).
struct VecArgs {
    const double* tab;                 // device: level tables, level-major, stride doubles per level
    const int* shape;                  // device: [nj, nl(0..nj-1), len of each group in consumption order]
    int stride;                        // doubles per level table
    int pad0;
    const double* sig;                 // device: sigma_n = sqrt(T / 2^(n+1)), n = 0..s
    const double* shift;               // device: straight-line level action, n = 0..s
    double a[kVecMaxDim], b[kVecMaxDim];   // endpoints after the mass rescaling
    RngKey key;
    uint64_t first_path;
    uint64_t n_paths;
    uint64_t n_chunks;                 // ceil(n_paths / kChunkPaths)
    int s;                             // N = 2^s
    int D;                             // s - U: levels walked with the explicit stack
    int hier;                          // every level (else level s only)
    double* partials;                  // device [level][chunk][4] or null
    double* dump;                      // device [path][s+1] or null
};

// LDS doubles per lane of the walk above the register subtrees (D levels): D level sums and the
// pending right endpoints of levels 2..D (level 1's right endpoint is b itself), dim each.
__host__ __device__ constexpr int vec_top_slots(int dim, int D) { return D + (D > 1 ? (D - 1) * dim : 0); }

// Dynamic LDS bytes: the Box-Muller table; per lane the walk's slots; per accumulator slot and level
// three sums.
inline size_t vec_lds_bytes(int dim, int D, int s) {
    return (size_t(kBoxMullerTable) + size_t(vec_top_slots(dim, D)) * kVecBlock +
            size_t(kChunkSlots * (s + 1) * 3)) * sizeof(double);
}

// Component evaluator (any polynomial V): a level-independent structure stream (A.shape, ints) and
// per-level coefficient arrays (A.tab, A.stride doubles per level); layout in pimc_vector_impl.hpp,
// PolyEvalRT.
#ifndef PIMC_POLY_U
#define PIMC_POLY_U 5
#endif
#ifndef PIMC_POLY_U3
#define PIMC_POLY_U3 7
#endif
// Subtree levels of the component evaluator (1..7) in d = 1, 2 and in d = 3, 4: deeper than the radial
// kernels' 3, because its cost is a pass over the structure per slice batch, and deeper subtrees give
// fewer, wider batches (the points that do not fit the registers live in scratch).
constexpr int kPolyU = PIMC_POLY_U;
constexpr int kPolyU3 = PIMC_POLY_U3;
constexpr int poly_subtree_levels(int dim) { return dim >= 3 ? kPolyU3 : kPolyU; }
constexpr int kPolyMaxSlots = 1 << 20;  // coefficient slots per level

// Launch the vector estimation kernel: dim 1..4; U = min(s, kVecU); `specialized` selects the
// evaluator with the compile-time shape of level p (dim 2 or 3, U = kVecU), else the evaluator
// that reads the shape array. hipErrorInvalidValue for an unsupported combination.
hipError_t launch_vector(const VecArgs& A, int dim, int p, int U, bool specialized, int grid, hipStream_t st);
int vector_resident_blocks(int dim, int p, int U, bool specialized, size_t lds_bytes, int device);

// The component evaluator: A.tab = coefficients, A.shape = structure stream.
hipError_t launch_vector_poly(const VecArgs& A, int dim, int U, int grid, hipStream_t st);
int vector_poly_resident(int dim, int U, size_t lds_bytes, int device);

// Per-dimension halves (one translation unit each).
hipError_t launch_vector_d1(const VecArgs& A, int p, int U, bool specialized, int grid, hipStream_t st);
hipError_t launch_vector_d2(const VecArgs& A, int p, int U, bool specialized, int grid, hipStream_t st);
hipError_t launch_vector_d3(const VecArgs& A, int p, int U, bool specialized, int grid, hipStream_t st);
int vector_resident_d1(int p, int U, bool specialized, size_t lds, int device);
int vector_resident_d2(int p, int U, bool specialized, size_t lds, int device);
int vector_resident_d3(int p, int U, bool specialized, size_t lds, int device);
hipError_t launch_vector_d4(const VecArgs& A, int p, int U, bool specialized, int grid, hipStream_t st);
int vector_resident_d4(int p, int U, bool specialized, size_t lds, int device);
// The component evaluator's kernels, one translation unit per dimension (pimc_vector_poly.hip).
template <int DIM>
hipError_t launch_vector_poly_dim(const VecArgs& A, int U, int grid, hipStream_t st);
template <int DIM>
int vector_poly_resident_dim(int U, size_t lds, int device);
// Subtrees of kPolySplitU levels or more (the deepest, poly_subtree_levels(DIM)) are compiled in a
// translation unit of their own per dimension (pimc_vector_poly.hip with PIMC_POLY_DEEP), in
// parallel with the shallower ones; launch_vector_poly_dim forwards to them.
constexpr int kPolySplitU = 7;
template <int DIM>
hipError_t launch_vector_poly_deep(const VecArgs& A, int grid, hipStream_t st);
template <int DIM>
int vector_poly_resident_deep(size_t lds, int device);

}  // namespace pimc
