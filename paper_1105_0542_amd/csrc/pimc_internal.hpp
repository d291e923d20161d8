// Internal interface between the host library (pimc_host.cpp) and the kernels (pimc_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pimc.h"
#include "pimc_device.hpp"

namespace pimc {

constexpr int kBlock = 256;            // threads per workgroup of the auxiliary kernels (4 waves)

// Canonical chunk of the estimators: kChunkPaths consecutive path indices, in kChunkGroups groups of
// 64 consecutive paths (the lanes of one wave). A group's per-level sums are a wave butterfly;
// group g is added to accumulator slot g mod kChunkSlots, each slot in increasing g, and the chunk
// sum is slot 0 + slot 1 + slot 2 + slot 3. The order is fixed by the path indices alone, so the
// chunk sums -- and the amplitudes -- do not depend on the workgroup size (64, 128 or 256 lanes:
// wave w of a workgroup of W waves takes groups w, w + W, ..., and no two waves share a slot), on
// the subtree depth or slice batch of the walker, on N (level n of an s-run is bitwise the n-run),
// or on which workgroup ran the chunk.
constexpr uint32_t kChunkPaths = PIMC_CHUNK_PATHS;
constexpr int kChunkGroups = int(kChunkPaths / 64);
constexpr int kChunkSlots = 4;

// Launch shape of the estimation walker: U bisection levels of each subtree in registers
// (2^U + 1 points), BS threads per workgroup, occupancy target WPE waves per SIMD (register budget
// 512/WPE), slices evaluated together coefficient-major (BATCH). Every shape gives the same bits.
template <int U_, int BS_, int WPE_, int BATCH_>
struct Shape {
    static constexpr int U = U_;
    static constexpr int BS = BS_;
    static constexpr int WPE = WPE_;
    static constexpr int BATCH = BATCH_;
    static_assert(BS_ == 64 || BS_ == 128 || BS_ == 256, "workgroup of 1, 2 or 4 waves");
};
// The default shapes: 256 threads, 2 waves per SIMD, 16 slices at once, U-level subtrees (the
// quartic kernels use U = 4: measured fastest on MI355X at p = 8, 12 and 18 for N from 64 to 1024;
// U = 5 needs more registers than 2 waves per SIMD leave and spills to scratch).
template <int U>
using DefaultShape = Shape<U, 256, 2, 16>;

// Arguments of one estimation launch (passed by value in the kernel argument segment, so every
// field is wave-uniform and scalar-loaded).
struct AmpArgs {
    const double* tab64;               // device: level tables, level-major
    const float* tab32;                // device: FP32 copy (PIMC_FP32_POLY)
    const int* gdeg;                   // device: generic shape, degree of each P_k
    int gK;                            // generic shape: number of P_k
    int gstride;                       // generic shape: doubles per level table
    double a, b;                       // endpoints (after the mass rescaling)
    double alpha;                      // Poeschl-Teller: tanh argument scale (after the mass rescaling)
    GenTables gen;                     // general-potential mode: derivative tables (coefficients in tab64)
    const double* sig;                 // device: sigma_n = sqrt(T / 2^(n+1)), n = 0..s (0 unused)
    const double* shift;               // device: straight-line level action S_ref,n, n = 0..s
    RngKey key;
    uint64_t first_path;               // path index of local path 0
    uint64_t n_paths;                  // local paths 0..n_paths-1
    uint64_t n_chunks;                 // ceil(n_paths / kChunkPaths)
    int s;                             // N = 2^s
    int D;                             // s - U: levels walked with the explicit stack
    int hier;                          // evaluate every level (else level s only)
    double* partials;                  // device [level][chunk][4] or null
    double* dump;                      // device [path][s+1] or null
    unsigned long long* queue;         // device chunk counter, 0 at launch (persistent kernel), or null
                                       // for a grid-stride loop over the chunks
};

// Tanh64P: the Poeschl-Teller tables with the compile-time shape of level p (K = p groups of degree
// p), U = 4.
enum class EvalKind { Quartic64, Quartic32, GenericEven64, GenericOdd64, Tanh64, Tanh64P, General64 };

// Dynamic LDS bytes of the estimation kernel: the Box-Muller table; per lane, 3D+2 slots of the
// explicit stack; per accumulator slot and level, three sums.
inline size_t amp_lds_bytes(int D, int s, int BS) {
    return (size_t(kBoxMullerTable) + size_t(3 * D + 2) * size_t(BS) + size_t(kChunkSlots * (s + 1) * 3)) *
           sizeof(double);
}

// Launch the estimation kernel; p selects the quartic specialization, U = s - D the unrolled
// subtree depth. Returns hipErrorInvalidValue for an unsupported combination.
hipError_t launch_amplitude(const AmpArgs& A, EvalKind kind, int p, int U, int grid, hipStream_t st);

// The compile-time shapes of level p with U = 4 (pimc_kernels_q64.hip, pimc_kernels_q32.hip,
// pimc_kernels_tanh.hip): hipErrorInvalidValue / 256 for p outside 1..kMaxP.
hipError_t launch_quartic64(const AmpArgs& A, int p, int U, int grid, hipStream_t st);
hipError_t launch_quartic32(const AmpArgs& A, int p, int U, int grid, hipStream_t st);
hipError_t launch_tanh_fixed(const AmpArgs& A, int p, int grid, hipStream_t st);
int resident_quartic64(int p, int U, size_t lds_bytes, int device);
int resident_quartic32(int p, int U, size_t lds_bytes, int device);
int resident_tanh_fixed(int p, size_t lds_bytes, int device);

// General-potential mode (pimc_general_kernels.hip): the evaluators generated for level p; the
// number of monomials of the level-p table (-1 outside 1..kGenMaxP).
hipError_t launch_general_compiled(const AmpArgs& A, int p, int U, int grid, hipStream_t st);
int general_compiled_resident(int p, int U, size_t lds_bytes, int device);
int general_compiled_nrec(int p);
// The levels above kGenInlineMaxP, one translation unit each (pimc_general_hi.hip built with
// PIMC_GEN_P = p): launch, resident workgroups per CU and monomial count of that level's evaluator.
template <int P>
hipError_t gen_hi_launch(const AmpArgs& A, int U, int grid, hipStream_t st);
template <int P>
int gen_hi_resident(int U, size_t lds_bytes, int device);
template <int P>
int gen_hi_nrec();
#define PIMC_GEN_HI_DECLARE(P)                                                         \
    template <>                                                                         \
    hipError_t gen_hi_launch<P>(const AmpArgs& A, int U, int grid, hipStream_t st);    \
    template <>                                                                         \
    int gen_hi_resident<P>(int U, size_t lds_bytes, int device);                        \
    template <>                                                                         \
    int gen_hi_nrec<P>();
PIMC_GEN_HI_DECLARE(11)
PIMC_GEN_HI_DECLARE(12)
PIMC_GEN_HI_DECLARE(13)
PIMC_GEN_HI_DECLARE(14)
PIMC_GEN_HI_DECLARE(15)
PIMC_GEN_HI_DECLARE(16)
PIMC_GEN_HI_DECLARE(17)
PIMC_GEN_HI_DECLARE(18)
#undef PIMC_GEN_HI_DECLARE

// Raw standard normals of heap nodes 1..n_nodes for k_paths paths: out[path][node-1] (device).
hipError_t launch_normals(const RngKey& key, uint64_t first_path, uint64_t k_paths, uint32_t n_nodes, double* out,
                          hipStream_t st);

// Canonical reduction: segment i = len[i] chunk sums of 4 doubles at partials + base[i], added in a
// fixed order that depends only on len[i]; out[i][4] (all device).
hipError_t launch_seg_reduce(const double* partials, const uint64_t* base, const uint64_t* len, uint64_t n_seg,
                             double* out, hipStream_t st);

// One task of a batch, as the persistent kernel reads it (device array, wave-uniform loads).
struct BatchTask {
    const double* tab;                 // level tables of the task's (system, T, p), quartic layout
    const double* sig;                 // sigma_n, n = 0..s
    const double* shift;               // S_ref,n, n = 0..s
    double* partials;                  // [slot][chunk][4]
    double a, b;                       // endpoints after the mass rescaling
    uint64_t n_paths;
    uint64_t n_chunks;
    uint64_t item0;                    // queue index of the task's chunk 0
    uint32_t stream;
    int s;
};

// A launch shape as the host sees it.
struct ShapeDesc {
    int U, BS, WPE, BATCH;
};

// Batched estimation (pimc_kernels_batch.hip). A class is the tasks of one level p with N = 16
// (n16: subtrees of at most 4 levels) or with N >= 32; shape selects one of its compiled launch
// shapes (0 = the default; levels 8, 12 and 18 have several for the autotuner, every other level
// only the default).
int batch_shape_count(int p, bool n16);
bool batch_shape(int p, bool n16, int idx, ShapeDesc& d);
hipError_t launch_batch(const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue, uint32_t grab,
                        const RngKey& key, int hier, int p, bool n16, int shape, int grid, size_t lds, hipStream_t st);
int batch_resident_blocks(int p, bool n16, int shape, size_t lds_bytes, int device);
hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st);

// Occupancy-derived number of resident workgroups of the estimation kernel on this device.
int amplitude_resident_blocks(EvalKind kind, int p, int U, size_t lds_bytes, int device);

}  // namespace pimc
