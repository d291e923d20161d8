// Internal interface between the host library (pimc_host.cpp) and the kernels (pimc_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pimc_device.hpp"

namespace pimc {

constexpr int kBlock = 256;            // threads per workgroup (4 waves); also the lanes of a chunk

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
    uint64_t n_chunks;                 // ceil(n_paths / (kBlock * ppl))
    uint32_t ppl;                      // paths per lane per chunk
    int s;                             // N = 2^s
    int D;                             // s - U: levels walked with the explicit stack
    int hier;                          // evaluate every level (else level s only)
    double* partials;                  // device [level][chunk][4] or null
    double* dump;                      // device [path][s+1] or null
};

// Tanh64P: the Poeschl-Teller tables with the compile-time shape of level p (K = p groups of degree
// p), U = 4.
enum class EvalKind { Quartic64, Quartic32, GenericEven64, GenericOdd64, Tanh64, Tanh64P, General64 };

// Dynamic LDS bytes of the estimation kernel: per lane, 3D+2 slots of the explicit stack; per wave
// and level, three accumulators.
inline size_t amp_lds_bytes(int D, int s) {
    return (size_t(3 * D + 2) * kBlock + size_t(4 * (s + 1) * 3)) * sizeof(double);
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
    uint32_t ppl;
    uint32_t stream;
    int s;
    int pad;
};

// Persistent batched estimation for one level p and subtree depth U (quartic kernels, U = 4 for
// s = 4, U = 5 for s >= 5).
hipError_t launch_batch(const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue, uint32_t grab,
                        const RngKey& key, int hier, int p, int U, int grid, size_t lds, hipStream_t st);
int batch_resident_blocks(int p, int U, size_t lds_bytes, int device);
hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st);

// Occupancy-derived number of resident workgroups of the estimation kernel on this device.
int amplitude_resident_blocks(EvalKind kind, int p, int U, size_t lds_bytes, int device);

}  // namespace pimc
