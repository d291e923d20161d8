// Spectrum from the space-discretized evolution operator: launchers shared by the kernels
// (pimc_spectrum.hip) and the host driver (pimc_spectrum_host.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pimc_device.hpp"

namespace pimc {

// The level-0 table of a problem with T = t (the short-time amplitude), device pointers.
struct SpecTable {
    const double* tab;      // folded P_k, highest power first, consecutive in k
    const int* deg;         // K degrees
    int K;
    int stride;             // doubles in the table
    int even;               // P_k in mid^2 (even potential) or mid
};

// M[i*ld + j] = pref * exp(-(y_j - y_i)^2/(2t) - t W_p) for the grid x_i = -L + (i + 1/2) D,
// y = sm x, i, j < n (device M, ld >= n).
hipError_t launch_evolution_matrix(const SpecTable& tb, double L, double D, double sm, double t, double pref,
                                   uint32_t n, double* M, uint64_t ld, hipStream_t st);
// Packed symmetric storage: tiles (I, J), I <= J, of kTile x kTile doubles, row-major within a tile,
// tile t at M + t * kTile^2 with map[t] = I << 16 | J in the order t = I*nb - I(I-1)/2 + (J - I),
// nb = ceil(n / kTile); elements beyond n are zero.
constexpr int kTile = 64;
hipError_t launch_evolution_tiles(const SpecTable& tb, double L, double D, double sm, double t, double pref,
                                  uint32_t n, const uint32_t* map, uint32_t ntiles, double* M, hipStream_t st);
// y = M x from the packed tiles: partial products per tile (prow, pcol: ntiles * kTile doubles each)
// then a fixed-order reduction per row block; x is read for indices < n only.
hipError_t launch_symv_tiles(const double* M, const uint32_t* map, uint32_t ntiles, uint32_t nb, uint32_t n,
                             const double* x, double* prow, double* pcol, double* y, hipStream_t st);
// y = M x (ld even; M and x 16-byte aligned).
hipError_t launch_gemv(const double* M, uint64_t ld, uint32_t n, const double* x, double* y, hipStream_t st);
// out[c] = <Q_c, w>, c < ncols (Q_c = Q + c*ldq); with diag non-null also *diag = out[diag_col].
hipError_t launch_col_dots(const double* Q, uint64_t ldq, uint32_t n, uint32_t ncols, const double* w, double* out,
                           hipStream_t st, double* diag = nullptr, uint32_t diag_col = 0);
// y = sum_c h[c] Q_c (subtract = 0) or y -= sum_c h[c] Q_c (subtract = 1).
hipError_t launch_combine_cols(const double* Q, uint64_t ldq, uint32_t n, uint32_t ncols, const double* h, double* y,
                               int subtract, hipStream_t st);
// beta[j] = |w|, qnext = w / beta[j].
hipError_t launch_normalize(const double* w, uint32_t n, double* beta, uint32_t j, double* qnext, hipStream_t st);

}  // namespace pimc
