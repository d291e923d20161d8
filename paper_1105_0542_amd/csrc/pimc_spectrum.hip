// Energy spectrum from the space-discretized evolution operator (the paper's application of
// short-time amplitudes): the matrix M_ij = D A_1^(p)(x_i, x_j; t) on a grid, and the kernels of
// a Lanczos iteration with full reorthogonalization that finds its largest eigenvalues
// exp(-t E_n). Everything stays on the device; every reduction has a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pimc_spectrum.hpp"

namespace pimc {

constexpr int kMatCols = 4;           // matrix elements per thread (consecutive columns)
#ifndef PIMC_SYMV_BLOCKS_PER_CU
#define PIMC_SYMV_BLOCKS_PER_CU 8
#endif
constexpr int kSymvBlocksPerCU = PIMC_SYMV_BLOCKS_PER_CU;   // workgroups of the tiled product per CU
constexpr double kGaussCut = 40.0;    // elements with (y_j - y_i)^2 / (2t) > kGaussCut are zero

// Element (i, j): pref * exp(-(y_j - y_i)^2 / (2t) - t W_p((y_i + y_j)/2, (y_j - y_i)/2; t)) with
// y = sqrt(m) x, x_i = -L + (i + 1/2) D, pref = D sqrt(m) / sqrt(2 pi t); exactly zero where the
// free-particle exponent (y_j - y_i)^2 / (2t) exceeds kGaussCut. The expansion in the half-deviation
// has a finite radius (Sec. 4), so far from the diagonal the truncated exponent may grow without
// bound where the true amplitude is below exp(-kGaussCut) of the free one.
template <bool EVEN>
__global__ void __launch_bounds__(256) k_evolution_matrix(SpecTable tb, double L, double D, double sm, double t,
                                                          double pref, uint32_t n, double* __restrict__ M,
                                                          uint64_t ld) {
    const uint32_t i = blockIdx.y;
    const uint32_t j0 = (blockIdx.x * 256u + threadIdx.x) * kMatCols;
    if (j0 >= n) return;
    const double yi = sm * ((double(i) + 0.5) * D - L);
    double qa[kMatCols], qb[kMatCols], S[kMatCols];
#pragma unroll
    for (int c = 0; c < kMatCols; ++c) {
        const uint32_t j = min(j0 + c, n - 1);
        qa[c] = yi;
        qb[c] = sm * ((double(j) + 0.5) * D - L);
    }
    const GenericEval64<EVEN> ev{tb.tab, tb.deg, tb.K, tb.stride};
    ev.template values<kMatCols>(0, qa, qb, S);
    double* row = M + uint64_t(i) * ld;
#pragma unroll
    for (int c = 0; c < kMatCols; ++c) {
        if (j0 + c < n) {
            const double dl = qb[c] - qa[c];
            const double g = (dl * dl) / (2.0 * t);
            row[j0 + c] = g > kGaussCut ? 0.0 : pref * exp_fp64(-g - S[c]);
        }
    }
}

// ---------------------------------------------------------------------------- packed symmetric form
// The matrix is exactly symmetric (its elements depend on (y_j - y_i)^2 and y_i + y_j only), so the
// eigenvalue iteration keeps only the tiles (I, J), I <= J, of kTile x kTile elements: tile t holds
// rows I*kTile.. and columns J*kTile.. row-major (kTile^2 doubles), diagonal tiles in full, elements
// beyond n zero; map[t] = I << 16 | J. Half the bytes to build and to stream per product.

// Tile t of the packed matrix: each thread computes kTile^2 / 256 elements, kMatCols consecutive
// columns at a time, with the arithmetic of k_evolution_matrix (identical elements).
template <bool EVEN>
__global__ void __launch_bounds__(256) k_evolution_tiles(SpecTable tb, double L, double D, double sm, double t,
                                                         double pref, uint32_t n, const uint32_t* __restrict__ map,
                                                         double* __restrict__ M) {
    const uint32_t code = map[blockIdx.x];
    const uint32_t I = code >> 16, J = code & 0xffffu;
    double* tile = M + uint64_t(blockIdx.x) * (kTile * kTile);
    const GenericEval64<EVEN> ev{tb.tab, tb.deg, tb.K, tb.stride};
    constexpr int kGroups = kTile / kMatCols;                       // column groups per tile row
    for (int task = threadIdx.x; task < kTile * kGroups; task += 256) {
        const int r = task / kGroups;
        const int c0 = (task % kGroups) * kMatCols;
        const uint32_t i = I * kTile + uint32_t(r);
        const uint32_t ii = min(i, n - 1);
        const double yi = sm * ((double(ii) + 0.5) * D - L);
        double qa[kMatCols], qb[kMatCols], S[kMatCols];
#pragma unroll
        for (int c = 0; c < kMatCols; ++c) {
            const uint32_t j = min(J * kTile + uint32_t(c0 + c), n - 1);
            qa[c] = yi;
            qb[c] = sm * ((double(j) + 0.5) * D - L);
        }
        ev.template values<kMatCols>(0, qa, qb, S);
#pragma unroll
        for (int c = 0; c < kMatCols; ++c) {
            const uint32_t j = J * kTile + uint32_t(c0 + c);
            double v = 0.0;
            if (i < n && j < n) {
                const double dl = qb[c] - qa[c];
                const double g = (dl * dl) / (2.0 * t);
                v = g > kGaussCut ? 0.0 : pref * exp_fp64(-g - S[c]);
            }
            tile[r * kTile + c0 + c] = v;
        }
    }
}

// Partial products of tile t: prow[t] = M_IJ x_J (rows of block I) and, off the diagonal,
// pcol[t] = M_IJ^T x_I (rows of block J). Wave w streams rows 16w..16w+15 (one row of 64 doubles per
// load, lane = column); the column partial accumulates in the lane, the sixteen row partials are
// reduced across the lanes by a halving butterfly (16 + 8 + ... values exchanged), after which
// row 16w + (lane >> 2) is held by lanes with lane & 3 == 0. Fixed order throughout.
// One step of the halving butterfly: lanes with bit MASK set keep the upper HALF of their values and
// send the lower half to the partner lane (and the other way round), then add what they receive.
template <int HALF, int MASK>
__device__ __forceinline__ void fold_rows(double (&v)[16], int lane) {
    if constexpr (HALF >= 1) {
        const bool hi = (lane & MASK) != 0;
#pragma unroll
        for (int k = 0; k < HALF; ++k) {
            const double send = hi ? v[k] : v[k + HALF];
            const double keep = hi ? v[k + HALF] : v[k];
            v[k] = keep + __shfl_xor(send, MASK, 64);
        }
        fold_rows<HALF / 2, MASK / 2>(v, lane);
    }
}

__global__ void __launch_bounds__(256) k_symv_tiles(const double* __restrict__ M, const uint32_t* __restrict__ map,
                                                    uint32_t ntiles, uint32_t n, const double* __restrict__ x,
                                                    double* __restrict__ prow, double* __restrict__ pcol) {
    static_assert(kTile == 64, "one lane per tile column");
    __shared__ double colpart[4][kTile];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // a few workgroups per CU, each streaming many tiles (one tile is only 32 KB)
    for (uint32_t tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        const uint32_t code = map[tt];
        const uint32_t I = code >> 16, J = code & 0xffffu;
        const uint32_t jc = J * kTile + uint32_t(lane);
        const double xj = jc < n ? x[jc] : 0.0;                     // x beyond n is not read
        const double* tile = M + uint64_t(tt) * (kTile * kTile) + uint64_t(wave) * 16 * kTile + lane;
        // first row of this wave: wave-uniform, so its x values come by scalar loads
        const uint32_t i0 = I * kTile + uint32_t(__builtin_amdgcn_readfirstlane(wave)) * 16;
        double v[16];
        double cs = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const double m = __builtin_nontemporal_load(tile + r * kTile);
            const uint32_t ri = i0 + uint32_t(r);
            const double xr = ri < n ? x[ri < n ? ri : n - 1] : 0.0;      // x beyond n is not used
            v[r] = m * xj;
            cs = fma(m, xr, cs);
        }
        // rows: 16 values per lane -> one row sum per group of four lanes
        fold_rows<8, 32>(v, lane);
        v[0] += __shfl_xor(v[0], 2, 64);
        v[0] += __shfl_xor(v[0], 1, 64);
        if ((lane & 3) == 0) prow[uint64_t(tt) * kTile + uint32_t(wave * 16 + (lane >> 2))] = v[0];
        if (I != J) {
            colpart[wave][lane] = cs;
            __syncthreads();
            if (wave == 0)
                pcol[uint64_t(tt) * kTile + uint32_t(lane)] =
                    ((colpart[0][lane] + colpart[1][lane]) + colpart[2][lane]) + colpart[3][lane];
            __syncthreads();                                        // colpart is reused by the next tile
        }
    }
}

// y for row block I (one workgroup per block, lane = row): the nb partials of the block in a fixed
// order, q = 0..nb-1 with q < I the column partial of tile (q, I) and q >= I the row partial of tile
// (I, q); wave w takes q = w, w + 4, ..., the four wave sums are added in wave order.
__global__ void __launch_bounds__(256) k_symv_reduce(const double* __restrict__ prow, const double* __restrict__ pcol,
                                                     uint32_t n, uint32_t nb, double* __restrict__ y) {
    __shared__ double part[4][kTile];
    const uint32_t I = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    double s = 0.0;
#pragma unroll 8
    for (uint32_t q = uint32_t(wave); q < nb; q += 4) {
        const uint32_t a = q < I ? q : I, b = q < I ? I : q;       // tile (a, b), a <= b
        const uint64_t t = uint64_t(a) * nb - uint64_t(a) * (a - (a > 0 ? 1 : 0)) / 2 + (b - a);
        s += q < I ? pcol[t * kTile + uint32_t(lane)] : prow[t * kTile + uint32_t(lane)];
    }
    part[wave][lane] = s;
    __syncthreads();
    if (wave == 0) {
        const uint32_t i = I * kTile + uint32_t(lane);
        if (i < n) y[i] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    }
}

// y = M x, M dense n x n with leading dimension ld (even, 16-byte aligned rows): a wave takes four
// consecutive rows, lanes stride the columns two at a time, then a fixed butterfly.
__global__ void __launch_bounds__(256) k_gemv4(const double* __restrict__ M, uint64_t ld, uint32_t n,
                                               const double* __restrict__ x, double* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    const uint32_t row0 = (blockIdx.x * 4u + (threadIdx.x >> 6)) * 4u;
    if (row0 >= n) return;
    const uint32_t nr = min(4u, n - row0);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double* r0 = M + uint64_t(row0) * ld;
    for (uint32_t c = 2u * lane; c < n; c += 128u) {
        if (c + 1 < n) {
            const double2 xv = *reinterpret_cast<const double2*>(x + c);
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
                if (r < nr) {
                    const double2 mv = *reinterpret_cast<const double2*>(r0 + r * ld + c);
                    acc[r] = fma(mv.x, xv.x, acc[r]);
                    acc[r] = fma(mv.y, xv.y, acc[r]);
                }
            }
        } else {
            const double xv = x[c];
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r)
                if (r < nr) acc[r] = fma(r0[r * ld + c], xv, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double v = acc[r];
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        acc[r] = v;
    }
    if (lane == 0)
        for (uint32_t r = 0; r < nr; ++r) y[row0 + r] = acc[r];
}

// Fixed-order sum of v over one workgroup of 256 threads (result valid in thread 0).
__device__ __forceinline__ double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    return red[0];
}

// out[c] = sum_i Q[c*ldq + i] w[i], c = 0..ncols-1: one workgroup per column.
// This thread's part of sum_i a[i] b[i] over i = threadIdx.x + 256 k: eight independent partial
// sums (eight loads in flight), combined pairwise in a fixed order.
__device__ __forceinline__ double dot_strided(const double* __restrict__ a, const double* __restrict__ b,
                                              uint32_t n) {
    double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    uint32_t i = threadIdx.x;
    for (; i + 7u * 256u < n; i += 8u * 256u) {
#pragma unroll
        for (int u = 0; u < 8; ++u) p[u] = fma(a[i + u * 256u], b[i + u * 256u], p[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (i + u * 256u < n) p[u] = fma(a[i + u * 256u], b[i + u * 256u], p[u]);
    return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
}

__global__ void __launch_bounds__(256) k_col_dots(const double* __restrict__ Q, uint64_t ldq, uint32_t n,
                                                  const double* __restrict__ w, double* __restrict__ out,
                                                  double* __restrict__ diag, uint32_t diag_col) {
    __shared__ double red[256];
    const uint32_t c = blockIdx.x;
    const double* q = Q + uint64_t(c) * ldq;
    double s = dot_strided(q, w, n);
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        out[c] = s;
        if (diag && c == diag_col) *diag = s;
    }
}

// y[i] (+)= sign * sum_{c < ncols} Q[c*ldq + i] h[c]: the Gram-Schmidt correction (sign -1, added to
// y) or a Ritz vector (sign +1, y overwritten).
__global__ void k_combine_cols(const double* __restrict__ Q, uint64_t ldq, uint32_t n, uint32_t ncols,
                               const double* __restrict__ h, double* __restrict__ y, int subtract) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (uint32_t c = 0; c < ncols; ++c) s = fma(Q[uint64_t(c) * ldq + i], h[c], s);
    y[i] = subtract ? y[i] - s : s;
}

// beta[j] = |w| (one workgroup).
__global__ void __launch_bounds__(256) k_norm(const double* __restrict__ w, uint32_t n, double* __restrict__ beta,
                                              uint32_t j) {
    __shared__ double red[256];
    double s = dot_strided(w, w, n);
    s = block_sum(s, red);
    if (threadIdx.x == 0) beta[j] = sqrt(s);
}

// q_{j+1} = w / beta[j] (zero vector if |w| = 0), over the whole vector in parallel (one workgroup
// doing both the norm and the scaling took as long as the two launches: 9.6 us against 4.3 + 4.7).
__global__ void k_scale_by_norm(const double* __restrict__ w, uint32_t n, const double* __restrict__ beta, uint32_t j,
                                double* __restrict__ qnext) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n) return;
    const double nrm = beta[j];
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    qnext[i] = w[i] * inv;
}

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return uint32_t((a + b - 1) / b); }

hipError_t launch_evolution_matrix(const SpecTable& tb, double L, double D, double sm, double t, double pref,
                                   uint32_t n, double* M, uint64_t ld, hipStream_t st) {
    if (n == 0 || ld < n) return hipErrorInvalidValue;
    const dim3 grid(cdiv(n, 256u * kMatCols), n);
    if (tb.even)
        hipLaunchKernelGGL(k_evolution_matrix<true>, grid, dim3(256), 0, st, tb, L, D, sm, t, pref, n, M, ld);
    else
        hipLaunchKernelGGL(k_evolution_matrix<false>, grid, dim3(256), 0, st, tb, L, D, sm, t, pref, n, M, ld);
    return hipGetLastError();
}

hipError_t launch_evolution_tiles(const SpecTable& tb, double L, double D, double sm, double t, double pref,
                                  uint32_t n, const uint32_t* map, uint32_t ntiles, double* M, hipStream_t st) {
    if (n == 0 || ntiles == 0) return hipErrorInvalidValue;
    if (tb.even)
        hipLaunchKernelGGL(k_evolution_tiles<true>, dim3(ntiles), dim3(256), 0, st, tb, L, D, sm, t, pref, n, map, M);
    else
        hipLaunchKernelGGL(k_evolution_tiles<false>, dim3(ntiles), dim3(256), 0, st, tb, L, D, sm, t, pref, n, map, M);
    return hipGetLastError();
}

hipError_t launch_symv_tiles(const double* M, const uint32_t* map, uint32_t ntiles, uint32_t nb, uint32_t n,
                             const double* x, double* prow, double* pcol, double* y, hipStream_t st) {
    if (n == 0 || ntiles != nb * (nb + 1) / 2 || nb != (n + kTile - 1) / kTile) return hipErrorInvalidValue;
    int ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 256;
    const uint32_t grid = std::min<uint32_t>(ntiles, uint32_t(kSymvBlocksPerCU * ncu));
    hipLaunchKernelGGL(k_symv_tiles, dim3(grid), dim3(256), 0, st, M, map, ntiles, n, x, prow, pcol);
    hipLaunchKernelGGL(k_symv_reduce, dim3(nb), dim3(256), 0, st, prow, pcol, n, nb, y);
    return hipGetLastError();
}

hipError_t launch_gemv(const double* M, uint64_t ld, uint32_t n, const double* x, double* y, hipStream_t st) {
    if (ld % 2 || (reinterpret_cast<uintptr_t>(M) & 15) || (reinterpret_cast<uintptr_t>(x) & 15))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemv4, dim3(cdiv(n, 16)), dim3(256), 0, st, M, ld, n, x, y);
    return hipGetLastError();
}

hipError_t launch_col_dots(const double* Q, uint64_t ldq, uint32_t n, uint32_t ncols, const double* w, double* out,
                           hipStream_t st, double* diag, uint32_t diag_col) {
    hipLaunchKernelGGL(k_col_dots, dim3(ncols), dim3(256), 0, st, Q, ldq, n, w, out, diag, diag_col);
    return hipGetLastError();
}

hipError_t launch_combine_cols(const double* Q, uint64_t ldq, uint32_t n, uint32_t ncols, const double* h, double* y,
                               int subtract, hipStream_t st) {
    hipLaunchKernelGGL(k_combine_cols, dim3(cdiv(n, 256)), dim3(256), 0, st, Q, ldq, n, ncols, h, y, subtract);
    return hipGetLastError();
}

hipError_t launch_normalize(const double* w, uint32_t n, double* beta, uint32_t j, double* qnext, hipStream_t st) {
    hipLaunchKernelGGL(k_norm, dim3(1), dim3(256), 0, st, w, n, beta, j);
    hipLaunchKernelGGL(k_scale_by_norm, dim3(cdiv(n, 256)), dim3(256), 0, st, w, n, beta, j, qnext);
    return hipGetLastError();
}

}  // namespace pimc
