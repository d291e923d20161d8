// Estimation kernels of the bisection PIMC amplitude (Sec. 4 of Balaz et al.) for gfx950: the walker
// (pimc_walker.hpp) with the runtime-shaped evaluators (any polynomial, Poeschl-Teller), raw normals,
// the canonical chunk reduction and the launch dispatch. The compile-time table shapes are
// instantiated in pimc_kernels_q64.hip, pimc_kernels_q32.hip, pimc_kernels_tanh.hip and
// pimc_general_kernels.hip (one translation unit per evaluator family, built in parallel) and the
// batched kernel in pimc_kernels_batch.hip and pimc_batch_p*.hip.
#include <hip/hip_runtime.h>

#include "pimc_walker.hpp"

namespace pimc {

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------- raw normals
// One thread per (path, node pair): nodes 2j and 2j+1 of path first_path + i, written where
// 1 <= node <= n_nodes.
__global__ void __launch_bounds__(kBlock) k_normals(RngKey key, uint64_t first_path, uint64_t k_paths,
                                                    uint32_t n_nodes, double* __restrict__ out) {
    __shared__ double bm[kBoxMullerTable];
    load_bm_table(bm, kBlock);
    __syncthreads();
    const uint32_t pairs = n_nodes / 2 + 1;
    const uint64_t gid = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (gid >= k_paths * pairs) return;
    const uint64_t i = gid / pairs;
    const uint32_t j = uint32_t(gid % pairs);
    const PathRng pr = path_rng(key, first_path + i);
    double ze, zo;
    normal_pair(key, pr, j, bm, ze, zo);
    double* o = out + i * n_nodes;
    const uint32_t he = 2 * j, ho = 2 * j + 1;
    if (he >= 1 && he <= n_nodes) o[he - 1] = ze;
    if (ho <= n_nodes) o[ho - 1] = zo;
}

hipError_t launch_normals(const RngKey& key, uint64_t first_path, uint64_t k_paths, uint32_t n_nodes, double* out,
                          hipStream_t st) {
    const uint64_t work = k_paths * (uint64_t(n_nodes) / 2 + 1);
    const uint64_t blocks = (work + kBlock - 1) / kBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_normals, dim3(uint32_t(blocks)), dim3(kBlock), 0, st, key, first_path, k_paths, n_nodes, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- chunk reduction
// Canonical reduction: segment i (one level of one run) is the sequence of chunk sums
// partials[base[i] + c*4 .. +3], c = 0..len[i]-1. One workgroup of kBlock threads per segment:
// thread t adds chunks t, t + kBlock, ... in order, then a fixed halving tree over the threads.
// The order depends only on the chunk count, so any run -- single or one task of a batch, any
// grid -- gives the same bits for the same chunks.
__global__ void __launch_bounds__(kBlock) k_seg_reduce(const double* __restrict__ partials,
                                                       const uint64_t* __restrict__ base,
                                                       const uint64_t* __restrict__ len,
                                                       double* __restrict__ out) {
    __shared__ double red[4][kBlock];
    const uint64_t seg = blockIdx.x;
    const int tid = threadIdx.x;
    const double* p = partials + base[seg];
    const uint64_t n = len[seg];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint64_t c = tid; c < n; c += kBlock) {
#pragma unroll
        for (int j = 0; j < 4; ++j) s[j] += p[c * 4 + j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) red[j][tid] = s[j];
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int j = 0; j < 4; ++j) red[j][tid] += red[j][tid + w];
        }
        __syncthreads();
    }
    if (tid < 4) out[seg * 4 + tid] = red[tid][0];
}

// ---------------------------------------------------------------------------- dispatch

template <bool EVEN>
static hipError_t launch_generic(const AmpArgs& A, int U, int grid, hipStream_t st) {
    GenericEval64<EVEN> ev{A.tab64, A.gdeg, A.gK, A.gstride};
    switch (U) {
        case 1: return launch_one<DefaultShape<1>>(A, ev, grid, st);
        case 2: return launch_one<DefaultShape<2>>(A, ev, grid, st);
        case 3: return launch_one<DefaultShape<3>>(A, ev, grid, st);
        case 4: return launch_one<DefaultShape<4>>(A, ev, grid, st);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_tanh(const AmpArgs& A, int U, int grid, hipStream_t st) {
    TanhEval64 ev{A.tab64, A.gdeg, A.gK, A.gstride, A.alpha};
    switch (U) {
        case 1: return launch_one<DefaultShape<1>>(A, ev, grid, st);
        case 2: return launch_one<DefaultShape<2>>(A, ev, grid, st);
        case 3: return launch_one<DefaultShape<3>>(A, ev, grid, st);
        case 4: return launch_one<DefaultShape<4>>(A, ev, grid, st);
        default: return hipErrorInvalidValue;
    }
}


hipError_t launch_amplitude(const AmpArgs& A, EvalKind kind, int p, int U, int grid, hipStream_t st) {
    switch (kind) {
        case EvalKind::Quartic64: return launch_quartic64(A, p, U, grid, st);
        case EvalKind::Quartic32: return launch_quartic32(A, p, U, grid, st);
        case EvalKind::GenericEven64: return launch_generic<true>(A, U, grid, st);
        case EvalKind::GenericOdd64: return launch_generic<false>(A, U, grid, st);
        case EvalKind::Tanh64: return launch_tanh(A, U, grid, st);
        case EvalKind::Tanh64P:
            if (U != 4) return hipErrorInvalidValue;
            return launch_tanh_fixed(A, p, grid, st);
        case EvalKind::General64: return launch_general_compiled(A, p, U, grid, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_seg_reduce(const double* partials, const uint64_t* base, const uint64_t* len, uint64_t n_seg,
                             double* out, hipStream_t st) {
    if (n_seg == 0) return hipSuccess;
    if (n_seg > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_seg_reduce, dim3(uint32_t(n_seg)), dim3(kBlock), 0, st, partials, base, len, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3((n + 63) / 64), dim3(64), 0, st, p, n, v);
    return hipGetLastError();
}



int amplitude_resident_blocks(EvalKind kind, int p, int U, size_t lds_bytes, int device) {
    switch (kind) {
        case EvalKind::Quartic64: return resident_quartic64(p, U, lds_bytes, device);
        case EvalKind::Quartic32: return resident_quartic32(p, U, lds_bytes, device);
        case EvalKind::GenericEven64:
        case EvalKind::GenericOdd64:
            switch (U) {
                case 1: return resident_one<DefaultShape<1>, GenericEval64<true>>(lds_bytes, device);
                case 2: return resident_one<DefaultShape<2>, GenericEval64<true>>(lds_bytes, device);
                case 3: return resident_one<DefaultShape<3>, GenericEval64<true>>(lds_bytes, device);
                default: return resident_one<DefaultShape<4>, GenericEval64<true>>(lds_bytes, device);
            }
        case EvalKind::Tanh64:
            switch (U) {
                case 1: return resident_one<DefaultShape<1>, TanhEval64>(lds_bytes, device);
                case 2: return resident_one<DefaultShape<2>, TanhEval64>(lds_bytes, device);
                case 3: return resident_one<DefaultShape<3>, TanhEval64>(lds_bytes, device);
                default: return resident_one<DefaultShape<4>, TanhEval64>(lds_bytes, device);
            }
        case EvalKind::Tanh64P:
            return resident_tanh_fixed(p, lds_bytes, device);
        case EvalKind::General64:
            return general_compiled_resident(p, U, lds_bytes, device);
    }
    return 256;
}

}  // namespace pimc
