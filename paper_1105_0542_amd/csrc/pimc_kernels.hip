// Estimation kernels of the bisection PIMC amplitude (Sec. 4 of Balaz et al.) for gfx950: the
// instantiations of the walker (pimc_walker.hpp) for the polynomial, Poeschl-Teller and FP32 slice
// evaluators, the persistent batched kernel, raw normals, the canonical chunk reduction and the
// launch dispatch.
#include <hip/hip_runtime.h>

#include "pimc_walker.hpp"

namespace pimc {

// ---------------------------------------------------------------------------- batched tasks
// Persistent kernel over the (task, chunk) items of one effective-action level p: each workgroup
// takes `grab` consecutive items at a time from an atomic counter until the queue is empty (every
// wave of every workgroup reaches the exit test with the same value). Items are numbered task by
// task (task t owns items item0[t] .. item0[t] + n_chunks[t] - 1), so an item maps to its task by
// binary search over the wave-uniform task records; the chunk itself is processed by the same code
// as a single-task launch, so results do not depend on which workgroup took which item.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return (uint64_t(hi) << 32) | lo;
}

template <int U, class Eval>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PIMC_WAVES_PER_EU)))
k_batch(const BatchTask* __restrict__ tasks, int n_tasks, uint64_t n_items, unsigned long long* queue,
        uint32_t grab, RngKey key, int hier, Eval ev0) {
    extern __shared__ double smem[];
    __shared__ unsigned long long s_item;
    const const_ptr<BatchTask> T = as_const(tasks);
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(queue, (unsigned long long)grab);
        __syncthreads();
        const uint64_t first = uniform_u64(s_item);
        if (first >= n_items) break;
        const uint64_t last = first + grab < n_items ? first + grab : n_items;
        for (uint64_t item = first; item < last; ++item) {
            int lo = 0, hi = n_tasks - 1;                  // last task with item0 <= item
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (T[mid].item0 <= item) lo = mid; else hi = mid - 1;
            }
            AmpArgs A;
            A.tab64 = T[lo].tab;
            A.tab32 = nullptr;
            A.gdeg = nullptr;
            A.gK = 0;
            A.gstride = 0;
            A.a = T[lo].a;
            A.b = T[lo].b;
            A.sig = T[lo].sig;
            A.shift = T[lo].shift;
            A.key = key;
            A.key.stream = T[lo].stream;
            A.first_path = 0;
            A.n_paths = T[lo].n_paths;
            A.n_chunks = T[lo].n_chunks;
            A.ppl = T[lo].ppl;
            A.s = T[lo].s;
            A.D = T[lo].s - U;
            A.hier = hier;
            A.partials = T[lo].partials;
            A.dump = nullptr;
            Eval ev = ev0;
            ev.tab = T[lo].tab;
            process_chunk<U, Eval>(ev, A, item - T[lo].item0, smem);
        }
    }
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------- raw normals
// One thread per (path, node pair): nodes 2j and 2j+1 of path first_path + i, written where
// 1 <= node <= n_nodes.
__global__ void __launch_bounds__(kBlock) k_normals(RngKey key, uint64_t first_path, uint64_t k_paths,
                                                    uint32_t n_nodes, double* __restrict__ out) {
    const uint32_t pairs = n_nodes / 2 + 1;
    const uint64_t gid = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (gid >= k_paths * pairs) return;
    const uint64_t i = gid / pairs;
    const uint32_t j = uint32_t(gid % pairs);
    const PathRng pr = path_rng(key, first_path + i);
    double ze, zo;
    normal_pair(key, pr, j, ze, zo);
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

template <int P>
static hipError_t launch_quartic(const AmpArgs& A, bool fp32, int grid, hipStream_t st) {
    if (fp32) {
        QuarticEval32<P> ev{A.tab32};
        return launch_one<4>(A, ev, grid, st);
    }
    QuarticEval64<P> ev{A.tab64};
    return launch_one<4>(A, ev, grid, st);
}

template <bool EVEN>
static hipError_t launch_generic(const AmpArgs& A, int U, int grid, hipStream_t st) {
    GenericEval64<EVEN> ev{A.tab64, A.gdeg, A.gK, A.gstride};
    switch (U) {
        case 1: return launch_one<1>(A, ev, grid, st);
        case 2: return launch_one<2>(A, ev, grid, st);
        case 3: return launch_one<3>(A, ev, grid, st);
        case 4: return launch_one<4>(A, ev, grid, st);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t launch_tanh_fixed(const AmpArgs& A, int p, int grid, hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p != P) return launch_tanh_fixed<P + 1>(A, p, grid, st);
        TanhEvalP<P> ev{A.tab64, A.alpha};
        return launch_one<4>(A, ev, grid, st);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int P>
static int resident_tanh_fixed(int p, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p != P) return resident_tanh_fixed<P + 1>(p, lds, device);
        return resident_one<4, TanhEvalP<P>>(lds, device);
    } else {
        return 256;
    }
}

static hipError_t launch_tanh(const AmpArgs& A, int U, int grid, hipStream_t st) {
    TanhEval64 ev{A.tab64, A.gdeg, A.gK, A.gstride, A.alpha};
    switch (U) {
        case 1: return launch_one<1>(A, ev, grid, st);
        case 2: return launch_one<2>(A, ev, grid, st);
        case 3: return launch_one<3>(A, ev, grid, st);
        case 4: return launch_one<4>(A, ev, grid, st);
        default: return hipErrorInvalidValue;
    }
}


template <int P>
static hipError_t quartic_dispatch(const AmpArgs& A, bool fp32, int p, int grid, hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p == P) return launch_quartic<P>(A, fp32, grid, st);
        return quartic_dispatch<P + 1>(A, fp32, p, grid, st);
    } else {
        return hipErrorInvalidValue;
    }
}

hipError_t launch_amplitude(const AmpArgs& A, EvalKind kind, int p, int U, int grid, hipStream_t st) {
    switch (kind) {
        case EvalKind::Quartic64:
        case EvalKind::Quartic32:
            if (U != 4) return hipErrorInvalidValue;
            return quartic_dispatch<1>(A, kind == EvalKind::Quartic32, p, grid, st);
        case EvalKind::GenericEven64: return launch_generic<true>(A, U, grid, st);
        case EvalKind::GenericOdd64: return launch_generic<false>(A, U, grid, st);
        case EvalKind::Tanh64: return launch_tanh(A, U, grid, st);
        case EvalKind::Tanh64P:
            if (U != 4) return hipErrorInvalidValue;
            return launch_tanh_fixed<1>(A, p, grid, st);
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

template <int P>
static hipError_t batch_quartic(const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue,
                                uint32_t grab, RngKey key, int hier, int p, int grid, size_t lds, hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p != P) return batch_quartic<P + 1>(tasks, n_tasks, n_items, queue, grab, key, hier, p, grid, lds, st);
        QuarticEval64<P> ev{nullptr};
        hipLaunchKernelGGL((k_batch<4, QuarticEval64<P>>), dim3(grid), dim3(kBlock), lds, st, tasks, n_tasks, n_items,
                           queue, grab, key, hier, ev);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

hipError_t launch_batch(const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue, uint32_t grab,
                        const RngKey& key, int hier, int p, int grid, size_t lds, hipStream_t st) {
    return batch_quartic<1>(tasks, n_tasks, n_items, queue, grab, key, hier, p, grid, lds, st);
}

template <int P>
static int batch_resident(int p, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p != P) return batch_resident<P + 1>(p, lds, device);
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<4, QuarticEval64<P>>, kBlock, lds) != hipSuccess)
            per_cu = 1;
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) ncu = 256;
        return (per_cu < 1 ? 1 : per_cu) * ncu;
    } else {
        return 256;
    }
}

int batch_resident_blocks(int p, size_t lds_bytes, int device) { return batch_resident<1>(p, lds_bytes, device); }


template <int P>
static int resident_quartic(bool fp32, int p, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p == P) return fp32 ? resident_one<4, QuarticEval32<P>>(lds, device) : resident_one<4, QuarticEval64<P>>(lds, device);
        return resident_quartic<P + 1>(fp32, p, lds, device);
    } else {
        return 256;
    }
}

int amplitude_resident_blocks(EvalKind kind, int p, int U, size_t lds_bytes, int device) {
    switch (kind) {
        case EvalKind::Quartic64: return resident_quartic<1>(false, p, lds_bytes, device);
        case EvalKind::Quartic32: return resident_quartic<1>(true, p, lds_bytes, device);
        case EvalKind::GenericEven64:
        case EvalKind::GenericOdd64:
            switch (U) {
                case 1: return resident_one<1, GenericEval64<true>>(lds_bytes, device);
                case 2: return resident_one<2, GenericEval64<true>>(lds_bytes, device);
                case 3: return resident_one<3, GenericEval64<true>>(lds_bytes, device);
                default: return resident_one<4, GenericEval64<true>>(lds_bytes, device);
            }
        case EvalKind::Tanh64:
            switch (U) {
                case 1: return resident_one<1, TanhEval64>(lds_bytes, device);
                case 2: return resident_one<2, TanhEval64>(lds_bytes, device);
                case 3: return resident_one<3, TanhEval64>(lds_bytes, device);
                default: return resident_one<4, TanhEval64>(lds_bytes, device);
            }
        case EvalKind::Tanh64P:
            return resident_tanh_fixed<1>(p, lds_bytes, device);
        case EvalKind::General64:
            return general_compiled_resident(p, U, lds_bytes, device);
    }
    return 256;
}

}  // namespace pimc
