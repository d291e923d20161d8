// Persistent batched estimation kernel (the walker of pimc_walker.hpp over an atomic queue of
// (task, chunk) items) for the quartic evaluators, and the launch-shape lists the autotuner picks
// from. Included by pimc_kernels_batch.hip (default shapes, every p) and one translation unit per
// tuned level p (pimc_batch_p*.hip), so the variants compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "pimc_walker.hpp"

namespace pimc {

template <class... Ss>
struct ShapeList {
    static constexpr int size = sizeof...(Ss);
};

// Candidate shapes of the tuned classes. Tasks with N >= 32 may use 4- or 5-level subtrees; tasks
// with N = 16 (s = 4) have at most 4. Shape 0 of each list is the default (the single-call shape).
using BatchShapesN32 = ShapeList<Shape<4, 256, 2, 16>, Shape<4, 256, 2, 8>, Shape<5, 256, 2, 16>, Shape<5, 256, 2, 8>,
                                 Shape<4, 128, 2, 16>, Shape<4, 256, 1, 16>, Shape<4, 256, 3, 8>, Shape<4, 64, 2, 16>>;
using BatchShapesN16 = ShapeList<Shape<4, 256, 2, 16>, Shape<4, 256, 2, 8>, Shape<4, 128, 2, 16>, Shape<4, 256, 3, 8>,
                                 Shape<4, 256, 1, 16>>;
using BatchDefaultN32 = ShapeList<DefaultShape<4>>;
using BatchDefaultN16 = ShapeList<DefaultShape<4>>;

// Persistent kernel over the (task, chunk) items of one class (level p, launch shape): each
// workgroup takes `grab` consecutive items at a time from an atomic counter until the queue is
// empty (every wave of every workgroup reaches the exit test with the same value). Items are
// numbered task by task (task t owns items item0[t] .. item0[t] + n_chunks[t] - 1), so an item maps
// to its task by binary search over the wave-uniform task records; the chunk itself is processed
// by the same code as a single-task launch, so results do not depend on which workgroup took which
// item, nor on the shape.
template <class S, class Eval>
__global__ void __launch_bounds__(S::BS) __attribute__((amdgpu_waves_per_eu(S::WPE)))
k_batch(const BatchTask* __restrict__ tasks, int n_tasks, uint64_t n_items, unsigned long long* queue,
        uint32_t grab, RngKey key, int hier, Eval ev0) {
    extern __shared__ double smem[];
    __shared__ unsigned long long s_item;
    const const_ptr<BatchTask> T = as_const(tasks);
    load_bm_table(smem, S::BS);
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
            A.s = T[lo].s;
            A.D = T[lo].s - S::U;
            A.hier = hier;
            A.partials = T[lo].partials;
            A.dump = nullptr;
            A.queue = nullptr;
            Eval ev = ev0;
            ev.tab = T[lo].tab;
            process_chunk<S, Eval>(ev, A, item - T[lo].item0, smem);
        }
    }
}

// Shape idx of a list: launch, occupancy and description.
template <int P, class List>
struct BatchLauncher;

template <int P>
struct BatchLauncher<P, ShapeList<>> {
    static hipError_t launch(int, const BatchTask*, int, uint64_t, unsigned long long*, uint32_t, const RngKey&, int, int,
                             size_t, hipStream_t) {
        return hipErrorInvalidValue;
    }
    static int resident(int, size_t, int) { return 0; }
    static bool desc(int, ShapeDesc&) { return false; }
};

template <int P, class S0, class... Ss>
struct BatchLauncher<P, ShapeList<S0, Ss...>> {
    using Rest = BatchLauncher<P, ShapeList<Ss...>>;
    static hipError_t launch(int idx, const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue,
                             uint32_t grab, const RngKey& key, int hier, int grid, size_t lds, hipStream_t st) {
        if (idx != 0) return Rest::launch(idx - 1, tasks, n_tasks, n_items, queue, grab, key, hier, grid, lds, st);
        QuarticEval64<P> ev{nullptr};
        hipLaunchKernelGGL((k_batch<S0, QuarticEval64<P>>), dim3(grid), dim3(S0::BS), lds, st, tasks, n_tasks, n_items,
                           queue, grab, key, hier, ev);
        return hipGetLastError();
    }
    static int resident(int idx, size_t lds, int device) {
        if (idx != 0) return Rest::resident(idx - 1, lds, device);
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<S0, QuarticEval64<P>>, S0::BS, lds) !=
            hipSuccess)
            per_cu = 1;
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) ncu = 256;
        return (per_cu < 1 ? 1 : per_cu) * ncu;
    }
    static bool desc(int idx, ShapeDesc& d) {
        if (idx != 0) return Rest::desc(idx - 1, d);
        d = ShapeDesc{S0::U, S0::BS, S0::WPE, S0::BATCH};
        return true;
    }
};

// The tuned classes of level P (defined in pimc_batch_p<P>.hip).
#define PIMC_BATCH_TUNED_DECL(P)                                                                                      \
    hipError_t launch_batch_tuned_##P(bool n16, int idx, const BatchTask* tasks, int n_tasks, uint64_t n_items,        \
                                      unsigned long long* queue, uint32_t grab, const RngKey& key, int hier, int grid,  \
                                      size_t lds, hipStream_t st);                                                      \
    int resident_batch_tuned_##P(bool n16, int idx, size_t lds, int device);

#define PIMC_BATCH_TUNED_DEF(P)                                                                                       \
    hipError_t launch_batch_tuned_##P(bool n16, int idx, const BatchTask* tasks, int n_tasks, uint64_t n_items,        \
                                      unsigned long long* queue, uint32_t grab, const RngKey& key, int hier, int grid,  \
                                      size_t lds, hipStream_t st) {                                                     \
        return n16 ? BatchLauncher<P, BatchShapesN16>::launch(idx, tasks, n_tasks, n_items, queue, grab, key, hier,    \
                                                             grid, lds, st)                                             \
                   : BatchLauncher<P, BatchShapesN32>::launch(idx, tasks, n_tasks, n_items, queue, grab, key, hier,    \
                                                             grid, lds, st);                                            \
    }                                                                                                                  \
    int resident_batch_tuned_##P(bool n16, int idx, size_t lds, int device) {                                          \
        return n16 ? BatchLauncher<P, BatchShapesN16>::resident(idx, lds, device)                                      \
                   : BatchLauncher<P, BatchShapesN32>::resident(idx, lds, device);                                     \
    }

PIMC_BATCH_TUNED_DECL(8)
PIMC_BATCH_TUNED_DECL(12)
PIMC_BATCH_TUNED_DECL(18)

}  // namespace pimc
