// Persistent batched estimation kernel (the walker of pimc_walker.hpp over an atomic queue of
// (task, chunk) items) for the quartic evaluators, p = 1..kMaxP.
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

template <int P>
static hipError_t batch_quartic(const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue,
                                uint32_t grab, RngKey key, int hier, int p, int U, int grid, size_t lds, hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p != P) return batch_quartic<P + 1>(tasks, n_tasks, n_items, queue, grab, key, hier, p, U, grid, lds, st);
        QuarticEval64<P> ev{nullptr};
        if (U == 5)
            hipLaunchKernelGGL((k_batch<5, QuarticEval64<P>>), dim3(grid), dim3(kBlock), lds, st, tasks, n_tasks,
                               n_items, queue, grab, key, hier, ev);
        else if (U == 4)
            hipLaunchKernelGGL((k_batch<4, QuarticEval64<P>>), dim3(grid), dim3(kBlock), lds, st, tasks, n_tasks,
                               n_items, queue, grab, key, hier, ev);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

hipError_t launch_batch(const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue, uint32_t grab,
                        const RngKey& key, int hier, int p, int U, int grid, size_t lds, hipStream_t st) {
    return batch_quartic<1>(tasks, n_tasks, n_items, queue, grab, key, hier, p, U, grid, lds, st);
}

template <int P>
static int batch_resident(int p, int U, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p != P) return batch_resident<P + 1>(p, U, lds, device);
        int per_cu = 0;
        const hipError_t e =
            U == 5 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<5, QuarticEval64<P>>, kBlock, lds)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<4, QuarticEval64<P>>, kBlock, lds);
        if (e != hipSuccess) per_cu = 1;
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) ncu = 256;
        return (per_cu < 1 ? 1 : per_cu) * ncu;
    } else {
        return 256;
    }
}

int batch_resident_blocks(int p, int U, size_t lds_bytes, int device) {
    return batch_resident<1>(p, U, lds_bytes, device);
}

}  // namespace pimc
