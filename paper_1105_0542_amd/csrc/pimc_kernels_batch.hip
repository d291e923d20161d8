// Batched estimation: dispatch of the persistent kernel (pimc_batch.hpp) by level p and launch
// shape. Levels 8, 12 and 18 (the configured batch classes) have the tuned shape lists, compiled in
// their own translation units; every other level has the default shapes only.
#include <hip/hip_runtime.h>

#include "pimc_batch.hpp"

namespace pimc {

namespace {

bool tuned_level(int p) { return p == 8 || p == 12 || p == 18; }

template <int P>
hipError_t launch_default(int p, bool n16, int idx, const BatchTask* tasks, int n_tasks, uint64_t n_items,
                          unsigned long long* queue, uint32_t grab, const RngKey& key, int hier, int grid, size_t lds,
                          hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p != P)
            return launch_default<P + 1>(p, n16, idx, tasks, n_tasks, n_items, queue, grab, key, hier, grid, lds, st);
        return n16 ? BatchLauncher<P, BatchDefaultN16>::launch(idx, tasks, n_tasks, n_items, queue, grab, key, hier, grid,
                                                               lds, st)
                   : BatchLauncher<P, BatchDefaultN32>::launch(idx, tasks, n_tasks, n_items, queue, grab, key, hier, grid,
                                                               lds, st);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int P>
int resident_default(int p, bool n16, int idx, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p != P) return resident_default<P + 1>(p, n16, idx, lds, device);
        return n16 ? BatchLauncher<P, BatchDefaultN16>::resident(idx, lds, device)
                   : BatchLauncher<P, BatchDefaultN32>::resident(idx, lds, device);
    } else {
        return 0;
    }
}

}  // namespace

int batch_shape_count(int p, bool n16) {
    if (tuned_level(p)) return n16 ? BatchShapesN16::size : BatchShapesN32::size;
    return 1;
}

bool batch_shape(int p, bool n16, int idx, ShapeDesc& d) {
    if (idx < 0 || idx >= batch_shape_count(p, n16)) return false;
    if (tuned_level(p))
        return n16 ? BatchLauncher<1, BatchShapesN16>::desc(idx, d) : BatchLauncher<1, BatchShapesN32>::desc(idx, d);
    return n16 ? BatchLauncher<1, BatchDefaultN16>::desc(idx, d) : BatchLauncher<1, BatchDefaultN32>::desc(idx, d);
}

hipError_t launch_batch(const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue, uint32_t grab,
                        const RngKey& key, int hier, int p, bool n16, int shape, int grid, size_t lds, hipStream_t st) {
    switch (p) {
        case 8: return launch_batch_tuned_8(n16, shape, tasks, n_tasks, n_items, queue, grab, key, hier, grid, lds, st);
        case 12: return launch_batch_tuned_12(n16, shape, tasks, n_tasks, n_items, queue, grab, key, hier, grid, lds, st);
        case 18: return launch_batch_tuned_18(n16, shape, tasks, n_tasks, n_items, queue, grab, key, hier, grid, lds, st);
        default:
            return launch_default<1>(p, n16, shape, tasks, n_tasks, n_items, queue, grab, key, hier, grid, lds, st);
    }
}

int batch_resident_blocks(int p, bool n16, int shape, size_t lds_bytes, int device) {
    switch (p) {
        case 8: return resident_batch_tuned_8(n16, shape, lds_bytes, device);
        case 12: return resident_batch_tuned_12(n16, shape, lds_bytes, device);
        case 18: return resident_batch_tuned_18(n16, shape, lds_bytes, device);
        default: return resident_default<1>(p, n16, shape, lds_bytes, device);
    }
}

}  // namespace pimc
