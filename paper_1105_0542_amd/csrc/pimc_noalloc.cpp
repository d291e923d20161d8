// The estimation entry point that allocates nothing (pimc_amplitude_noalloc, include/pimc.h): the
// device buffers of one pimc_amplitude call -- the parameter block (tables, bridge widths,
// reference actions), the canonical-chunk sums, the segment list and the reduced sums -- live in a
// file-scope device workspace instead of buffers grown with hipMalloc. Every GPU the library runs on
// holds its own copy of the workspace until the process ends; its address on each device is looked
// up once, when the first context on that device is created.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "pimc.h"
#include "pimc_host_common.hpp"

using namespace pimc_host;

namespace {

// Layout of the workspace: parameter block, segment list (base, length per level), reduced sums
// (4 doubles per level), then the chunk sums.
constexpr size_t kPrmBytes = size_t(256) << 10;
constexpr size_t kSegBytes = size_t(PIMC_MAX_S + 1) * 2 * 8;
constexpr size_t kRedBytes = size_t(PIMC_MAX_S + 1) * 4 * 8;
constexpr size_t kSegOff = kPrmBytes;
constexpr size_t kRedOff = (kSegOff + kSegBytes + 255) & ~size_t(255);
constexpr size_t kPartOff = (kRedOff + kRedBytes + 255) & ~size_t(255);
static_assert(kPartOff < PIMC_NOALLOC_BYTES, "workspace layout");

static __device__ __align__(256) unsigned char scratch[PIMC_NOALLOC_BYTES];

std::mutex g_mutex;
std::vector<void*> g_addr;          // device address of `scratch` on each device (null: not looked up)
std::vector<int> g_status;          // hipError_t of the lookup on each device

}  // namespace

namespace pimc_host {

// With `device` current: look up the workspace's address on this device once. Called by
// pimc_create; the result (and any error) is kept for pimc_amplitude_noalloc.
void noalloc_setup(int device) {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (device < 0) return;
    if (size_t(device) >= g_addr.size()) {
        g_addr.resize(size_t(device) + 1, nullptr);
        g_status.resize(size_t(device) + 1, int(hipErrorNotReady));
    }
    if (g_addr[size_t(device)]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_status[size_t(device)] = int(e);
    if (e == hipSuccess) g_addr[size_t(device)] = ptr;
}

}  // namespace pimc_host

extern "C" {

int pimc_amplitude_noalloc(pimc_ctx* c, const pimc_potential* V, double m, double a, double b, double T, uint32_t N,
                           int p, uint64_t n_samples, uint64_t seed, uint32_t stream, uint32_t flags,
                           pimc_level_result* out) {
    int st = check_args(V, m, a, b, T, N, p, n_samples);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        if (size_t(c->device) < g_addr.size()) base = g_addr[size_t(c->device)];
        if (!base) {
            const int e = size_t(c->device) < g_status.size() ? g_status[size_t(c->device)] : int(hipErrorNotReady);
            return ctx_fail(c, PIMC_EDEVICE, "workspace address on device %d not available: %s", c->device,
                            hipGetErrorString(hipError_t(e)));
        }
    }
    HIP_TRY(c, hipSetDevice(c->device));
    Problem P;
    char why[256] = "";
    st = build_problem(V, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    unsigned char* w = static_cast<unsigned char*>(base);
    DeviceWork work;
    work.prm = w;
    work.prm_cap = kPrmBytes;
    work.seg = reinterpret_cast<uint64_t*>(w + kSegOff);
    work.seg_cap = kSegBytes;
    work.red = reinterpret_cast<double*>(w + kRedOff);
    work.red_cap = kRedBytes;
    work.partials = reinterpret_cast<double*>(w + kPartOff);
    work.partial_cap = PIMC_NOALLOC_BYTES - kPartOff;
    return amplitude_core(c, P, n_samples, seed, stream, flags, out, &work);
}

}  // extern "C"
