// Host-side pieces shared by the estimation, batch and learned-proposal entry points: the context,
// error reporting, device buffer growth, the per-problem tables and the assembly of a level result.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <vector>

#include "pimc.h"
#include "pimc_internal.hpp"
#include "pimc_general.hpp"

struct pimc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char err[512] = "";
    // device buffers, grown on demand
    void* d_prm = nullptr;          size_t prm_bytes = 0;
    double* d_partials = nullptr;   size_t partial_bytes = 0;
    double* d_red = nullptr;        size_t red_bytes = 0;
    uint64_t* d_seg = nullptr;      size_t seg_bytes = 0;
    std::vector<uint64_t> h_seg;    // segment base/len of the last reduction (kept alive for the async copy)
    double* d_dump = nullptr;       size_t dump_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // last estimation
    const double* last_partials_ptr = nullptr;   // chunk partials of the last run (context buffer or workspace)
    uint64_t last_chunks = 0, last_chunk_paths = 0;
    int last_s = -1;
    bool last_hier = false;
    std::vector<double> last_shift;
    double last_ms = 0.0;
};

namespace pimc_host {

extern thread_local char g_thread_error[512];

void set_thread_error(const char* fmt, ...);
// Record an error on the context (and the thread) and return status.
int ctx_fail(pimc_ctx* c, int status, const char* fmt, ...);
// Grow a device buffer to at least need bytes (contents are not kept).
int ensure(pimc_ctx* c, void** buf, size_t* have, size_t need);

#define HIP_TRY(ctx, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ctx_fail((ctx), PIMC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Problem {
    int s = 0, p = 0;
    bool even = true;
    pimc::EvalKind kind = pimc::EvalKind::GenericEven64;
    int U = 1, D = 0;
    double a = 0, b = 0, T = 0, pref = 1.0, K0 = 0.0;
    std::vector<int> deg;            // per k in the evaluation variable
    int stride = 0;                  // doubles per level table
    std::vector<double> tab;         // (s+1) * stride, the folded tables (mid-point form)
    std::vector<double> tab_dev;     // the same as uploaded for the estimation kernels
    std::vector<float> tab32;
    std::vector<double> sig;         // s+1
    std::vector<double> shift;       // s+1
    double level0_action = 0.0;      // T W_p((a+b)/2, (b-a)/2; T)
    double alpha = 0.0;              // Poeschl-Teller: tables in u = tanh^2(alpha mid) (after the mass rescaling)
    // general-potential mode
    pimc::GenPotential gen;                  // derivative tables (coefficients in tab)
};

// Tables, bridge widths and straight-line reference actions of one problem after the mass
// rescaling; returns a status and a reason in why.
int build_problem(const pimc_potential* V, double m, double a, double b, double T, uint32_t N, int p, uint32_t flags,
                  Problem& P, char* why, size_t whylen);
// The same for the modified Poeschl-Teller potential -lambda/cosh^2(alpha x) (tables in
// u = tanh^2(alpha' mid), alpha' = alpha/sqrt(m)).
int build_problem_mpt(double lambda, double alpha, double m, double a, double b, double T, uint32_t N, int p,
                      uint32_t flags, Problem& P, char* why, size_t whylen);
// The same for the general-potential mode (derivative symbols, p <= kGenMaxP).
int build_problem_general(const pimc_general_potential* V, double m, double a, double b, double T, uint32_t N, int p,
                          uint32_t flags, Problem& P, char* why, size_t whylen);
int check_general(const pimc_general_potential* V, double m, double a, double b, double T, uint32_t N, int p,
                  uint64_t n_samples);
// Estimation / per-path actions of a built problem (shared by every potential family).
// Fixed device buffers of one estimation (the no-allocation entry point's workspace) instead of
// the context's growable ones; the capacities are checked, never grown.
struct DeviceWork {
    void* prm = nullptr;            size_t prm_cap = 0;
    double* partials = nullptr;     size_t partial_cap = 0;
    double* red = nullptr;          size_t red_cap = 0;
    uint64_t* seg = nullptr;        size_t seg_cap = 0;
};
int amplitude_core(pimc_ctx* c, const Problem& P, uint64_t n_samples, uint64_t seed, uint32_t stream, uint32_t flags,
                   pimc_level_result* out, const DeviceWork* work = nullptr);
int path_actions_core(pimc_ctx* c, const Problem& P, uint64_t seed, uint32_t stream, uint32_t flags,
                      uint64_t first_path, uint64_t k_paths, double* S_out);
extern const uint32_t kKnownFlags;
// Level result from the canonical sums (n, sum d, sum d^2, non-finite count) with d = w - 1 and
// log prefactor logbase; true when the result is not finite.
bool assemble_level(const double* red, double logbase, pimc_level_result& r);
int check_args(const pimc_potential* V, double m, double a, double b, double T, uint32_t N, int p,
               uint64_t n_samples);
// With `device` current: look up the device address of the no-allocation workspace once per device
// (pimc_noalloc.cpp); called by pimc_create.
void noalloc_setup(int device);
int log2_exact(uint32_t N);

}  // namespace pimc_host
