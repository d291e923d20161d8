// Host side of the C ABI declared in include/pimc.h: argument validation, the mass rescaling, the
// FP64 effective-action tables per bisection level, launches on the context's HIP stream and the
// assembly of amplitude +- error per level (Sec. 4 of Balaz et al.).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <fstream>
#include <map>
#include <sstream>
#include <thread>
#include <tuple>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "pimc.h"
#include "pimc_internal.hpp"
#include "pimc_tables.hpp"
#include "pimc_host_common.hpp"

using namespace pimc;
using namespace pimc_host;

namespace pimc_host {

thread_local char g_thread_error[512] = "";

void set_thread_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_thread_error, sizeof(g_thread_error), fmt, ap);
    va_end(ap);
}


int ctx_fail(pimc_ctx* c, int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) std::snprintf(c->err, sizeof(c->err), "%s", buf);
    std::snprintf(g_thread_error, sizeof(g_thread_error), "%s", buf);
    return status;
}

int ensure(pimc_ctx* c, void** buf, size_t* have, size_t need) {
    if (need <= *have) return PIMC_OK;
    if (*buf) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipFree(*buf));
        *buf = nullptr;
        *have = 0;
    }
    size_t alloc = std::max(need, size_t(1) << 16);
    hipError_t e = hipMalloc(buf, alloc);
    if (e != hipSuccess) return ctx_fail(c, PIMC_ENOMEM, "hipMalloc(%zu) failed: %s", alloc, hipGetErrorString(e));
    *have = alloc;
    return PIMC_OK;
}

bool finite(double v) { return std::isfinite(v); }

int log2_exact(uint32_t N) {
    int s = 0;
    while ((1u << s) < N) ++s;
    return s;
}

// ------------------------------------------------------------------------------------- problem
PolyD rescaled_potential(const pimc_potential* V, double m) {
    PolyD poly(V->coef, V->coef + V->degree + 1);
    if (m != 1.0) {
        const double inv = 1.0 / std::sqrt(m);
        double f = 1.0;
        for (size_t j = 0; j < poly.size(); ++j) {
            poly[j] *= f;
            f *= inv;
        }
    }
    return poly_trim(poly);
}

std::vector<int> quartic_xdegrees(int p) {
    std::vector<int> x;
    int K = 0;
    for (int k = 0; k < p; ++k) {
        int d = -1;
        for (int m = k; m < p; ++m) d = std::max(d, kQuarticDegrees.d[m][k]);
        x.push_back(d);
        if (d >= 0) K = k + 1;
    }
    x.resize(size_t(K));
    return x;
}

// K_0(a,b;T) = (2 pi T)^(-1/2) exp(-(b-a)^2/(2T)): the free kernel (W = 0 in the ideal-action form,
// Sec. 2.1), the prefactor of every estimate.
double free_kernel(double a, double b, double T) {
    return std::exp(-(b - a) * (b - a) / (2.0 * T)) / std::sqrt(2.0 * M_PI * T);
}

// Potential part of eq.(SNp) on the straight line from a to b at level n (2^n slices).
double straight_line_action(const LevelTable& lt, double a, double b, int n) {
    const int M = 1 << n;
    double acc = 0.0;
    for (int k = 0; k < M; ++k) {
        const double q0 = a + (b - a) * double(k) / double(M);
        const double q1 = a + (b - a) * double(k + 1) / double(M);
        acc += eval_level(lt, q0, q1);
    }
    return acc;
}

// Amplitude, error and diagnostics of one level from its canonical sums red = (n, sum d, sum d^2,
// non-finite count), with log of the prefactor K_0 sqrt(m) e^{-S_ref}. Returns true when the
// result is not finite.
bool assemble_level(const double* red, double logbase, pimc_level_result& r) {
    const double cnt = red[0];
    const double sd = red[1];
    const double sd2 = red[2];
    const double nb = red[3];
    const double mean = sd / cnt;
    double var;
    if (std::isnan(sd) || std::isnan(sd2)) {
        var = std::numeric_limits<double>::quiet_NaN();
    } else if (!std::isfinite(sd2)) {
        var = std::numeric_limits<double>::infinity();   // second moment beyond FP64 range
    } else {
        var = (sd2 - sd * mean) / (cnt - 1.0);               // sd*mean <= sd2: no overflow
        if (var < 0) var = 0;
    }
    const double base = std::exp(logbase);
    r.amp = base * (1.0 + mean);
    r.err = base * std::sqrt(var / cnt);
    r.log_amp = logbase + std::log1p(mean);
    r.relvar = var / ((1.0 + mean) * (1.0 + mean));
    const double sw = cnt + sd;
    const double sw2 = cnt + 2.0 * sd + sd2;
    // one weight beyond the FP64 range of its square dominates the sum: ESS is 1
    r.ess = !std::isfinite(sw2) && std::isfinite(sw) ? 1.0 : (sw2 > 0 ? sw * sw / sw2 : 0.0);
    r.n = uint64_t(cnt);
    r.n_nonfinite = uint64_t(nb);
    return nb > 0 || !std::isfinite(r.amp) || !std::isfinite(r.err);
}


int build_problem(const pimc_potential* V, double m, double a, double b, double T, uint32_t N, int p,
                  uint32_t flags, Problem& P, char* why, size_t whylen) {
    P.s = log2_exact(N);
    P.p = p;
    P.T = T;
    const double sm = std::sqrt(m);
    P.a = a * sm;
    P.b = b * sm;
    P.pref = sm;
    P.K0 = free_kernel(P.a, P.b, T);
    const PolyD Vt = rescaled_potential(V, m);
    P.even = potential_is_even(Vt);
    const int dV = int(Vt.size()) - 1;
    const Coefficients C = effective_coefficients(Vt, p);
    const bool fp32 = (flags & PIMC_FP32_POLY) != 0;
    std::vector<int> xdeg;
    if (P.even && dV <= 4 && P.s >= 4) {
        P.kind = fp32 ? EvalKind::Quartic32 : EvalKind::Quartic64;
        xdeg = quartic_xdegrees(p);
        // subtrees of 4 levels (the default launch shape; the batch autotuner also times 5)
        P.U = 4;
    } else {
        if (fp32) {
            std::snprintf(why, whylen, "FP32 polynomials need an even potential of degree <= 4 and N >= 16");
            return PIMC_EUNSUPPORTED;
        }
        P.kind = P.even ? EvalKind::GenericEven64 : EvalKind::GenericOdd64;
        xdeg = table_xdegrees(C);
        P.U = std::min(P.s, 4);
    }
    // The table layout must cover every non-zero coefficient.
    for (int k = 0; k < C.p; ++k)
        for (int mm = k; mm < C.p; ++mm) {
            const int have = int(C.c[mm][k].size()) - 1;
            if (have >= 0 && (k >= int(xdeg.size()) || have > xdeg[size_t(k)])) {
                std::snprintf(why, whylen, "internal: coefficient c_{%d,%d} exceeds the table shape", mm, k);
                return PIMC_EUNSUPPORTED;
            }
        }
    if (P.s == 0) P.U = 0;
    P.D = P.s - P.U;
    P.deg.clear();
    for (int d : xdeg) P.deg.push_back(P.even ? d / 2 : d);
    P.stride = 0;
    for (int d : P.deg) P.stride += d + 1;
    P.tab.assign(size_t(P.s + 1) * size_t(P.stride), 0.0);
    std::vector<LevelTable> levels;
    for (int n = 0; n <= P.s; ++n) {
        const double eps = std::ldexp(T, -n);
        LevelTable lt = fold_level(C, P.even, eps, xdeg);
        std::copy(lt.coef.begin(), lt.coef.end(), P.tab.begin() + size_t(n) * size_t(P.stride));
        levels.push_back(std::move(lt));
    }
    // device copies: the quartic evaluators square the endpoint sum, the generic ones the mid-point
    P.tab_dev = P.tab;
    if (P.kind == EvalKind::Quartic64 || P.kind == EvalKind::Quartic32)
        for (int n = 0; n <= P.s; ++n) scale_for_endpoint_sum(P.tab_dev.data() + size_t(n) * size_t(P.stride), P.deg);
    P.tab32.resize(P.tab_dev.size());
    for (size_t i = 0; i < P.tab_dev.size(); ++i) {
        const double v = P.tab_dev[i];
        P.tab32[i] = (std::fabs(v) < double(std::numeric_limits<float>::min())) ? 0.0f : float(v);
    }
    P.sig.assign(size_t(P.s + 1), 0.0);
    for (int n = 1; n <= P.s; ++n) P.sig[size_t(n)] = std::sqrt(T / std::ldexp(1.0, n + 1));
    P.shift.assign(size_t(P.s + 1), 0.0);
    for (int n = 0; n <= P.s; ++n) P.shift[size_t(n)] = straight_line_action(levels[size_t(n)], P.a, P.b, n);
    P.level0_action = P.shift[0];
    return PIMC_OK;
}

int build_problem_mpt(double lambda, double alpha, double m, double a, double b, double T, uint32_t N, int p,
                      uint32_t flags, Problem& P, char* why, size_t whylen) {
    if (flags & PIMC_FP32_POLY) {
        std::snprintf(why, whylen, "FP32 polynomials need an even polynomial potential of degree <= 4");
        return PIMC_EUNSUPPORTED;
    }
    P.s = log2_exact(N);
    P.p = p;
    P.T = T;
    const double sm = std::sqrt(m);
    P.a = a * sm;
    P.b = b * sm;
    P.pref = sm;
    P.K0 = free_kernel(P.a, P.b, T);
    P.alpha = alpha / sm;
    P.even = true;
    P.kind = EvalKind::Tanh64;
    P.U = std::min(P.s, 4);
    if (P.s == 0) P.U = 0;
    P.D = P.s - P.U;
    const PolyD Vy = {-lambda, 0.0, lambda};                    // -lambda (1 - tanh^2)
    const Coefficients C = effective_coefficients(Vy, p, TanhDerivative{P.alpha});
    const std::vector<int> ydeg = table_xdegrees(C);
    for (int d : ydeg)
        if (d % 2) {
            std::snprintf(why, whylen, "internal: odd power of tanh in the Poeschl-Teller table");
            return PIMC_EUNSUPPORTED;
        }
    P.deg.clear();
    for (int d : ydeg) P.deg.push_back(d / 2);
    P.stride = 0;
    for (int d : P.deg) P.stride += d + 1;
    // the usual shape (K = p groups of degree p) has compile-time kernels for N >= 16
    bool fixed = P.U == 4 && p <= PIMC_MAX_P && int(P.deg.size()) == p;
    for (int d : P.deg) fixed = fixed && d == p;
    if (fixed) P.kind = EvalKind::Tanh64P;
    P.tab.assign(size_t(P.s + 1) * size_t(P.stride), 0.0);
    std::vector<LevelTable> levels;
    for (int n = 0; n <= P.s; ++n) {
        LevelTable lt = fold_level(C, true, std::ldexp(T, -n), ydeg);
        lt.tanh_alpha = P.alpha;
        std::copy(lt.coef.begin(), lt.coef.end(), P.tab.begin() + size_t(n) * size_t(P.stride));
        levels.push_back(std::move(lt));
    }
    P.tab_dev = P.tab;
    P.tab32.assign(P.tab.size(), 0.0f);
    P.sig.assign(size_t(P.s + 1), 0.0);
    for (int n = 1; n <= P.s; ++n) P.sig[size_t(n)] = std::sqrt(T / std::ldexp(1.0, n + 1));
    P.shift.assign(size_t(P.s + 1), 0.0);
    for (int n = 0; n <= P.s; ++n) P.shift[size_t(n)] = straight_line_action(levels[size_t(n)], P.a, P.b, n);
    P.level0_action = P.shift[0];
    return PIMC_OK;
}

int check_mpt(const pimc_mpt* V, double m, double a, double b, double T, uint32_t N, int p, uint64_t n_samples) {
    if (!V) { set_thread_error("potential is NULL"); return PIMC_EINVAL; }
    if (!std::isfinite(V->lambda)) { set_thread_error("lambda must be finite"); return PIMC_EINVAL; }
    if (!std::isfinite(V->alpha) || V->alpha <= 0) { set_thread_error("alpha must be finite and > 0"); return PIMC_EINVAL; }
    pimc_potential zero{};
    return check_args(&zero, m, a, b, T, N, p, n_samples);
}

// Upload tables and per-level constants (into the context's buffer, or into work->prm); fill the
// kernel arguments except the output pointers.
int stage_problem(pimc_ctx* c, const Problem& P, uint64_t seed, uint32_t stream, AmpArgs& A,
                  const DeviceWork* work = nullptr) {
    const size_t nlev = size_t(P.s + 1);
    const size_t n_tab = P.tab.size();
    // layout: sig[nlev] shift[nlev] tab64[n_tab] tab32[n_tab] deg[K]
    const size_t off_shift = nlev * 8;
    const size_t off_tab = 2 * nlev * 8;
    const size_t off_tab32 = off_tab + n_tab * 8;
    const size_t off_deg = (off_tab32 + n_tab * 4 + 15) & ~size_t(15);
    // general-potential mode: derivative tables
    const size_t off_dpoly = (off_deg + P.deg.size() * 4 + 15) & ~size_t(15);
    const size_t off_dsech = off_dpoly + P.gen.dpoly.size() * 8;
    // the chunk counter of the persistent kernel, on its own 256-byte line
    const size_t off_queue = (off_dsech + P.gen.dsech.size() * 8 + 255) & ~size_t(255);
    const size_t total = off_queue + 256;
    std::vector<unsigned char> host(total, 0);
    std::memcpy(host.data(), P.sig.data(), nlev * 8);
    std::memcpy(host.data() + off_shift, P.shift.data(), nlev * 8);
    if (n_tab) {
        std::memcpy(host.data() + off_tab, P.tab_dev.data(), n_tab * 8);
        std::memcpy(host.data() + off_tab32, P.tab32.data(), n_tab * 4);
    }
    if (!P.deg.empty()) std::memcpy(host.data() + off_deg, P.deg.data(), P.deg.size() * 4);
    if (!P.gen.dpoly.empty()) std::memcpy(host.data() + off_dpoly, P.gen.dpoly.data(), P.gen.dpoly.size() * 8);
    if (!P.gen.dsech.empty()) std::memcpy(host.data() + off_dsech, P.gen.dsech.data(), P.gen.dsech.size() * 8);
    void* prm = nullptr;
    if (work) {
        if (total > work->prm_cap)
            return ctx_fail(c, PIMC_EINVAL, "tables need %zu bytes, the workspace holds %zu", total, work->prm_cap);
        prm = work->prm;
    } else {
        const int st = ensure(c, &c->d_prm, &c->prm_bytes, total);
        if (st) return st;
        prm = c->d_prm;
    }
    HIP_TRY(c, hipMemcpyAsync(prm, host.data(), total, hipMemcpyHostToDevice, c->stream));
    // the host vector must stay valid until the copy has read it
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unsigned char* base = static_cast<unsigned char*>(prm);
    std::memset(&A, 0, sizeof(A));
    A.sig = reinterpret_cast<const double*>(base);
    A.shift = reinterpret_cast<const double*>(base + off_shift);
    A.tab64 = reinterpret_cast<const double*>(base + off_tab);
    A.tab32 = reinterpret_cast<const float*>(base + off_tab32);
    A.gdeg = reinterpret_cast<const int*>(base + off_deg);
    A.queue = reinterpret_cast<unsigned long long*>(base + off_queue);
    A.gK = int(P.deg.size());
    A.gstride = P.stride;
    A.a = P.a;
    A.b = P.b;
    A.alpha = P.alpha;
    if (P.kind == EvalKind::General64) {
        GenTables& g = A.gen;
        g.dpoly = reinterpret_cast<const double*>(base + off_dpoly);
        g.dsech = reinterpret_cast<const double*>(base + off_dsech);
        g.n_sech = int(P.gen.sech_A.size());
        g.n_gauss = int(P.gen.gauss_B.size());
        for (int i = 0; i < g.n_sech; ++i) g.sech_a[i] = P.gen.sech_a[size_t(i)];
        for (int i = 0; i < g.n_gauss; ++i) {
            g.gB[i] = P.gen.gauss_B[size_t(i)];
            g.gb[i] = P.gen.gauss_b[size_t(i)];
            g.gsb[i] = std::sqrt(P.gen.gauss_b[size_t(i)]);
        }
    }
    A.key.seed_lo = uint32_t(seed);
    A.key.seed_hi = uint32_t(seed >> 32);
    A.key.stream = stream;
    A.s = P.s;
    A.D = P.D;
    return PIMC_OK;
}

int launch_grid(pimc_ctx* c, const Problem& P, uint64_t n_chunks) {
    const int resident = amplitude_resident_blocks(P.kind, P.p, P.U, amp_lds_bytes(P.D, P.s, 256), c->device);
    const uint64_t g = std::min<uint64_t>(n_chunks, uint64_t(std::max(resident, 1)));
    return int(std::max<uint64_t>(g, 1));
}

int check_args(const pimc_potential* V, double m, double a, double b, double T, uint32_t N, int p,
               uint64_t n_samples) {
    if (!V) { set_thread_error("potential is NULL"); return PIMC_EINVAL; }
    if (V->degree < 0 || V->degree > PIMC_MAX_DEGREE) {
        set_thread_error("potential degree %d outside 0..%d", V->degree, PIMC_MAX_DEGREE);
        return PIMC_EINVAL;
    }
    for (int j = 0; j <= V->degree; ++j)
        if (!finite(V->coef[j])) { set_thread_error("potential coefficient %d is not finite", j); return PIMC_EINVAL; }
    if (!finite(m) || m <= 0) { set_thread_error("mass must be finite and > 0"); return PIMC_EINVAL; }
    if (!finite(a) || !finite(b)) { set_thread_error("endpoints must be finite"); return PIMC_EINVAL; }
    if (!finite(T) || T <= 0) { set_thread_error("T must be finite and > 0"); return PIMC_EINVAL; }
    if (N == 0 || (N & (N - 1)) != 0 || N > (1u << PIMC_MAX_S)) {
        set_thread_error("N = %u is not a power of two in 1..2^%d", N, PIMC_MAX_S);
        return PIMC_EINVAL;
    }
    if (p < 1 || p > PIMC_MAX_P) { set_thread_error("p = %d outside 1..%d", p, PIMC_MAX_P); return PIMC_EINVAL; }
    if (n_samples < 2) { set_thread_error("need at least 2 samples"); return PIMC_EINVAL; }
    return PIMC_OK;
}

extern const uint32_t kKnownFlags = PIMC_FP32_POLY | PIMC_HIERARCHY;

// Estimation of every requested level of a built problem (the body shared by the potentials), with
// the context's device buffers or the fixed ones of `work`.
int amplitude_core(pimc_ctx* c, const Problem& P, uint64_t n_samples, uint64_t seed, uint32_t stream, uint32_t flags,
                   pimc_level_result* out, const DeviceWork* work) {
    int st;
    const int nlev = P.s + 1;
    const bool hier = (flags & PIMC_HIERARCHY) != 0;
    for (int n = 0; n < nlev; ++n) out[n] = pimc_level_result{};
    // level 0: the analytic short-time amplitude (Sec. 4.2), error 0
    out[0].log_amp = std::log(P.pref * P.K0) - P.level0_action;
    out[0].amp = std::exp(out[0].log_amp);
    out[0].n = n_samples;
    out[0].ess = double(n_samples);
    c->last_s = P.s;
    c->last_shift = P.shift;
    if (P.s == 0) return PIMC_OK;

    const uint64_t chunk_paths = kChunkPaths;
    const uint64_t n_chunks = (n_samples + chunk_paths - 1) / chunk_paths;
    const int slots = hier ? nlev : 1;            // partial slot of level n: n, or 0 for level s alone
    const size_t partial_bytes = size_t(slots) * n_chunks * 4 * 8;
    double* partials;
    double* red_dev;
    uint64_t* seg;
    if (work) {
        if (partial_bytes > work->partial_cap || size_t(slots) * 32 > work->red_cap || size_t(slots) * 16 > work->seg_cap)
            return ctx_fail(c, PIMC_EINVAL,
                            "%llu samples x %d levels need %zu bytes of chunk sums, the workspace holds %zu",
                            (unsigned long long)n_samples, slots, partial_bytes, work->partial_cap);
        partials = work->partials;
        red_dev = work->red;
        seg = work->seg;
    } else {
        st = ensure(c, reinterpret_cast<void**>(&c->d_partials), &c->partial_bytes, partial_bytes);
        if (st) return st;
        st = ensure(c, reinterpret_cast<void**>(&c->d_red), &c->red_bytes, size_t(slots) * 4 * 8);
        if (st) return st;
        st = ensure(c, reinterpret_cast<void**>(&c->d_seg), &c->seg_bytes, size_t(slots) * 2 * 8);
        if (st) return st;
        partials = c->d_partials;
        red_dev = c->d_red;
        seg = c->d_seg;
    }
    AmpArgs A;
    st = stage_problem(c, P, seed, stream, A, work);
    if (st) return st;
    c->h_seg.assign(size_t(slots) * 2, 0);
    for (int k = 0; k < slots; ++k) {
        c->h_seg[size_t(k)] = uint64_t(k) * n_chunks * 4;
        c->h_seg[size_t(slots + k)] = n_chunks;
    }
    HIP_TRY(c, hipMemcpyAsync(seg, c->h_seg.data(), c->h_seg.size() * 8, hipMemcpyHostToDevice, c->stream));
    A.first_path = 0;
    A.n_paths = n_samples;
    A.n_chunks = n_chunks;
    A.hier = hier ? 1 : 0;
    A.partials = partials;
    A.dump = nullptr;
    const int grid = launch_grid(c, P, n_chunks);
    HIP_TRY(c, launch_fill_u64(A.queue, 1, 0ull, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    HIP_TRY(c, launch_amplitude(A, P.kind, P.p, P.U, grid, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
    HIP_TRY(c, launch_seg_reduce(partials, seg, seg + slots, uint64_t(slots), red_dev, c->stream));
    double red[4 * (PIMC_MAX_S + 1)];
    HIP_TRY(c, hipMemcpyAsync(red, red_dev, size_t(slots) * 4 * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms = ms;
    c->last_partials_ptr = partials;
    c->last_chunks = n_chunks;
    c->last_chunk_paths = chunk_paths;
    c->last_hier = hier;
    bool nonfinite = false;
    for (int n = 1; n < nlev; ++n) {
        if (!hier && n != P.s) continue;
        const size_t k = size_t(hier ? n : 0);
        if (assemble_level(&red[k * 4], std::log(P.pref * P.K0) - P.shift[size_t(n)], out[n])) nonfinite = true;
    }
    return nonfinite ? PIMC_WNONFINITE : PIMC_OK;
}


// Per-path level actions of a built problem by the estimation kernels (shared by the potentials).
int path_actions_core(pimc_ctx* c, const Problem& P, uint64_t seed, uint32_t stream, uint32_t flags,
                      uint64_t first_path, uint64_t k_paths, double* S_out) {
    int st;
    const size_t nlev = size_t(P.s + 1);
    if (P.s == 0) {
        for (uint64_t i = 0; i < k_paths; ++i) S_out[i] = P.level0_action;
        return PIMC_OK;
    }
    AmpArgs A;
    st = stage_problem(c, P, seed, stream, A);
    if (st) return st;
    st = ensure(c, reinterpret_cast<void**>(&c->d_dump), &c->dump_bytes, size_t(k_paths) * nlev * 8);
    if (st) return st;
    const uint64_t chunk_paths = kChunkPaths;
    A.first_path = first_path;
    A.n_paths = k_paths;
    A.n_chunks = (k_paths + chunk_paths - 1) / chunk_paths;
    A.hier = (flags & PIMC_HIERARCHY) ? 1 : 0;
    A.partials = nullptr;
    A.dump = c->d_dump;
    const int grid = launch_grid(c, P, A.n_chunks);
    HIP_TRY(c, launch_fill_u64(A.queue, 1, 0ull, c->stream));
    HIP_TRY(c, launch_amplitude(A, P.kind, P.p, P.U, grid, c->stream));
    HIP_TRY(c, hipMemcpyAsync(S_out, c->d_dump, size_t(k_paths) * nlev * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // level 0 is the same straight slice for every path: report it for every path
    for (uint64_t i = 0; i < k_paths; ++i)
        if (!(flags & PIMC_HIERARCHY)) S_out[i * nlev] = 0.0;
    return PIMC_OK;
}


}  // namespace

// ============================================================================================ C ABI
extern "C" {

const char* pimc_strerror(int status) {
    switch (status) {
        case PIMC_OK: return "ok";
        case PIMC_EINVAL: return "invalid argument";
        case PIMC_EUNSUPPORTED: return "unsupported request";
        case PIMC_ENOMEM: return "out of memory";
        case PIMC_EDEVICE: return "device (HIP) error";
        case PIMC_WNONFINITE: return "warning: non-finite weights in the sums";
        case PIMC_WNOTCONVERGED: return "warning: iteration limit reached before the tolerance";
        default: return "unknown status";
    }
}

const char* pimc_last_error(const pimc_ctx* ctx) { return ctx ? ctx->err : g_thread_error; }

int pimc_check_problem(const pimc_potential* V, double m, double a, double b, double T, uint32_t N, int p,
                       uint64_t n_samples) {
    return check_args(V, m, a, b, T, N, p, n_samples);
}

int pimc_level_table(const pimc_potential* V, double m, double T, int p, uint32_t level, double* out, size_t cap,
                     size_t* n_out, int* n_k, int* deg, int* is_even) {
    int st = check_args(V, m, 0.0, 0.0, T, 1u << std::min<uint32_t>(level, PIMC_MAX_S), 1, 2);
    if (st) return st;
    if (p < 1 || p > PIMC_MAX_P_SHORT_TIME) {
        set_thread_error("p = %d outside 1..%d", p, PIMC_MAX_P_SHORT_TIME);
        return PIMC_EINVAL;
    }
    if (level > PIMC_MAX_S) { set_thread_error("level > %d", PIMC_MAX_S); return PIMC_EINVAL; }
    const PolyD Vt = rescaled_potential(V, m);
    const bool even = potential_is_even(Vt);
    const Coefficients C = effective_coefficients(Vt, p);
    const std::vector<int> xdeg = table_xdegrees(C);
    const LevelTable lt = fold_level(C, even, std::ldexp(T, -int(level)), xdeg);
    if (n_out) *n_out = lt.coef.size();
    if (n_k) *n_k = int(lt.deg.size());
    if (deg)
        for (size_t k = 0; k < lt.deg.size(); ++k) deg[k] = lt.deg[k];
    if (is_even) *is_even = even ? 1 : 0;
    if (!out || cap < lt.coef.size()) {
        set_thread_error("output capacity %zu < %zu", cap, lt.coef.size());
        return PIMC_EINVAL;
    }
    std::copy(lt.coef.begin(), lt.coef.end(), out);
    return PIMC_OK;
}

int pimc_create(pimc_ctx** out, int device, void* hip_stream) {
    if (!out) { set_thread_error("out is NULL"); return PIMC_EINVAL; }
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        set_thread_error("no HIP device available (%s)", e == hipSuccess ? "0 devices" : hipGetErrorString(e));
        return PIMC_EDEVICE;
    }
    if (device < 0 || device >= ndev) { set_thread_error("device %d outside 0..%d", device, ndev - 1); return PIMC_EINVAL; }
    pimc_ctx* c = new (std::nothrow) pimc_ctx();
    if (!c) { set_thread_error("out of host memory"); return PIMC_ENOMEM; }
    c->device = device;
    e = hipSetDevice(device);
    if (e == hipSuccess && hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else if (e == hipSuccess) {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        c->own_stream = (e == hipSuccess);
    }
    if (e == hipSuccess) e = hipEventCreate(&c->ev0);
    if (e == hipSuccess) e = hipEventCreate(&c->ev1);
    if (e == hipSuccess) noalloc_setup(device);
    if (e != hipSuccess) {
        set_thread_error("context setup failed: %s", hipGetErrorString(e));
        pimc_destroy(c);
        return PIMC_EDEVICE;
    }
    *out = c;
    return PIMC_OK;
}

int pimc_destroy(pimc_ctx* c) {
    if (!c) return PIMC_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->d_prm);
    (void)hipFree(c->d_partials);
    (void)hipFree(c->d_red);
    (void)hipFree(c->d_seg);
    (void)hipFree(c->d_dump);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return PIMC_OK;
}

int pimc_amplitude(pimc_ctx* c, const pimc_potential* V, double m, double a, double b, double T, uint32_t N, int p,
                   uint64_t n_samples, uint64_t seed, uint32_t stream, uint32_t flags, pimc_level_result* out) {
    int st = check_args(V, m, a, b, T, N, p, n_samples);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    HIP_TRY(c, hipSetDevice(c->device));
    Problem P;
    char why[256] = "";
    st = build_problem(V, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return amplitude_core(c, P, n_samples, seed, stream, flags, out);
}

int pimc_path_actions(pimc_ctx* c, const pimc_potential* V, double m, double a, double b, double T, uint32_t N,
                      int p, uint64_t seed, uint32_t stream, uint32_t flags, uint64_t first_path, uint64_t k_paths,
                      double* S_out) {
    int st = check_args(V, m, a, b, T, N, p, 2);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!S_out && k_paths) return ctx_fail(c, PIMC_EINVAL, "S_out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    if (k_paths == 0) return PIMC_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    Problem P;
    char why[256] = "";
    st = build_problem(V, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return path_actions_core(c, P, seed, stream, flags, first_path, k_paths, S_out);
}

int pimc_amplitude_mpt(pimc_ctx* c, const pimc_mpt* V, double m, double a, double b, double T, uint32_t N, int p,
                       uint64_t n_samples, uint64_t seed, uint32_t stream, uint32_t flags, pimc_level_result* out) {
    int st = check_mpt(V, m, a, b, T, N, p, n_samples);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    HIP_TRY(c, hipSetDevice(c->device));
    Problem P;
    char why[256] = "";
    st = build_problem_mpt(V->lambda, V->alpha, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return amplitude_core(c, P, n_samples, seed, stream, flags, out);
}

int pimc_path_actions_mpt(pimc_ctx* c, const pimc_mpt* V, double m, double a, double b, double T, uint32_t N, int p,
                          uint64_t seed, uint32_t stream, uint32_t flags, uint64_t first_path, uint64_t k_paths,
                          double* S_out) {
    int st = check_mpt(V, m, a, b, T, N, p, 2);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!S_out && k_paths) return ctx_fail(c, PIMC_EINVAL, "S_out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    if (k_paths == 0) return PIMC_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    Problem P;
    char why[256] = "";
    st = build_problem_mpt(V->lambda, V->alpha, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return path_actions_core(c, P, seed, stream, flags, first_path, k_paths, S_out);
}

int pimc_level_table_mpt(const pimc_mpt* V, double m, double T, int p, uint32_t level, double* out, size_t cap,
                         size_t* n_out, int* n_k, int* deg) {
    int st = check_mpt(V, m, 0.0, 0.0, T, 1u << std::min<uint32_t>(level, PIMC_MAX_S), 1, 2);
    if (st) return st;
    if (p < 1 || p > PIMC_MAX_P_SHORT_TIME) {
        set_thread_error("p = %d outside 1..%d", p, PIMC_MAX_P_SHORT_TIME);
        return PIMC_EINVAL;
    }
    if (level > PIMC_MAX_S) { set_thread_error("level > %d", PIMC_MAX_S); return PIMC_EINVAL; }
    const double am = V->alpha / std::sqrt(m);
    const Coefficients C = effective_coefficients(PolyD{-V->lambda, 0.0, V->lambda}, p, TanhDerivative{am});
    const std::vector<int> ydeg = table_xdegrees(C);
    const LevelTable lt = fold_level(C, true, std::ldexp(T, -int(level)), ydeg);
    if (n_out) *n_out = lt.coef.size();
    if (n_k) *n_k = int(lt.deg.size());
    if (deg)
        for (size_t k = 0; k < lt.deg.size(); ++k) deg[k] = lt.deg[k];
    if (!out || cap < lt.coef.size()) {
        set_thread_error("output capacity %zu < %zu", cap, lt.coef.size());
        return PIMC_EINVAL;
    }
    std::copy(lt.coef.begin(), lt.coef.end(), out);
    return PIMC_OK;
}

int pimc_last_partials(pimc_ctx* c, uint32_t level, uint64_t first_chunk, uint64_t n_chunks, double* out,
                       uint64_t* chunk_paths, uint64_t* total_chunks, double* shift) {
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (c->last_s < 1 || !c->last_partials_ptr) return ctx_fail(c, PIMC_EINVAL, "no estimation has run on this context");
    if (int(level) > c->last_s) return ctx_fail(c, PIMC_EINVAL, "level %u > s = %d", level, c->last_s);
    if (!c->last_hier && int(level) != c->last_s)
        return ctx_fail(c, PIMC_EINVAL, "the last run estimated level %d only", c->last_s);
    const uint64_t slot = c->last_hier ? level : 0;
    if (first_chunk + n_chunks > c->last_chunks || first_chunk + n_chunks < first_chunk)
        return ctx_fail(c, PIMC_EINVAL, "chunks out of range (%llu total)", (unsigned long long)c->last_chunks);
    if (chunk_paths) *chunk_paths = c->last_chunk_paths;
    if (total_chunks) *total_chunks = c->last_chunks;
    if (shift) *shift = c->last_shift[level];
    if (n_chunks == 0) return PIMC_OK;
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    const double* src = c->last_partials_ptr + (slot * c->last_chunks + first_chunk) * 4;
    HIP_TRY(c, hipMemcpyAsync(out, src, n_chunks * 4 * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIMC_OK;
}

int pimc_normals(pimc_ctx* c, uint64_t seed, uint32_t stream, uint64_t first_path, uint64_t k_paths, uint32_t n_nodes,
                 double* out) {
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (n_nodes == 0 || n_nodes > (1u << PIMC_MAX_S) - 1)
        return ctx_fail(c, PIMC_EINVAL, "n_nodes = %u outside 1..2^%d-1", n_nodes, PIMC_MAX_S);
    if (k_paths == 0) return PIMC_OK;
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    if (k_paths > (uint64_t(1) << 40) / n_nodes) return ctx_fail(c, PIMC_EINVAL, "request too large");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t bytes = size_t(k_paths) * n_nodes * 8;
    int st = ensure(c, reinterpret_cast<void**>(&c->d_dump), &c->dump_bytes, bytes);
    if (st) return st;
    RngKey key{uint32_t(seed), uint32_t(seed >> 32), stream};
    HIP_TRY(c, launch_normals(key, first_path, k_paths, n_nodes, c->d_dump, c->stream));
    HIP_TRY(c, hipMemcpyAsync(out, c->d_dump, bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIMC_OK;
}

int pimc_last_kernel_ms(pimc_ctx* c, double* ms) {
    if (!c || !ms) { set_thread_error("NULL argument"); return PIMC_EINVAL; }
    *ms = c->last_ms;
    return PIMC_OK;
}

}  // extern "C"

// ============================================================================================ batch
struct pimc_batch {
    pimc_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;              // capture/replay stream (owned)
    uint32_t flags = 0;
    uint64_t seed = 0;
    int s_max = 0;
    size_t n_tasks = 0;
    // per task (caller order)
    std::vector<int> t_s;
    std::vector<double> t_logpref;             // log(sqrt(m) K_0) after the mass rescaling
    std::vector<double> t_level0;              // T W_p at level 0
    std::vector<uint64_t> t_n;
    std::vector<std::vector<double>> t_shift;  // S_ref,n
    std::vector<uint64_t> t_seg;               // first segment of the task
    // kernel classes: the tasks of one level p with N = 16, or with N >= 32
    struct Class {
        int p;
        bool n16;
        int shape = 0;                         // launch shape (batch_shape)
        ShapeDesc d{};
        int n_tasks = 0;
        size_t first = 0;                      // first position in the device task array
        uint64_t n_items = 0;
        int smax = 0;                          // largest s of the class
        size_t lds = 0;
        int resident = 0;
        double tuned_ms = 0.0, default_ms = 0.0;
    };
    std::vector<Class> classes;
    // device
    void* d_blob = nullptr;
    BatchTask* d_tasks = nullptr;
    double* d_partials = nullptr;
    uint64_t* d_seg = nullptr;
    double* d_red = nullptr;
    unsigned long long* d_queue = nullptr;
    double* h_red = nullptr;                   // pinned
    pimc_level_result* h_out = nullptr;        // pinned staging of results bound for device memory
    uint64_t n_seg = 0;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int grid_mult_x2 = 2;                      // grid = resident * grid_mult_x2 / 2
    uint32_t grab = 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double last_ms = 0.0;
    char err[512] = "";
};

namespace {

int batch_fail(pimc_batch* b, int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (b) std::snprintf(b->err, sizeof(b->err), "%s", buf);
    if (b && b->ctx) std::snprintf(b->ctx->err, sizeof(b->ctx->err), "%s", buf);
    std::snprintf(g_thread_error, sizeof(g_thread_error), "%s", buf);
    return status;
}

#define HIP_TRY_B(b, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return batch_fail((b), PIMC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

void destroy_graph(pimc_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

int class_grid(const pimc_batch* b, const pimc_batch::Class& C) { return std::max(1, C.resident * b->grid_mult_x2 / 2); }

// The launch of class k's persistent kernel on `st` (its queue must be reset first).
hipError_t launch_class(pimc_batch* b, size_t k, hipStream_t st) {
    const auto& C = b->classes[k];
    RngKey key{uint32_t(b->seed), uint32_t(b->seed >> 32), 0u};
    const int hier = (b->flags & PIMC_HIERARCHY) ? 1 : 0;
    return launch_batch(b->d_tasks + C.first, C.n_tasks, C.n_items, b->d_queue + k, b->grab, key, hier, C.p, C.n16,
                        C.shape, class_grid(b, C), C.lds, st);
}

// Shape idx for class k: its description, LDS bytes and resident workgroups.
int set_class_shape(pimc_batch* b, size_t k, int idx) {
    auto& C = b->classes[k];
    ShapeDesc d;
    if (!batch_shape(C.p, C.n16, idx, d))
        return batch_fail(b, PIMC_EINVAL, "class %zu (p = %d): shape %d outside 0..%d", k, C.p, idx,
                          batch_shape_count(C.p, C.n16) - 1);
    C.shape = idx;
    C.d = d;
    C.lds = amp_lds_bytes(C.smax - d.U, C.smax, d.BS);
    C.resident = batch_resident_blocks(C.p, C.n16, idx, C.lds, b->ctx->device);
    if (C.resident <= 0) return batch_fail(b, PIMC_EDEVICE, "class %zu: no resident workgroups for shape %d", k, idx);
    return PIMC_OK;
}

// Capture: reset the queues (a fill kernel, no memset node), one persistent launch per class, the
// canonical reduction, and the copy of the sums to pinned host memory.
int capture_graph(pimc_batch* b) {
    destroy_graph(b);
    HIP_TRY_B(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_fill_u64(b->d_queue, int(b->classes.size()), 0ull, b->stream);
    for (size_t k = 0; k < b->classes.size() && e == hipSuccess; ++k) e = launch_class(b, k, b->stream);
    if (e == hipSuccess)
        e = launch_seg_reduce(b->d_partials, b->d_seg, b->d_seg + b->n_seg, b->n_seg, b->d_red, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_red, b->d_red, b->n_seg * 4 * 8, hipMemcpyDeviceToHost, b->stream);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return batch_fail(b, PIMC_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return batch_fail(b, PIMC_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e2));
    b->graph = g;
    HIP_TRY_B(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return PIMC_OK;
}

// Device time of class k alone with its current shape: queue reset, one launch (eager, on the
// batch stream).
int time_class(pimc_batch* b, size_t k, double* ms) {
    HIP_TRY_B(b, launch_fill_u64(b->d_queue + k, 1, 0ull, b->stream));
    HIP_TRY_B(b, hipEventRecord(b->e0, b->stream));
    HIP_TRY_B(b, launch_class(b, k, b->stream));
    HIP_TRY_B(b, hipEventRecord(b->e1, b->stream));
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
    float f = 0.f;
    HIP_TRY_B(b, hipEventElapsedTime(&f, b->e0, b->e1));
    *ms = f;
    return PIMC_OK;
}

int check_task(const pimc_task& t, int n_systems) {
    if (t.system >= uint32_t(n_systems)) { set_thread_error("task system %u >= %d", t.system, n_systems); return PIMC_EINVAL; }
    return PIMC_OK;
}

}  // namespace

extern "C" {

int pimc_batch_create(pimc_ctx* c, const pimc_potential* systems, int n_systems, const pimc_task* tasks, size_t n_tasks,
                      uint64_t seed, uint32_t flags, pimc_batch** out) {
    if (!out) { set_thread_error("out is NULL"); return PIMC_EINVAL; }
    *out = nullptr;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!systems || n_systems < 1 || !tasks || n_tasks == 0) return ctx_fail(c, PIMC_EINVAL, "empty batch");
    if (flags & ~uint32_t(PIMC_HIERARCHY))
        return ctx_fail(c, (flags & PIMC_FP32_POLY) ? PIMC_EUNSUPPORTED : PIMC_EINVAL,
                        "batches support the FP64 path with or without PIMC_HIERARCHY");
    if (n_tasks > (size_t(1) << 31)) return ctx_fail(c, PIMC_EINVAL, "too many tasks");
    for (size_t i = 0; i < n_tasks; ++i) {
        const pimc_task& t = tasks[i];
        int st = check_task(t, n_systems);
        if (!st) st = check_args(&systems[t.system], t.m, t.a, t.b, t.T, t.N, t.p, t.n_samples);
        if (st) return ctx_fail(c, st, "task %zu: %s", i, g_thread_error);
        if (t.N < 16) return ctx_fail(c, PIMC_EUNSUPPORTED, "task %zu: batches need N >= 16", i);
        const PolyD V = rescaled_potential(&systems[t.system], t.m);
        if (!potential_is_even(V) || V.size() > 5)
            return ctx_fail(c, PIMC_EUNSUPPORTED, "task %zu: batches need an even potential of degree <= 4", i);
    }
    HIP_TRY(c, hipSetDevice(c->device));
    pimc_batch* b = new (std::nothrow) pimc_batch();
    if (!b) return ctx_fail(c, PIMC_ENOMEM, "out of host memory");
    b->ctx = c;
    b->flags = flags;
    b->seed = seed;
    b->n_tasks = n_tasks;
    const bool hier = (flags & PIMC_HIERARCHY) != 0;
    auto fail = [&](int st) { pimc_batch_destroy(b); return st; };

    // ---- tables per (system, mass, p, T), levels 0..s_max of that combination
    using Key = std::tuple<uint32_t, double, int, double>;
    std::map<Key, int> combo_smax;
    for (size_t i = 0; i < n_tasks; ++i) {
        const Key k{tasks[i].system, tasks[i].m, tasks[i].p, tasks[i].T};
        combo_smax[k] = std::max(combo_smax[k], log2_exact(tasks[i].N));
    }
    std::map<std::tuple<uint32_t, double, int>, Coefficients> coef_cache;
    std::map<Key, size_t> combo_off;                         // offset (doubles) of level 0 in the blob
    std::map<Key, std::vector<LevelTable>> combo_levels;
    std::vector<double> blob;
    for (const auto& kv : combo_smax) {
        const auto& [sys, m, p, T] = kv.first;
        auto ck = std::make_tuple(sys, m, p);
        if (!coef_cache.count(ck)) coef_cache[ck] = effective_coefficients(rescaled_potential(&systems[sys], m), p);
        const Coefficients& C = coef_cache[ck];
        const std::vector<int> xdeg = quartic_xdegrees(p);
        combo_off[kv.first] = blob.size();
        auto& lv = combo_levels[kv.first];
        for (int n = 0; n <= kv.second; ++n) {
            lv.push_back(fold_level(C, true, std::ldexp(T, -n), xdeg));
            const size_t at = blob.size();
            blob.insert(blob.end(), lv.back().coef.begin(), lv.back().coef.end());
            scale_for_endpoint_sum(blob.data() + at, lv.back().deg);     // quartic evaluator form
        }
    }
    // ---- per task: sigma, S_ref, chunking; device order grouped by p, then N = 16 before N >= 32
    auto is_n16 = [&](size_t i) { return tasks[i].N == 16; };
    std::vector<size_t> order(n_tasks);
    for (size_t i = 0; i < n_tasks; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
        return tasks[x].p != tasks[y].p ? tasks[x].p < tasks[y].p : (is_n16(x) && !is_n16(y));
    });
    b->t_s.resize(n_tasks);
    b->t_logpref.resize(n_tasks);
    b->t_level0.resize(n_tasks);
    b->t_n.resize(n_tasks);
    b->t_shift.resize(n_tasks);
    b->t_seg.resize(n_tasks);
    std::vector<size_t> t_sig_off(n_tasks), t_shift_off(n_tasks);
    // straight-line reference actions, in parallel over tasks (the same host routine as single runs)
    {
        const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        for (unsigned w = 0; w < nth; ++w)
            pool.emplace_back([&, w]() {
                for (size_t i = w; i < n_tasks; i += nth) {
                    const pimc_task& t = tasks[i];
                    const int s = log2_exact(t.N);
                    const double sm = std::sqrt(t.m);
                    const double a = t.a * sm, bb = t.b * sm;
                    const auto& lv = combo_levels.at(Key{t.system, t.m, t.p, t.T});
                    std::vector<double> sh(size_t(s + 1), 0.0);
                    for (int n = 0; n <= s; ++n) {
                        if (!hier && n != s && n != 0) continue;
                        sh[size_t(n)] = straight_line_action(lv[size_t(n)], a, bb, n);
                    }
                    b->t_s[i] = s;
                    b->t_n[i] = t.n_samples;
                    b->t_logpref[i] = std::log(sm * free_kernel(a, bb, t.T));
                    b->t_level0[i] = sh[0];
                    b->t_shift[i] = std::move(sh);
                }
            });
        for (auto& th : pool) th.join();
    }
    for (size_t i = 0; i < n_tasks; ++i) {
        b->s_max = std::max(b->s_max, b->t_s[i]);
        t_sig_off[i] = blob.size();
        for (int n = 0; n <= b->t_s[i]; ++n) blob.push_back(n ? std::sqrt(tasks[i].T / std::ldexp(1.0, n + 1)) : 0.0);
        t_shift_off[i] = blob.size();
        blob.insert(blob.end(), b->t_shift[i].begin(), b->t_shift[i].end());
    }
    // partial slots and segments
    std::vector<uint64_t> t_chunks(n_tasks), t_part_off(n_tasks);
    uint64_t part_total = 0;
    std::vector<uint64_t> seg_base, seg_len;
    for (size_t pos = 0; pos < n_tasks; ++pos) {
        const size_t i = order[pos];
        t_chunks[i] = (tasks[i].n_samples + kChunkPaths - 1) / kChunkPaths;
        const int slots = hier ? b->t_s[i] + 1 : 1;
        t_part_off[i] = part_total;
        b->t_seg[i] = seg_base.size();
        for (int k = 0; k < slots; ++k) {
            seg_base.push_back((part_total + uint64_t(k) * t_chunks[i]) * 4);
            seg_len.push_back(t_chunks[i]);
        }
        part_total += uint64_t(slots) * t_chunks[i];
    }
    b->n_seg = seg_base.size();
    // ---- device buffers
    int st;
    auto dmalloc = [&](void** p, size_t bytes) -> int {
        const hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) return batch_fail(b, PIMC_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        return PIMC_OK;
    };
    if ((st = dmalloc(&b->d_blob, blob.size() * 8))) return fail(st);
    if ((st = dmalloc(reinterpret_cast<void**>(&b->d_tasks), n_tasks * sizeof(BatchTask)))) return fail(st);
    if ((st = dmalloc(reinterpret_cast<void**>(&b->d_partials), part_total * 4 * 8))) return fail(st);
    if ((st = dmalloc(reinterpret_cast<void**>(&b->d_seg), b->n_seg * 2 * 8))) return fail(st);
    if ((st = dmalloc(reinterpret_cast<void**>(&b->d_red), b->n_seg * 4 * 8))) return fail(st);
    if ((st = dmalloc(reinterpret_cast<void**>(&b->d_queue), 64 * 8))) return fail(st);
    {
        const hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->h_red), std::max<size_t>(b->n_seg * 4 * 8, 64), 0);
        if (e != hipSuccess) return fail(batch_fail(b, PIMC_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e)));
    }
    const double* dblob = static_cast<const double*>(b->d_blob);
    std::vector<BatchTask> dt(n_tasks);
    for (size_t pos = 0; pos < n_tasks; ++pos) {
        const size_t i = order[pos];
        const pimc_task& t = tasks[i];
        BatchTask& r = dt[pos];
        r.tab = dblob + combo_off.at(Key{t.system, t.m, t.p, t.T});
        r.sig = dblob + t_sig_off[i];
        r.shift = dblob + t_shift_off[i];
        r.partials = b->d_partials + t_part_off[i] * 4;
        const double sm = std::sqrt(t.m);
        r.a = t.a * sm;
        r.b = t.b * sm;
        r.n_paths = t.n_samples;
        r.n_chunks = t_chunks[i];
        r.stream = t.stream;
        r.s = b->t_s[i];
    }
    // classes and item numbering
    for (size_t pos = 0; pos < n_tasks;) {
        pimc_batch::Class C;
        C.p = tasks[order[pos]].p;
        C.n16 = is_n16(order[pos]);
        C.first = pos;
        while (pos < n_tasks && tasks[order[pos]].p == C.p && is_n16(order[pos]) == C.n16) {
            dt[pos].item0 = C.n_items;
            C.n_items += dt[pos].n_chunks;
            C.smax = std::max(C.smax, dt[pos].s);
            ++C.n_tasks;
            ++pos;
        }
        b->classes.push_back(C);
    }
    if (b->classes.size() > 64) return fail(batch_fail(b, PIMC_EUNSUPPORTED, "more than 64 kernel classes"));
    for (size_t k = 0; k < b->classes.size(); ++k)
        if ((st = set_class_shape(b, k, 0))) return fail(st);
    std::vector<uint64_t> seg(b->n_seg * 2);
    std::copy(seg_base.begin(), seg_base.end(), seg.begin());
    std::copy(seg_len.begin(), seg_len.end(), seg.begin() + b->n_seg);
    HIP_TRY_B(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    HIP_TRY_B(b, hipEventCreate(&b->e0));
    HIP_TRY_B(b, hipEventCreate(&b->e1));
    HIP_TRY_B(b, hipMemcpyAsync(b->d_blob, blob.data(), blob.size() * 8, hipMemcpyHostToDevice, b->stream));
    HIP_TRY_B(b, hipMemcpyAsync(b->d_tasks, dt.data(), dt.size() * sizeof(BatchTask), hipMemcpyHostToDevice, b->stream));
    HIP_TRY_B(b, hipMemcpyAsync(b->d_seg, seg.data(), seg.size() * 8, hipMemcpyHostToDevice, b->stream));
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
    if ((st = capture_graph(b))) return fail(st);
    *out = b;
    return PIMC_OK;
}

int pimc_batch_set_tuning(pimc_batch* b, int grid_mult_x2, uint32_t grab) {
    if (!b) { set_thread_error("batch is NULL"); return PIMC_EINVAL; }
    if (grid_mult_x2 < 1 || grid_mult_x2 > 8 || grab < 1 || grab > 64)
        return batch_fail(b, PIMC_EINVAL, "tuning out of range (grid_mult_x2 1..8, grab 1..64)");
    b->grid_mult_x2 = grid_mult_x2;
    b->grab = grab;
    return capture_graph(b);
}

int pimc_batch_n_classes(const pimc_batch* b) { return b ? int(b->classes.size()) : 0; }

int pimc_batch_class_info(const pimc_batch* b, int k, pimc_batch_class* out) {
    if (!b || !out) { set_thread_error("NULL argument"); return PIMC_EINVAL; }
    if (k < 0 || size_t(k) >= b->classes.size()) {
        set_thread_error("class %d outside 0..%zu", k, b->classes.size() - 1);
        return PIMC_EINVAL;
    }
    const auto& C = b->classes[size_t(k)];
    out->p = C.p;
    out->n16 = C.n16 ? 1 : 0;
    out->n_tasks = uint64_t(C.n_tasks);
    out->n_items = C.n_items;
    out->shape = C.shape;
    out->n_shapes = batch_shape_count(C.p, C.n16);
    out->subtree_levels = C.d.U;
    out->block = C.d.BS;
    out->waves_per_eu = C.d.WPE;
    out->slice_batch = C.d.BATCH;
    out->tuned_ms = C.tuned_ms;
    out->default_ms = C.default_ms;
    return PIMC_OK;
}

int pimc_batch_set_shape(pimc_batch* b, int k, int shape) {
    if (!b) { set_thread_error("batch is NULL"); return PIMC_EINVAL; }
    if (k < 0 || size_t(k) >= b->classes.size())
        return batch_fail(b, PIMC_EINVAL, "class %d outside 0..%zu", k, b->classes.size() - 1);
    HIP_TRY_B(b, hipSetDevice(b->ctx->device));
    const int st = set_class_shape(b, size_t(k), shape);
    if (st) return st;
    return capture_graph(b);
}

// Assemble every task from the reduced sums into out (host memory).
static int batch_assemble(pimc_batch* b, pimc_level_result* out) {
    const bool hier = (b->flags & PIMC_HIERARCHY) != 0;
    const size_t stride = size_t(b->s_max + 1);
    bool nonfinite = false;
    for (size_t i = 0; i < b->n_tasks; ++i) {
        pimc_level_result* r = out + i * stride;
        for (size_t n = 0; n < stride; ++n) r[n] = pimc_level_result{};
        const int s = b->t_s[i];
        r[0].amp = std::exp(b->t_logpref[i] - b->t_level0[i]);
        r[0].log_amp = b->t_logpref[i] - b->t_level0[i];
        r[0].n = b->t_n[i];
        r[0].ess = double(b->t_n[i]);
        for (int n = 1; n <= s; ++n) {
            if (!hier && n != s) continue;
            const double* red = b->h_red + (b->t_seg[i] + size_t(hier ? n : 0)) * 4;
            if (assemble_level(red, b->t_logpref[i] - b->t_shift[i][size_t(n)], r[n])) nonfinite = true;
        }
    }
    return nonfinite ? PIMC_WNONFINITE : PIMC_OK;
}

int pimc_batch_run_to(pimc_batch* b, pimc_level_result* out, int out_on_device, double* ms) {
    if (!b) { set_thread_error("batch is NULL"); return PIMC_EINVAL; }
    if (!out) return batch_fail(b, PIMC_EINVAL, "out is NULL");
    HIP_TRY_B(b, hipSetDevice(b->ctx->device));
    HIP_TRY_B(b, hipEventRecord(b->e0, b->stream));
    HIP_TRY_B(b, hipGraphLaunch(b->exec, b->stream));
    HIP_TRY_B(b, hipEventRecord(b->e1, b->stream));
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
    float fms = 0.f;
    HIP_TRY_B(b, hipEventElapsedTime(&fms, b->e0, b->e1));
    b->last_ms = fms;
    if (ms) *ms = fms;
    if (!out_on_device) return batch_assemble(b, out);
    const size_t count = b->n_tasks * size_t(b->s_max + 1);
    if (!b->h_out) {
        const hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->h_out), count * sizeof(pimc_level_result), 0);
        if (e != hipSuccess) return batch_fail(b, PIMC_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    const int st = batch_assemble(b, b->h_out);
    pimc_ctx* c = b->ctx;
    HIP_TRY_B(b, hipMemcpyAsync(out, b->h_out, count * sizeof(pimc_level_result), hipMemcpyHostToDevice, c->stream));
    HIP_TRY_B(b, hipStreamSynchronize(c->stream));            // the staging buffer is reused by the next run
    return st;
}

int pimc_batch_run(pimc_batch* b, pimc_level_result* out, double* ms) { return pimc_batch_run_to(b, out, 0, ms); }

int pimc_batch_autotune(pimc_batch* b, const char* cache_path, int* grid_mult_x2, uint32_t* grab) {
    if (!b) { set_thread_error("batch is NULL"); return PIMC_EINVAL; }
    HIP_TRY_B(b, hipSetDevice(b->ctx->device));
    // cache key: device architecture, the classes (p, N = 16 or not), the largest s, flags
    hipDeviceProp_t prop;
    HIP_TRY_B(b, hipGetDeviceProperties(&prop, b->ctx->device));
    std::ostringstream key;
    key << prop.gcnArchName << "|c";
    for (const auto& C : b->classes) key << ":" << C.p << (C.n16 ? "n16" : "n32");
    key << "|s" << b->s_max << "|f" << b->flags;
    const size_t nc = b->classes.size();
    int st;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int g;
            unsigned gr;
            if (!(ls >> k >> g >> gr) || k != key.str()) continue;
            std::vector<int> shapes(nc);
            bool ok = true;
            for (size_t i = 0; i < nc && ok; ++i) ok = bool(ls >> shapes[i]);
            if (!ok) continue;
            for (size_t i = 0; i < nc; ++i)
                if ((st = set_class_shape(b, i, shapes[i]))) return st;
            if (grid_mult_x2) *grid_mult_x2 = g;
            if (grab) *grab = gr;
            return pimc_batch_set_tuning(b, g, gr);
        }
    }
    // 1. per class: every candidate shape, timed alone (default grid and grab)
    b->grid_mult_x2 = 2;
    b->grab = 1;
    for (size_t k = 0; k < nc; ++k) {
        auto& C = b->classes[k];
        const int n = batch_shape_count(C.p, C.n16);
        double best = 1e300;
        int best_i = 0;
        for (int i = 0; i < n; ++i) {
            if ((st = set_class_shape(b, k, i))) return st;
            double ms = 0.0;
            if ((st = time_class(b, k, &ms))) return st;
            if (i == 0) C.default_ms = ms;
            if (ms < best) {
                best = ms;
                best_i = i;
            }
        }
        if ((st = set_class_shape(b, k, best_i))) return st;
        C.tuned_ms = best;
    }
    // 2. grid size and grab over the whole graph with the chosen shapes
    std::vector<pimc_level_result> scratch(b->n_tasks * size_t(b->s_max + 1));
    double best = 1e300;
    int best_g = 2;
    uint32_t best_gr = 1;
    const int gs[] = {1, 2, 4};
    const uint32_t grs[] = {1, 4, 16};
    for (int g : gs)
        for (uint32_t gr : grs) {
            if ((st = pimc_batch_set_tuning(b, g, gr))) return st;
            double ms = 0;
            st = pimc_batch_run(b, scratch.data(), &ms);
            if (st < 0) return st;
            if (ms < best) {
                best = ms;
                best_g = g;
                best_gr = gr;
            }
        }
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << key.str() << " " << best_g << " " << best_gr;
        for (const auto& C : b->classes) o << " " << C.shape;
        o << "\n";
    }
    if (grid_mult_x2) *grid_mult_x2 = best_g;
    if (grab) *grab = best_gr;
    return pimc_batch_set_tuning(b, best_g, best_gr);
}

int pimc_batch_destroy(pimc_batch* b) {
    if (!b) return PIMC_OK;
    if (b->ctx) (void)hipSetDevice(b->ctx->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    destroy_graph(b);
    (void)hipFree(b->d_blob);
    (void)hipFree(b->d_tasks);
    (void)hipFree(b->d_partials);
    (void)hipFree(b->d_seg);
    (void)hipFree(b->d_red);
    (void)hipFree(b->d_queue);
    if (b->h_red) (void)hipHostFree(b->h_red);
    if (b->h_out) (void)hipHostFree(b->h_out);
    if (b->e0) (void)hipEventDestroy(b->e0);
    if (b->e1) (void)hipEventDestroy(b->e1);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return PIMC_OK;
}

const char* pimc_batch_last_error(const pimc_batch* b) { return b ? b->err : g_thread_error; }

int pimc_amplitude_batch(pimc_ctx* c, const pimc_potential* systems, int n_systems, const pimc_task* tasks,
                         size_t n_tasks, uint64_t seed, uint32_t flags, pimc_level_result* out, int out_on_device) {
    pimc_batch* b = nullptr;
    int st = pimc_batch_create(c, systems, n_systems, tasks, n_tasks, seed, flags, &b);
    if (st) return st;
    st = pimc_batch_run_to(b, out, out_on_device, nullptr);
    pimc_batch_destroy(b);
    return st;
}

}  // extern "C"
