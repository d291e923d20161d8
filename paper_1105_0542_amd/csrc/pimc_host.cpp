// Host side of the C ABI declared in include/pimc.h: argument validation, the mass rescaling, the
// FP64 effective-action tables per bisection level, launches on the context's HIP stream and the
// assembly of amplitude +- error per level (Sec. 4 of Balaz et al.).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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

using namespace pimc;

namespace {

thread_local char g_thread_error[512] = "";

void set_thread_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_thread_error, sizeof(g_thread_error), fmt, ap);
    va_end(ap);
}

}  // namespace

struct pimc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char err[512] = "";
    // device buffers, grown on demand
    void* d_prm = nullptr;          size_t prm_bytes = 0;
    double* d_partials = nullptr;   size_t partial_bytes = 0;
    double* d_red = nullptr;        size_t red_bytes = 0;
    double* d_dump = nullptr;       size_t dump_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // last estimation
    uint64_t last_chunks = 0, last_chunk_paths = 0;
    int last_s = -1;
    std::vector<double> last_shift;
    double last_ms = 0.0;
};

namespace {

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

#define HIP_TRY(ctx, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ctx_fail((ctx), PIMC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

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
struct Problem {
    int s = 0, p = 0;
    bool even = true;
    EvalKind kind = EvalKind::GenericEven64;
    int U = 1, D = 0;
    double a = 0, b = 0, T = 0, pref = 1.0, K0 = 0.0;
    std::vector<int> deg;            // per k in the evaluation variable
    int stride = 0;                  // doubles per level table
    std::vector<double> tab;         // (s+1) * stride
    std::vector<float> tab32;
    std::vector<double> sig;         // s+1
    std::vector<double> shift;       // s+1
    double level0_action = 0.0;      // T W_p((a+b)/2, (b-a)/2; T)
};

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

int build_problem(const pimc_potential* V, double m, double a, double b, double T, uint32_t N, int p,
                  uint32_t flags, Problem& P, char* why, size_t whylen) {
    P.s = log2_exact(N);
    P.p = p;
    P.T = T;
    const double sm = std::sqrt(m);
    P.a = a * sm;
    P.b = b * sm;
    P.pref = sm;
    P.K0 = std::exp(-(P.b - P.a) * (P.b - P.a) / (2.0 * T)) / std::sqrt(2.0 * M_PI * T);
    const PolyD Vt = rescaled_potential(V, m);
    P.even = potential_is_even(Vt);
    const int dV = int(Vt.size()) - 1;
    const Coefficients C = effective_coefficients(Vt, p);
    const bool fp32 = (flags & PIMC_FP32_POLY) != 0;
    std::vector<int> xdeg;
    if (P.even && dV <= 4 && P.s >= 4) {
        P.kind = fp32 ? EvalKind::Quartic32 : EvalKind::Quartic64;
        xdeg = quartic_xdegrees(p);
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
    P.tab32.resize(P.tab.size());
    for (size_t i = 0; i < P.tab.size(); ++i) {
        const double v = P.tab[i];
        P.tab32[i] = (std::fabs(v) < double(std::numeric_limits<float>::min())) ? 0.0f : float(v);
    }
    P.sig.assign(size_t(P.s + 1), 0.0);
    for (int n = 1; n <= P.s; ++n) P.sig[size_t(n)] = std::sqrt(T / std::ldexp(1.0, n + 1));
    P.shift.assign(size_t(P.s + 1), 0.0);
    for (int n = 0; n <= P.s; ++n) {
        const int M = 1 << n;
        double acc = 0.0;
        for (int k = 0; k < M; ++k) {
            const double q0 = P.a + (P.b - P.a) * double(k) / double(M);
            const double q1 = P.a + (P.b - P.a) * double(k + 1) / double(M);
            acc += eval_level(levels[size_t(n)], q0, q1);
        }
        P.shift[size_t(n)] = acc;
    }
    P.level0_action = P.shift[0];
    return PIMC_OK;
}

uint32_t paths_per_lane(int s) { return s >= 10 ? 1u : (1u << (10 - s)); }

// Upload tables and per-level constants; fill the kernel arguments except the output pointers.
int stage_problem(pimc_ctx* c, const Problem& P, uint64_t seed, uint32_t stream, AmpArgs& A) {
    const size_t nlev = size_t(P.s + 1);
    const size_t n_tab = P.tab.size();
    // layout: sig[nlev] shift[nlev] tab64[n_tab] tab32[n_tab] deg[K]
    const size_t off_shift = nlev * 8;
    const size_t off_tab = 2 * nlev * 8;
    const size_t off_tab32 = off_tab + n_tab * 8;
    const size_t off_deg = (off_tab32 + n_tab * 4 + 15) & ~size_t(15);
    const size_t total = off_deg + P.deg.size() * 4 + 16;
    std::vector<unsigned char> host(total, 0);
    std::memcpy(host.data(), P.sig.data(), nlev * 8);
    std::memcpy(host.data() + off_shift, P.shift.data(), nlev * 8);
    if (n_tab) {
        std::memcpy(host.data() + off_tab, P.tab.data(), n_tab * 8);
        std::memcpy(host.data() + off_tab32, P.tab32.data(), n_tab * 4);
    }
    if (!P.deg.empty()) std::memcpy(host.data() + off_deg, P.deg.data(), P.deg.size() * 4);
    int st = ensure(c, &c->d_prm, &c->prm_bytes, total);
    if (st) return st;
    HIP_TRY(c, hipMemcpyAsync(c->d_prm, host.data(), total, hipMemcpyHostToDevice, c->stream));
    // the host vector must stay valid until the copy has read it
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unsigned char* base = static_cast<unsigned char*>(c->d_prm);
    std::memset(&A, 0, sizeof(A));
    A.sig = reinterpret_cast<const double*>(base);
    A.shift = reinterpret_cast<const double*>(base + off_shift);
    A.tab64 = reinterpret_cast<const double*>(base + off_tab);
    A.tab32 = reinterpret_cast<const float*>(base + off_tab32);
    A.gdeg = reinterpret_cast<const int*>(base + off_deg);
    A.gK = int(P.deg.size());
    A.gstride = P.stride;
    A.a = P.a;
    A.b = P.b;
    A.key.seed_lo = uint32_t(seed);
    A.key.seed_hi = uint32_t(seed >> 32);
    A.key.stream = stream;
    A.s = P.s;
    A.D = P.D;
    return PIMC_OK;
}

int launch_grid(pimc_ctx* c, const Problem& P, uint64_t n_chunks) {
    const int resident = amplitude_resident_blocks(P.kind, P.p, P.U, amp_lds_bytes(P.D, P.s), c->device);
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

const uint32_t kKnownFlags = PIMC_FP32_POLY | PIMC_HIERARCHY;

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
    int st = check_args(V, m, 0.0, 0.0, T, 1u << std::min<uint32_t>(level, PIMC_MAX_S), p, 2);
    if (st) return st;
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
    const int nlev = P.s + 1;
    const bool hier = (flags & PIMC_HIERARCHY) != 0;
    for (int n = 0; n < nlev; ++n) out[n] = pimc_level_result{};
    // level 0: the analytic short-time amplitude (Sec. 4.2), error 0
    out[0].amp = P.pref * P.K0 * std::exp(-P.level0_action);
    out[0].log_amp = std::log(P.pref * P.K0) - P.level0_action;
    out[0].n = n_samples;
    out[0].ess = double(n_samples);
    c->last_s = P.s;
    c->last_shift = P.shift;
    if (P.s == 0) return PIMC_OK;

    AmpArgs A;
    st = stage_problem(c, P, seed, stream, A);
    if (st) return st;
    const uint32_t ppl = paths_per_lane(P.s);
    const uint64_t chunk_paths = uint64_t(kBlock) * ppl;
    const uint64_t n_chunks = (n_samples + chunk_paths - 1) / chunk_paths;
    st = ensure(c, reinterpret_cast<void**>(&c->d_partials), &c->partial_bytes, size_t(nlev) * n_chunks * 4 * 8);
    if (st) return st;
    st = ensure(c, reinterpret_cast<void**>(&c->d_red), &c->red_bytes, size_t(nlev) * 4 * 8);
    if (st) return st;
    A.first_path = 0;
    A.n_paths = n_samples;
    A.n_chunks = n_chunks;
    A.ppl = ppl;
    A.hier = hier ? 1 : 0;
    A.partials = c->d_partials;
    A.dump = nullptr;
    const int grid = launch_grid(c, P, n_chunks);
    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    HIP_TRY(c, launch_amplitude(A, P.kind, P.p, P.U, grid, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
    HIP_TRY(c, launch_reduce(c->d_partials, n_chunks, nlev, c->d_red, c->stream));
    std::vector<double> red(size_t(nlev) * 4);
    HIP_TRY(c, hipMemcpyAsync(red.data(), c->d_red, red.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms = ms;
    c->last_chunks = n_chunks;
    c->last_chunk_paths = chunk_paths;
    bool nonfinite = false;
    for (int n = 1; n < nlev; ++n) {
        if (!hier && n != P.s) continue;
        const double cnt = red[size_t(n) * 4 + 0];
        const double sd = red[size_t(n) * 4 + 1];
        const double sd2 = red[size_t(n) * 4 + 2];
        const double nb = red[size_t(n) * 4 + 3];
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
        const double logbase = std::log(P.pref * P.K0) - P.shift[size_t(n)];
        const double base = std::exp(logbase);
        pimc_level_result& r = out[n];
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
        if (nb > 0 || !std::isfinite(r.amp) || !std::isfinite(r.err)) nonfinite = true;
    }
    return nonfinite ? PIMC_WNONFINITE : PIMC_OK;
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
    const uint32_t ppl = paths_per_lane(P.s);
    const uint64_t chunk_paths = uint64_t(kBlock) * ppl;
    A.first_path = first_path;
    A.n_paths = k_paths;
    A.n_chunks = (k_paths + chunk_paths - 1) / chunk_paths;
    A.ppl = ppl;
    A.hier = (flags & PIMC_HIERARCHY) ? 1 : 0;
    A.partials = nullptr;
    A.dump = c->d_dump;
    const int grid = launch_grid(c, P, A.n_chunks);
    HIP_TRY(c, launch_amplitude(A, P.kind, P.p, P.U, grid, c->stream));
    HIP_TRY(c, hipMemcpyAsync(S_out, c->d_dump, size_t(k_paths) * nlev * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // level 0 is the same straight slice for every path: report it for every path
    for (uint64_t i = 0; i < k_paths; ++i)
        if (!(flags & PIMC_HIERARCHY)) S_out[i * nlev] = 0.0;
    return PIMC_OK;
}

int pimc_last_partials(pimc_ctx* c, uint32_t level, uint64_t first_chunk, uint64_t n_chunks, double* out,
                       uint64_t* chunk_paths, uint64_t* total_chunks, double* shift) {
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (c->last_s < 1 || !c->d_partials) return ctx_fail(c, PIMC_EINVAL, "no estimation has run on this context");
    if (int(level) > c->last_s) return ctx_fail(c, PIMC_EINVAL, "level %u > s = %d", level, c->last_s);
    if (first_chunk + n_chunks > c->last_chunks || first_chunk + n_chunks < first_chunk)
        return ctx_fail(c, PIMC_EINVAL, "chunks out of range (%llu total)", (unsigned long long)c->last_chunks);
    if (chunk_paths) *chunk_paths = c->last_chunk_paths;
    if (total_chunks) *total_chunks = c->last_chunks;
    if (shift) *shift = c->last_shift[level];
    if (n_chunks == 0) return PIMC_OK;
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    const double* src = c->d_partials + (uint64_t(level) * c->last_chunks + first_chunk) * 4;
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
