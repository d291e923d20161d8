// Host side of the general-potential entry points (pimc_amplitude_general, pimc_path_actions_general
// in include/pimc.h): the derivative-symbol coefficients of eq.(1Drec)/(diagonal), computed once
// per p and cached, their monomials in the canonical order of the evaluators generated at build time,
// the scale factors of each bisection level; the derivative tables of the potential after the mass
// rescaling; the straight-line reference actions. Estimation and per-path actions then run through
// the shared walker kernels with the evaluator of level p.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>

#include "pimc.h"
#include "pimc_host_common.hpp"

using namespace pimc;
using namespace pimc_host;

static_assert(PIMC_GEN_MAX_P == kGenMaxP, "general-mode level limit of the public header");
static_assert(PIMC_GEN_MAX_TERMS == kGenMaxTerms, "general-mode term limit of the public header");
static_assert(PIMC_MAX_DEGREE == 8, "the derivative tables and their device evaluation hold rows of degree 8");

namespace {

struct LevelMonomials {
    SymCoefficients C;
    std::vector<GenMono> M;
};

// The symbolic coefficients and canonical monomials of level p, computed once per process.
const LevelMonomials& cached_monomials(int p) {
    static std::mutex mu;
    static std::map<int, std::unique_ptr<LevelMonomials>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(p);
    if (it == cache.end()) {
        auto L = std::make_unique<LevelMonomials>();
        L->C = symbolic_coefficients(p);
        L->M = canonical_monomials(L->C);
        it = cache.emplace(p, std::move(L)).first;
    }
    return *it->second;
}

double straight_line_general(const GenPotential& G, const std::vector<GenMono>& M, const double* scales, double a,
                             double b, int n) {
    const int N = 1 << n;
    double acc = 0.0;
    for (int k = 0; k < N; ++k) {
        const double q0 = a + (b - a) * double(k) / double(N);
        const double q1 = a + (b - a) * double(k + 1) / double(N);
        acc += gen_eval_slice(G, M, scales, q0, q1);
    }
    return acc;
}

}  // namespace

namespace pimc_host {

int check_general(const pimc_general_potential* V, double m, double a, double b, double T, uint32_t N, int p,
                  uint64_t n_samples) {
    if (!V) { set_thread_error("potential is NULL"); return PIMC_EINVAL; }
    if (V->degree < 0 || V->degree > PIMC_MAX_DEGREE) {
        set_thread_error("degree %d outside 0..%d", V->degree, PIMC_MAX_DEGREE);
        return PIMC_EINVAL;
    }
    for (int j = 0; j <= V->degree; ++j)
        if (!std::isfinite(V->coef[j])) { set_thread_error("coefficient %d is not finite", j); return PIMC_EINVAL; }
    if (V->n_sech2 < 0 || V->n_sech2 > PIMC_GEN_MAX_TERMS || V->n_gauss < 0 || V->n_gauss > PIMC_GEN_MAX_TERMS) {
        set_thread_error("term counts outside 0..%d", PIMC_GEN_MAX_TERMS);
        return PIMC_EINVAL;
    }
    for (int i = 0; i < V->n_sech2; ++i)
        if (!std::isfinite(V->sech2_A[i]) || !std::isfinite(V->sech2_alpha[i]) || V->sech2_alpha[i] <= 0) {
            set_thread_error("sech^2 term %d: A finite, alpha finite and > 0", i);
            return PIMC_EINVAL;
        }
    for (int i = 0; i < V->n_gauss; ++i)
        if (!std::isfinite(V->gauss_B[i]) || !std::isfinite(V->gauss_beta[i]) || V->gauss_beta[i] <= 0) {
            set_thread_error("Gaussian term %d: B finite, beta finite and > 0", i);
            return PIMC_EINVAL;
        }
    if (p < 1 || p > PIMC_GEN_MAX_P) { set_thread_error("p = %d outside 1..%d", p, PIMC_GEN_MAX_P); return PIMC_EINVAL; }
    pimc_potential zero{};
    return check_args(&zero, m, a, b, T, N, p, n_samples);
}

int build_problem_general(const pimc_general_potential* V, double m, double a, double b, double T, uint32_t N, int p,
                          uint32_t flags, Problem& P, char* why, size_t whylen) {
    if (flags & PIMC_FP32_POLY) {
        std::snprintf(why, whylen, "FP32 polynomials need an even polynomial potential of degree <= 4");
        return PIMC_EUNSUPPORTED;
    }
    if (log2_exact(N) > 20) {
        std::snprintf(why, whylen, "N too large");
        return PIMC_EINVAL;
    }
    P.s = log2_exact(N);
    P.p = p;
    P.T = T;
    const double sm = std::sqrt(m);
    P.a = a * sm;
    P.b = b * sm;
    P.pref = sm;
    P.K0 = std::exp(-(P.b - P.a) * (P.b - P.a) / (2.0 * T)) / std::sqrt(2.0 * M_PI * T);
    P.even = false;
    P.kind = EvalKind::General64;
    P.U = std::min(P.s, gen_subtree_levels(p));
    if (P.s == 0) P.U = 0;
    P.D = P.s - P.U;
    // the potential after the mass rescaling V(y / sqrt(m))
    GenPotential& G = P.gen;
    G.J = 2 * p - 2;
    G.poly.assign(size_t(V->degree) + 1, 0.0);
    double f = 1.0;
    for (int j = 0; j <= V->degree; ++j) {
        G.poly[size_t(j)] = V->coef[j] * f;
        f /= sm;
    }
    G.poly = poly_trim(G.poly);
    G.sech_A.clear();
    G.sech_a.clear();
    G.gauss_B.clear();
    G.gauss_b.clear();
    for (int i = 0; i < V->n_sech2; ++i) {
        G.sech_A.push_back(V->sech2_A[i]);
        G.sech_a.push_back(V->sech2_alpha[i] / sm);
    }
    for (int i = 0; i < V->n_gauss; ++i) {
        G.gauss_B.push_back(V->gauss_B[i]);
        G.gauss_b.push_back(V->gauss_beta[i] / m);
    }
    gen_potential_tables(G);
    const LevelMonomials& L = cached_monomials(p);
    const int nrec = int(L.M.size());
    if (general_compiled_nrec(p) != nrec) {
        std::snprintf(why, whylen, "internal: the evaluator compiled for p = %d expects %d monomials, the recursion gives %d",
                      p, general_compiled_nrec(p), nrec);
        return PIMC_EUNSUPPORTED;
    }
    P.deg.clear();
    const int stride = G.J + 2;
    P.stride = stride;
    P.tab.assign(size_t(P.s + 1) * size_t(stride), 0.0);
    for (int n = 0; n <= P.s; ++n) level_scales(G.J, std::ldexp(T, -n), P.tab.data() + size_t(n) * size_t(stride));
    P.tab_dev = P.tab;
    P.tab32.assign(P.tab.size(), 0.0f);
    P.sig.assign(size_t(P.s + 1), 0.0);
    for (int n = 1; n <= P.s; ++n) P.sig[size_t(n)] = std::sqrt(T / std::ldexp(1.0, n + 1));
    P.shift.assign(size_t(P.s + 1), 0.0);
    for (int n = 0; n <= P.s; ++n)
        P.shift[size_t(n)] =
            straight_line_general(G, L.M, P.tab.data() + size_t(n) * size_t(stride), P.a, P.b, n);
    P.level0_action = P.shift[0];
    return PIMC_OK;
}

}  // namespace pimc_host

extern "C" {

int pimc_amplitude_general(pimc_ctx* c, const pimc_general_potential* V, double m, double a, double b, double T,
                           uint32_t N, int p, uint64_t n_samples, uint64_t seed, uint32_t stream, uint32_t flags,
                           pimc_level_result* out) {
    int st = check_general(V, m, a, b, T, N, p, n_samples);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    HIP_TRY(c, hipSetDevice(c->device));
    Problem P;
    char why[256] = "";
    st = build_problem_general(V, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return amplitude_core(c, P, n_samples, seed, stream, flags, out);
}

int pimc_path_actions_general(pimc_ctx* c, const pimc_general_potential* V, double m, double a, double b, double T,
                              uint32_t N, int p, uint64_t seed, uint32_t stream, uint32_t flags, uint64_t first_path,
                              uint64_t k_paths, double* S_out) {
    int st = check_general(V, m, a, b, T, N, p, 2);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!S_out && k_paths) return ctx_fail(c, PIMC_EINVAL, "S_out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    if (k_paths == 0) return PIMC_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    Problem P;
    char why[256] = "";
    st = build_problem_general(V, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return path_actions_core(c, P, seed, stream, flags, first_path, k_paths, S_out);
}

}  // extern "C"
