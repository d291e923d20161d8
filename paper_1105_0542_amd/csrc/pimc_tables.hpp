// Host-side effective-action tables (FP64) and the compile-time table shape of the anharmonic
// oscillator. Independent of any device code.
//
// The coefficients c_{m,k}(x) of W = sum_{m,k} c_{m,k}(x) eps^(m-k) xbar^(2k) (eq.(ansatz)) follow
// from eq.(1Drec) with c_{0,0} = V and the diagonal eq.(diagonal), each m computed diagonal first
// and then k = m-1 .. 0 (Fig. 1 of Balaz et al.). For a polynomial V every c_{m,k} is a polynomial
// in x; here they are carried in FP64 (a polynomial of degree d has d+1 coefficients).
//
// The GPU evaluates  eps W_p = sum_k dlt^(2k) P_k(u)  with dlt = q_{k+1} - q_k = 2 xbar, so
// P_k = eps 4^-k sum_{m=k}^{p-1} eps^(m-k) c_{m,k}(x), and u = x^2 when V is even (then every
// c_{m,k} is even in x) or u = x otherwise.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace pimc {

constexpr int kMaxP = 18;

using PolyD = std::vector<double>;   // index = power of x

inline PolyD poly_trim(PolyD a) {
    while (!a.empty() && a.back() == 0.0) a.pop_back();
    return a;
}
inline PolyD poly_der(const PolyD& a, int times = 1) {
    PolyD r = a;
    for (int t = 0; t < times; ++t) {
        if (r.size() <= 1) return {};
        PolyD d(r.size() - 1);
        for (size_t i = 1; i < r.size(); ++i) d[i - 1] = r[i] * double(i);
        r.swap(d);
    }
    return r;
}
inline void poly_axpy(PolyD& y, double a, const PolyD& x) {   // y += a x
    if (y.size() < x.size()) y.resize(x.size(), 0.0);
    for (size_t i = 0; i < x.size(); ++i) y[i] += a * x[i];
}
inline PolyD poly_mul(const PolyD& a, const PolyD& b) {
    if (a.empty() || b.empty()) return {};
    PolyD r(a.size() + b.size() - 1, 0.0);
    for (size_t i = 0; i < a.size(); ++i)
        for (size_t j = 0; j < b.size(); ++j) r[i + j] += a[i] * b[j];
    return r;
}

// General-potential mode: highest level p, derivative order and number of sech^2 / Gaussian terms.
// Levels up to kGenInlineMaxP use evaluators inlined into the walker over several slices at once;
// the higher ones (up to 24,196 monomials at p = 18) one out-of-line function per level that takes
// one slice, so that each level's straight-line code exists once per kernel.
constexpr int kGenMaxP = 18;
constexpr int kGenInlineMaxP = 10;
constexpr int kGenMaxJ = 2 * kGenMaxP - 2;
constexpr int kGenMaxTerms = 4;
// General mode, per level p: bisection levels of a subtree held in registers and slices evaluated
// together by the generated code (for 5 <= p <= kGenInlineMaxP: PIMC_GEN_U_HI, PIMC_GEN_B_HI; above,
// subtrees of 3 levels whose slices go to the out-of-line evaluator in pairs).
#ifndef PIMC_GEN_U_HI
#define PIMC_GEN_U_HI 1
#endif
#ifndef PIMC_GEN_B_HI
#define PIMC_GEN_B_HI 2
#endif
constexpr int gen_subtree_levels(int p) { return p <= 4 ? 2 : p <= kGenInlineMaxP ? PIMC_GEN_U_HI : 3; }
constexpr int gen_block_slices(int p) { return p <= 4 ? 4 : PIMC_GEN_B_HI; }
static_assert(PIMC_GEN_U_HI >= 1 && PIMC_GEN_U_HI <= 4, "general-mode subtree levels");

// c[m][k], 0 <= k <= m < p, FP64.
struct Coefficients {
    int p = 0;
    std::vector<std::vector<PolyD>> c;
};

// d/dx of a polynomial in x.
struct XDerivative {
    PolyD operator()(const PolyD& a, int times = 1) const { return poly_der(a, times); }
};

// d/dx of a polynomial in y = tanh(alpha x): alpha (1 - y^2) d/dy (polynomials in y stay
// polynomials; the modified Poeschl-Teller potential -lambda/cosh^2(alpha x) is -lambda (1 - y^2)).
struct TanhDerivative {
    double alpha;
    PolyD operator()(const PolyD& a, int times = 1) const {
        PolyD r = a;
        for (int t = 0; t < times; ++t) {
            const PolyD d = poly_der(r);
            PolyD out(d.size() + 2, 0.0);
            for (size_t i = 0; i < d.size(); ++i) {
                out[i] += alpha * d[i];
                out[i + 2] -= alpha * d[i];
            }
            r = poly_trim(out);
        }
        return r;
    }
};

// eq.(1Drec) and eq.(diagonal) with the derivative `der` (coefficients as polynomials in the
// variable `der` differentiates).
template <class Der>
inline Coefficients effective_coefficients(const PolyD& V, int p, const Der& der) {
    Coefficients C;
    C.p = p;
    C.c.assign(p, std::vector<PolyD>(p));
    C.c[0][0] = poly_trim(V);
    double fact = 1.0;                                           // (2m+1)!
    std::vector<std::vector<PolyD>> d1(p, std::vector<PolyD>(p)); // first derivatives
    d1[0][0] = der(C.c[0][0]);
    for (int m = 1; m < p; ++m) {
        fact *= double(2 * m) * double(2 * m + 1);
        PolyD diag = der(C.c[0][0], 2 * m);                      // eq.(diagonal)
        for (double& v : diag) v /= fact;
        C.c[m][m] = poly_trim(diag);
        for (int k = m - 1; k >= 0; --k) {                       // eq.(1Drec)
            PolyD rhs;
            poly_axpy(rhs, double((2 * k + 2) * (2 * k + 1)), C.c[m][k + 1]);
            poly_axpy(rhs, 1.0, der(C.c[m - 1][k], 2));
            for (int l = 0; l <= m - 2; ++l)
                for (int r = std::max(0, k - m + l + 2); r <= std::min(k, l); ++r)
                    poly_axpy(rhs, -1.0, poly_mul(d1[l][r], d1[m - l - 2][k - r]));
            for (int l = 1; l <= m - 2; ++l)
                for (int r = std::max(0, k - m + l + 2); r <= std::min(k, l); ++r) {
                    const int f = 2 * r * (2 * k - 2 * r + 2);
                    if (f) poly_axpy(rhs, -double(f), poly_mul(C.c[l][r], C.c[m - l - 1][k - r + 1]));
                }
            for (double& v : rhs) v /= double(8 * (m + k + 1));
            C.c[m][k] = poly_trim(rhs);
        }
        for (int k = 0; k <= m; ++k) d1[m][k] = der(C.c[m][k]);
    }
    return C;
}

inline Coefficients effective_coefficients(const PolyD& V, int p) { return effective_coefficients(V, p, XDerivative{}); }

// Folded table of one level: for k = 0..K-1 the coefficients of P_k(u) from the highest power
// deg[k] down to 0.
struct LevelTable {
    bool even = true;
    double tanh_alpha = 0.0;       // > 0: the variable is u = tanh^2(tanh_alpha * mid)
    std::vector<int> deg;          // per k, in the variable u
    std::vector<double> coef;      // concatenated, highest power first
};

inline bool potential_is_even(const PolyD& V) {
    for (size_t j = 1; j < V.size(); j += 2)
        if (V[j] != 0.0) return false;
    return true;
}

// Shape (number of P_k and their degrees) is a property of the coefficient structure, not of eps:
// it is taken from the degree bound `xdeg` so that every level of a run has the same layout.
inline LevelTable fold_level(const Coefficients& C, bool even, double eps, const std::vector<int>& xdeg) {
    LevelTable t;
    t.even = even;
    const int p = C.p;
    const int K = int(xdeg.size());
    for (int k = 0; k < K; ++k) {
        // Q(x) = sum_m eps^(m-k) c_{m,k}(x), then * eps * 4^-k
        PolyD Q;
        double ep = 1.0;
        for (int m = k; m < p; ++m) {
            poly_axpy(Q, ep, C.c[m][k]);
            ep *= eps;
        }
        const double scale = eps * std::ldexp(1.0, -2 * k);
        const int dx = xdeg[k];
        const int du = even ? dx / 2 : dx;
        t.deg.push_back(du);
        for (int e = du; e >= 0; --e) {
            const size_t px = size_t(even ? 2 * e : e);
            t.coef.push_back(px < Q.size() ? Q[px] * scale : 0.0);
        }
    }
    return t;
}

// Device form of an even table for evaluators that square the endpoint sum (qa + qb) instead of
// the mid-point: the coefficient of u^e is multiplied by 4^-e, so with u' = (qa + qb)^2 = 4 mid^2
// every Horner step is the unscaled one times an exact power of two (the same results bit for bit).
// coef: one level (deg.size() blocks, highest power first).
inline void scale_for_endpoint_sum(double* coef, const std::vector<int>& deg) {
    size_t off = 0;
    for (int d : deg) {
        for (int i = 0; i <= d; ++i) coef[off + size_t(i)] = std::ldexp(coef[off + size_t(i)], -2 * (d - i));
        off += size_t(d) + 1;
    }
}

// Degree (in x) of each P_k at level p: the largest degree among c_{m,k}, m = k..p-1, with
// trailing all-zero k dropped.
inline std::vector<int> table_xdegrees(const Coefficients& C) {
    std::vector<int> xdeg;
    for (int k = 0; k < C.p; ++k) {
        int d = -1;
        for (int m = k; m < C.p; ++m) d = std::max(d, int(C.c[m][k].size()) - 1);
        xdeg.push_back(d);
    }
    while (!xdeg.empty() && xdeg.back() < 0) xdeg.pop_back();
    for (int& d : xdeg) d = std::max(d, 0);
    return xdeg;
}

// Horner evaluation of one folded table on the host (used for the straight-line reference action
// and the analytic level-0 amplitude).
inline double eval_level(const LevelTable& t, double qa, double qb) {
    const double mid = 0.5 * (qa + qb);
    const double dl = qb - qa;
    double u;
    if (t.tanh_alpha > 0.0) {
        const double y = std::tanh(t.tanh_alpha * mid);
        u = y * y;
    } else {
        u = t.even ? mid * mid : mid;
    }
    const double z = dl * dl;
    double acc = 0.0;
    size_t off = t.coef.size();
    for (int k = int(t.deg.size()) - 1; k >= 0; --k) {
        off -= size_t(t.deg[k]) + 1;
        double v = t.coef[off];
        for (int e = 1; e <= t.deg[k]; ++e) v = v * u + t.coef[off + e];
        acc = (k == int(t.deg.size()) - 1) ? v : acc * z + v;
    }
    return acc;
}

// ----------------------------------------------------------------------------------------------
// Compile-time shape of the anharmonic-oscillator table (V even, degree 4): the degree recursion
// of eq.(1Drec)/(diagonal) with generic coefficients. deg(c_{0,0}) = 4; a product adds degrees, a
// derivative lowers by one, a zero polynomial has degree -1.
struct DegreeTable {
    int d[kMaxP][kMaxP];
};

constexpr int deg_der(int d, int times) { return d - times >= 0 ? d - times : -1; }
constexpr int deg_mul(int a, int b) { return (a < 0 || b < 0) ? -1 : a + b; }
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }

constexpr DegreeTable degree_table(int dV) {
    DegreeTable t{};
    for (int m = 0; m < kMaxP; ++m)
        for (int k = 0; k < kMaxP; ++k) t.d[m][k] = -1;
    t.d[0][0] = dV;
    for (int m = 1; m < kMaxP; ++m) {
        t.d[m][m] = deg_der(dV, 2 * m);
        for (int k = m - 1; k >= 0; --k) {
            int d = imax(t.d[m][k + 1], deg_der(t.d[m - 1][k], 2));
            for (int l = 0; l <= m - 2; ++l)
                for (int r = imax(0, k - m + l + 2); r <= imin(k, l); ++r)
                    d = imax(d, deg_mul(deg_der(t.d[l][r], 1), deg_der(t.d[m - l - 2][k - r], 1)));
            for (int l = 1; l <= m - 2; ++l)
                for (int r = imax(0, k - m + l + 2); r <= imin(k, l); ++r)
                    if (r > 0) d = imax(d, deg_mul(t.d[l][r], t.d[m - l - 1][k - r + 1]));
            t.d[m][k] = d;
        }
    }
    return t;
}

constexpr DegreeTable kQuarticDegrees = degree_table(4);

// Shape of the quartic table at level p: K polynomials P_k(y), y-degrees DY[k], offsets, size E.
template <int P>
struct QuarticShape {
    static constexpr int xdeg(int k) {
        int d = -1;
        for (int m = k; m < P; ++m) d = imax(d, kQuarticDegrees.d[m][k]);
        return d;
    }
    static constexpr int count_k() {
        int K = 0;
        for (int k = 0; k < P; ++k)
            if (xdeg(k) >= 0) K = k + 1;
        return K;
    }
    static constexpr int K = count_k();
    static constexpr int dy(int k) { return xdeg(k) < 0 ? 0 : xdeg(k) / 2; }
    static constexpr int off(int k) {
        int o = 0;
        for (int i = 0; i < k; ++i) o += dy(i) + 1;
        return o;
    }
    static constexpr int E = off(K);
};

static_assert(QuarticShape<18>::K == 8 && QuarticShape<18>::E == 48, "quartic table shape at p=18");
static_assert(QuarticShape<12>::K == 6 && QuarticShape<12>::E == 27, "quartic table shape at p=12");
static_assert(QuarticShape<4>::K == 3 && QuarticShape<4>::E == 8, "quartic table shape at p=4");

}  // namespace pimc
