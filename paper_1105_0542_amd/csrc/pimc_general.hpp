// General-potential mode (host side): the effective potential in the derivative symbols
// v_j = V^(j)(x) (Sec. 3.1/3.2: for a general V the c_{m,k} are expressions in V and its
// derivatives up to order 2p-2). eq.(1Drec) and eq.(diagonal) run on polynomials in v_0..v_J with
// the derivation d v_j/dx = v_{j+1}; the result does not depend on V and is computed once per p.
// In the dimensionless form (level_scales) the coefficients are the same at every bisection level and
// only the derivative values and dlt^2 are scaled per level; the device evaluators, generated from the
// same canonical monomial order at build time with the coefficients as constants, form the products
// of the scaled derivative values at each slice mid-point and sum eps W_p.
//
// Potentials of this mode: V(x) = sum_n c_n x^n + sum_i A_i / cosh^2(a_i x) + sum_i B_i exp(-b_i x^2),
// whose derivatives come from tables computed here: the polynomial's derivative coefficients, the
// polynomials S_j(t) in t = tanh(a x) with d^j/dx^j (A/cosh^2(a x)) = A a^j S_j(t), S_0 = 1 - t^2,
// S_{j+1} = (1 - t^2) S_j'(t), kept as S_j = sech^2(a x) R_j(t) with R_0 = 1,
// R_{j+1} = -2t R_j + (1 - t^2) R_j' (sech^2 from e^(-2|a x|), accurate where tanh^2 rounds to 1),
// and Hermite polynomials for the Gaussians.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <vector>

#include "pimc_tables.hpp"

namespace pimc {

using SymMono = std::vector<uint8_t>;            // exponent of each symbol v_0..v_{J+1}
using SymPoly = std::map<SymMono, double>;

inline void sym_axpy(SymPoly& y, double a, const SymPoly& x) {
    for (const auto& kv : x) {
        auto it = y.find(kv.first);
        if (it == y.end())
            y.emplace(kv.first, a * kv.second);
        else
            it->second += a * kv.second;
    }
}

inline SymPoly sym_mul(const SymPoly& a, const SymPoly& b) {
    SymPoly out;
    for (const auto& ka : a)
        for (const auto& kb : b) {
            SymMono m(ka.first.size());
            for (size_t i = 0; i < m.size(); ++i) m[i] = uint8_t(ka.first[i] + kb.first[i]);
            out[m] += ka.second * kb.second;
        }
    return out;
}

inline SymPoly sym_der(const SymPoly& a, int times = 1) {
    SymPoly r = a;
    for (int t = 0; t < times; ++t) {
        SymPoly out;
        for (const auto& kv : r)
            for (size_t j = 0; j + 1 < kv.first.size(); ++j)
                if (kv.first[j]) {
                    SymMono m = kv.first;
                    m[j] -= 1;
                    m[j + 1] += 1;
                    out[m] += kv.second * double(kv.first[j]);
                }
        r.swap(out);
    }
    return r;
}

struct SymCoefficients {
    int p = 0;
    int J = 0;                                   // highest derivative order, 2p - 2
    std::vector<std::vector<SymPoly>> c;         // c[m][k]
};

// eq.(diagonal) then eq.(1Drec) for k = m-1..0 (Fig. 1), c_{0,0} = v_0.
inline SymCoefficients symbolic_coefficients(int p) {
    SymCoefficients C;
    C.p = p;
    C.J = 2 * p - 2;
    const size_t nv = size_t(C.J) + 2;
    C.c.assign(p, std::vector<SymPoly>(p));
    SymMono v0(nv, 0);
    v0[0] = 1;
    C.c[0][0][v0] = 1.0;
    std::vector<std::vector<SymPoly>> d1(p, std::vector<SymPoly>(p));
    d1[0][0] = sym_der(C.c[0][0]);
    double fact = 1.0;
    for (int m = 1; m < p; ++m) {
        fact *= double(2 * m) * double(2 * m + 1);
        SymMono vm(nv, 0);
        vm[size_t(2 * m)] = 1;
        C.c[m][m][vm] = 1.0 / fact;
        for (int k = m - 1; k >= 0; --k) {
            SymPoly rhs;
            sym_axpy(rhs, double((2 * k + 2) * (2 * k + 1)), C.c[m][k + 1]);
            sym_axpy(rhs, 1.0, sym_der(C.c[m - 1][k], 2));
            for (int l = 0; l <= m - 2; ++l)
                for (int r = std::max(0, k - m + l + 2); r <= std::min(k, l); ++r)
                    sym_axpy(rhs, -1.0, sym_mul(d1[l][r], d1[m - l - 2][k - r]));
            for (int l = 1; l <= m - 2; ++l)
                for (int r = std::max(0, k - m + l + 2); r <= std::min(k, l); ++r) {
                    const int f = 2 * r * (2 * k - 2 * r + 2);
                    if (f) sym_axpy(rhs, -double(f), sym_mul(C.c[l][r], C.c[m - l - 1][k - r + 1]));
                }
            SymPoly out;
            for (const auto& kv : rhs)
                if (kv.second != 0.0) out.emplace(kv.first, kv.second / double(8 * (m + k + 1)));
            C.c[m][k].swap(out);
        }
        for (int k = 0; k <= m; ++k) d1[m][k] = sym_der(C.c[m][k]);
    }
    return C;
}

// One monomial of the level-p effective potential: coefficient c of prod_i v_{f[i]} in c_{m,k}.
struct GenMono {
    int k = 0, m = 0;
    std::vector<uint8_t> f;                      // factor indices, ascending (v_j repeated e_j times)
    double c = 0.0;
};

// Every monomial of every c_{m,k} in the order in which the compiled evaluators consume them:
// k from p-1 down to 0 (Horner in dlt^2), then factor lists in lexicographic order, so that
// consecutive monomials share the longest possible prefix of factors (a prefix tree walked depth
// first). A factor list determines m (its weight is 2m + 2), so the order is total.
inline std::vector<GenMono> canonical_monomials(const SymCoefficients& C) {
    std::vector<GenMono> out;
    for (int k = C.p - 1; k >= 0; --k) {
        std::vector<GenMono> grp;
        for (int m = k; m < C.p; ++m)
            for (const auto& kv : C.c[size_t(m)][size_t(k)]) {
                GenMono g;
                g.k = k;
                g.m = m;
                g.c = kv.second;
                for (size_t j = 0; j < kv.first.size(); ++j)
                    for (int e = 0; e < kv.first[j]; ++e) g.f.push_back(uint8_t(j));
                grp.push_back(std::move(g));
            }
        std::sort(grp.begin(), grp.end(), [](const GenMono& a, const GenMono& b) { return a.f < b.f; });
        out.insert(out.end(), grp.begin(), grp.end());
    }
    return out;
}

// Per-level scale factors of the dimensionless form. A monomial of c_{m,k} with factor list f has
// weight sum_f (j_f + 2) = 2m + 2, so its term eps^(m-k+1) 4^-k dlt^(2k) prod_f v_(j_f) equals
// (dlt^2 / (4 eps))^k prod_f (eps^(1 + j_f/2) v_(j_f)): with the scaled derivatives
// vt_j = eps^(1 + j/2) v_j and zt = dlt^2 / (4 eps), eps W_p = sum_k zt^k sum c prod vt_f, whose
// coefficients c do not depend on the level. out[j] = eps^(1 + j/2) for j <= J, out[J+1] = 1/(4 eps).
inline void level_scales(int J, double eps, double* out) {
    for (int j = 0; j <= J; ++j) out[j] = std::pow(eps, 1.0 + 0.5 * double(j));
    out[J + 1] = 0.25 / eps;
}

// Derivative tables of a potential of this mode (after the mass rescaling).
struct GenPotential {
    int J = 0;
    std::vector<double> poly;                    // c_n
    std::vector<double> dpoly;                   // (J+1) rows x 9: coefficients of V^(j)
    int pdeg = -1;
    std::vector<double> sech_A, sech_a;          // terms A / cosh^2(a x)
    std::vector<double> dsech;                   // per term (J+1) rows x (J+1): A a^j R_j
    std::vector<double> gauss_B, gauss_b;        // terms B exp(-b x^2)
};

inline void gen_potential_tables(GenPotential& G) {
    const int J = G.J;
    G.pdeg = int(G.poly.size()) - 1;
    G.dpoly.assign(size_t(J + 1) * 9, 0.0);
    PolyD d = G.poly;
    for (int j = 0; j <= J; ++j) {
        for (size_t n = 0; n < d.size() && n < 9; ++n) G.dpoly[size_t(j) * 9 + n] = d[n];
        d = poly_der(d);
    }
    G.dsech.assign(G.sech_A.size() * size_t(J + 1) * size_t(J + 1), 0.0);
    for (size_t i = 0; i < G.sech_A.size(); ++i) {
        PolyD R = {1.0};                                        // R_0 = 1
        double scale = G.sech_A[i];
        for (int j = 0; j <= J; ++j) {
            double* row = G.dsech.data() + (i * size_t(J + 1) + size_t(j)) * size_t(J + 1);
            for (size_t n = 0; n < R.size() && n <= size_t(J); ++n) row[n] = scale * R[n];
            // S_j = (1 - t^2) R_j and S_{j+1} = (1 - t^2) S_j' give R_{j+1} = -2t R_j + (1 - t^2) R_j'
            const PolyD dR = poly_der(R);
            PolyD nx(std::max(R.size() + 1, dR.size() + 2), 0.0);
            for (size_t n = 0; n < R.size(); ++n) nx[n + 1] -= 2.0 * R[n];
            for (size_t n = 0; n < dR.size(); ++n) {
                nx[n] += dR[n];
                nx[n + 2] -= dR[n];
            }
            R = poly_trim(nx);
            scale *= G.sech_a[i];
        }
    }
}

// sech^2(y) = 4w / (1 + w)^2 with w = e^(-2|y|): no cancellation anywhere (1 - tanh^2 loses every
// digit once tanh rounds towards 1), no overflow for large |y|.
inline double sech2_of(double y) {
    const double w = std::exp(-2.0 * std::fabs(y));
    const double d = 1.0 + w;
    return 4.0 * w / (d * d);
}

// v_j = V^(j)(x), j = 0..J (the device evaluates the same formulas).
inline void gen_derivatives(const GenPotential& G, double x, double* v) {
    const int J = G.J;
    for (int j = 0; j <= J; ++j) {
        const int dg = G.pdeg - j;
        double acc = 0.0;
        if (dg >= 0) {
            acc = G.dpoly[size_t(j) * 9 + size_t(dg)];
            for (int n = dg - 1; n >= 0; --n) acc = std::fma(acc, x, G.dpoly[size_t(j) * 9 + size_t(n)]);
        }
        v[j] = acc;
    }
    for (size_t i = 0; i < G.sech_A.size(); ++i) {
        const double y = G.sech_a[i] * x;
        const double t = std::tanh(y);
        const double s2 = sech2_of(y);
        for (int j = 0; j <= J; ++j) {
            const double* row = G.dsech.data() + (i * size_t(J + 1) + size_t(j)) * size_t(J + 1);
            double acc = row[j];
            for (int n = j - 1; n >= 0; --n) acc = std::fma(acc, t, row[n]);
            v[j] = std::fma(s2, acc, v[j]);
        }
    }
    for (size_t i = 0; i < G.gauss_B.size(); ++i) {
        // d^j/dx^j B e^{-b x^2} = B (-sqrt b)^j H_j(sqrt(b) x) e^{-b x^2}, H_{j+1} = 2y H_j - 2j H_{j-1}
        const double sb = std::sqrt(G.gauss_b[i]);
        const double y = sb * x;
        double e = G.gauss_B[i] * std::exp(-G.gauss_b[i] * x * x);
        double hm = 0.0, h = 1.0;
        for (int j = 0; j <= J; ++j) {
            v[j] += e * h;
            const double hn = 2.0 * y * h - 2.0 * double(j) * hm;
            hm = h;
            h = hn;
            e *= -sb;
        }
    }
}

// Value of the prefix-tree node at depth d whose monomials are M[r0..r1) (all share their first d
// factors, in lexicographic order): its own coefficient (the monomial of exactly d factors, which
// comes first) plus v_j times the value of each child j; a leaf child contributes its coefficient.
// The generated evaluators do the same operations in the same order.
inline double gen_tree_node(const std::vector<GenMono>& M, size_t r0, size_t r1, size_t d, const double* v) {
    bool has_c = false;
    double c = 0.0;
    if (M[r0].f.size() == d) {
        has_c = true;
        c = M[r0].c;
        ++r0;
    }
    double a = 0.0;
    bool first = true;
    for (size_t c0 = r0; c0 < r1;) {
        const int j = M[c0].f[d];
        size_t c1 = c0;
        while (c1 < r1 && M[c1].f[d] == j) ++c1;
        const double t = (c1 - c0 == 1 && M[c0].f.size() == d + 1) ? M[c0].c : gen_tree_node(M, c0, c1, d + 1, v);
        a = (first && !has_c) ? v[j] * t : std::fma(v[j], t, first ? c : a);
        first = false;
        c0 = c1;
    }
    return a;
}

// eps W_p of one slice from the canonical monomials and one level's scale factors (level_scales),
// formed as the compiled evaluators form it: scaled derivatives, per power of zt the prefix-tree sum
// (gen_tree_node), Horner in zt.
inline double gen_eval_slice(const GenPotential& G, const std::vector<GenMono>& M, const double* scales, double qa,
                             double qb) {
    const double x = 0.5 * (qa + qb);
    const double dl = qb - qa;
    const double z = dl * dl * scales[G.J + 1];
    std::vector<double> v(size_t(G.J) + 1);
    gen_derivatives(G, x, v.data());
    for (int j = 0; j <= G.J; ++j) v[size_t(j)] *= scales[j];
    double acc = 0.0;
    int k_prev = -1;
    bool first = true;
    for (size_t r0 = 0; r0 < M.size();) {
        size_t r1 = r0;
        while (r1 < M.size() && M[r1].k == M[r0].k) ++r1;
        if (!first)
            for (int k = k_prev - 1; k > M[r0].k; --k) acc = acc * z;   // a k without monomials
        const double g = gen_tree_node(M, r0, r1, 0, v.data());
        acc = first ? g : std::fma(acc, z, g);
        first = false;
        k_prev = M[r0].k;
        r0 = r1;
    }
    for (int k = k_prev - 1; k >= 0; --k) acc = acc * z;
    return acc;
}

}  // namespace pimc
