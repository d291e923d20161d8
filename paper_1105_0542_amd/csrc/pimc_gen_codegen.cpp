// Build-time generator of the general-potential slice evaluators (the counterpart of the generated
// Wp() functions of Sec. 3.1/3.2): for every level p = 1..kGenMaxP it runs eq.(1Drec)/(diagonal) on
// polynomials in the derivative symbols v_j = V^(j) (pimc_general.hpp), takes the monomials in
// canonical order and writes straight-line device code that forms their products from the scaled
// derivative values held in registers and sums them, coefficient by coefficient, into the Horner
// scheme in zt = dlt^2 / (4 eps):
//
//   template <> struct GenCompiled<p> {
//       static constexpr int J, NREC;        // highest derivative, number of monomials
//       template <int W> static void eval(vt[W][J+1], zt[W], acc[W]);
//   };
//
// In this dimensionless form (pimc_general.hpp: level_scales) the coefficients do not depend on the
// bisection level, so they are written into the code as exact hexadecimal constants. Consecutive
// monomials share prefixes of their factor lists; the prefix products are kept (q2, q3, ...:
// products of the first 2, 3, ... factors) and formed again only when the prefix changes. The
// monomials of one power of zt go round-robin into kGenAcc partial sums (independent dependency
// chains), added pairwise at the end of the group.
// Usage: pimc_gen_codegen <output header>.
#include <cstdio>
#include <string>
#include <vector>

#include "pimc_general.hpp"

using namespace pimc;

namespace {

std::string vref(int factor) { return "v[i][" + std::to_string(factor) + "]"; }

// Expression of the product of the first d factors of f (d >= 1).
std::string prefix(const std::vector<uint8_t>& f, int d) {
    return d == 1 ? vref(f[0]) : "q" + std::to_string(d) + "[i]";
}

// Sum of the first n partial accumulators of a group, pairwise in a fixed order (gen_group_sum).
std::string group_sum(int n) {
    std::vector<std::string> t;
    for (int a = 0; a < n; ++a) t.push_back("g" + std::to_string(a) + "[i]");
    while (t.size() > 1) {
        std::vector<std::string> u;
        for (size_t a = 0; a + 1 < t.size(); a += 2) u.push_back("(" + t[a] + " + " + t[a + 1] + ")");
        if (t.size() % 2) u.push_back(t.back());
        t.swap(u);
    }
    return t[0];
}

void emit_level(FILE* o, int p) {
    const SymCoefficients C = symbolic_coefficients(p);
    const std::vector<GenMono> M = canonical_monomials(C);
    size_t maxdeg = 1;
    for (const GenMono& g : M) maxdeg = std::max(maxdeg, g.f.size());
    std::fprintf(o, "template <>\nstruct GenCompiled<%d> {\n", p);
    std::fprintf(o, "    static constexpr int J = %d;\n    static constexpr int NREC = %zu;\n", C.J, M.size());
    std::fprintf(o, "    template <int W>\n");
    std::fprintf(o, "    __device__ __forceinline__ static void eval(const double (&v)[W][J + 1], const double (&z)[W],\n"
                    "                                                double (&acc)[W]) {\n");
    for (int a = 0; a < kGenAcc; ++a) std::fprintf(o, "        double g%d[W];\n", a);
    for (size_t d = 2; d < maxdeg; ++d) std::fprintf(o, "        double q%zu[W];\n", d);
    std::vector<std::vector<uint8_t>> held(maxdeg + 1);   // held[d]: the factors whose product q<d> holds
    int k_prev = -1;
    bool first_group = true;
    for (size_t r0 = 0; r0 < M.size();) {
        size_t r1 = r0;
        while (r1 < M.size() && M[r1].k == M[r0].k) ++r1;
        if (!first_group)
            for (int k = k_prev - 1; k > M[r0].k; --k)   // a k without monomials
                std::fprintf(o, "#pragma unroll\n        for (int i = 0; i < W; ++i) acc[i] = acc[i] * z[i];\n");
        std::fprintf(o, "        // k = %d\n", M[r0].k);
        for (size_t r = r0; r < r1; ++r) {
            const GenMono& g = M[r];
            const int a = int((r - r0) % size_t(kGenAcc));
            const bool first_use = r - r0 < size_t(kGenAcc);
            // prefix products still held from earlier monomials are reused; the others are formed
            const size_t n = g.f.size();
            std::string body;
            for (size_t d = 2; d + 1 <= n; ++d) {
                const std::vector<uint8_t> want(g.f.begin(), g.f.begin() + long(d));
                if (held[d] == want) continue;
                body += "q" + std::to_string(d) + "[i] = " + prefix(g.f, int(d - 1)) + " * " + vref(g.f[d - 1]) + "; ";
                held[d] = want;
            }
            const std::string val = n == 1 ? vref(g.f[0]) : prefix(g.f, int(n - 1)) + " * " + vref(g.f[n - 1]);
            const std::string ga = "g" + std::to_string(a) + "[i]";
            body += first_use ? ga + " = c * (" + val + ");" : ga + " = fma(c, " + val + ", " + ga + ");";
            std::fprintf(o, "        {\n            const double c = %a;   // monomial %zu\n#pragma unroll\n"
                            "            for (int i = 0; i < W; ++i) { %s }\n        }\n", g.c, r, body.c_str());
        }
        const std::string sum = group_sum(int(std::min(r1 - r0, size_t(kGenAcc))));
        std::fprintf(o, "#pragma unroll\n        for (int i = 0; i < W; ++i) acc[i] = %s;\n",
                     first_group ? sum.c_str() : ("fma(acc[i], z[i], " + sum + ")").c_str());
        first_group = false;
        k_prev = M[r0].k;
        r0 = r1;
    }
    for (int k = k_prev - 1; k >= 0; --k)
        std::fprintf(o, "#pragma unroll\n        for (int i = 0; i < W; ++i) acc[i] = acc[i] * z[i];\n");
    std::fprintf(o, "    }\n};\n\n");
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s <output header>\n", argv[0]);
        return 2;
    }
    FILE* o = std::fopen(argv[1], "w");
    if (!o) {
        std::perror(argv[1]);
        return 1;
    }
    std::fprintf(o, "// Generated by pimc_gen_codegen from the derivative-symbol recursion; not edited by hand.\n");
    std::fprintf(o, "#pragma once\n\nnamespace pimc {\n\n");
    for (int p = 1; p <= kGenMaxP; ++p) emit_level(o, p);
    std::fprintf(o, "}  // namespace pimc\n");
    return std::fclose(o) == 0 ? 0 : 1;
}
