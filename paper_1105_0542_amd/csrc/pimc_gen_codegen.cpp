// Build-time generator of the general-potential slice evaluators (the counterpart of the generated
// Wp() functions of Sec. 3.1/3.2): for every level p = 1..kGenMaxP it runs eq.(1Drec)/(diagonal) on
// polynomials in the derivative symbols v_j = V^(j) (pimc_general.hpp), takes the monomials in
// canonical order and writes straight-line device code that sums them from the scaled derivative
// values held in registers, per power of zt = dlt^2 / (4 eps) by a multivariate Horner scheme over the
// prefix tree of their factor lists, and then by the Horner scheme in zt:
//
//   template <> struct GenCompiled<p> {
//       static constexpr int J, NREC;        // highest derivative, number of monomials
//       template <int W> static void eval(vt[W][J+1], zt[W], acc[W]);
//   };
//
// In this dimensionless form (pimc_general.hpp: level_scales) the coefficients do not depend on the
// bisection level, so they are written into the code as exact hexadecimal constants. The monomials of
// one power of zt, in lexicographic order of their factor lists, are the depth-first walk of a prefix
// tree; a node's value is its own coefficient plus v_j times the value of each child j, so every tree
// edge costs one fma and only one partial sum per depth (a0, a1, ...) is live.
// Usage: pimc_gen_codegen <output header>.
#include <cstdio>
#include <string>
#include <vector>

#include "pimc_general.hpp"

using namespace pimc;

namespace {

std::string vref(int factor) { return "v[i][" + std::to_string(factor) + "]"; }
std::string aref(int depth) { return "a" + std::to_string(depth) + "[i]"; }

// Emits the value T of the prefix-tree node at depth d whose monomials are M[r0..r1) (all share
// their first d factors) into a<d>, following gen_tree_node: the node's own coefficient (a monomial
// of exactly d factors, first in lexicographic order) starts the sum, then each child j adds
// v_j T(child), a leaf child with its constant directly.
void emit_node(FILE* o, const std::vector<GenMono>& M, size_t r0, size_t r1, size_t d, const std::string& ind) {
    std::string init;                             // the node's coefficient, if it has one
    if (M[r0].f.size() == d) {
        char buf[64];
        std::snprintf(buf, sizeof(buf), "%a", M[r0].c);
        init = buf;
        ++r0;
    }
    bool first = true;
    for (size_t c0 = r0; c0 < r1;) {
        const int j = M[c0].f[d];
        size_t c1 = c0;
        while (c1 < r1 && M[c1].f[d] == j) ++c1;
        std::string t;                            // T(child)
        if (c1 - c0 == 1 && M[c0].f.size() == d + 1) {
            char buf[64];
            std::snprintf(buf, sizeof(buf), "%a", M[c0].c);
            t = buf;
            std::fprintf(o, "%s// monomial %zu\n", ind.c_str(), c0);
        } else {
            emit_node(o, M, c0, c1, d + 1, ind);
            t = aref(int(d + 1));
        }
        std::string rhs;
        if (first && init.empty())
            rhs = vref(j) + " * " + t;
        else
            rhs = "fma(" + vref(j) + ", " + t + ", " + (first ? init : aref(int(d))) + ")";
        std::fprintf(o, "%s#pragma unroll\n%sfor (int i = 0; i < W; ++i) %s = %s;\n", ind.c_str(), ind.c_str(),
                     aref(int(d)).c_str(), rhs.c_str());
        first = false;
        c0 = c1;
    }
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
    for (size_t d = 0; d < maxdeg; ++d) std::fprintf(o, "        double a%zu[W];\n", d);
    const std::string ind = "        ";
    int k_prev = -1;
    bool first_group = true;
    for (size_t r0 = 0; r0 < M.size();) {
        size_t r1 = r0;
        while (r1 < M.size() && M[r1].k == M[r0].k) ++r1;
        if (!first_group)
            for (int k = k_prev - 1; k > M[r0].k; --k)   // a k without monomials
                std::fprintf(o, "#pragma unroll\n        for (int i = 0; i < W; ++i) acc[i] = acc[i] * z[i];\n");
        std::fprintf(o, "        // k = %d\n", M[r0].k);
        emit_node(o, M, r0, r1, 0, ind);
        std::fprintf(o, "#pragma unroll\n        for (int i = 0; i < W; ++i) acc[i] = %s;\n",
                     first_group ? "a0[i]" : "fma(acc[i], z[i], a0[i])");
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
