// Build-time generator of the general-potential slice evaluators (the counterpart of the generated
// Wp() functions of Sec. 3.1/3.2): for every level p = 1..kGenMaxP it runs eq.(1Drec)/(diagonal) on
// polynomials in the derivative symbols v_j = V^(j) (pimc_general.hpp), takes the monomials in
// canonical order and writes straight-line device code that sums them from the scaled derivative
// values held in registers, per power of zt = dlt^2 / (4 eps) by a multivariate Horner scheme over the
// prefix tree of their factor lists, and then by the Horner scheme in zt:
//
//   template <> struct GenCompiled<p> {
//       static constexpr int J, NREC;        // highest derivative, number of monomials
//       template <int W> static void eval(vt[W][J+1], zt[W], acc[W]);    // p <= kGenInlineMaxP
//       static double eval1(vt[J+1], zt);                                 // p > kGenInlineMaxP
//       static void eval2(vt0, vt1, zt0, zt1, r0, r1);                    // (two slices)
//   };
//
// Levels up to kGenInlineMaxP go into one header with loops over the W slices; each higher level into
// a header of its own, pimc_general_gen_p<p>.hpp, as loop-free code for one and for two slices
// (thousands of one-statement loops make the compiler's loop passes take minutes on these sizes).
// The two-slice form lets every instruction of the long code serve two slices (the code is
// streamed through the instruction cache once per call; its literal coefficients are shared).
//
// In this dimensionless form (pimc_general.hpp: level_scales) the coefficients do not depend on the
// bisection level, so they are written into the code as exact hexadecimal constants. The monomials of
// one power of zt, in lexicographic order of their factor lists, are the depth-first walk of a prefix
// tree; a node's value is its own coefficient plus v_j times the value of each child j, so every tree
// edge costs one fma and only one partial sum per depth (a0, a1, ...) is live.
// Usage: pimc_gen_codegen <output header>.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "pimc_general.hpp"

using namespace pimc;

namespace {

// Statement form: with loops over the W slices (inline evaluators), or written out for g_w slices
// whose variables carry the slice number (out-of-line evaluators). Coefficients are literals.
bool g_scalar = false;
int g_w = 1;

// '@' stands for the slice number in the statement templates of the out-of-line form
std::string vref(int factor) { return (g_scalar ? "v@[" : "v[i][") + std::to_string(factor) + "]"; }
std::string aref(int depth) { return "a" + std::to_string(depth) + (g_scalar ? "_@" : "[i]"); }

std::string coef(double c) {
    char buf[64];
    std::snprintf(buf, sizeof(buf), "%a", c);
    return buf;
}

// One statement `lhs = rhs;` over the slices.
void emit_stmt(FILE* o, const std::string& ind, const std::string& lhs, const std::string& rhs) {
    if (g_scalar) {
        for (int i = 0; i < g_w; ++i) {
            std::string st = lhs + " = " + rhs + ";";
            for (size_t q = st.find('@'); q != std::string::npos; q = st.find('@', q)) st.replace(q, 1, std::to_string(i));
            std::fprintf(o, "%s%s\n", ind.c_str(), st.c_str());
        }
    } else {
        std::fprintf(o, "%s#pragma unroll\n%sfor (int i = 0; i < W; ++i) %s = %s;\n", ind.c_str(), ind.c_str(),
                     lhs.c_str(), rhs.c_str());
    }
}

// Emits the value T of the prefix-tree node at depth d whose monomials are M[r0..r1) (all share
// their first d factors) into a<d>, following gen_tree_node: the node's own coefficient (a monomial
// of exactly d factors, first in lexicographic order) starts the sum, then each child j adds
// v_j T(child), a leaf child with its constant directly.
void emit_node(FILE* o, const std::vector<GenMono>& M, size_t r0, size_t r1, size_t d, const std::string& ind) {
    std::string init;                             // the node's coefficient, if it has one
    if (M[r0].f.size() == d) {
        init = coef(M[r0].c);
        ++r0;
    }
    bool first = true;
    for (size_t c0 = r0; c0 < r1;) {
        const int j = M[c0].f[d];
        size_t c1 = c0;
        while (c1 < r1 && M[c1].f[d] == j) ++c1;
        std::string t;                            // T(child)
        if (c1 - c0 == 1 && M[c0].f.size() == d + 1) {
            t = coef(M[c0].c);
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
        emit_stmt(o, ind, aref(int(d)), rhs);
        first = false;
        c0 = c1;
    }
}

// The body of one evaluator: per power k of zt (highest first) the prefix-tree sum, Horner in zt.
void emit_body(FILE* o, const std::vector<GenMono>& M) {
    const std::string acc = g_scalar ? "acc@" : "acc[i]";
    const std::string z = g_scalar ? "z@" : "z[i]";
    const std::string ind = "        ";
    int k_prev = -1;
    bool first_group = true;
    for (size_t r0 = 0; r0 < M.size();) {
        size_t r1 = r0;
        while (r1 < M.size() && M[r1].k == M[r0].k) ++r1;
        if (!first_group)
            for (int k = k_prev - 1; k > M[r0].k; --k)   // a k without monomials
                emit_stmt(o, ind, acc, acc + " * " + z);
        std::fprintf(o, "        // k = %d\n", M[r0].k);
        emit_node(o, M, r0, r1, 0, ind);
        emit_stmt(o, ind, acc, first_group ? aref(0) : "fma(" + acc + ", " + z + ", " + aref(0) + ")");
        first_group = false;
        k_prev = M[r0].k;
        r0 = r1;
    }
    for (int k = k_prev - 1; k >= 0; --k) emit_stmt(o, ind, acc, acc + " * " + z);
}

void emit_level(FILE* o, int p) {
    const SymCoefficients C = symbolic_coefficients(p);
    const std::vector<GenMono> M = canonical_monomials(C);
    size_t maxdeg = 1;
    for (const GenMono& g : M) maxdeg = std::max(maxdeg, g.f.size());
    g_scalar = p > kGenInlineMaxP;
    if (!g_scalar) {
        std::fprintf(o, "template <>\nstruct GenCompiled<%d> {\n", p);
        std::fprintf(o, "    static constexpr int J = %d;\n    static constexpr int NREC = %zu;\n", C.J, M.size());
        std::fprintf(o, "    template <int W>\n");
        std::fprintf(o, "    __device__ __forceinline__ static void eval(const double (&v)[W][J + 1], const double (&z)[W],\n"
                        "                                                double (&acc)[W]) {\n");
        for (size_t d = 0; d < maxdeg; ++d) std::fprintf(o, "        double a%zu[W];\n", d);
        emit_body(o, M);
        std::fprintf(o, "    }\n};\n\n");
        return;
    }
    // out of line: eval1 (one slice) and eval2 (two slices, each formed exactly as eval1 forms it)
    std::string body[2];
    for (int w = 1; w <= 2; ++w) {
        g_w = w;
        char* buf = nullptr;
        size_t len = 0;
        FILE* mem = open_memstream(&buf, &len);
        for (size_t d = 0; d < maxdeg; ++d)
            for (int i = 0; i < w; ++i) std::fprintf(mem, "        double a%zu_%d;\n", d, i);
        for (int i = 0; i < w; ++i) std::fprintf(mem, "        double acc%d;\n", i);
        emit_body(mem, M);
        std::fclose(mem);
        body[w - 1].assign(buf, len);
        std::free(buf);
    }
    std::fprintf(o, "template <>\nstruct GenCompiled<%d> {\n", p);
    std::fprintf(o, "    static constexpr int J = %d;\n    static constexpr int NREC = %zu;\n", C.J, M.size());
    std::fprintf(o, "    __device__ __forceinline__ static double eval1(const double (&v0)[J + 1], double z0) {\n");
    std::fputs(body[0].c_str(), o);
    std::fprintf(o, "        return acc0;\n    }\n");
    std::fprintf(o, "    __device__ __forceinline__ static void eval2(const double (&v0)[J + 1], const double (&v1)[J + 1],\n"
                    "                                                 double z0, double z1, double& r0, double& r1) {\n");
    std::fputs(body[1].c_str(), o);
    std::fprintf(o, "        r0 = acc0;\n        r1 = acc1;\n    }\n};\n\n");
}

bool write_header(const std::string& path, int p0, int p1) {
    FILE* o = std::fopen(path.c_str(), "w");
    if (!o) {
        std::perror(path.c_str());
        return false;
    }
    std::fprintf(o, "// Generated by pimc_gen_codegen from the derivative-symbol recursion; not edited by hand.\n");
    std::fprintf(o, "#pragma once\n\nnamespace pimc {\n\n");
    for (int p = p0; p <= p1; ++p) emit_level(o, p);
    std::fprintf(o, "}  // namespace pimc\n");
    return std::fclose(o) == 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 3) {
        std::fprintf(stderr, "usage: %s <header of levels 1..%d> <directory of the per-level headers>\n", argv[0],
                     kGenInlineMaxP);
        return 2;
    }
    if (!write_header(argv[1], 1, kGenInlineMaxP)) return 1;
    for (int p = kGenInlineMaxP + 1; p <= kGenMaxP; ++p)
        if (!write_header(std::string(argv[2]) + "/pimc_general_gen_p" + std::to_string(p) + ".hpp", p, p)) return 1;
    return 0;
}
