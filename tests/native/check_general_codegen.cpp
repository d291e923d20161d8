// Host check of the generated general-potential evaluators (pimc_general_gen.hpp for p <= 10 and
// pimc_general_gen_p<p>.hpp above): for every level p the straight-line code with its reused prefix
// products and its constant coefficients must equal the direct evaluation of
// sum_k z^k sum_r c_r prod v_f over the monomials of the symbolic recursion, for random derivative
// values and z. Prints the worst relative error (to the sum of absolute terms) per p.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#define __device__
#define __forceinline__ inline
template <class T> using const_ptr = const T*;
#include "pimc_general.hpp"
namespace pimc { template <int P> struct GenCompiled; }
// Built once per out-of-line level (CHECK_LEVEL = 11..18, that level's header only) and once
// without CHECK_LEVEL for the inline levels 1..10, so that the test can compile the parts in parallel.
#ifdef CHECK_LEVEL
#define CHECK_STR2(x) #x
#define CHECK_STR(x) CHECK_STR2(x)
#define CHECK_HEADER2(p) CHECK_STR(pimc_general_gen_p##p.hpp)
#define CHECK_HEADER(p) CHECK_HEADER2(p)
#include CHECK_HEADER(CHECK_LEVEL)
#else
#include "pimc_general_gen.hpp"
#endif
using namespace pimc;
// one slice through the form the generator wrote for level P
template <int P> void eval_two(double (&v)[2][GenCompiled<P>::J + 1], double (&z)[2], double (&acc)[2]) {
    if constexpr (P <= kGenInlineMaxP) {
        GenCompiled<P>::template eval<2>(v, z, acc);
    } else {
        // the pair form must give the one-slice form's bits for each slice
        double r0, r1;
        GenCompiled<P>::eval2(v[0], v[1], z[0], z[1], r0, r1);
        for (int i = 0; i < 2; ++i) acc[i] = GenCompiled<P>::eval1(v[i], z[i]);
        if (r0 != acc[0] || r1 != acc[1]) acc[0] = acc[1] = 1e300;   // reported as a huge error
    }
}
template <int P> double run(std::mt19937_64& rng) {
    const SymCoefficients C = symbolic_coefficients(P);
    const auto M = canonical_monomials(C);
    if ((int)M.size() != GenCompiled<P>::NREC) { printf("NREC mismatch %d\n", P); return 1e9; }
    std::uniform_real_distribution<double> U(-1.5, 1.5);
    double v[2][GenCompiled<P>::J + 1], z[2], acc[2];
    double worst = 0;
    const int trials = P <= kGenInlineMaxP ? 50 : 4;
    for (int trial = 0; trial < trials; ++trial) {
        for (int i = 0; i < 2; ++i) { for (auto& x : v[i]) x = U(rng); z[i] = U(rng) * U(rng); }
        eval_two<P>(v, z, acc);
        for (int i = 0; i < 2; ++i) {
            // definition: sum_k z^k sum_{mono of k} c_r prod v
            long double ref = 0, scale = 0;
            for (size_t r = 0; r < M.size(); ++r) {
                long double pr = M[r].c;
                for (auto f : M[r].f) pr *= v[i][f];
                ref += pr * std::pow((long double)z[i], M[r].k);
                scale += std::fabs((double)(pr * std::pow((long double)z[i], M[r].k)));
            }
            worst = std::max(worst, (double)(std::fabs(acc[i] - ref) / (scale + 1e-300)));
        }
    }
    return worst;
}
int main() {
    std::mt19937_64 rng(7);
#ifdef CHECK_LEVEL
    printf("%g\n", run<CHECK_LEVEL>(rng));
#else
    static_assert(kGenInlineMaxP == 10, "one call per level below");
    printf("%g %g %g %g %g %g %g %g %g %g\n", run<1>(rng), run<2>(rng), run<3>(rng), run<4>(rng), run<5>(rng),
           run<6>(rng), run<7>(rng), run<8>(rng), run<9>(rng), run<10>(rng));
#endif
}
