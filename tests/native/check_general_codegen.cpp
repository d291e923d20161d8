// Host check of the generated general-potential evaluators (pimc_general_gen.hpp): for every level p
// the straight-line code with its reused prefix products and its constant coefficients must equal the
// direct evaluation of sum_k z^k sum_r c_r prod v_f over the monomials of the symbolic recursion, for
// random derivative values and z. Prints the worst relative error (to the sum of absolute terms) per p.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#define __device__
#define __forceinline__ inline
template <class T> using const_ptr = const T*;
#include "pimc_general.hpp"
namespace pimc { template <int P> struct GenCompiled; }
#include "pimc_general_gen.hpp"
using namespace pimc;
template <int P> double run(std::mt19937_64& rng) {
    const SymCoefficients C = symbolic_coefficients(P);
    const auto M = canonical_monomials(C);
    if ((int)M.size() != GenCompiled<P>::NREC) { printf("NREC mismatch %d\n", P); return 1e9; }
    std::uniform_real_distribution<double> U(-1.5, 1.5);
    double v[2][GenCompiled<P>::J + 1], z[2], acc[2];
    double worst = 0;
    for (int trial = 0; trial < 50; ++trial) {
        for (int i = 0; i < 2; ++i) { for (auto& x : v[i]) x = U(rng); z[i] = U(rng) * U(rng); }
        GenCompiled<P>::template eval<2>(v, z, acc);
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
    static_assert(kGenMaxP == 10, "one call per level below");
    printf("%g %g %g %g %g %g %g %g %g %g\n", run<1>(rng), run<2>(rng), run<3>(rng), run<4>(rng), run<5>(rng),
           run<6>(rng), run<7>(rng), run<8>(rng), run<9>(rng), run<10>(rng));
}
