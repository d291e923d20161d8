// Host check of the FP64 elementary functions of the device code (pimc_math.hpp), compiled for the
// CPU. The hardware reciprocal and reciprocal-square-root estimates are replaced by the exact values
// perturbed by a relative 2^-22 (the estimates are accurate to about 2^-23), so the Newton steps are
// exercised. Prints the worst error in units of the last place (against long double references) of
// tanh_fp64, exp_fp64, -2 ln u, sqrt and (sin, cos)(2 pi u) over their argument ranges (the
// Box-Muller pair with the table of pimc_math.hpp, read from host memory here), with the extreme
// and bucket-boundary uniforms added to the random ones.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#define __device__
#define __forceinline__ inline
static double __builtin_amdgcn_rcp(double x) { return (1.0 / x) * (1.0 + 0x1p-22); }
static double __builtin_amdgcn_rsq(double x) { return (1.0 / std::sqrt(x)) * (1.0 - 0x1p-22); }
#include "pimc_math.hpp"
using namespace pimc;

static double ulp_err(double got, long double ref) {
    if (ref == 0.0L) return got == 0.0 ? 0.0 : 1e300;
    const double r = double(ref);
    const double u = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
    return double(std::fabs((long double)got - ref) / (long double)u);
}

int main() {
    std::mt19937_64 rng(11);
    double w_tanh = 0, w_exp = 0, w_log = 0, w_sqrt = 0, w_sc = 0;
    for (int i = 0; i < 400000; ++i) {
        // tanh over |y| up to 25, log-uniform magnitudes down to 1e-12, both signs
        const double mag = std::pow(10.0, std::uniform_real_distribution<double>(-12.0, 1.4)(rng));
        const double y = (rng() & 1) ? mag : -mag;
        w_tanh = std::max(w_tanh, ulp_err(tanh_fp64(y), std::tanh((long double)y)));
        // exp over [-740, 700]
        const double x = std::uniform_real_distribution<double>(-740.0, 700.0)(rng);
        w_exp = std::max(w_exp, ulp_err(exp_fp64(x), std::exp((long double)x)));
        const double xs = std::uniform_real_distribution<double>(-3.0, 3.0)(rng);
        w_exp = std::max(w_exp, ulp_err(exp_fp64(xs), std::exp((long double)xs)));
        // -2 ln u and (sin, cos)(2 pi u) for u = K 2^-53 from two 32-bit words
        uint64_t bits = rng();
        if (i < 4096) {
            // extremes (u -> 0, u -> 1) and the neighbourhoods of the table's bucket boundaries
            const uint64_t K0 = (i & 1) ? (uint64_t(1) << 53) - 1 - 2 * uint64_t(i) : 1 + 2 * uint64_t(i);
            const uint64_t Kb = ((uint64_t(64 + (i >> 6)) << 46) + (uint64_t(i & 63) - 32)) | 1;   // near c-bucket edges
            const uint64_t K = (i & 2) ? K0 : (Kb >> (i % 7));
            bits = ((K | 1) << 11) | (rng() & 0x7FF);
        }
        const uint32_t lo = uint32_t(bits), hi = uint32_t(bits >> 32);
        const uint64_t K = ((uint64_t(hi) << 32 | lo) >> 11) | 1u;
        const long double u = (long double)K * 0x1p-53L;
        const double L = neg2_log_u53(lo, hi, kBMTable);
        w_log = std::max(w_log, ulp_err(L, -2.0L * std::log(u)));
        w_sqrt = std::max(w_sqrt, ulp_err(sqrt_pos(L), std::sqrt((long double)L)));
        double sn, cs;
        sincos_2pi_u53(lo, hi, kBMTable, sn, cs);
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * u;
        // absolute error in ulps of 1 (the normals use r * sin, r * cos; near zeros relative error is
        // not meaningful)
        w_sc = std::max(w_sc, double(std::fabs((long double)sn - std::sin(a)) / 0x1p-53L));
        w_sc = std::max(w_sc, double(std::fabs((long double)cs - std::cos(a)) / 0x1p-53L));
    }
    std::printf("%g %g %g %g %g\n", w_tanh, w_exp, w_log, w_sqrt, w_sc);
    return 0;
}
