// Command-line front end of libpimc.so with the argument order of the paper's program (Sec. 4.2):
// propagation time T, endpoints a and b, largest bisection level s, number of Monte Carlo samples,
// seed, then the potential's coefficients V(q) = sum_j coef_j q^j. The effective-action level p,
// the mass and the precision are options (the paper fixes p at compile time). Prints the amplitude
// and its Monte Carlo error for every level n = 0..s; level 0 is analytic and prints error 0.
// With --dim d (Sec. 2.2, several coordinates) the endpoints are d coordinates each and the
// coefficients those of a rotation-invariant V(q) = sum_n coef_n (q.q)^n (the 2D anharmonic
// oscillator of Sec. 3.3 is --dim 2 with coefficients 0 A/2 g/24).
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "pimc.h"

namespace {

void usage(const char* prog) {
    std::printf(
        "usage: %s [options] T a b s Nmc seed coef0 [coef1 ... coef8]\n"
        "  Estimates the imaginary-time amplitude A_N^(p)(a,b;T) for N = 2^n, n = 0..s, of a particle in\n"
        "  V(q) = coef0 + coef1 q + ... (hbar = 1) from Nmc bisection paths with the level-p effective action.\n"
        "options:\n"
        "  -p P         effective-action level, 1..%d (default 18)\n"
        "  -m M         mass (default 1)\n"
        "  --stream S   Philox stream (default 0)\n"
        "  --fp32       FP32 slice polynomials (FP64 sums)\n"
        "  --level-s    estimate level s only (default: every level from the same paths)\n"
        "  --device D   HIP device (default 0)\n"
        "  --dim D      D coordinates (2..%d): arguments T a_1..a_D b_1..b_D s Nmc seed coef0 [coef1 [coef2]]\n"
        "               with V(q) = coef0 + coef1 (q.q) + coef2 (q.q)^2\n"
        "output: one line per level: n N amplitude error\n",
        prog, PIMC_MAX_P, PIMC_MAX_DIM);
}

bool parse_double(const char* s, double& v) {
    char* end = nullptr;
    errno = 0;
    v = std::strtod(s, &end);
    return errno == 0 && end && *end == '\0' && end != s;
}

bool parse_u64(const char* s, unsigned long long& v) {
    char* end = nullptr;
    errno = 0;
    v = std::strtoull(s, &end, 0);
    return errno == 0 && end && *end == '\0' && end != s && s[0] != '-';
}

// Several coordinates: T a_1..a_d b_1..b_d s Nmc seed coef0 [coef1 [coef2]], V = sum_n coef_n (q.q)^n.
int run_radial(const std::vector<const char*>& pos, int dim, int p, double m, uint32_t stream, uint32_t flags,
               int device) {
    const size_t fixed = 1 + 2 * size_t(dim) + 3;
    if (pos.size() < fixed + 1 || pos.size() > fixed + PIMC_MAX_RADIAL_DEGREE + 1) {
        std::fprintf(stderr, "expected T, %d + %d endpoint coordinates, s Nmc seed and 1..%d coefficients\n", dim, dim,
                     PIMC_MAX_RADIAL_DEGREE + 1);
        return 2;
    }
    double T;
    double a[PIMC_MAX_DIM] = {0.0}, b[PIMC_MAX_DIM] = {0.0};
    unsigned long long s, nmc, seed;
    bool ok = parse_double(pos[0], T);
    for (int c = 0; c < dim; ++c) ok = ok && parse_double(pos[1 + c], a[c]) && parse_double(pos[1 + dim + c], b[c]);
    const size_t k = 1 + 2 * size_t(dim);
    ok = ok && parse_u64(pos[k], s) && parse_u64(pos[k + 1], nmc) && parse_u64(pos[k + 2], seed) && s <= PIMC_MAX_S;
    if (!ok) {
        std::fprintf(stderr, "cannot parse T, the endpoints, s, Nmc or seed\n");
        return 2;
    }
    pimc_radial_potential V;
    std::memset(&V, 0, sizeof(V));
    V.dim = dim;
    V.degree = int(pos.size() - fixed) - 1;
    for (size_t j = fixed; j < pos.size(); ++j)
        if (!parse_double(pos[j], V.coef[j - fixed])) { std::fprintf(stderr, "bad coefficient %s\n", pos[j]); return 2; }
    pimc_ctx* ctx = nullptr;
    int st = pimc_create(&ctx, device, nullptr);
    if (st != PIMC_OK) {
        std::fprintf(stderr, "pimc_create: %s\n", pimc_last_error(nullptr));
        return 1;
    }
    std::vector<pimc_level_result> out(s + 1);
    st = pimc_amplitude_radial(ctx, &V, m, a, b, T, 1u << s, p, nmc, seed, stream, flags, out.data());
    if (st < 0) {
        std::fprintf(stderr, "pimc_amplitude_radial: %s\n", pimc_last_error(ctx));
        pimc_destroy(ctx);
        return st == PIMC_EINVAL ? 2 : 1;
    }
    for (unsigned long long n = 0; n <= s; ++n) {
        if (out[n].n == 0) continue;
        std::printf("%llu %llu %.17g %.17g\n", n, 1ull << n, out[n].amp, out[n].err);
    }
    if (st == PIMC_WNONFINITE) std::fprintf(stderr, "warning: %s\n", pimc_strerror(st));
    pimc_destroy(ctx);
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) {
        usage(argv[0]);
        return 0;
    }
    int p = 18, device = 0, dim = 0;
    double m = 1.0;
    unsigned long long stream = 0;
    uint32_t flags = PIMC_HIERARCHY;
    std::vector<const char*> pos;
    for (int i = 1; i < argc; ++i) {
        const std::string a = argv[i];
        auto next = [&](const char* what) -> const char* {
            if (i + 1 >= argc) {
                std::fprintf(stderr, "%s needs a value\n", what);
                std::exit(2);
            }
            return argv[++i];
        };
        if (a == "-h" || a == "--help") {
            usage(argv[0]);
            return 0;
        } else if (a == "-p") {
            p = std::atoi(next("-p"));
        } else if (a == "-m") {
            if (!parse_double(next("-m"), m)) { std::fprintf(stderr, "bad mass\n"); return 2; }
        } else if (a == "--stream") {
            if (!parse_u64(next("--stream"), stream) || stream > 0xffffffffull) { std::fprintf(stderr, "bad stream\n"); return 2; }
        } else if (a == "--dim") {
            dim = std::atoi(next("--dim"));
            if (dim < 2 || dim > PIMC_MAX_DIM) { std::fprintf(stderr, "--dim needs 2..%d\n", PIMC_MAX_DIM); return 2; }
        } else if (a == "--device") {
            device = std::atoi(next("--device"));
        } else if (a == "--fp32") {
            flags |= PIMC_FP32_POLY;
        } else if (a == "--level-s") {
            flags &= ~uint32_t(PIMC_HIERARCHY);
        } else {
            pos.push_back(argv[i]);
        }
    }
    if (dim > 0) return run_radial(pos, dim, p, m, uint32_t(stream), flags, device);
    if (pos.size() < 7 || pos.size() > 6 + PIMC_MAX_DEGREE + 1) {
        std::fprintf(stderr, "expected T a b s Nmc seed and 1..%d coefficients\n", PIMC_MAX_DEGREE + 1);
        return 2;
    }
    double T, a, b;
    unsigned long long s, nmc, seed;
    if (!parse_double(pos[0], T) || !parse_double(pos[1], a) || !parse_double(pos[2], b) || !parse_u64(pos[3], s) ||
        !parse_u64(pos[4], nmc) || !parse_u64(pos[5], seed) || s > PIMC_MAX_S) {
        std::fprintf(stderr, "cannot parse T a b s Nmc seed\n");
        return 2;
    }
    pimc_potential V;
    std::memset(&V, 0, sizeof(V));
    V.degree = int(pos.size()) - 7;
    for (size_t j = 6; j < pos.size(); ++j)
        if (!parse_double(pos[j], V.coef[j - 6])) { std::fprintf(stderr, "bad coefficient %s\n", pos[j]); return 2; }
    const uint32_t N = 1u << s;
    int st = pimc_check_problem(&V, m, a, b, T, N, p, nmc);
    if (st != PIMC_OK) {
        std::fprintf(stderr, "invalid problem: %s\n", pimc_last_error(nullptr));
        return 2;
    }
    pimc_ctx* ctx = nullptr;
    st = pimc_create(&ctx, device, nullptr);
    if (st != PIMC_OK) {
        std::fprintf(stderr, "pimc_create: %s\n", pimc_last_error(nullptr));
        return 1;
    }
    std::vector<pimc_level_result> out(s + 1);
    st = pimc_amplitude(ctx, &V, m, a, b, T, N, p, nmc, seed, uint32_t(stream), flags, out.data());
    if (st < 0) {
        std::fprintf(stderr, "pimc_amplitude: %s\n", pimc_last_error(ctx));
        pimc_destroy(ctx);
        return 1;
    }
    for (unsigned long long n = 0; n <= s; ++n) {
        if (out[n].n == 0) continue;
        std::printf("%llu %llu %.17g %.17g\n", n, 1ull << n, out[n].amp, out[n].err);
    }
    if (st == PIMC_WNONFINITE) std::fprintf(stderr, "warning: %s\n", pimc_strerror(st));
    pimc_destroy(ctx);
    return 0;
}
