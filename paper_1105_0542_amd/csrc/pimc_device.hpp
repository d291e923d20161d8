// Device building blocks of the bisection estimator on CDNA4 (gfx950), wave64.
//
//  * normal_pair: one Philox4x32-10 call (Salmon et al., SC'11) per pair of heap nodes (2j, 2j+1)
//    of a path, counter (j, path_lo32, path_hi32, stream), key (seed_lo32, seed_hi32); two 53-bit
//    uniforms u = ((b >> 11) | 1) 2^-53 (open interval, no ln 0); Box-Muller r = sqrt(-2 ln u1),
//    theta = 2 pi u2; node 2j gets r cos(theta), node 2j+1 gets r sin(theta). ln, sin and cos use
//    the table reductions of pimc_math.hpp with the table in LDS. This replaces the
//    SPRNG uniforms and cosine-only Box-Muller of Sec. 4.1 with a generator that any lane can
//    evaluate for any node without state.
//    Within one wave the node index j and the stream are uniform, and the path words are constant
//    over a path: the first two Philox rounds therefore need no per-node vector multiply (their
//    multiplications are either scalar or hoisted per path), leaving 16 of 20 per-lane 32x32->64
//    products per call; each round's two three-input xors are single v_bitop3 instructions.
//  * Bisection (Sec. 4.1): the point of heap node h (level n = floor(log2 h)+1, offset
//    i = h - 2^(n-1)) is sigma_n z_h + (left + right)/2 with sigma_n^2 = T/2^(n+1), the conditional
//    (Brownian-bridge) width that makes the kinetic term and normalizations integrate out to the
//    free kernel.
//  * Slice action eps W_p (Sec. 2.1, eq.(ansatz) at level p): sum_k z^k P_k(y), y = mid^2,
//    z = dlt^2, Horner in y for each P_k then in z (the quartic evaluators take y = (2 mid)^2 with
//    the coefficient of y^e pre-scaled by 4^-e: exact, and one multiply fewer per slice). Evaluated for W slices at once, coefficient-
//    major, so that every table coefficient (wave-uniform, scalar-loaded) feeds W independent FMA
//    chains.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pimc_math.hpp"
#include "pimc_tables.hpp"

namespace pimc {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;
constexpr int kMaxLevels = 21;          // s <= 20

// Read-only, wave-uniform data (tables, per-level constants) is read through the constant address
// space: the kernels never write it, so the compiler may use scalar loads (one load per wave,
// kept in SGPRs) instead of per-lane vector loads.
template <class T>
using const_ptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ const_ptr<T> as_const(const T* p) {
    return (const_ptr<T>)(p);
}

__device__ __forceinline__ void mulhilo(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
    const uint64_t p = uint64_t(a) * uint64_t(b);
    hi = uint32_t(p >> 32);
    lo = uint32_t(p);
}

// Per-path Philox state that does not depend on the node: results of round 1's path-dependent
// product and round 2's product of a path-only word.
struct PathRng {
    uint32_t x1;        // round-1 output word 1  = lo(M1 * path_hi)
    uint32_t r2hi;      // round-2 hi(M0 * x0), x0 = hi(M1*path_hi) ^ path_lo ^ k0
    uint32_t r2lo;      // round-2 lo(M0 * x0)
};

struct RngKey {
    uint32_t seed_lo, seed_hi, stream;
};

__device__ __forceinline__ PathRng path_rng(const RngKey& key, uint64_t path) {
    const uint32_t plo = uint32_t(path), phi = uint32_t(path >> 32);
    uint32_t h1, l1;
    mulhilo(kPhiloxM1, phi, h1, l1);
    const uint32_t x0 = h1 ^ plo ^ key.seed_lo;            // round 1, key index 0
    PathRng r;
    r.x1 = l1;
    mulhilo(kPhiloxM0, x0, r.r2hi, r.r2lo);                // round 2 product of word 0
    return r;
}

// Philox4x32-10 of counter (j, path_lo, path_hi, stream) -> 4 words.
__device__ __forceinline__ void philox_node_pair(const RngKey& key, const PathRng& pr, uint32_t j,
                                                 uint32_t& o0, uint32_t& o1, uint32_t& o2, uint32_t& o3) {
    uint32_t k0 = key.seed_lo, k1 = key.seed_hi;
    // round 1: word 0 product hi/lo(M0 * j) is wave-uniform; the path product is in pr
    uint32_t h0, l0;
    mulhilo(kPhiloxM0, j, h0, l0);
    const uint32_t x2 = h0 ^ key.stream ^ k1;
    const uint32_t x3 = l0;
    // round 2
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    uint32_t h1, l1;
    mulhilo(kPhiloxM1, x2, h1, l1);                        // wave-uniform product
    uint32_t c0 = h1 ^ pr.x1 ^ k0;
    uint32_t c1 = l1;
    uint32_t c2 = pr.r2hi ^ x3 ^ k1;
    uint32_t c3 = pr.r2lo;
#pragma unroll
    for (int r = 2; r < 10; ++r) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
        uint32_t a_hi, a_lo, b_hi, b_lo;
        mulhilo(kPhiloxM0, c0, a_hi, a_lo);
        mulhilo(kPhiloxM1, c2, b_hi, b_lo);
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(b_hi, c1, k0, 0x96);   // b_hi ^ c1 ^ k0
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(a_hi, c3, k1, 0x96);   // a_hi ^ c3 ^ k1
        c0 = n0;
        c1 = b_lo;
        c2 = n2;
        c3 = a_lo;
    }
    o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}

// Standard normals of heap nodes 2j (even) and 2j+1 (odd); bm: the Box-Muller table (LDS).
__device__ __forceinline__ void normal_pair(const RngKey& key, const PathRng& pr, uint32_t j, const double* bm,
                                            double& z_even, double& z_odd) {
    uint32_t o0, o1, o2, o3;
    philox_node_pair(key, pr, j, o0, o1, o2, o3);
    const double r = sqrt_pos(neg2_log_u53(o0, o1, bm));
    double sn, cs;
    sincos_2pi_u53(o2, o3, bm, sn, cs);
    z_even = r * cs;
    z_odd = r * sn;
}

// Copy the Box-Muller table into LDS: every thread of the workgroup (nthreads of them) takes part;
// a barrier must follow before the first normal is drawn.
__device__ __forceinline__ void load_bm_table(double* lds, int nthreads) {
    for (int i = threadIdx.x; i < kBoxMullerTable; i += nthreads) lds[i] = kBMTable[i];
}

// Normal sources of the bisection walker: pair(j, z_even, z_odd) gives the normals of heap nodes
// 2j and 2j+1 (node 0 does not exist; its value is ignored).
struct PhiloxSource {
    RngKey key;
    PathRng pr;
    const double* bm;
    __device__ __forceinline__ void pair(uint32_t j, double& ze, double& zo) const { normal_pair(key, pr, j, bm, ze, zo); }
};

// Normals held in device memory, feature-major: node h of path `path` at z[(h-1)*ld + path].
struct MemorySource {
    const double* z;
    uint64_t ld;
    uint64_t path;
    __device__ __forceinline__ void pair(uint32_t j, double& ze, double& zo) const {
        ze = j ? z[uint64_t(2 * j - 1) * ld + path] : 0.0;
        zo = z[uint64_t(2 * j) * ld + path];
    }
};

// ---------------------------------------------------------------------------------------------
// Slice evaluators. eval<W>(level, qa, qb, S) adds eps_level W_p of the slices (qa[i], qb[i]) to S
// one at a time in index order, so a level action is always the left-to-right sum of its slices
// whatever the batching (level n of an s-run is then bitwise the n-run).

// Anharmonic oscillator (even, degree <= 4) at compile-time level P, FP64.
template <int P>
struct QuarticEval64 {
    using Shape = QuarticShape<P>;
    const double* __restrict__ tab;   // level-major, Shape::E doubles per level
    // Hide the table address from loop-invariant code motion: coefficients are then re-read from
    // the scalar cache where they are used instead of being hoisted (and spilled) across the path.
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab)); }
    template <int W>
    __device__ __forceinline__ void eval(int level, const double (&qa)[W], const double (&qb)[W], double& S) const {
        const_ptr<double> t = as_const(tab) + level * Shape::E;
        double y[W], z[W], acc[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const double sum = qa[i] + qb[i];           // 2 mid: the table is scaled for (2 mid)^2
            const double dl = qb[i] - qa[i];
            y[i] = sum * sum;
            z[i] = dl * dl;
        }
#pragma unroll
        for (int k = Shape::K - 1; k >= 0; --k) {
            // one P_k's coefficients at a time in scalar registers (see launder())
            asm volatile("" : "+s"(t));
            double v[W];
            const double c0 = t[Shape::off(k)];
#pragma unroll
            for (int i = 0; i < W; ++i) v[i] = c0;
#pragma unroll
            for (int e = 1; e <= Shape::dy(k); ++e) {
                const double c = t[Shape::off(k) + e];
#pragma unroll
                for (int i = 0; i < W; ++i) v[i] = fma(v[i], y[i], c);
            }
#pragma unroll
            for (int i = 0; i < W; ++i) acc[i] = (k == Shape::K - 1) ? v[i] : fma(acc[i], z[i], v[i]);
        }
#pragma unroll
        for (int i = 0; i < W; ++i) S += acc[i];
    }
};

// Same, with the polynomials in FP32 (table rounded to FP32, tiny entries flushed on the host);
// mid-point and deviation are formed in FP64 and rounded, every slice value is widened to FP64
// before it is added.
template <int P>
struct QuarticEval32 {
    using Shape = QuarticShape<P>;
    const float* __restrict__ tab;
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab)); }
    template <int W>
    __device__ __forceinline__ void eval(int level, const double (&qa)[W], const double (&qb)[W], double& S) const {
        const const_ptr<float> t = as_const(tab) + level * Shape::E;
        float y[W], z[W], acc[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const float sum = float(qa[i] + qb[i]);     // 2 mid: the table is scaled for (2 mid)^2
            const float dl = float(qb[i] - qa[i]);
            y[i] = sum * sum;
            z[i] = dl * dl;
        }
#pragma unroll
        for (int k = Shape::K - 1; k >= 0; --k) {
            float v[W];
            const float c0 = t[Shape::off(k)];
#pragma unroll
            for (int i = 0; i < W; ++i) v[i] = c0;
#pragma unroll
            for (int e = 1; e <= Shape::dy(k); ++e) {
                const float c = t[Shape::off(k) + e];
#pragma unroll
                for (int i = 0; i < W; ++i) v[i] = fmaf(v[i], y[i], c);
            }
#pragma unroll
            for (int i = 0; i < W; ++i) acc[i] = (k == Shape::K - 1) ? v[i] : fmaf(acc[i], z[i], v[i]);
        }
#pragma unroll
        for (int i = 0; i < W; ++i) S += double(acc[i]);
    }
};

// The modified Poeschl-Teller potential -lambda/cosh^2(alpha x): runtime shape in
// u = tanh^2(alpha mid) (the coefficients of eq.(1D-MPTansatz) as polynomials in tanh^2).
struct TanhEval64 {
    const double* __restrict__ tab;
    const int* __restrict__ deg;      // device, K entries
    int K;
    int stride;
    double alpha;
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab)); }
    template <int W>
    __device__ __forceinline__ void eval(int level, const double (&qa)[W], const double (&qb)[W], double& S) const {
        const const_ptr<double> t = as_const(tab) + level * stride;
        double u[W], z[W], acc[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const double mid = 0.5 * (qa[i] + qb[i]);
            const double dl = qb[i] - qa[i];
            const double y = tanh_fp64(alpha * mid);
            u[i] = y * y;
            z[i] = dl * dl;
            acc[i] = 0.0;
        }
        int off = stride;
        for (int k = K - 1; k >= 0; --k) {
            const int d = as_const(deg)[k];
            off -= d + 1;
            double v[W];
            const double c0 = t[off];
#pragma unroll
            for (int i = 0; i < W; ++i) v[i] = c0;
            for (int e = 1; e <= d; ++e) {
                const double c = t[off + e];
#pragma unroll
                for (int i = 0; i < W; ++i) v[i] = fma(v[i], u[i], c);
            }
#pragma unroll
            for (int i = 0; i < W; ++i) acc[i] = (k == K - 1) ? v[i] : fma(acc[i], z[i], v[i]);
        }
#pragma unroll
        for (int i = 0; i < W; ++i) S += acc[i];
    }
};

// v = c[0] u^D + c[1] u^(D-1) + ... + c[D], by Horner from the leading coefficient.
template <int W, int D>
__device__ __forceinline__ void horner_group(const_ptr<double> c, const double (&u)[W], double (&v)[W]) {
    const double c0 = c[0];
#pragma unroll
    for (int i = 0; i < W; ++i) v[i] = c0;
#pragma unroll
    for (int e = 1; e <= D; ++e) {
        const double ce = c[e];
#pragma unroll
        for (int i = 0; i < W; ++i) v[i] = fma(v[i], u[i], ce);
    }
}

// The same tables with their shape fixed at compile time: the Poeschl-Teller fold has K = P groups
// P_k(u) of degree P each (P(P+1) coefficients per level), so each group's Horner scheme unrolls and
// its coefficients are scalar-loaded where they are used. Same operations in the same order as
// TanhEval64 (bitwise equal results).
template <int P>
struct TanhEvalP {
    static constexpr int E = P * (P + 1);
    const double* __restrict__ tab;
    double alpha;
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab)); }
    template <int W>
    __device__ __forceinline__ void eval(int level, const double (&qa)[W], const double (&qb)[W], double& S) const {
        const_ptr<double> t = as_const(tab) + level * E;
        double u[W], z[W], acc[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const double mid = 0.5 * (qa[i] + qb[i]);
            const double dl = qb[i] - qa[i];
            const double y = tanh_fp64(alpha * mid);
            u[i] = y * y;
            z[i] = dl * dl;
            acc[i] = 0.0;
        }
        // group P-1, then the others in a loop that is not unrolled: each group's P+1 coefficients
        // are loaded in its own iteration, so a level's table (P(P+1) doubles) is never held in
        // scalar registers (unrolled, the compiler loaded it whole and spilled it into VGPR lanes)
        horner_group<W, P>(t + (P - 1) * (P + 1), u, acc);
#pragma unroll 1
        for (int k = P - 2; k >= 0; --k) {
            double v[W];
            horner_group<W, P>(t + k * (P + 1), u, v);
#pragma unroll
            for (int i = 0; i < W; ++i) acc[i] = fma(acc[i], z[i], v[i]);
        }
#pragma unroll
        for (int i = 0; i < W; ++i) S += acc[i];
    }
};

// General-potential mode: the derivative tables of V = poly + sum A/cosh^2(a x) + sum B exp(-b x^2)
// (see pimc_general.hpp); the slice evaluators themselves are generated per p at build time
// (pimc_general_device.hpp).
struct GenTables {
    const double* dpoly;                         // (J+1) x 9: coefficients of V^(j) of the polynomial part
    const double* dsech;                         // per term (J+1) x (J+1): A a^j R_j(t)
    int n_sech;
    int n_gauss;
    double sech_a[kGenMaxTerms];
    double gB[kGenMaxTerms], gb[kGenMaxTerms], gsb[kGenMaxTerms];
};

// Any polynomial potential: runtime shape (K polynomials, degrees deg[k]) in u = x^2 (EVEN) or x.
template <bool EVEN>
struct GenericEval64 {
    const double* __restrict__ tab;
    const int* __restrict__ deg;      // device, K entries
    int K;
    int stride;
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab)); }
    template <int W>
    __device__ __forceinline__ void eval(int level, const double (&qa)[W], const double (&qb)[W], double& S) const {
        const const_ptr<double> t = as_const(tab) + level * stride;
        double u[W], z[W], acc[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const double mid = 0.5 * (qa[i] + qb[i]);
            const double dl = qb[i] - qa[i];
            u[i] = EVEN ? mid * mid : mid;
            z[i] = dl * dl;
            acc[i] = 0.0;
        }
        // P_k stored consecutively for k = 0..K-1; walk them from the last one.
        int off = stride;
        for (int k = K - 1; k >= 0; --k) {
            const int d = as_const(deg)[k];
            off -= d + 1;
            double v[W];
            const double c0 = t[off];
#pragma unroll
            for (int i = 0; i < W; ++i) v[i] = c0;
            for (int e = 1; e <= d; ++e) {
                const double c = t[off + e];
#pragma unroll
                for (int i = 0; i < W; ++i) v[i] = fma(v[i], u[i], c);
            }
#pragma unroll
            for (int i = 0; i < W; ++i) acc[i] = (k == K - 1) ? v[i] : fma(acc[i], z[i], v[i]);
        }
#pragma unroll
        for (int i = 0; i < W; ++i) S += acc[i];
    }
    // The W slice values separately (no accumulation): out[i] = sum_k z_i^k P_k(u_i).
    template <int W>
    __device__ __forceinline__ void values(int level, const double (&qa)[W], const double (&qb)[W], double (&out)[W]) const {
        const const_ptr<double> t = as_const(tab) + level * stride;
        double u[W], z[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const double mid = 0.5 * (qa[i] + qb[i]);
            const double dl = qb[i] - qa[i];
            u[i] = EVEN ? mid * mid : mid;
            z[i] = dl * dl;
            out[i] = 0.0;
        }
        int off = stride;
        for (int k = K - 1; k >= 0; --k) {
            const int d = as_const(deg)[k];
            off -= d + 1;
            double v[W];
            const double c0 = t[off];
#pragma unroll
            for (int i = 0; i < W; ++i) v[i] = c0;
            for (int e = 1; e <= d; ++e) {
                const double c = t[off + e];
#pragma unroll
                for (int i = 0; i < W; ++i) v[i] = fma(v[i], u[i], c);
            }
#pragma unroll
            for (int i = 0; i < W; ++i) out[i] = (k == K - 1) ? v[i] : fma(out[i], z[i], v[i]);
        }
    }
};

// ---------------------------------------------------------------------------------------------
// Wave64 sum of a double (butterfly over the 64 lanes; every lane ends with the total, added in
// the same fixed order for any launch).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace pimc
