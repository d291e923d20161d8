// FP64 elementary functions for the Box-Muller step, specialized to the arguments it sees, and the
// tanh and exp of the slice evaluators of non-polynomial potentials.
//
// The bisection offsets need r = sqrt(-2 ln u1) and (cos, sin)(2 pi u2) for uniforms u = K 2^-53
// with K odd, 1 <= K < 2^53 (so 2^-53 <= u <= 1 - 2^-53). Knowing the argument ranges removes the
// special-case handling (zero, negative, infinite, denormal inputs, Payne-Hanek reduction) and the
// extra-precision steps of general-purpose library routines; what remains are short polynomials.
// Each routine is written from the mathematics stated next to it, with constants rounded once to
// nearest from their exact values (gen_math_coeffs.py prints them). Their results agree with
// correctly rounded references to a few ulp (checked against the oracle's normals).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pimc {

// 2/(2k+3), k = 0..9: ln m = 2 atanh(s) = 2s + s^3 sum_k 2 s^(2k)/(2k+3), s = (m-1)/(m+1).
// For m in [sqrt(1/2), sqrt(2)), |s| <= 0.1716, s^2 <= 0.0295, and the first omitted term is below
// 2^-55 relative to 2s.
__device__ constexpr double kLogP[10] = {
    0x1.5555555555555p-1, 0x1.999999999999ap-2, 0x1.2492492492492p-2, 0x1.c71c71c71c71cp-3,
    0x1.745d1745d1746p-3, 0x1.3b13b13b13b14p-3, 0x1.1111111111111p-3, 0x1.e1e1e1e1e1e1ep-4,
    0x1.af286bca1af28p-4, 0x1.8618618618618p-4};
// ln 2 = kLn2Hi + kLn2Lo, kLn2Hi with 32 significant bits (E * kLn2Hi exact for |E| < 2^21).
constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;

// Taylor coefficients of sin(2 pi r) / r and cos(2 pi r) in w = r^2 for |r| <= 1/8 (|2 pi r| <=
// pi/4): (-1)^i (2pi)^(2i+1)/(2i+1)!, i = 0..8 and (-1)^i (2pi)^(2i)/(2i)!, i = 0..9; the first
// omitted terms are below 1e-19 and 2e-18 of the leading term.
__device__ constexpr double kSinC[9] = {
    0x1.921fb54442d18p+2, -0x1.4abbce625be53p+5, 0x1.466bc6775aae2p+6, -0x1.32d2cce62bd86p+6,
    0x1.50783487ee782p+5, -0x1.e3074fde8871fp+3, 0x1.e8f434d018d63p+1, -0x1.6fadb9f155744p-1,
    0x1.aaec32af93359p-4};
__device__ constexpr double kCosC[10] = {
    0x1.0000000000000p+0, -0x1.3bd3cc9be45dep+4, 0x1.03c1f081b5ac4p+6, -0x1.55d3c7e3cbffap+6,
    0x1.e1f506891babbp+5, -0x1.a6d1f2a204a8cp+4, 0x1.f9d38a3763cc3p+2, -0x1.b6e24f44b128fp+0,
    0x1.20c62c2f2d7f5p-2, -0x1.2a0c591af8314p-5};

// -2 ln(u), u = K 2^-53, K = (((uint64)hi << 32 | lo) >> 11) | 1.
// K = m 2^e with m in [sqrt(1/2), sqrt(2)) exactly (frexp plus one exact doubling), so
// ln u = ln m + (e - 53) ln 2, and ln m by the atanh series above; s = (m-1)/(m+1) with m-1 exact
// and the quotient from the hardware reciprocal estimate refined by Newton steps.
__device__ __forceinline__ double neg2_log_odd53(uint32_t lo, uint32_t hi) {
    const double Kd = fma(double(hi), 0x1p21, double((lo >> 11) | 1u));   // exact integer < 2^53
    int e;
    double m = frexp(Kd, &e);                       // Kd = m 2^e, m in [1/2, 1)
    if (m < kSqrtHalf) {
        m = m + m;
        e -= 1;
    }
    const double f = m - 1.0;                       // exact
    const double t = 2.0 + f;                       // m + 1
    double r = __builtin_amdgcn_rcp(t);
    r = fma(r, fma(-t, r, 1.0), r);
    r = fma(r, fma(-t, r, 1.0), r);
    double s = f * r;
    s = fma(r, fma(-t, s, f), s);                   // s = f / t
    const double w = s * s;
    double P = kLogP[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) P = fma(P, w, kLogP[k]);
    const double lnm = fma(s * w, P, s + s);
    const double E = double(e - 53);
    const double lnu = fma(E, kLn2Hi, fma(E, kLn2Lo, lnm));
    return -2.0 * lnu;
}

// sqrt(x) for 2^-60 < x < 2^10 (finite, normal, positive): reciprocal square-root estimate, two
// coupled Newton steps on (sqrt x, 1/(2 sqrt x)), then a final correction of sqrt x.
__device__ __forceinline__ double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = 0.5 * y;
    double rr = fma(-g, h, 0.5);
    g = fma(g, rr, g);
    h = fma(h, rr, h);
    rr = fma(-g, h, 0.5);
    g = fma(g, rr, g);
    h = fma(h, rr, h);
    const double d = fma(-g, g, x);
    return fma(h, d, g);
}

// (sin, cos)(2 pi t) for t in [0, 1] a multiple of 2^-53: t = k/4 + r with k = round(4t) and
// |r| <= 1/8 exactly, the polynomials above for 2 pi r, and the quarter-turn identities for k.
__device__ __forceinline__ void sincos_2pi(double t, double& sn, double& cs) {
    const double k = rint(4.0 * t);
    const double r = fma(-0.25, k, t);              // exact
    const double w = r * r;
    double S = kSinC[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) S = fma(S, w, kSinC[i]);
    S = r * S;
    double C = kCosC[9];
#pragma unroll
    for (int i = 8; i >= 0; --i) C = fma(C, w, kCosC[i]);
    const int q = int(k) & 3;
    double a = (q & 1) ? C : S;                     // sin(2 pi r + q pi/2)
    double c = (q & 1) ? S : C;                     // cos(2 pi r + q pi/2)
    sn = (q & 2) ? -a : a;
    cs = ((q + 1) & 2) ? -c : c;
}

// 1/k!, k = 2..13 (each rounded once to nearest): e^r - 1 = r + r^2 sum_k r^(k-2)/k!. For
// |r| <= ln2/2 the first omitted term r^14/14! is below 5e-18 relative to r.
__device__ constexpr double kExpC[12] = {
    0x1.0000000000000p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,
    0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19,
    0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};
constexpr double kLog2e = 0x1.71547652b82fep+0;

// e^r - 1 for |r| <= ln2/2 (plus the rounding of the reduction), without cancellation.
__device__ __forceinline__ double expm1_reduced(double r) {
    double q = kExpC[11];
#pragma unroll
    for (int k = 10; k >= 0; --k) q = fma(q, r, kExpC[k]);
    return fma(r * r, q, r);
}

// Cody-Waite reduction x = n ln2 + r, |r| <= ln2/2 (n * kLn2Hi exact for |n| < 2^21).
__device__ __forceinline__ double reduce_ln2(double x, double& n) {
    n = rint(x * kLog2e);
    const double r = fma(-n, kLn2Hi, x);
    return fma(-n, kLn2Lo, r);
}

// tanh(y) = sign(y) e/(e + 2) with e = e^(2|y|) - 1 = 2^n expm1(r) + (2^n - 1) (both terms exact,
// one rounding, no cancellation for small |y|); the quotient from the hardware reciprocal estimate
// refined by Newton steps. For |y| > 20, 1 - tanh|y| < 2^-56 and the result is 1 (the formula
// itself already rounds to 1 above 55 ln2 / 2 = 19.06). A few ulp.
__device__ __forceinline__ double tanh_fp64(double y) {
    const double a = fabs(y);
    const double ac = a > 20.0 ? 20.0 : a;           // keeps n in range; NaN passes through
    double n;
    const double r = reduce_ln2(ac + ac, n);
    const int ni = int(n);
    const double e = ldexp(expm1_reduced(r), ni) + (ldexp(1.0, ni) - 1.0);
    const double d = e + 2.0;
    double rc = __builtin_amdgcn_rcp(d);
    rc = fma(rc, fma(-d, rc, 1.0), rc);
    rc = fma(rc, fma(-d, rc, 1.0), rc);
    double t = e * rc;
    t = fma(rc, fma(-d, t, e), t);
    t = a > 20.0 ? 1.0 : t;
    return copysign(t, y);
}

// e^x for finite x: 2^n (1 + expm1(r)); 0 below -746 (where e^x rounds to zero), infinity above
// 710. About 1 ulp for normal results.
__device__ __forceinline__ double exp_fp64(double x) {
    double n;
    const double r = reduce_ln2(x < -746.0 ? -746.0 : (x > 710.0 ? 710.0 : x), n);
    const double e = ldexp(1.0 + expm1_reduced(r), int(n));
    return x < -746.0 ? 0.0 : e;
}

}  // namespace pimc
