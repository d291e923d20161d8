// FP64 elementary functions for the Box-Muller step, specialized to the arguments it sees, and the
// tanh and exp of the slice evaluators of non-polynomial potentials.
//
// The bisection offsets need r = sqrt(-2 ln u1) and (cos, sin)(2 pi u2) for uniforms u = K 2^-53
// with K odd, 1 <= K < 2^53 (so 2^-53 <= u <= 1 - 2^-53). Knowing the argument ranges removes the
// special-case handling (zero, negative, infinite, denormal inputs, Payne-Hanek reduction) and the
// extra-precision steps of general-purpose library routines; what remains are table reductions
// and short polynomials. Each routine is written from the mathematics stated next to it, with
// constants rounded once to nearest from their exact values (gen_math_coeffs.py prints them).
// Their results agree with correctly rounded references to a few ulp (host checks against long
// double, and the oracle's normals).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pimc {

// ln 2 = kLn2Hi + kLn2Lo, kLn2Hi with 32 significant bits (E * kLn2Hi exact for |E| < 2^21).
constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;

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

// ---------------------------------------------------------------------------------------------
// Box-Muller with table reductions (the normals of the bisection offsets). Both uniforms of a pair
// come as 53-bit odd integers K = (hi << 21) | ((lo >> 11) | 1), u = K 2^-53 (open interval).
//
// -2 ln u: K = 2^e m with m in [1, 2) (exponent and mantissa read off the bits of K as a double,
// which is exact). The top six mantissa bits select c_i = 1 + (i + 1/2)/64; r = m / c_i - 1 is
// formed as fma(m, 1/c_i rounded, -1) (|r| <= 1/128) and ln m = ln c_i + log1p(r), where ln c_i
// stands for -ln of the rounded reciprocal (so the rounding of 1/c_i cancels exactly). Buckets
// i >= 27 (m > sqrt 2) carry a factor 1/2 into the exponent, so that for u -> 1 the result is
// log1p(r) alone: the last bucket uses c = 2 exactly (reciprocal 1/2, table term 0), where r is
// exact and no cancellation occurs. -2 log1p(r) is its Taylor series to r^8 (first omitted term
// below 2^-56 relative to r). The table stores, per bucket, the rounded 1/c_i and A_i = -2 ln c_i
// (with -ln 2 folded in for i >= 27); -2 ln u = E (-2 ln 2) + A_i - 2 log1p(r) with
// E = e - 53 (+1 for i >= 27), the product with ln 2 split into an exact part and a remainder.
//
// (sin, cos)(2 pi u): 64 u = k + J 2^-47 with k = round(64 u) (mod 64) and |J| <= 2^46 an exact
// integer (no rounding in the reduction); sin and cos of the remainder angle 2 pi J 2^-53
// (|angle| <= pi/64) by their Taylor series to degree 7 and 8, with the powers of 2^-53 folded into
// the coefficients, then the angle-addition formulas with the table's (sin, cos)(2 pi k/64).
//
// The 256 doubles of the table live in LDS (copied once per workgroup); the functions take its
// address. Constants are rounded once to nearest from their exact values (gen_math_coeffs.py).
constexpr int kBoxMullerTable = 256;
constexpr double kM2Ln2Hi = -0x1.62e42fee00000p+0;     // -2 ln 2, high part (32 significant bits)
constexpr double kM2Ln2Lo = -0x1.a39ef35793c76p-32;     // -2 ln 2 - kM2Ln2Hi
__device__ constexpr double kBMLogP[8] = {
    -0x1.0000000000000p+1, 0x1.0000000000000p+0, -0x1.5555555555555p-1, 0x1.0000000000000p-1,
    -0x1.999999999999ap-2, 0x1.5555555555555p-2, -0x1.2492492492492p-2, 0x1.0000000000000p-2};
__device__ constexpr double kBMSin[4] = {
    0x1.921fb54442d18p-51, -0x1.4abbce625be53p-154,
    0x1.466bc6775aae2p-259, -0x1.32d2cce62bd86p-365};
__device__ constexpr double kBMCos[4] = {
    -0x1.3bd3cc9be45dep-102, 0x1.03c1f081b5ac4p-206,
    -0x1.55d3c7e3cbffap-312, 0x1.e1f506891babbp-419};
__device__ constexpr double kBMTable[kBoxMullerTable] = {
    0x1.fc07f01fc07f0p-1, -0x1.fe02a6b106799p-7, 0x1.f44659e4a4271p-1, -0x1.7b91b07d5b126p-5,
    0x1.ecc07b301ecc0p-1, -0x1.39e87b9febd68p-4, 0x1.e573ac901e574p-1, -0x1.b42dd711971b9p-4,
    0x1.de5d6e3f8868ap-1, -0x1.16536eea37ae3p-3, 0x1.d77b654b82c34p-1, -0x1.51b073f06183cp-3,
    0x1.d0cb58f6ec074p-1, -0x1.8c345d6319b23p-3, 0x1.ca4b3055ee191p-1, -0x1.c5e548f5bc743p-3,
    0x1.c3f8f01c3f8f0p-1, -0x1.fec9131dbeabcp-3, 0x1.bdd2b899406f7p-1, -0x1.1b72ad52f67a2p-2,
    0x1.b7d6c3dda338bp-1, -0x1.371fc201e8f75p-2, 0x1.b2036406c80d9p-1, -0x1.526e5e3a1b438p-2,
    0x1.ac5701ac5701bp-1, -0x1.6d60fe719d21bp-2, 0x1.a6d01a6d01a6dp-1, -0x1.87fa06520c911p-2,
    0x1.a16d3f97a4b02p-1, -0x1.a23bc1fe2b561p-2, 0x1.9c2d14ee4a102p-1, -0x1.bc286742d8cd4p-2,
    0x1.970e4f80cb872p-1, -0x1.d5c216b4fbb94p-2, 0x1.920fb49d0e229p-1, -0x1.ef0adcbdc5935p-2,
    0x1.8d3018d3018d3p-1, -0x1.0402594b4d041p-1, 0x1.886e5f0abb04ap-1, -0x1.1058bf9ae4ad4p-1,
    0x1.83c977ab2beddp-1, -0x1.1c898c16999fbp-1, 0x1.7f405fd017f40p-1, -0x1.2895a13de86a4p-1,
    0x1.7ad2208e0ecc3p-1, -0x1.347dd9a987d56p-1, 0x1.767dce434a9b1p-1, -0x1.404308686a7e4p-1,
    0x1.724287f46debcp-1, -0x1.4be5f957778a1p-1, 0x1.6e1f76b4337c7p-1, -0x1.5767717455a6cp-1,
    0x1.6a13cd1537290p-1, -0x1.62c82f2b9c796p-1, 0x1.661ec6a5122f9p-1, 0x1.57bf753c8d1fbp-1,
    0x1.623fa77016240p-1, 0x1.4c9e09e172c3dp-1, 0x1.5e75bb8d015e7p-1, 0x1.419b423d5e8c6p-1,
    0x1.5ac056b015ac0p-1, 0x1.36b6776be1116p-1, 0x1.571ed3c506b3ap-1, 0x1.2bef07cdc9355p-1,
    0x1.5390948f40febp-1, 0x1.214456d0eb8d5p-1, 0x1.5015015015015p-1, 0x1.16b5ccbacfb73p-1,
    0x1.4cab88725af6ep-1, 0x1.0c42d676162e2p-1, 0x1.49539e3b2d067p-1, 0x1.01eae5626c691p-1,
    0x1.460cbc7f5cf9ap-1, 0x1.ef5ade4dcffe5p-2, 0x1.42d6625d51f87p-1, 0x1.db13db0d48941p-2,
    0x1.3fb013fb013fbp-1, 0x1.c6ffbc6f00f71p-2, 0x1.3c995a47babe7p-1, 0x1.b31d8575bce3bp-2,
    0x1.3991c2c187f63p-1, 0x1.9f6c407089663p-2, 0x1.3698df3de0748p-1, 0x1.8beafeb38fe8fp-2,
    0x1.33ae45b57bcb2p-1, 0x1.7898d85444c74p-2, 0x1.30d190130d190p-1, 0x1.6574ebe8c1339p-2,
    0x1.2e025c04b8097p-1, 0x1.527e5e4a1b58dp-2, 0x1.2b404ad012b40p-1, 0x1.3fb45a59928cap-2,
    0x1.288b01288b013p-1, 0x1.2d1610c86813dp-2, 0x1.25e22708092f1p-1, 0x1.1aa2b7e23f729p-2,
    0x1.23456789abcdfp-1, 0x1.08598b59e3a07p-2, 0x1.20b470c67c0d9p-1, 0x1.ec739830a1126p-3,
    0x1.1e2ef3b3fb874p-1, 0x1.c885801bc4b20p-3, 0x1.1bb4a4046ed29p-1, 0x1.a4e7640b1bc38p-3,
    0x1.19453808ca29cp-1, 0x1.8197e2f40e3f0p-3, 0x1.16e0689427379p-1, 0x1.5e95a4d9791cdp-3,
    0x1.1485f0e0acd3bp-1, 0x1.3bdf5a7d1ee5ep-3, 0x1.12358e75d3033p-1, 0x1.1973bd1465561p-3,
    0x1.0fef010fef011p-1, 0x1.eea31c006b87cp-4, 0x1.0db20a88f4696p-1, 0x1.aaef2d0fb1108p-4,
    0x1.0b7e6ec259dc8p-1, 0x1.67c94f2d4bb65p-4, 0x1.0953f39010954p-1, 0x1.252f32f8d1840p-4,
    0x1.073260a47f7c6p-1, 0x1.c63d2ec14aad7p-5, 0x1.05197f7d73404p-1, 0x1.432a925980cbcp-5,
    0x1.03091b51f5e1ap-1, 0x1.82448a388a283p-6, 0x1.0000000000000p-1, 0x0.0p+0,
    0x0.0p+0, 0x1.0000000000000p+0, 0x1.917a6bc29b42cp-4, 0x1.fd88da3d12526p-1,
    0x1.8f8b83c69a60bp-3, 0x1.f6297cff75cb0p-1, 0x1.294062ed59f06p-2, 0x1.e9f4156c62ddap-1,
    0x1.87de2a6aea963p-2, 0x1.d906bcf328d46p-1, 0x1.e2b5d3806f63bp-2, 0x1.c38b2f180bdb1p-1,
    0x1.1c73b39ae68c8p-1, 0x1.a9b66290ea1a3p-1, 0x1.44cf325091dd6p-1, 0x1.8bc806b151741p-1,
    0x1.6a09e667f3bcdp-1, 0x1.6a09e667f3bcdp-1, 0x1.8bc806b151741p-1, 0x1.44cf325091dd6p-1,
    0x1.a9b66290ea1a3p-1, 0x1.1c73b39ae68c8p-1, 0x1.c38b2f180bdb1p-1, 0x1.e2b5d3806f63bp-2,
    0x1.d906bcf328d46p-1, 0x1.87de2a6aea963p-2, 0x1.e9f4156c62ddap-1, 0x1.294062ed59f06p-2,
    0x1.f6297cff75cb0p-1, 0x1.8f8b83c69a60bp-3, 0x1.fd88da3d12526p-1, 0x1.917a6bc29b42cp-4,
    0x1.0000000000000p+0, 0x1.77d4c76273645p-204, 0x1.fd88da3d12526p-1, -0x1.917a6bc29b42cp-4,
    0x1.f6297cff75cb0p-1, -0x1.8f8b83c69a60bp-3, 0x1.e9f4156c62ddap-1, -0x1.294062ed59f06p-2,
    0x1.d906bcf328d46p-1, -0x1.87de2a6aea963p-2, 0x1.c38b2f180bdb1p-1, -0x1.e2b5d3806f63bp-2,
    0x1.a9b66290ea1a3p-1, -0x1.1c73b39ae68c8p-1, 0x1.8bc806b151741p-1, -0x1.44cf325091dd6p-1,
    0x1.6a09e667f3bcdp-1, -0x1.6a09e667f3bcdp-1, 0x1.44cf325091dd6p-1, -0x1.8bc806b151741p-1,
    0x1.1c73b39ae68c8p-1, -0x1.a9b66290ea1a3p-1, 0x1.e2b5d3806f63bp-2, -0x1.c38b2f180bdb1p-1,
    0x1.87de2a6aea963p-2, -0x1.d906bcf328d46p-1, 0x1.294062ed59f06p-2, -0x1.e9f4156c62ddap-1,
    0x1.8f8b83c69a60bp-3, -0x1.f6297cff75cb0p-1, 0x1.917a6bc29b42cp-4, -0x1.fd88da3d12526p-1,
    0x1.77d4c76273645p-203, -0x1.0000000000000p+0, -0x1.917a6bc29b42cp-4, -0x1.fd88da3d12526p-1,
    -0x1.8f8b83c69a60bp-3, -0x1.f6297cff75cb0p-1, -0x1.294062ed59f06p-2, -0x1.e9f4156c62ddap-1,
    -0x1.87de2a6aea963p-2, -0x1.d906bcf328d46p-1, -0x1.e2b5d3806f63bp-2, -0x1.c38b2f180bdb1p-1,
    -0x1.1c73b39ae68c8p-1, -0x1.a9b66290ea1a3p-1, -0x1.44cf325091dd6p-1, -0x1.8bc806b151741p-1,
    -0x1.6a09e667f3bcdp-1, -0x1.6a09e667f3bcdp-1, -0x1.8bc806b151741p-1, -0x1.44cf325091dd6p-1,
    -0x1.a9b66290ea1a3p-1, -0x1.1c73b39ae68c8p-1, -0x1.c38b2f180bdb1p-1, -0x1.e2b5d3806f63bp-2,
    -0x1.d906bcf328d46p-1, -0x1.87de2a6aea963p-2, -0x1.e9f4156c62ddap-1, -0x1.294062ed59f06p-2,
    -0x1.f6297cff75cb0p-1, -0x1.8f8b83c69a60bp-3, -0x1.fd88da3d12526p-1, -0x1.917a6bc29b42cp-4,
    -0x1.0000000000000p+0, 0x1.dcc40d4ec52eap-199, -0x1.fd88da3d12526p-1, 0x1.917a6bc29b42cp-4,
    -0x1.f6297cff75cb0p-1, 0x1.8f8b83c69a60bp-3, -0x1.e9f4156c62ddap-1, 0x1.294062ed59f06p-2,
    -0x1.d906bcf328d46p-1, 0x1.87de2a6aea963p-2, -0x1.c38b2f180bdb1p-1, 0x1.e2b5d3806f63bp-2,
    -0x1.a9b66290ea1a3p-1, 0x1.1c73b39ae68c8p-1, -0x1.8bc806b151741p-1, 0x1.44cf325091dd6p-1,
    -0x1.6a09e667f3bcdp-1, 0x1.6a09e667f3bcdp-1, -0x1.44cf325091dd6p-1, 0x1.8bc806b151741p-1,
    -0x1.1c73b39ae68c8p-1, 0x1.a9b66290ea1a3p-1, -0x1.e2b5d3806f63bp-2, 0x1.c38b2f180bdb1p-1,
    -0x1.87de2a6aea963p-2, 0x1.d906bcf328d46p-1, -0x1.294062ed59f06p-2, 0x1.e9f4156c62ddap-1,
    -0x1.8f8b83c69a60bp-3, 0x1.f6297cff75cb0p-1, -0x1.917a6bc29b42cp-4, 0x1.fd88da3d12526p-1};

template <class To, class From>
__device__ __forceinline__ To bits_as(const From& v) {
    return __builtin_bit_cast(To, v);
}

// -2 ln u for u = K 2^-53, K = (hi << 21) | ((lo >> 11) | 1); tab: the table above.
__device__ __forceinline__ double neg2_log_u53(uint32_t lo, uint32_t hi, const double* tab) {
    const double Kd = fma(double(hi), 0x1p21, double((lo >> 11) | 1u));   // exact integer in [1, 2^53)
    const uint64_t kb = bits_as<uint64_t>(Kd);
    const uint32_t kh = uint32_t(kb >> 32);
    const uint32_t X = (kh >> 14) & 0x1FFFFu;        // biased exponent (11 bits), top 6 mantissa bits
    const uint32_t i = X & 63u;
    const int E = int(X + (37u - 1076u * 64u)) >> 6;  // e - 53, +1 for buckets i >= 27
    const double m = bits_as<double>((uint64_t((kh & 0x000FFFFFu) | 0x3FF00000u) << 32) | (kb & 0xFFFFFFFFull));
    const double r = fma(m, tab[2 * i], -1.0);
    double P = kBMLogP[7];
#pragma unroll
    for (int n = 6; n >= 0; --n) P = fma(P, r, kBMLogP[n]);
    P = P * r;                                      // -2 log1p(r)
    const double Ed = double(E);
    return fma(Ed, kM2Ln2Hi, tab[2 * i + 1]) + fma(Ed, kM2Ln2Lo, P);
}

// (sin, cos)(2 pi u) for u = K 2^-53, K = (hi << 21) | ((lo >> 11) | 1); tab: the table above.
__device__ __forceinline__ void sincos_2pi_u53(uint32_t lo, uint32_t hi, const double* tab, double& sn, double& cs) {
    const uint32_t k = (hi + 0x2000000u) >> 26;      // round(64 u) mod 64 (K is odd: no ties)
    const int hs = int(hi << 6) >> 6;                // hi - k 2^26, in [-2^25, 2^25)
    const double J = fma(double(hs), 0x1p21, double((lo >> 11) | 1u));   // K - k 2^47, exact
    const double w = J * J;
    double S = kBMSin[3];
    S = fma(S, w, kBMSin[2]);
    S = fma(S, w, kBMSin[1]);
    S = fma(S, w, kBMSin[0]);
    S = S * J;                                      // sin(2 pi J 2^-53)
    double C = kBMCos[3];
    C = fma(C, w, kBMCos[2]);
    C = fma(C, w, kBMCos[1]);
    C = fma(C, w, kBMCos[0]);
    C = C * w;                                      // cos(2 pi J 2^-53) - 1
    const double s0 = tab[128 + 2 * k], c0 = tab[129 + 2 * k];
    sn = fma(c0, S, fma(s0, C, s0));
    cs = fma(-s0, S, fma(c0, C, c0));
}

}  // namespace pimc
