// General-potential mode on the device: per slice, the derivatives v_j = V^(j)(mid), j <= J = 2p-2,
// in registers (from the tables of pimc_general.hpp: the polynomial part by Horner per derivative,
// one tanh and one exp per sech^2 term with sech^2 times the polynomials R_j(tanh), one exp per
// Gaussian term with the Hermite recurrence), scaled per bisection level to vt_j = eps^(1 + j/2) v_j, then
// eps W_p = sum_k zt^k sum c prod vt_f with zt = dlt^2 / (4 eps) by the straight-line code generated
// for level p at build time (GenCompiled<p>, pimc_general_gen.hpp), whose coefficients c are
// compile-time constants (the same at every level); the per-level scale factors are scalar loads.
// Levels above kGenInlineMaxP (GenSliceEval) evaluate one slice per call of an out-of-line function
// gen_slice_hi<p>, instantiated only in the translation unit that includes that level's generated
// header (pimc_general_hi.hip), so that its straight-line code is emitted once per kernel.
#pragma once

#include "pimc_device.hpp"

namespace pimc {
template <int P>
struct GenCompiled;
}  // namespace pimc

#include "pimc_general_gen.hpp"

namespace pimc {

template <int J>
__device__ __forceinline__ void gen_derivatives_dev(const GenTables& g, double x, double (&v)[J + 1]) {
    // V^(j) of the polynomial part (degree <= 8, zero-padded rows: a leading zero coefficient leaves
    // the Horner value unchanged), fully unrolled so that the wave-uniform coefficients are
    // independent scalar loads
    const const_ptr<double> dp = as_const(g.dpoly);
    constexpr int JP = J < 8 ? J : 8;
#pragma unroll
    for (int j = 0; j <= JP; ++j) {
        double acc = dp[j * 9 + 8 - j];
#pragma unroll
        for (int n = 7 - j; n >= 0; --n) acc = fma(acc, x, dp[j * 9 + n]);
        v[j] = acc;
    }
#pragma unroll
    for (int j = JP + 1; j <= J; ++j) v[j] = 0.0;
    const const_ptr<double> ds = as_const(g.dsech);
    for (int t = 0; t < g.n_sech; ++t) {
        // A a^j S_j(tanh) = sech^2 * (A a^j R_j(tanh)), sech^2 = 4w/(1+w)^2 with w = e^(-2|a x|)
        const double y = g.sech_a[t] * x;
        const double th = tanh_fp64(y);
        const double w = exp_fp64(-2.0 * fabs(y));
        const double dw = 1.0 + w;
        const double s2 = 4.0 * w / (dw * dw);
#pragma unroll
        for (int j = 0; j <= J; ++j) {
            const int row = (t * (J + 1) + j) * (J + 1);
            double acc = ds[row + j];
#pragma unroll
            for (int n = j - 1; n >= 0; --n) acc = fma(acc, th, ds[row + n]);
            v[j] = fma(s2, acc, v[j]);
        }
    }
    for (int t = 0; t < g.n_gauss; ++t) {
        // d^j/dx^j B e^{-b x^2} = B (-sqrt b)^j H_j(sqrt(b) x) e^{-b x^2}, H_{j+1} = 2y H_j - 2j H_{j-1}
        const double y = g.gsb[t] * x;
        double e = g.gB[t] * exp_fp64(-g.gb[t] * x * x);
        double hm = 0.0, h = 1.0;
#pragma unroll
        for (int j = 0; j <= J; ++j) {
            v[j] += e * h;
            const double hn = 2.0 * y * h - 2.0 * double(j) * hm;
            hm = h;
            h = hn;
            e *= -g.gsb[t];
        }
    }
}

template <int P>
struct GenCompiledEval {
    static constexpr int J = 2 * P - 2;
    const double* __restrict__ tab;      // level-major, J + 2 per level: eps^(1 + j/2), j <= J, then 1/(4 eps)
    GenTables g;
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab)); }
    template <int W>
    __device__ __forceinline__ void eval(int level, const double (&qa)[W], const double (&qb)[W], double& S) const {
        static_assert(GenCompiled<P>::J == J, "generated evaluator of another level");
        // the level is wave-uniform (the walk does not depend on the lane): keep the table address in
        // scalar registers
        const int lv = __builtin_amdgcn_readfirstlane(level);
        const_ptr<double> t = as_const(tab) + lv * (J + 2);
        // slices evaluated together (each holds J+1 derivative values in registers)
        constexpr int B = W < gen_block_slices(P) ? W : gen_block_slices(P);
#pragma unroll
        for (int b0 = 0; b0 < W; b0 += B) {
            double v[B][J + 1], z[B], acc[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const double x = 0.5 * (qa[b0 + i] + qb[b0 + i]);
                const double dl = qb[b0 + i] - qa[b0 + i];
                z[i] = dl * dl * t[J + 1];
                gen_derivatives_dev<J>(g, x, v[i]);
#pragma unroll
                for (int j = 0; j <= J; ++j) v[i][j] *= t[j];
            }
            GenCompiled<P>::template eval<B>(v, z, acc);
#pragma unroll
            for (int i = 0; i < B; ++i) S += acc[i];
        }
    }
};

// eps W_p of one slice (qa, qb) at the level whose scale factors are t[0..J+1] (p > kGenInlineMaxP).
template <int P>
__device__ __forceinline__ void gen_scaled_derivatives(const GenTables& g, const double* t, double qa, double qb,
                                                       double (&v)[2 * P - 1], double& z) {
    constexpr int J = 2 * P - 2;
    const double x = 0.5 * (qa + qb);
    const double dl = qb - qa;
    gen_derivatives_dev<J>(g, x, v);
#pragma unroll
    for (int j = 0; j <= J; ++j) v[j] *= t[j];
    z = dl * dl * t[J + 1];
}

template <int P>
__device__ __noinline__ double gen_slice_hi(const GenTables g, const double* t, double qa, double qb) {
    static_assert(GenCompiled<P>::J == 2 * P - 2, "generated evaluator of another level");
    double v[2 * P - 1], z;
    gen_scaled_derivatives<P>(g, t, qa, qb, v, z);
    return GenCompiled<P>::eval1(v, z);
}

// Two slices per call, each formed exactly as gen_slice_hi forms it (the same bits): every
// instruction of the long straight-line code then serves two slices.
template <int P>
__device__ __noinline__ void gen_slices2_hi(const GenTables g, const double* t, double qa0, double qb0, double qa1,
                                            double qb1, double& r0, double& r1) {
    double v0[2 * P - 1], v1[2 * P - 1], z0, z1;
    gen_scaled_derivatives<P>(g, t, qa0, qb0, v0, z0);
    gen_scaled_derivatives<P>(g, t, qa1, qb1, v1, z1);
    GenCompiled<P>::eval2(v0, v1, z0, z1, r0, r1);
}

template <int P>
struct GenSliceEval {
    static constexpr int J = 2 * P - 2;
    const double* __restrict__ tab;      // level-major, J + 2 per level: eps^(1 + j/2), j <= J, then 1/(4 eps)
    GenTables g;
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab)); }
    template <int W>
    __device__ __forceinline__ void eval(int level, const double (&qa)[W], const double (&qb)[W], double& S) const {
        const int lv = __builtin_amdgcn_readfirstlane(level);
        const double* t = tab + lv * (J + 2);
        if constexpr (W == 1) {
            S += gen_slice_hi<P>(g, t, qa[0], qb[0]);
        } else {
            static_assert(W % 2 == 0, "slices in pairs");
#pragma unroll
            for (int i = 0; i < W; i += 2) {
                double r0, r1;
                gen_slices2_hi<P>(g, t, qa[i], qb[i], qa[i + 1], qb[i + 1], r0, r1);
                S += r0;
                S += r1;
            }
        }
    }
};

}  // namespace pimc
