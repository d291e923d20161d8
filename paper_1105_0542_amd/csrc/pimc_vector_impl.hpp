// Vector estimation kernels (several coordinates, Sec. 2.2 with the bisection estimator of Sec. 4),
// included once per dimension by pimc_vector_d{1,2,3,4}.hip and pimc_vector_poly.hip.
//
// The walk is the one of the one-dimensional kernels, with a point of DIM coordinates per node: one
// lane owns one path; the bottom U bisection levels of each subtree live in registers, the levels
// above keep one pending right endpoint per level in LDS; every level-n slice is evaluated as soon as
// both its endpoints exist. Coordinate c of heap node h takes the normal of generator call
// (h >> 1) + c * 2^20 (so coordinate 0 is the one-dimensional path). The normal of a pending right
// child is drawn again when the walk returns to it instead of being kept (one more generator call per
// coordinate for every 2^U leaves; it halves the LDS per lane).
//
// Per level, each path's weight enters as d = exp(-(S_n - S_ref,n)) - 1, summed per canonical chunk
// (kChunkPaths paths, the order of the one-dimensional kernels, pimc_internal.hpp), then over chunks
// by k_seg_reduce: the result does not depend on the grid.
#pragma once

#include "pimc_vector.hpp"

namespace pimc {
namespace vec {

template <int DIM>
struct VecSource {
    RngKey key;
    PathRng pr;
    const double* bm;                  // Box-Muller table (LDS)
    // Normals of heap nodes 2j and 2j+1 in every coordinate.
    __device__ __forceinline__ void pair(uint32_t j, double (&ze)[DIM], double (&zo)[DIM]) const {
#pragma unroll
        for (int c = 0; c < DIM; ++c) normal_pair(key, pr, j + uint32_t(c) * kCoordPairStride, bm, ze[c], zo[c]);
    }
    // Normal of heap node h in every coordinate.
    __device__ __forceinline__ void node(uint32_t h, double (&z)[DIM]) const {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            double e, o;
            normal_pair(key, pr, (h >> 1) + uint32_t(c) * kCoordPairStride, bm, e, o);
            z[c] = (h & 1u) ? o : e;
        }
    }
};

// Invariants of B slices from their endpoints (x4: the tables are pre-scaled).
template <int DIM, int B>
__device__ __forceinline__ void invariants(const double (&qa)[B][DIM], const double (&qb)[B][DIM], double (&u)[B],
                                           double (&w2)[B], double (&z)[B]) {
#pragma unroll
    for (int i = 0; i < B; ++i) {
        double su = 0.0, sw = 0.0, sz = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const double s = qa[i][c] + qb[i][c];
            const double d = qb[i][c] - qa[i][c];
            su = fma(s, s, su);
            sw = fma(s, d, sw);
            sz = fma(d, d, sz);
        }
        u[i] = su;
        w2[i] = sw * sw;
        z[i] = sz;
    }
}

// Level tables with the compile-time shape of level P. The group loops are template recursions so
// that every length and offset is a constant of the front end.
template <int P, int B, int J, int L>
__device__ __forceinline__ void radial_groups_l(const_ptr<double> t, const double (&u)[B], const double (&z)[B],
                                                double (&zs)[B]) {
    if constexpr (L >= 0) {
        constexpr int len = radial_len(P, J + L, J);
        constexpr int off = radial_off(P, J, L);
        constexpr bool top = (L == radial_nl(P, J) - 1);
        double v[B];
        if constexpr (len == 0) {
#pragma unroll
            for (int i = 0; i < B; ++i) v[i] = 0.0;
        } else {
            const double c0 = t[off];
#pragma unroll
            for (int i = 0; i < B; ++i) v[i] = c0;
#pragma unroll
            for (int e = 1; e < len; ++e) {
                const double c = t[off + e];
#pragma unroll
                for (int i = 0; i < B; ++i) v[i] = fma(v[i], u[i], c);
            }
        }
#pragma unroll
        for (int i = 0; i < B; ++i) zs[i] = top ? v[i] : fma(zs[i], z[i], v[i]);
        radial_groups_l<P, B, J, L - 1>(t, u, z, zs);
    }
}

template <int P, int B, int J>
__device__ __forceinline__ void radial_groups_j(const_ptr<double> t, const double (&u)[B], const double (&w2)[B],
                                                const double (&z)[B], double (&acc)[B]) {
    if constexpr (J >= 0) {
        asm volatile("" : "+s"(t));
        double zs[B];
        radial_groups_l<P, B, J, radial_nl(P, J) - 1>(t, u, z, zs);
        constexpr bool top = (J == radial_nj(P) - 1);
#pragma unroll
        for (int i = 0; i < B; ++i) acc[i] = top ? zs[i] : fma(acc[i], w2[i], zs[i]);
        radial_groups_j<P, B, J - 1>(t, u, w2, z, acc);
    }
}

template <int P, int DIM>
struct RadialEval {
    const double* __restrict__ tab;
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab)); }
    template <int B>
    __device__ __forceinline__ void eval(int level, const double (&qa)[B][DIM], const double (&qb)[B][DIM],
                                         double& S) const {
        constexpr int E = radial_size(P);
        constexpr int NJ = radial_nj(P);
        const const_ptr<double> t = as_const(tab) + level * E;
        double u[B], w2[B], z[B], acc[B];
        invariants<DIM, B>(qa, qb, u, w2, z);
        radial_groups_j<P, B, NJ - 1>(t, u, w2, z, acc);
        if constexpr (NJ > 0) {
#pragma unroll
            for (int i = 0; i < B; ++i) S += acc[i];
        }
    }
};

// The same layout with the shape read from the shape array (any p, any s).
template <int DIM>
struct RadialEvalRT {
    const double* __restrict__ tab;
    const int* __restrict__ shape;
    int stride;
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab)); }
    template <int B>
    __device__ __forceinline__ void eval(int level, const double (&qa)[B][DIM], const double (&qb)[B][DIM],
                                         double& S) const {
        const const_ptr<double> t = as_const(tab) + level * stride;
        const const_ptr<int> sh = as_const(shape);
        double u[B], w2[B], z[B], acc[B];
        invariants<DIM, B>(qa, qb, u, w2, z);
        const int nj = sh[0];
        int g = 1 + nj;                     // index of the next group length
        int off = 0;
        for (int j = nj - 1; j >= 0; --j) {
            const int nl = sh[1 + j];
            double zs[B];
            for (int l = nl - 1; l >= 0; --l) {
                const int len = sh[g++];
                double v[B];
#pragma unroll
                for (int i = 0; i < B; ++i) v[i] = 0.0;
                if (len > 0) {
                    const double c0 = t[off];
#pragma unroll
                    for (int i = 0; i < B; ++i) v[i] = c0;
                    for (int e = 1; e < len; ++e) {
                        const double c = t[off + e];
#pragma unroll
                        for (int i = 0; i < B; ++i) v[i] = fma(v[i], u[i], c);
                    }
                }
                off += len;
#pragma unroll
                for (int i = 0; i < B; ++i) zs[i] = (l == nl - 1) ? v[i] : fma(zs[i], z[i], v[i]);
            }
#pragma unroll
            for (int i = 0; i < B; ++i) acc[i] = (j == nj - 1) ? zs[i] : fma(acc[i], w2[i], zs[i]);
        }
        if (nj > 0) {
#pragma unroll
            for (int i = 0; i < B; ++i) S += acc[i];
        }
    }
};

// Any polynomial V (component route): eps W_p of a slice is a polynomial in the 2 DIM variables
// y_c = qb_c - qa_c (c < DIM) and y_{DIM+c} = qa_c + qb_c, evaluated by a multivariate Horner scheme
// over the prefix tree of its monomials (exponents of y_0, y_1, ... from high to low). The tree is a
// level-independent structure stream of ints (pre-order); only the coefficients depend on the level.
//   node at depth v < 2 DIM - 1:  [n >= 1 children] then per child [gap | tail << 8] and the child's
//       node; a_v = first child's value y_{v+1}^tail, then per child a_v = a_v y_v^gap + (child value)
//       y_{v+1}^tail;
//   node at depth 2 DIM - 1:      [L >= 1]: the dense Horner chain in y_{2 DIM - 1} over the next L
//       coefficients of the level's array (zeros fill the exponents that are absent);
//   stream head: [tail of the root]; the slice value is a_0 y_0^tail.
// Every count and exponent is wave-uniform (scalar loads through the constant address space), so the
// depth-nested loops are scalar branches around B-wide vector FMAs; a_v and the running pointers have
// one register home per depth (no interpreter dispatch, no copies between depths).
#ifndef PIMC_POLY_UNROLL
#define PIMC_POLY_UNROLL 4
#endif
constexpr int kPolyUnroll = PIMC_POLY_UNROLL;   // coefficients per scalar load group of a chain

template <int DIM>
struct PolyEvalRT {
    static constexpr int NV = 2 * DIM;
    const double* __restrict__ tab;      // coefficients, level-major, stride doubles per level
    const int* __restrict__ code;        // structure stream
    int stride;
    __device__ __forceinline__ void launder() { asm volatile("" : "+s"(tab), "+s"(code)); }

    // a = a * y + t in a's registers. Written as fma(), the compiler picks the two-operand form that
    // accumulates into t's registers and then copies the result back to a at every iteration of a
    // node's child loop (B 64-bit moves per child); the three-operand instruction with a tied to its
    // destination needs no copy. Same operation, same rounding.
    __device__ __forceinline__ static void fma_into(double& a, double y, double t) {
        asm("v_fma_f64 %0, %0, %1, %2" : "+v"(a) : "v"(y), "v"(t));
    }

    // x[i] *= y[i]^e for a wave-uniform e >= 0 (a scalar loop around B multiplies).
    template <int B>
    __device__ __forceinline__ static void times_pow(double (&x)[B], const double (&y)[B], int e) {
        for (int k = 0; k < e; ++k) {
#pragma unroll
            for (int i = 0; i < B; ++i) x[i] *= y[i];
        }
    }

    // The node's value into out. A chain starts from its first coefficient and a node of the two
    // deepest internal levels from its first child's value (the same bits as starting from 0:
    // fma(0, y, t) = t); every node has at least one child and every chain at least one coefficient.
    template <int V, int B>
    __device__ __forceinline__ static void node(const_ptr<int>& s, const_ptr<double>& c, const double (&y)[NV][B],
                                                double (&out)[B]) {
        if constexpr (V == NV - 1) {
            const int L = s[0];
            s += 1;
            const double c0 = c[0];
#pragma unroll
            for (int i = 0; i < B; ++i) out[i] = c0;
            int j = 1;
            for (; j + kPolyUnroll <= L; j += kPolyUnroll) {
                double cq[kPolyUnroll];
#pragma unroll
                for (int q = 0; q < kPolyUnroll; ++q) cq[q] = c[j + q];
#pragma unroll
                for (int q = 0; q < kPolyUnroll; ++q) {
#pragma unroll
                    for (int i = 0; i < B; ++i) out[i] = fma(out[i], y[V][i], cq[q]);
                }
            }
            for (; j < L; ++j) {
                const double c1 = c[j];
#pragma unroll
                for (int i = 0; i < B; ++i) out[i] = fma(out[i], y[V][i], c1);
            }
            c += L;
        } else {
            const int n = s[0];
            int k = 0;
            if constexpr (V >= NV - 3) {
                // the two deepest internal levels (most of the nodes) let the first child write the
                // accumulator; above them it is zeroed, which keeps one copy of a child's code per
                // level instead of two (2^(2 DIM - 1) copies of the chain loop when peeled throughout)
                const int h0 = s[1];
                s += 2;
                node<V + 1, B>(s, c, y, out);
                times_pow<B>(out, y[V + 1], h0 >> 8);
                k = 1;
            } else {
                s += 1;
#pragma unroll
                for (int i = 0; i < B; ++i) out[i] = 0.0;
            }
            for (; k < n; ++k) {
                const int h = s[0];
                s += 1;
                times_pow<B>(out, y[V], (h & 255) - 1);
                double t[B];
                node<V + 1, B>(s, c, y, t);
                times_pow<B>(t, y[V + 1], h >> 8);
#pragma unroll
                for (int i = 0; i < B; ++i) fma_into(out[i], y[V][i], t[i]);
            }
        }
    }

    template <int B>
    __device__ __forceinline__ void eval(int level, const double (&qa)[B][DIM], const double (&qb)[B][DIM],
                                         double& S) const {
        const int lv = __builtin_amdgcn_readfirstlane(level);
        const_ptr<double> c = as_const(tab) + lv * stride;
        const_ptr<int> s = as_const(code);
        double y[NV][B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                y[k][i] = qb[i][k] - qa[i][k];
                y[DIM + k][i] = qa[i][k] + qb[i][k];
            }
        }
        const int tail = s[0];
        s += 1;
        double v[B];
        node<0, B>(s, c, y, v);
        times_pow<B>(v, y[0], tail);
#pragma unroll
        for (int i = 0; i < B; ++i) S += v[i];
    }
};

// ---------------------------------------------------------------------------- subtree (registers)
template <int DIM, int U, int L>
__device__ __forceinline__ void gen_level(const VecArgs& A, const VecSource<DIM>& src, uint32_t root, int D,
                                          double (&q)[(1 << U) + 1][DIM]) {
    if constexpr (L <= U) {
        constexpr int step = 1 << (U - L);
        const double sg = as_const(A.sig)[D + L];
#pragma unroll
        for (int i2 = 0; i2 < (1 << (L - 2)); ++i2) {
            const uint32_t parent = (root << (L - 2)) + uint32_t(i2);   // node of sub-level L-1
            double ze[DIM], zo[DIM];
            src.pair(parent, ze, zo);                                    // children 2*parent, 2*parent+1
            const int jl = (4 * i2 + 1) * step;
            const int jr = (4 * i2 + 3) * step;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                q[jl][c] = sg * ze[c] + 0.5 * (q[jl - step][c] + q[jl + step][c]);
                q[jr][c] = sg * zo[c] + 0.5 * (q[jr - step][c] + q[jr + step][c]);
            }
        }
        gen_level<DIM, U, L + 1>(A, src, root, D, q);
    }
}

// Add the 2^L slices of sub-level L (point stride 2^(U-L)) at tree level `level` to S, left to right.
template <int DIM, int U, int L, class Eval>
__device__ __forceinline__ void level_sum(const Eval& ev, int level, const double (&q)[(1 << U) + 1][DIM],
                                          double& S) {
    constexpr int W = 1 << L;
    constexpr int ST = 1 << (U - L);
    constexpr int B = W < kVecBatch ? W : kVecBatch;
#pragma unroll
    for (int b0 = 0; b0 < W; b0 += B) {
        double qa[B][DIM], qb[B][DIM];
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                qa[i][c] = q[(b0 + i) * ST][c];
                qb[i][c] = q[(b0 + i + 1) * ST][c];
            }
        ev.template eval<B>(level, qa, qb, S);
    }
}

template <int DIM, int U, int L, class Eval>
__device__ __forceinline__ void hier_levels(const Eval& ev, int D, const double (&q)[(1 << U) + 1][DIM],
                                            double (&Ssub)[U + 1]) {
    if constexpr (L < U) {
        level_sum<DIM, U, L, Eval>(ev, D + L, q, Ssub[L]);
        hier_levels<DIM, U, L + 1, Eval>(ev, D, q, Ssub);
    }
}

// Subtree rooted at heap node `root` (level D+1) over the level-D slice (qL, qR) with root normal z.
template <int DIM, int U, class Eval>
__device__ __forceinline__ void run_subtree(const Eval& ev_in, const VecArgs& A, const VecSource<DIM>& src,
                                            uint32_t root, int D, const double (&qL)[DIM], const double (&qR)[DIM],
                                            const double (&zroot)[DIM], double (&Ssub)[U + 1]) {
    Eval ev = ev_in;
    ev.launder();
    double q[(1 << U) + 1][DIM];
    const double sg = as_const(A.sig)[D + 1];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        q[0][c] = qL[c];
        q[1 << U][c] = qR[c];
        q[1 << (U - 1)][c] = sg * zroot[c] + 0.5 * (qL[c] + qR[c]);
    }
    gen_level<DIM, U, 2>(A, src, root, D, q);
    if (A.hier) hier_levels<DIM, U, 0, Eval>(ev, D, q, Ssub);
    level_sum<DIM, U, U, Eval>(ev, D + U, q, Ssub[U]);
}

// ---------------------------------------------------------------------------- one path
// top: this lane's LDS slots (stride kVecBlock): S_top[n] at slot n (n < D); the pending right
// endpoint of level L (L = 2..D), coordinate c, at slot D + (L-2)*DIM + c.
template <int DIM, int U, class Eval>
__device__ __forceinline__ void walk_path(const Eval& ev, const VecArgs& A, const VecSource<DIM>& src, double* top,
                                          double (&Ssub)[U + 1]) {
    const int D = A.D;
#pragma unroll
    for (int j = 0; j <= U; ++j) Ssub[j] = 0.0;
    double a[DIM], b[DIM], z1[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        a[c] = A.a[c];
        b[c] = A.b[c];
    }
    {
        double unused[DIM];
        src.pair(0u, unused, z1);                    // node 1 = sine output of call 0
    }
    if (D == 0) {
        run_subtree<DIM, U, Eval>(ev, A, src, 1u, 0, a, b, z1, Ssub);
        return;
    }
    for (int n = 0; n < D; ++n) top[n * kVecBlock] = 0.0;
    double* R = top + D * kVecBlock;
    const uint32_t nTop = 1u << (D - 1);             // level-D nodes nTop .. 2 nTop - 1
    double qlast[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) qlast[c] = a[c];
    for (uint32_t J = 0; J < nTop; ++J) {
        int L;
        uint32_t node;
        double qL[DIM], qR[DIM], z[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) qL[c] = qlast[c];
        if (J == 0) {
            L = 1;
            node = 1u;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                qR[c] = b[c];
                z[c] = z1[c];
            }
        } else {
            const int t = __builtin_ctz(J);
            L = D - t;
            node = (nTop + J) >> t;
#pragma unroll
            for (int c = 0; c < DIM; ++c) qR[c] = R[((L - 2) * DIM + c) * kVecBlock];
            src.node(node, z);
        }
        double qm[DIM], zl[DIM], zr[DIM];
        while (true) {
            if (A.hier) {
                double qa1[1][DIM], qb1[1][DIM];
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    qa1[0][c] = qL[c];
                    qb1[0][c] = qR[c];
                }
                double St = top[(L - 1) * kVecBlock];
                ev.template eval<1>(L - 1, qa1, qb1, St);
                top[(L - 1) * kVecBlock] = St;
            }
            const double sg = as_const(A.sig)[L];
#pragma unroll
            for (int c = 0; c < DIM; ++c) qm[c] = sg * z[c] + 0.5 * (qL[c] + qR[c]);
            src.pair(node, zl, zr);
            if (L == D) break;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                R[((L - 1) * DIM + c) * kVecBlock] = qR[c];   // right child of `node`: (qm, qR), level L+1
                qR[c] = qm[c];
                z[c] = zl[c];
            }
            node = 2u * node;
            ++L;
        }
        run_subtree<DIM, U, Eval>(ev, A, src, 2u * node, D, qL, qm, zl, Ssub);
        run_subtree<DIM, U, Eval>(ev, A, src, 2u * node + 1u, D, qm, qR, zr, Ssub);
#pragma unroll
        for (int c = 0; c < DIM; ++c) qlast[c] = qR[c];
    }
}

// ---------------------------------------------------------------------------- estimation kernel
__device__ __forceinline__ void reduce_level(const VecArgs& A, double* a, int lane, int n, double S, bool valid) {
    const double d = valid ? expm1(-(S - as_const(A.shift)[n])) : 0.0;
    const bool bad = valid && !isfinite(d);
    const double sd = wave_sum(d);
    const double sd2 = wave_sum(d * d);
    const unsigned long long badmask = __ballot(bad);
    if (lane == 0) {
        a[0] += sd;
        a[1] += sd2;
        a[2] += double(__popcll(badmask));
    }
}

// One canonical chunk c: paths c*kChunkPaths + 64 g + lane, groups g = wave, wave + 4, ... (the
// order of the one-dimensional kernels); writes the chunk's four sums per evaluated level to
// A.partials[(slot * n_chunks + c) * 4] and/or the per-path level actions to A.dump. smem: the
// Box-Muller table, the per-lane stack, the accumulator slots.
template <int DIM, int U, class Eval>
__device__ __forceinline__ void process_chunk(const Eval& ev, const VecArgs& A, uint64_t c, double* smem) {
    constexpr int WAVES = kVecBlock / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int D = A.D;
    const int nlev = A.s + 1;
    const double* bm = smem;
    double* top = smem + kBoxMullerTable + tid;
    double* acc = smem + kBoxMullerTable + size_t(vec_top_slots(DIM, D)) * kVecBlock;
    const uint64_t first = c * kChunkPaths;
    if (A.partials) {
        for (int i = tid; i < kChunkSlots * nlev * 3; i += kVecBlock) acc[i] = 0.0;
        __syncthreads();
    }
    for (int g = wave; g < kChunkGroups; g += WAVES) {
        const uint64_t group0 = first + uint64_t(g) * 64;
        if (group0 >= A.n_paths) break;                   // wave-uniform: the rest of the chunk is empty
        const uint64_t local = group0 + uint64_t(lane);
        const bool valid = local < A.n_paths;
        double Ssub[U + 1];
        const VecSource<DIM> src{A.key, path_rng(A.key, A.first_path + local), bm};
        walk_path<DIM, U, Eval>(ev, A, src, top, Ssub);
        if (A.dump && valid) {
            double* o = A.dump + local * uint64_t(nlev);
            for (int n = 0; n < D; ++n) o[n] = A.hier ? top[n * kVecBlock] : 0.0;
#pragma unroll
            for (int j = 0; j <= U; ++j) o[D + j] = (A.hier || j == U) ? Ssub[j] : 0.0;
        }
        if (A.partials) {
            double* a = acc + (g % kChunkSlots) * nlev * 3;
            if (A.hier) {
                for (int n = 0; n < D; ++n) reduce_level(A, a + n * 3, lane, n, top[n * kVecBlock], valid);
#pragma unroll
                for (int j = 0; j < U; ++j) reduce_level(A, a + (D + j) * 3, lane, D + j, Ssub[j], valid);
            }
            reduce_level(A, a + (D + U) * 3, lane, D + U, Ssub[U], valid);
        }
    }
    if (A.partials) {
        __syncthreads();
        const int slots = A.hier ? nlev : 1;
        if (tid < slots) {
            const int lev = A.hier ? tid : nlev - 1;
            const uint64_t rem = A.n_paths - first;
            const double cnt = double(rem < kChunkPaths ? rem : kChunkPaths);
            double s1 = 0.0, s2 = 0.0, nb = 0.0;
            for (int q = 0; q < kChunkSlots; ++q) {
                const double* a = acc + (q * nlev + lev) * 3;
                s1 += a[0];
                s2 += a[1];
                nb += a[2];
            }
            double* o = A.partials + (uint64_t(tid) * A.n_chunks + c) * 4;
            o[0] = cnt;
            o[1] = s1;
            o[2] = s2;
            o[3] = nb;
        }
        __syncthreads();
    }
}

template <int DIM, int U, class Eval>
__global__ void __launch_bounds__(kVecBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_amplitude_vec(VecArgs A, Eval ev) {
    extern __shared__ double smem[];
    load_bm_table(smem, kVecBlock);
    __syncthreads();
    for (uint64_t c = blockIdx.x; c < A.n_chunks; c += gridDim.x) process_chunk<DIM, U, Eval>(ev, A, c, smem);
}

// ---------------------------------------------------------------------------- dispatch
template <int DIM, int U, class Eval>
inline hipError_t launch_one(const VecArgs& A, const Eval& ev, int grid, hipStream_t st) {
    const size_t lds = vec_lds_bytes(DIM, A.D, A.s);
    hipLaunchKernelGGL((k_amplitude_vec<DIM, U, Eval>), dim3(grid), dim3(kVecBlock), lds, st, A, ev);
    return hipGetLastError();
}

template <int DIM, int U, class Eval>
inline int resident_one(size_t lds, int device) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_amplitude_vec<DIM, U, Eval>, kVecBlock, lds) != hipSuccess)
        per_cu = 1;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) ncu = 256;
    return (per_cu < 1 ? 1 : per_cu) * ncu;
}

template <int DIM>
inline hipError_t launch_rt(const VecArgs& A, int U, int grid, hipStream_t st) {
    const RadialEvalRT<DIM> ev{A.tab, A.shape, A.stride};
    switch (U) {
        case 1: return launch_one<DIM, 1>(A, ev, grid, st);
        case 2: return launch_one<DIM, 2>(A, ev, grid, st);
        case 3: return launch_one<DIM, 3>(A, ev, grid, st);
        case 4: return launch_one<DIM, 4>(A, ev, grid, st);
        default: return hipErrorInvalidValue;
    }
}

template <int DIM>
inline int resident_rt(int U, size_t lds, int device) {
    switch (U) {
        case 1: return resident_one<DIM, 1, RadialEvalRT<DIM>>(lds, device);
        case 2: return resident_one<DIM, 2, RadialEvalRT<DIM>>(lds, device);
        case 3: return resident_one<DIM, 3, RadialEvalRT<DIM>>(lds, device);
        default: return resident_one<DIM, 4, RadialEvalRT<DIM>>(lds, device);
    }
}

// UMAX: the deepest subtree instantiated by the caller's translation unit (the deepest of all may be
// compiled in a unit of its own).
template <int DIM, int UMAX = poly_subtree_levels(DIM)>
inline hipError_t launch_poly(const VecArgs& A, int U, int grid, hipStream_t st) {
    const PolyEvalRT<DIM> ev{A.tab, A.shape, A.stride};
    switch (U) {
        case 1: return launch_one<DIM, 1>(A, ev, grid, st);
        case 2: return launch_one<DIM, 2>(A, ev, grid, st);
        case 3: return launch_one<DIM, 3>(A, ev, grid, st);
        case 4: if constexpr (UMAX >= 4) return launch_one<DIM, 4>(A, ev, grid, st); break;
        case 5: if constexpr (UMAX >= 5) return launch_one<DIM, 5>(A, ev, grid, st); break;
        case 6: if constexpr (UMAX >= 6) return launch_one<DIM, 6>(A, ev, grid, st); break;
        case 7: if constexpr (UMAX >= 7) return launch_one<DIM, 7>(A, ev, grid, st); break;
        default: break;
    }
    return hipErrorInvalidValue;
}

template <int DIM, int UMAX = poly_subtree_levels(DIM)>
inline int resident_poly(int U, size_t lds, int device) {
    switch (U) {
        case 1: return resident_one<DIM, 1, PolyEvalRT<DIM>>(lds, device);
        case 2: return resident_one<DIM, 2, PolyEvalRT<DIM>>(lds, device);
        case 4: if constexpr (UMAX >= 4) return resident_one<DIM, 4, PolyEvalRT<DIM>>(lds, device); break;
        case 5: if constexpr (UMAX >= 5) return resident_one<DIM, 5, PolyEvalRT<DIM>>(lds, device); break;
        case 6: if constexpr (UMAX >= 6) return resident_one<DIM, 6, PolyEvalRT<DIM>>(lds, device); break;
        case 7: if constexpr (UMAX >= 7) return resident_one<DIM, 7, PolyEvalRT<DIM>>(lds, device); break;
        default: break;
    }
    return resident_one<DIM, 3, PolyEvalRT<DIM>>(lds, device);
}

template <int DIM, int P>
inline hipError_t launch_spec(const VecArgs& A, int p, int grid, hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p != P) return launch_spec<DIM, P + 1>(A, p, grid, st);
        const RadialEval<P, DIM> ev{A.tab};
        return launch_one<DIM, kVecU>(A, ev, grid, st);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int DIM, int P>
inline int resident_spec(int p, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p != P) return resident_spec<DIM, P + 1>(p, lds, device);
        return resident_one<DIM, kVecU, RadialEval<P, DIM>>(lds, device);
    } else {
        return 256;
    }
}

}  // namespace vec
}  // namespace pimc
