// The bisection walker and estimation kernel template of the PIMC amplitude (Sec. 4 of Balaz et al.)
// for gfx950, shared by the translation units that instantiate it with their slice evaluators.
//
// One lane owns one path at a time. The path is built depth first, left to right, and never
// leaves the lane: the bottom U bisection levels of each subtree live in registers (2^U + 1
// points), the levels above them keep one pending right endpoint and one cached sibling normal per
// level in LDS. Every level-n slice is evaluated as soon as both of its endpoints exist, which for
// n < s is the moment its midpoint (a level-(n+1) node) is generated; the level-s slices are the
// leaves. Levels D..s of a subtree are evaluated coefficient-major over the slices of the level
// (up to BATCH at once) so that each wave-uniform table coefficient feeds independent FMA chains.
//
// Per level, each path's weight enters as d = exp(-(S_n - S_ref,n)) - 1 (a shift by the
// straight-line action only changes rounding); a wave butterfly sums d and d^2 over a group of 64
// consecutive paths, and lane 0 adds the group sum to the group's accumulator slot (canonical
// chunk, pimc_internal.hpp); at the end of a chunk the slots are added in slot order and written to
// the chunk's record. The chunk records are summed in chunk order by k_seg_reduce, so the result is
// bitwise independent of the launch shape, of the grid size, of which workgroup ran which chunk,
// and of whether the run was launched alone or as one task of a batch.
#pragma once

#include <hip/hip_runtime.h>

#include "pimc_internal.hpp"

namespace pimc {

// ---------------------------------------------------------------------------- subtree (registers)
template <int U, int L, class Src>
__device__ __forceinline__ void gen_level(const AmpArgs& A, const Src& src, uint32_t root, int D,
                                          double (&q)[(1 << U) + 1]) {
    if constexpr (L <= U) {
        constexpr int step = 1 << (U - L);
        const double sg = as_const(A.sig)[D + L];
#pragma unroll
        for (int i2 = 0; i2 < (1 << (L - 2)); ++i2) {
            const uint32_t parent = (root << (L - 2)) + uint32_t(i2);   // node of sub-level L-1
            double ze, zo;
            src.pair(parent, ze, zo);                                    // children 2*parent, 2*parent+1
            const int jl = (4 * i2 + 1) * step;
            const int jr = (4 * i2 + 3) * step;
            q[jl] = sg * ze + 0.5 * (q[jl - step] + q[jl + step]);
            q[jr] = sg * zo + 0.5 * (q[jr - step] + q[jr + step]);
        }
        gen_level<U, L + 1, Src>(A, src, root, D, q);
    }
}

// Add the 2^L slices of sub-level L (point stride 2^(U-L)) at tree level `level` to S, left to right.
template <int U, int BATCH, int L, class Eval>
__device__ __forceinline__ void level_sum(const Eval& ev, int level, const double (&q)[(1 << U) + 1], double& S) {
    constexpr int W = 1 << L;
    constexpr int ST = 1 << (U - L);
    constexpr int B = W < BATCH ? W : BATCH;
#pragma unroll
    for (int b0 = 0; b0 < W; b0 += B) {
        double qa[B], qb[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            qa[i] = q[(b0 + i) * ST];
            qb[i] = q[(b0 + i + 1) * ST];
        }
        ev.template eval<B>(level, qa, qb, S);
    }
}

template <int U, int BATCH, int L, class Eval>
__device__ __forceinline__ void hier_levels(const Eval& ev, int D, const double (&q)[(1 << U) + 1],
                                            double (&Ssub)[U + 1]) {
    if constexpr (L < U) {
        level_sum<U, BATCH, L, Eval>(ev, D + L, q, Ssub[L]);
        hier_levels<U, BATCH, L + 1, Eval>(ev, D, q, Ssub);
    }
}

// Subtree rooted at heap node `root` (level D+1) over the level-D slice (qL, qR) with root normal z.
template <int U, int BATCH, class Eval, class Src>
__device__ __forceinline__ void run_subtree(const Eval& ev_in, const AmpArgs& A, const Src& src,
                                            uint32_t root, int D, double qL, double qR, double zroot,
                                            double (&Ssub)[U + 1]) {
    Eval ev = ev_in;
    ev.launder();
    double q[(1 << U) + 1];
    q[0] = qL;
    q[1 << U] = qR;
    q[1 << (U - 1)] = as_const(A.sig)[D + 1] * zroot + 0.5 * (qL + qR);
    gen_level<U, 2, Src>(A, src, root, D, q);
    if (A.hier) hier_levels<U, BATCH, 0, Eval>(ev, D, q, Ssub);
    level_sum<U, BATCH, U, Eval>(ev, D + U, q, Ssub[U]);
}

// ---------------------------------------------------------------------------- one path
// top: this lane's LDS slots (stride BS): S_top[n] at slot n (n < D), pending right endpoint
// of level L at slot D+L, pending normal at slot 2D+1+L (L = 2..D).
template <int U, int BS, int BATCH, class Eval, class Src>
__device__ __forceinline__ void walk_path(const Eval& ev, const AmpArgs& A, const Src& src, double* top,
                                          double (&Ssub)[U + 1]) {
    const int D = A.D;
#pragma unroll
    for (int j = 0; j <= U; ++j) Ssub[j] = 0.0;
    double z0_unused, z1;
    src.pair(0u, z0_unused, z1);                      // node 1 = sine output of call 0
    if (D == 0) {
        run_subtree<U, BATCH, Eval, Src>(ev, A, src, 1u, 0, A.a, A.b, z1, Ssub);
        return;
    }
    for (int n = 0; n < D; ++n) top[n * BS] = 0.0;
    double* R = top + D * BS;
    double* Z = top + (2 * D + 1) * BS;
    const uint32_t nTop = 1u << (D - 1);             // level-D nodes nTop .. 2 nTop - 1
    double qlast = A.a;
    for (uint32_t J = 0; J < nTop; ++J) {
        int L;
        uint32_t node;
        double qL = qlast, qR, z;
        if (J == 0) {
            L = 1;
            node = 1u;
            qR = A.b;
            z = z1;
        } else {
            const int t = __builtin_ctz(J);
            L = D - t;
            node = (nTop + J) >> t;
            qR = R[L * BS];
            z = Z[L * BS];
        }
        double qm, zl, zr;
        while (true) {
            if (A.hier) {
                const double qa1[1] = {qL};
                const double qb1[1] = {qR};
                double St = top[(L - 1) * BS];
                ev.template eval<1>(L - 1, qa1, qb1, St);
                top[(L - 1) * BS] = St;
            }
            qm = as_const(A.sig)[L] * z + 0.5 * (qL + qR);
            src.pair(node, zl, zr);
            if (L == D) break;
            R[(L + 1) * BS] = qR;                     // right child of `node`: (qm, qR), normal zr
            Z[(L + 1) * BS] = zr;
            qR = qm;
            z = zl;
            node = 2u * node;
            ++L;
        }
        run_subtree<U, BATCH, Eval, Src>(ev, A, src, 2u * node, D, qL, qm, zl, Ssub);
        run_subtree<U, BATCH, Eval, Src>(ev, A, src, 2u * node + 1u, D, qm, qR, zr, Ssub);
        qlast = qR;
    }
}

// ---------------------------------------------------------------------------- estimation kernel
// Adds the group sums of level n (d and d^2 by a wave butterfly, the non-finite count by a ballot)
// to the accumulator slot `a` (lane 0 only).
__device__ __forceinline__ void reduce_level(const AmpArgs& A, double* a, int lane, int n, double S, bool valid) {
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

// One canonical chunk c of the run described by A: paths c*kChunkPaths + 64 g + lane, groups
// g = wave, wave + W, ... (W waves per workgroup). Writes the chunk's four sums per evaluated level
// to A.partials[(slot * n_chunks + c) * 4] (slot = level with every level evaluated, else 0 for
// level s) and/or the per-path level actions to A.dump. smem: the Box-Muller table, the per-lane
// stack, the accumulator slots.
template <class S, class Eval>
__device__ __forceinline__ void process_chunk(const Eval& ev, const AmpArgs& A, uint64_t c, double* smem) {
    constexpr int U = S::U;
    constexpr int BS = S::BS;
    constexpr int WAVES = BS / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int D = A.D;
    const int nlev = A.s + 1;
    const double* bm = smem;
    double* top = smem + kBoxMullerTable + tid;
    double* acc = smem + kBoxMullerTable + size_t(3 * D + 2) * BS;
    const uint64_t first = c * kChunkPaths;
    if (A.partials) {
        for (int i = tid; i < kChunkSlots * nlev * 3; i += BS) acc[i] = 0.0;
        __syncthreads();
    }
    for (int g = wave; g < kChunkGroups; g += WAVES) {
        const uint64_t group0 = first + uint64_t(g) * 64;
        if (group0 >= A.n_paths) break;                   // wave-uniform: the rest of the chunk is empty
        const uint64_t local = group0 + uint64_t(lane);
        const bool valid = local < A.n_paths;
        double Ssub[U + 1];
        const PhiloxSource src{A.key, path_rng(A.key, A.first_path + local), bm};
        walk_path<U, BS, S::BATCH, Eval, PhiloxSource>(ev, A, src, top, Ssub);
        if (A.dump && valid) {
            double* o = A.dump + local * uint64_t(nlev);
            for (int n = 0; n < D; ++n) o[n] = A.hier ? top[n * BS] : 0.0;
#pragma unroll
            for (int j = 0; j <= U; ++j) o[D + j] = (A.hier || j == U) ? Ssub[j] : 0.0;
        }
        if (A.partials) {
            double* a = acc + (g % kChunkSlots) * nlev * 3;
            if (A.hier) {
                for (int n = 0; n < D; ++n) reduce_level(A, a + n * 3, lane, n, top[n * BS], valid);
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

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return (uint64_t(hi) << 32) | lo;
}

// With A.queue: a persistent kernel whose workgroups take chunks one at a time from the counter
// until it passes n_chunks (the work balances itself across CUs and XCDs; every wave of a workgroup
// reaches the exit test with the same value). Without: a grid-stride loop over the chunks.
template <class S, class Eval>
__global__ void __launch_bounds__(S::BS) __attribute__((amdgpu_waves_per_eu(S::WPE)))
k_amplitude(AmpArgs A, Eval ev) {
    extern __shared__ double smem[];
    __shared__ unsigned long long s_chunk;
    load_bm_table(smem, S::BS);
    if (A.queue) {
        while (true) {
            __syncthreads();
            if (threadIdx.x == 0) s_chunk = atomicAdd(A.queue, 1ull);
            __syncthreads();
            const uint64_t c = uniform_u64(s_chunk);
            if (c >= A.n_chunks) break;
            process_chunk<S, Eval>(ev, A, c, smem);
        }
    } else {
        __syncthreads();
        for (uint64_t c = blockIdx.x; c < A.n_chunks; c += gridDim.x) process_chunk<S, Eval>(ev, A, c, smem);
    }
}

template <class S, class Eval>
inline hipError_t launch_one(const AmpArgs& A, const Eval& ev, int grid, hipStream_t st) {
    const size_t lds = amp_lds_bytes(A.D, A.s, S::BS);
    hipLaunchKernelGGL((k_amplitude<S, Eval>), dim3(grid), dim3(S::BS), lds, st, A, ev);
    return hipGetLastError();
}

template <class S, class Eval>
inline int resident_one(size_t lds, int device) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_amplitude<S, Eval>, S::BS, lds) != hipSuccess)
        per_cu = 1;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) ncu = 256;
    return (per_cu < 1 ? 1 : per_cu) * ncu;
}

}  // namespace pimc
