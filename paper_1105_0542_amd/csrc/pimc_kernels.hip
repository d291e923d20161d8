// Estimation kernels of the bisection PIMC amplitude (Sec. 4 of Balaz et al.) for gfx950.
//
// One lane owns one path at a time. The path is built depth first, left to right, and never
// leaves the lane: the bottom U bisection levels of each subtree live in registers (2^U + 1
// points), the levels above them keep one pending right endpoint and one cached sibling normal per
// level in LDS. Every level-n slice is evaluated as soon as both of its endpoints exist, which for
// n < s is the moment its midpoint (a level-(n+1) node) is generated; the level-s slices are the
// leaves. Levels D..s of a subtree are evaluated coefficient-major over all slices of the level
// (up to 8 at once) so that each wave-uniform table coefficient feeds independent FMA chains.
//
// Per level, each path's weight enters as d = exp(-(S_n - S_ref,n)) - 1 (a shift by the
// straight-line action only changes rounding); a wave butterfly sums d and d^2, lane 0 adds the
// wave sum to a per-wave LDS accumulator, and at the end of a canonical chunk (kBlock*ppl
// consecutive paths, lanes in a fixed order) the four wave accumulators are added in wave order and
// written to the chunk's slot. The chunk slots are summed in chunk order by k_seg_reduce, so the
// result is bitwise independent of the grid size, of which workgroup ran which chunk, and of
// whether the run was launched alone or as one task of a batch.
#include <hip/hip_runtime.h>

#include "pimc_internal.hpp"

// Occupancy target of the estimation kernel (waves per SIMD) and the number of slices evaluated
// together, coefficient-major (measured best on MI355X at p = 18: 2 waves, all 16 leaves at once).
#ifndef PIMC_WAVES_PER_EU
#define PIMC_WAVES_PER_EU 2
#endif
#ifndef PIMC_BATCH
#define PIMC_BATCH 16
#endif

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
template <int U, int L, class Eval>
__device__ __forceinline__ void level_sum(const Eval& ev, int level, const double (&q)[(1 << U) + 1], double& S) {
    constexpr int W = 1 << L;
    constexpr int ST = 1 << (U - L);
    constexpr int B = W < PIMC_BATCH ? W : PIMC_BATCH;
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

template <int U, int L, class Eval>
__device__ __forceinline__ void hier_levels(const Eval& ev, int D, const double (&q)[(1 << U) + 1],
                                            double (&Ssub)[U + 1]) {
    if constexpr (L < U) {
        level_sum<U, L, Eval>(ev, D + L, q, Ssub[L]);
        hier_levels<U, L + 1, Eval>(ev, D, q, Ssub);
    }
}

// Subtree rooted at heap node `root` (level D+1) over the level-D slice (qL, qR) with root normal z.
template <int U, class Eval, class Src>
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
    if (A.hier) hier_levels<U, 0, Eval>(ev, D, q, Ssub);
    level_sum<U, U, Eval>(ev, D + U, q, Ssub[U]);
}

// ---------------------------------------------------------------------------- one path
// top: this lane's LDS slots (stride kBlock): S_top[n] at slot n (n < D), pending right endpoint
// of level L at slot D+L, pending normal at slot 2D+1+L (L = 2..D).
template <int U, class Eval, class Src>
__device__ __forceinline__ void walk_path(const Eval& ev, const AmpArgs& A, const Src& src, double* top,
                                          double (&Ssub)[U + 1]) {
    const int D = A.D;
#pragma unroll
    for (int j = 0; j <= U; ++j) Ssub[j] = 0.0;
    double z0_unused, z1;
    src.pair(0u, z0_unused, z1);                      // node 1 = sine output of call 0
    if (D == 0) {
        run_subtree<U, Eval, Src>(ev, A, src, 1u, 0, A.a, A.b, z1, Ssub);
        return;
    }
    for (int n = 0; n < D; ++n) top[n * kBlock] = 0.0;
    double* R = top + D * kBlock;
    double* Z = top + (2 * D + 1) * kBlock;
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
            qR = R[L * kBlock];
            z = Z[L * kBlock];
        }
        double qm, zl, zr;
        while (true) {
            if (A.hier) {
                const double qa1[1] = {qL};
                const double qb1[1] = {qR};
                double St = top[(L - 1) * kBlock];
                ev.template eval<1>(L - 1, qa1, qb1, St);
                top[(L - 1) * kBlock] = St;
            }
            qm = as_const(A.sig)[L] * z + 0.5 * (qL + qR);
            src.pair(node, zl, zr);
            if (L == D) break;
            R[(L + 1) * kBlock] = qR;                 // right child of `node`: (qm, qR), normal zr
            Z[(L + 1) * kBlock] = zr;
            qR = qm;
            z = zl;
            node = 2u * node;
            ++L;
        }
        run_subtree<U, Eval, Src>(ev, A, src, 2u * node, D, qL, qm, zl, Ssub);
        run_subtree<U, Eval, Src>(ev, A, src, 2u * node + 1u, D, qm, qR, zr, Ssub);
        qlast = qR;
    }
}

// ---------------------------------------------------------------------------- estimation kernel
__device__ __forceinline__ void reduce_level(const AmpArgs& A, double* acc, int nlev, int wave, int lane,
                                             int n, double S, bool valid) {
    const double d = valid ? expm1(-(S - as_const(A.shift)[n])) : 0.0;
    const bool bad = valid && !isfinite(d);
    const double sd = wave_sum(d);
    const double sd2 = wave_sum(d * d);
    const unsigned long long badmask = __ballot(bad);
    if (lane == 0) {
        double* a = acc + (wave * nlev + n) * 3;
        a[0] += sd;
        a[1] += sd2;
        a[2] += double(__popcll(badmask));
    }
}

// One canonical chunk c of the run described by A: paths c*CH .. c*CH+CH-1 (CH = kBlock * ppl),
// lane tid takes paths c*CH + r*kBlock + tid for r = 0..ppl-1 in order. Writes the chunk's four
// sums per evaluated level to A.partials[(slot * n_chunks + c) * 4] (slot = level with every level
// evaluated, else 0 for level s) and/or the per-path level actions to A.dump.
template <int U, class Eval>
__device__ __forceinline__ void process_chunk(const Eval& ev, const AmpArgs& A, uint64_t c, double* smem) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int D = A.D;
    const int nlev = A.s + 1;
    double* top = smem + tid;
    double* acc = smem + size_t(3 * D + 2) * kBlock;
    const uint64_t CH = uint64_t(kBlock) * A.ppl;
    if (A.partials) {
        for (int i = tid; i < 4 * nlev * 3; i += kBlock) acc[i] = 0.0;
        __syncthreads();
    }
    for (uint32_t r = 0; r < A.ppl; ++r) {
        const uint64_t local = c * CH + uint64_t(r) * kBlock + uint64_t(tid);
        const bool valid = local < A.n_paths;
        double Ssub[U + 1];
        const PhiloxSource src{A.key, path_rng(A.key, A.first_path + local)};
        walk_path<U, Eval, PhiloxSource>(ev, A, src, top, Ssub);
        if (A.dump && valid) {
            double* o = A.dump + local * uint64_t(nlev);
            for (int n = 0; n < D; ++n) o[n] = A.hier ? top[n * kBlock] : 0.0;
#pragma unroll
            for (int j = 0; j <= U; ++j) o[D + j] = (A.hier || j == U) ? Ssub[j] : 0.0;
        }
        if (A.partials) {
            if (A.hier) {
                for (int n = 0; n < D; ++n) reduce_level(A, acc, nlev, wave, lane, n, top[n * kBlock], valid);
#pragma unroll
                for (int j = 0; j < U; ++j) reduce_level(A, acc, nlev, wave, lane, D + j, Ssub[j], valid);
            }
            reduce_level(A, acc, nlev, wave, lane, D + U, Ssub[U], valid);
        }
    }
    if (A.partials) {
        __syncthreads();
        const int slots = A.hier ? nlev : 1;
        if (tid < slots) {
            const int lev = A.hier ? tid : nlev - 1;
            const uint64_t rem = A.n_paths - c * CH;
            const double cnt = double(rem < CH ? rem : CH);
            double s1 = 0.0, s2 = 0.0, nb = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) {
                const double* a = acc + (w * nlev + lev) * 3;
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

template <int U, class Eval>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PIMC_WAVES_PER_EU)))
k_amplitude(AmpArgs A, Eval ev) {
    extern __shared__ double smem[];
    for (uint64_t c = blockIdx.x; c < A.n_chunks; c += gridDim.x) process_chunk<U, Eval>(ev, A, c, smem);
}

// ---------------------------------------------------------------------------- batched tasks
// Persistent kernel over the (task, chunk) items of one effective-action level p: each workgroup
// takes `grab` consecutive items at a time from an atomic counter until the queue is empty (every
// wave of every workgroup reaches the exit test with the same value). Items are numbered task by
// task (task t owns items item0[t] .. item0[t] + n_chunks[t] - 1), so an item maps to its task by
// binary search over the wave-uniform task records; the chunk itself is processed by the same code
// as a single-task launch, so results do not depend on which workgroup took which item.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return (uint64_t(hi) << 32) | lo;
}

template <int U, class Eval>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PIMC_WAVES_PER_EU)))
k_batch(const BatchTask* __restrict__ tasks, int n_tasks, uint64_t n_items, unsigned long long* queue,
        uint32_t grab, RngKey key, int hier, Eval ev0) {
    extern __shared__ double smem[];
    __shared__ unsigned long long s_item;
    const const_ptr<BatchTask> T = as_const(tasks);
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(queue, (unsigned long long)grab);
        __syncthreads();
        const uint64_t first = uniform_u64(s_item);
        if (first >= n_items) break;
        const uint64_t last = first + grab < n_items ? first + grab : n_items;
        for (uint64_t item = first; item < last; ++item) {
            int lo = 0, hi = n_tasks - 1;                  // last task with item0 <= item
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (T[mid].item0 <= item) lo = mid; else hi = mid - 1;
            }
            AmpArgs A;
            A.tab64 = T[lo].tab;
            A.tab32 = nullptr;
            A.gdeg = nullptr;
            A.gK = 0;
            A.gstride = 0;
            A.a = T[lo].a;
            A.b = T[lo].b;
            A.sig = T[lo].sig;
            A.shift = T[lo].shift;
            A.key = key;
            A.key.stream = T[lo].stream;
            A.first_path = 0;
            A.n_paths = T[lo].n_paths;
            A.n_chunks = T[lo].n_chunks;
            A.ppl = T[lo].ppl;
            A.s = T[lo].s;
            A.D = T[lo].s - U;
            A.hier = hier;
            A.partials = T[lo].partials;
            A.dump = nullptr;
            Eval ev = ev0;
            ev.tab = T[lo].tab;
            process_chunk<U, Eval>(ev, A, item - T[lo].item0, smem);
        }
    }
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------- raw normals
// One thread per (path, node pair): nodes 2j and 2j+1 of path first_path + i, written where
// 1 <= node <= n_nodes.
__global__ void __launch_bounds__(kBlock) k_normals(RngKey key, uint64_t first_path, uint64_t k_paths,
                                                    uint32_t n_nodes, double* __restrict__ out) {
    const uint32_t pairs = n_nodes / 2 + 1;
    const uint64_t gid = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (gid >= k_paths * pairs) return;
    const uint64_t i = gid / pairs;
    const uint32_t j = uint32_t(gid % pairs);
    const PathRng pr = path_rng(key, first_path + i);
    double ze, zo;
    normal_pair(key, pr, j, ze, zo);
    double* o = out + i * n_nodes;
    const uint32_t he = 2 * j, ho = 2 * j + 1;
    if (he >= 1 && he <= n_nodes) o[he - 1] = ze;
    if (ho <= n_nodes) o[ho - 1] = zo;
}

hipError_t launch_normals(const RngKey& key, uint64_t first_path, uint64_t k_paths, uint32_t n_nodes, double* out,
                          hipStream_t st) {
    const uint64_t work = k_paths * (uint64_t(n_nodes) / 2 + 1);
    const uint64_t blocks = (work + kBlock - 1) / kBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_normals, dim3(uint32_t(blocks)), dim3(kBlock), 0, st, key, first_path, k_paths, n_nodes, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- chunk reduction
// Canonical reduction: segment i (one level of one run) is the sequence of chunk sums
// partials[base[i] + c*4 .. +3], c = 0..len[i]-1. One workgroup of kBlock threads per segment:
// thread t adds chunks t, t + kBlock, ... in order, then a fixed halving tree over the threads.
// The order depends only on the chunk count, so any run -- single or one task of a batch, any
// grid -- gives the same bits for the same chunks.
__global__ void __launch_bounds__(kBlock) k_seg_reduce(const double* __restrict__ partials,
                                                       const uint64_t* __restrict__ base,
                                                       const uint64_t* __restrict__ len,
                                                       double* __restrict__ out) {
    __shared__ double red[4][kBlock];
    const uint64_t seg = blockIdx.x;
    const int tid = threadIdx.x;
    const double* p = partials + base[seg];
    const uint64_t n = len[seg];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint64_t c = tid; c < n; c += kBlock) {
#pragma unroll
        for (int j = 0; j < 4; ++j) s[j] += p[c * 4 + j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) red[j][tid] = s[j];
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int j = 0; j < 4; ++j) red[j][tid] += red[j][tid + w];
        }
        __syncthreads();
    }
    if (tid < 4) out[seg * 4 + tid] = red[tid][0];
}

// ---------------------------------------------------------------------------- dispatch
template <int U, class Eval>
static hipError_t launch_one(const AmpArgs& A, const Eval& ev, int grid, hipStream_t st) {
    const size_t lds = amp_lds_bytes(A.D, A.s);
    hipLaunchKernelGGL((k_amplitude<U, Eval>), dim3(grid), dim3(kBlock), lds, st, A, ev);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_quartic(const AmpArgs& A, bool fp32, int grid, hipStream_t st) {
    if (fp32) {
        QuarticEval32<P> ev{A.tab32};
        return launch_one<4>(A, ev, grid, st);
    }
    QuarticEval64<P> ev{A.tab64};
    return launch_one<4>(A, ev, grid, st);
}

template <bool EVEN>
static hipError_t launch_generic(const AmpArgs& A, int U, int grid, hipStream_t st) {
    GenericEval64<EVEN> ev{A.tab64, A.gdeg, A.gK, A.gstride};
    switch (U) {
        case 1: return launch_one<1>(A, ev, grid, st);
        case 2: return launch_one<2>(A, ev, grid, st);
        case 3: return launch_one<3>(A, ev, grid, st);
        case 4: return launch_one<4>(A, ev, grid, st);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_tanh(const AmpArgs& A, int U, int grid, hipStream_t st) {
    TanhEval64 ev{A.tab64, A.gdeg, A.gK, A.gstride, A.alpha};
    switch (U) {
        case 1: return launch_one<1>(A, ev, grid, st);
        case 2: return launch_one<2>(A, ev, grid, st);
        case 3: return launch_one<3>(A, ev, grid, st);
        case 4: return launch_one<4>(A, ev, grid, st);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_general(const AmpArgs& A, int U, int grid, hipStream_t st) {
    GeneralEval64 ev{A.gen};
    switch (U) {
        case 1: return launch_one<1>(A, ev, grid, st);
        case 2: return launch_one<2>(A, ev, grid, st);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t quartic_dispatch(const AmpArgs& A, bool fp32, int p, int grid, hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p == P) return launch_quartic<P>(A, fp32, grid, st);
        return quartic_dispatch<P + 1>(A, fp32, p, grid, st);
    } else {
        return hipErrorInvalidValue;
    }
}

hipError_t launch_amplitude(const AmpArgs& A, EvalKind kind, int p, int U, int grid, hipStream_t st) {
    switch (kind) {
        case EvalKind::Quartic64:
        case EvalKind::Quartic32:
            if (U != 4) return hipErrorInvalidValue;
            return quartic_dispatch<1>(A, kind == EvalKind::Quartic32, p, grid, st);
        case EvalKind::GenericEven64: return launch_generic<true>(A, U, grid, st);
        case EvalKind::GenericOdd64: return launch_generic<false>(A, U, grid, st);
        case EvalKind::Tanh64: return launch_tanh(A, U, grid, st);
        case EvalKind::General64: return launch_general(A, U, grid, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_seg_reduce(const double* partials, const uint64_t* base, const uint64_t* len, uint64_t n_seg,
                             double* out, hipStream_t st) {
    if (n_seg == 0) return hipSuccess;
    if (n_seg > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_seg_reduce, dim3(uint32_t(n_seg)), dim3(kBlock), 0, st, partials, base, len, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3((n + 63) / 64), dim3(64), 0, st, p, n, v);
    return hipGetLastError();
}

template <int P>
static hipError_t batch_quartic(const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue,
                                uint32_t grab, RngKey key, int hier, int p, int grid, size_t lds, hipStream_t st) {
    if constexpr (P <= kMaxP) {
        if (p != P) return batch_quartic<P + 1>(tasks, n_tasks, n_items, queue, grab, key, hier, p, grid, lds, st);
        QuarticEval64<P> ev{nullptr};
        hipLaunchKernelGGL((k_batch<4, QuarticEval64<P>>), dim3(grid), dim3(kBlock), lds, st, tasks, n_tasks, n_items,
                           queue, grab, key, hier, ev);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

hipError_t launch_batch(const BatchTask* tasks, int n_tasks, uint64_t n_items, unsigned long long* queue, uint32_t grab,
                        const RngKey& key, int hier, int p, int grid, size_t lds, hipStream_t st) {
    return batch_quartic<1>(tasks, n_tasks, n_items, queue, grab, key, hier, p, grid, lds, st);
}

template <int P>
static int batch_resident(int p, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p != P) return batch_resident<P + 1>(p, lds, device);
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<4, QuarticEval64<P>>, kBlock, lds) != hipSuccess)
            per_cu = 1;
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) ncu = 256;
        return (per_cu < 1 ? 1 : per_cu) * ncu;
    } else {
        return 256;
    }
}

int batch_resident_blocks(int p, size_t lds_bytes, int device) { return batch_resident<1>(p, lds_bytes, device); }

template <int U, class Eval>
static int resident_one(size_t lds, int device) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_amplitude<U, Eval>, kBlock, lds) != hipSuccess) per_cu = 1;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) ncu = 256;
    return (per_cu < 1 ? 1 : per_cu) * ncu;
}

template <int P>
static int resident_quartic(bool fp32, int p, size_t lds, int device) {
    if constexpr (P <= kMaxP) {
        if (p == P) return fp32 ? resident_one<4, QuarticEval32<P>>(lds, device) : resident_one<4, QuarticEval64<P>>(lds, device);
        return resident_quartic<P + 1>(fp32, p, lds, device);
    } else {
        return 256;
    }
}

int amplitude_resident_blocks(EvalKind kind, int p, int U, size_t lds_bytes, int device) {
    switch (kind) {
        case EvalKind::Quartic64: return resident_quartic<1>(false, p, lds_bytes, device);
        case EvalKind::Quartic32: return resident_quartic<1>(true, p, lds_bytes, device);
        case EvalKind::GenericEven64:
        case EvalKind::GenericOdd64:
            switch (U) {
                case 1: return resident_one<1, GenericEval64<true>>(lds_bytes, device);
                case 2: return resident_one<2, GenericEval64<true>>(lds_bytes, device);
                case 3: return resident_one<3, GenericEval64<true>>(lds_bytes, device);
                default: return resident_one<4, GenericEval64<true>>(lds_bytes, device);
            }
        case EvalKind::Tanh64:
            switch (U) {
                case 1: return resident_one<1, TanhEval64>(lds_bytes, device);
                case 2: return resident_one<2, TanhEval64>(lds_bytes, device);
                case 3: return resident_one<3, TanhEval64>(lds_bytes, device);
                default: return resident_one<4, TanhEval64>(lds_bytes, device);
            }
        case EvalKind::General64:
            return U == 1 ? resident_one<1, GeneralEval64>(lds_bytes, device)
                          : resident_one<2, GeneralEval64>(lds_bytes, device);
    }
    return 256;
}

}  // namespace pimc
