// Learned-proposal kernels (gfx950): affine couplings over the bisection normals.
//
// Per-path tensors are feature-major, X[(h-1)*ld + path] for heap node h, so every per-coordinate
// access of consecutive paths is coalesced. The conditioner inputs are rounded to bfloat16, the two
// MLP layers run on v_mfma_f32_16x16x32_bf16 as weights x activations (operand lanes:
// A[l%16][8(l/16)+i], B[8(l/16)+i][l%16], C[4(l/16)+j][l%16]), and the MFMA output layout puts
// s_hat and t of the same (coordinate, path) in the same lane, so the FP64 affine update and
// log-det follow without another exchange. The training backward uses v_mfma_f32_16x16x4f32
// (A[l%16][l/16], B[l/16][l%16], the same C layout).
#include <hip/hip_runtime.h>

#include "pimc_flow.hpp"
#include "pimc_internal.hpp"
#include "pimc_math.hpp"

namespace pimc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));


// C(16x16) += A(16 rows x K) * BT(16 rows x K)^T; rows K-contiguous, strides in elements.
__device__ __forceinline__ floatx4 mma16(const __bf16* A, int lda, const __bf16* BT, int ldb, int K, floatx4 c) {
    const int l = threadIdx.x & 63;
    for (int ks = 0; ks < K; ks += 32) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(A + (l & 15) * lda + ks + 8 * (l >> 4));
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(BT + (l & 15) * ldb + ks + 8 * (l >> 4));
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    return c;
}

// Conditioner nonlinearities in FP32 from the hardware exp2 and reciprocal (about 1 ulp each; the
// conditioner only has to be deterministic, its rounding never biases the estimator).
__device__ __forceinline__ float sigmoid_fast(float v) { return __builtin_amdgcn_rcpf(1.0f + __expf(-v)); }
__device__ __forceinline__ float silu(float v) { return v * sigmoid_fast(v); }
// tanh x = 1 - 2 / (e^{2x} + 1); |x| clamped to 15, where tanh is 1 in FP32.
__device__ __forceinline__ float tanh_fast(float x) {
    x = fminf(fmaxf(x, -15.0f), 15.0f);
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * x) + 1.0f);
}
// e^s in FP64 for |s| <= 2 (the affine log-scales): Cody-Waite reduction s = k ln2 + r with
// |r| <= ln2/2 (k*kLn2Hi exact), e^r by its Taylor series to degree 13 (truncation < 5e-18), and
// the exact scaling by 2^k. Error about 1 ulp.
__device__ __forceinline__ double exp_logscale(double s) {
    const double k = rint(s * 1.4426950408889634);
    double r = fma(-k, kLn2Hi, s);
    r = fma(-k, kLn2Lo, r);
    double p = 1.0 / 6227020800.0;                                   // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, int(k));
}

// ------------------------------------------------------------------------------------ training
// The training step works on tiles of kTP = 16 paths, the MFMA's column count (256 workgroups of
// four waves at a batch of 4096):
//  * k_train_fwd carries a tile through the base normals and every coupling in LDS -- the same
//    bf16 MFMA products and FP64 affine update as the fused estimation kernel -- and keeps each
//    layer's input X_c (FP64 planes [h-1][path]) for the backward;
//  * k_train_bwd recomputes each layer from X_c with the same products and back-propagates through
//    it on FP32 MFMA (v_mfma_f32_16x16x4f32): the bf16 weights and activations of the forward enter
//    as exact FP32 values, so the gradient is the derivative of the map the forward computes, up to
//    FP32 accumulation. It writes, per layer, the output and pre-activation gradients (FP32) and the
//    conditioner inputs and hidden activations (bf16) as [row][path] planes;
//  * k_flow_wgrad_part / k_flow_wgrad_sum form the parameter gradients from those planes, split
//    over batch slices and summed in a fixed order.
// One tile per CU leaves no other workgroup to cover a memory wait, so both tile kernels keep
// their global loads off the critical path: each wave holds its weight fragments of a layer in
// registers (bf16x8 operand vectors, 48 VGPRs forward, 96 backward plus the biases) and reloads
// them for the next layer right after their last use, and the backward loads the next layer's
// input X_{c-1} into registers at the start of layer c and moves it to LDS at the end.
constexpr int kTP = 16;                        // paths per training tile
constexpr int kFusedMaxD = 127;                // coordinates of a tile (N <= 128)
constexpr int kTileRegs = (kFusedMaxD * kTP + kBlock - 1) / kBlock;   // tile doubles per thread
constexpr int kTLdA = kFlowK + 8;              // xa [P][in] row stride (bf16 elements)
constexpr int kTLdH = kFlowH + 8;              // hs [P][hid] row stride (bf16 elements)
constexpr int kTLdG = kFlowH + 4;              // go, gp [P][row] row stride (floats)

// Operand vector of a 16 x 32 block of a row-major bf16 matrix: rows r0 + (l & 15), columns
// k0 + 8 (l >> 4) .. + 7 (the A layout of the bf16 MFMA; the FP32 products below take the same
// vector, see fma16_f32).
__device__ __forceinline__ bf16x8 frag(const __bf16* M, int ld, int r0, int k0) {
    const int l = threadIdx.x & 63;
    return *reinterpret_cast<const bf16x8*>(M + (r0 + (l & 15)) * ld + k0 + 8 * (l >> 4));
}

// Weight operands of one layer held by a wave: hidden rows 32w + 16mb (W1), output rows 16w (s_hat)
// and 64 + 16w (t) of W2, and the biases of this lane's output slots.
struct FwdFrags {
    bf16x8 w1[2][2];        // [mb][k block of 32 inputs]
    bf16x8 w2[2][4];        // [s, t][k block of 32 hidden]
    float b1[2][4];         // hidden 32w + 16mb + 4(l>>4) + j
    float b2[2][4];         // output 16w + 4(l>>4) + j (s_hat), 64 + ... (t)
};
struct BwdFrags {
    bf16x8 w2t[2][4];       // W2T rows 32w + 16mb, k block of 32 outputs
    bf16x8 w1t[4];          // W1T rows 16w, k block of 32 hidden
};

__device__ __forceinline__ void load_w1(FwdFrags& F, const FlowLayerDev& L) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) F.w1[mb][kb] = frag(L.W1, kFlowK, 32 * w + 16 * mb, 32 * kb);
#pragma unroll
        for (int j = 0; j < 4; ++j) F.b1[mb][j] = L.b1[32 * w + 16 * mb + 4 * (l >> 4) + j];
    }
}
__device__ __forceinline__ void load_w2(FwdFrags& F, const FlowLayerDev& L) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 0; o < 2; ++o) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) F.w2[o][kb] = frag(L.W2, kFlowH, 64 * o + 16 * w, 32 * kb);
#pragma unroll
        for (int j = 0; j < 4; ++j) F.b2[o][j] = L.b2[64 * o + 16 * w + 4 * (l >> 4) + j];
    }
}
__device__ __forceinline__ void load_w2t(BwdFrags& F, const FlowLayerDev& L) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) F.w2t[mb][kb] = frag(L.W2T, kFlowH, 32 * w + 16 * mb, 32 * kb);
}
__device__ __forceinline__ void load_w1t(BwdFrags& F, const FlowLayerDev& L) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) F.w1t[kb] = frag(L.W1T, kFlowH, 16 * w, 32 * kb);
}

// C(16 x 16) += A(16 x 128) B, A from fragments (bf16, exact in FP32) and B^T rows from LDS (FP32,
// [column][k], stride ldb), on v_mfma_f32_16x16x4f32. The k index is permuted against the
// instruction's own order: in product q of k block kb, lane l supplies k = 32kb + 8(l>>4) + q for
// both operands, so each lane reads 8 consecutive k of A (one fragment) and of B (two 16-byte LDS
// reads); the sum over k is the same, in another rounding order.
__device__ __forceinline__ floatx4 fma16_f32(const bf16x8 (&a)[4], const float* BT, int ldb, floatx4 c) {
    const int l = threadIdx.x & 63;
    const float* br = BT + (l & 15) * ldb + 8 * (l >> 4);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const floatx4 b0 = *reinterpret_cast<const floatx4*>(br + 32 * kb);
        const floatx4 b1 = *reinterpret_cast<const floatx4*>(br + 32 * kb + 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) c = __builtin_amdgcn_mfma_f32_16x16x4f32(float(a[kb][q]), b0[q], c, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) c = __builtin_amdgcn_mfma_f32_16x16x4f32(float(a[kb][4 + q]), b1[q], c, 0, 0, 0);
    }
    return c;
}

// The masks of every layer type into LDS: masks[type][0..63] conditioner coordinates, [64..127]
// transformed coordinates (heap node - 1).
__device__ __forceinline__ void train_masks(const FlowNet& net, int* masks) {
    int v[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) v[it] = net.masks[threadIdx.x + it * kBlock];
#pragma unroll
    for (int it = 0; it < 2; ++it) masks[threadIdx.x + it * kBlock] = v[it];
}
static_assert(2 * kBlock == 4 * 128, "two mask entries per thread");

// x_A tile of layer L: bf16 [P][in] from the FP64 tile X[(h-1)*kTP + P] (inputs beyond dA are 0).
__device__ __forceinline__ void train_xa(const FlowLayerDev& L, const int* am, const double* X, __bf16* xa) {
    for (int i = threadIdx.x; i < kTP * kFlowK; i += kBlock) {
        const int P = i % kTP, k = i / kTP;
        xa[P * kTLdA + k] = (__bf16)(float)(k < L.dA ? X[am[k] * kTP + P] : 0.0);
    }
}

// Hidden layer of the tile: wave w computes hidden rows 32w..32w+31 for the 16 paths;
// pre-activation (with bias) returned in pre[mb][j] for hid = 32w + 16mb + 4(l>>4) + j, path
// l & 15; h = silu(pre) stored to hs [P][hid] as bf16.
__device__ __forceinline__ void train_hidden(const FwdFrags& F, const __bf16* xa, __bf16* hs, floatx4 (&pre)[2]) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const __bf16* xr = xa + (l & 15) * kTLdA + 8 * (l >> 4);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w1[mb][kb], *reinterpret_cast<const bf16x8*>(xr + 32 * kb), c,
                                                        0, 0, 0);
        pre[mb] = c;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int hid = 32 * w + 16 * mb + 4 * (l >> 4) + j;
            pre[mb][j] += F.b1[mb][j];
            hs[(l & 15) * kTLdH + hid] = (__bf16)silu(pre[mb][j]);
        }
    }
}

// Output layer: wave w computes s_hat rows 16w..16w+15 (os) and t rows 64+16w.. (ot); lane l, slot
// j holds coordinate 16w + 4(l>>4) + j of path l & 15, bias included.
__device__ __forceinline__ void train_output(const FwdFrags& F, const __bf16* hs, floatx4& os, floatx4& ot) {
    const int l = threadIdx.x & 63;
    const __bf16* hr = hs + (l & 15) * kTLdH + 8 * (l >> 4);
    floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const bf16x8 h = *reinterpret_cast<const bf16x8*>(hr + 32 * kb);
        c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w2[0][kb], h, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w2[1][kb], h, c1, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        os[j] = c0[j] + F.b2[0][j];
        ot[j] = c1[j] + F.b2[1][j];
    }
}

// Base normals (the plain sampler's, stream key.stream + *step), every coupling; X_c (c = 0..L) to
// the planes Xg + c*plane ([h-1][path], ld), |u|^2/2 and log det per path.
__global__ void __launch_bounds__(kBlock) k_train_fwd(FlowNet net, RngKey key, const int* step, uint64_t n, int D,
                                                      double* __restrict__ Xg, uint64_t ld, uint64_t plane,
                                                      double* __restrict__ hu2, double* __restrict__ logdet) {
    constexpr int kG = kBlock / kTP;             // thread groups of the normals
    __shared__ double X[kFusedMaxD * kTP];
    __shared__ __attribute__((aligned(16))) __bf16 xa[kTP * kTLdA];
    __shared__ __attribute__((aligned(16))) __bf16 hs[kTP * kTLdH];      // also the Box-Muller table at first
    __shared__ int masks[4 * 128];
    __shared__ double red[kG][kTP];
    __shared__ double redl[4][kTP];
    static_assert(sizeof(hs) >= kBoxMullerTable * sizeof(double), "table fits the hidden tile");
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int P = l & 15;
    const uint64_t p0 = uint64_t(blockIdx.x) * kTP;
    FwdFrags F;
    load_w1(F, net.layer[0]);
    load_w2(F, net.layer[0]);
    train_masks(net, masks);
    {   // base normals: thread (Pn = t % kTP, g = t / kTP) takes node pairs j = g, g + kG, ...
        double* bm = reinterpret_cast<double*>(hs);
        load_bm_table(bm, kBlock);
        __syncthreads();
        RngKey k = key;
        if (step) k.stream += uint32_t(*step);
        const int Pn = t % kTP, g = t / kTP;
        const PathRng pr = path_rng(k, p0 + uint64_t(Pn));
        double u2 = 0.0;
        for (int j = g; 2 * j <= D; j += kG) {
            double ze, zo;
            normal_pair(k, pr, uint32_t(j), bm, ze, zo);
            if (j > 0) {
                X[(2 * j - 1) * kTP + Pn] = ze;
                u2 += ze * ze;
            }
            if (2 * j + 1 <= D) {
                X[(2 * j) * kTP + Pn] = zo;
                u2 += zo * zo;
            }
        }
        red[g][Pn] = u2;
    }
    double ldet = 0.0;                               // this wave's share of log det of path P
    for (int c = 0; c < net.n_layers; ++c) {
        const FlowLayerDev& L = net.layer[c];
        const FlowLayerDev& Ln = net.layer[c + 1 < net.n_layers ? c + 1 : c];
        const int* am = masks + (c % 4) * 128;
        __syncthreads();                             // X complete; hs, xa free
        for (int i = t; i < D * kTP; i += kBlock) {
            const uint64_t Pi = p0 + uint64_t(i % kTP);
            if (Pi < n) Xg[uint64_t(c) * plane + uint64_t(i / kTP) * ld + Pi] = X[i];
        }
        train_xa(L, am, X, xa);
        __syncthreads();
        floatx4 pre[2];
        train_hidden(F, xa, hs, pre);
        load_w1(F, Ln);
        __syncthreads();
        floatx4 os, ot;
        train_output(F, hs, os, ot);
        load_w2(F, Ln);
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 16 * w + 4 * (l >> 4) + j;
            if (k < L.dB) {
                const float sv = 2.0f * tanh_fast(0.5f * os[j]);
                const int a = am[64 + k] * kTP + P;
                X[a] = X[a] * exp_logscale(double(sv)) + double(ot[j]);
                v += double(sv);
            }
        }
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        ldet += v;
    }
    if (l < kTP) redl[w][l] = ldet;
    __syncthreads();
    for (int i = t; i < D * kTP; i += kBlock) {
        const uint64_t Pi = p0 + uint64_t(i % kTP);
        if (Pi < n) Xg[uint64_t(net.n_layers) * plane + uint64_t(i / kTP) * ld + Pi] = X[i];
    }
    if (t < kTP && p0 + t < n) {
        double u2 = 0.0, ld2 = 0.0;
        for (int g = 0; g < kG; ++g) u2 += red[g][t];
        for (int q = 0; q < 4; ++q) ld2 += redl[q][t];
        hu2[p0 + t] = 0.5 * u2;
        logdet[p0 + t] = ld2;
    }
}

// Backward through every layer, last first: G = alpha_i d l_i / d z (the action gradient Gg scaled
// by the path's loss weight as it is loaded) becomes the gradient for each layer's input; the planes
// of TrainPlanes (leading dimension pl.ld) are written for the weight gradients.
__global__ void __launch_bounds__(kBlock) k_train_bwd(FlowNet net, const double* __restrict__ Xg, const double* __restrict__ Gg,
                                                      uint64_t ld, uint64_t plane, uint64_t n, int D,
                                                      const double* __restrict__ alpha, TrainPlanes pl) {
    __shared__ double G[kFusedMaxD * kTP];
    __shared__ double Xb[2][kFusedMaxD * kTP];
    __shared__ __attribute__((aligned(16))) __bf16 xa[kTP * kTLdA];
    __shared__ __attribute__((aligned(16))) __bf16 hs[kTP * kTLdH];
    __shared__ __attribute__((aligned(16))) float go[kTP * kTLdG];
    __shared__ __attribute__((aligned(16))) float gp[kTP * kTLdG];
    __shared__ int masks[4 * 128];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int P = l & 15;
    const uint64_t p0 = uint64_t(blockIdx.x) * kTP;
    const bool valid = p0 + uint64_t(P) < n;
    const double al = valid ? alpha[p0 + P] : 0.0;
    const uint64_t pld = pl.ld;
    const int L0 = net.n_layers - 1;
    FwdFrags F;
    BwdFrags B;
    load_w1(F, net.layer[L0]);
    load_w2(F, net.layer[L0]);
    load_w2t(B, net.layer[L0]);
    load_w1t(B, net.layer[L0]);
    train_masks(net, masks);
    {   // thread t always takes path t % kTP of the tile (kBlock is a multiple of kTP)
        static_assert(kBlock % kTP == 0, "tile columns per thread");
        const uint64_t Pt = p0 + uint64_t(t % kTP);
        const double at = Pt < n ? alpha[Pt] : 0.0;
        double gv[kTileRegs], xv[kTileRegs];
#pragma unroll
        for (int it = 0; it < kTileRegs; ++it) {
            const int i = t + it * kBlock;
            const bool ok = i < D * kTP && Pt < n;
            const uint64_t o = uint64_t(i / kTP) * ld + Pt;
            gv[it] = ok ? Gg[o] : 0.0;
            xv[it] = ok ? Xg[uint64_t(L0) * plane + o] : 0.0;
        }
#pragma unroll
        for (int it = 0; it < kTileRegs; ++it) {
            const int i = t + it * kBlock;
            if (i < D * kTP) {
                G[i] = gv[it] * at;
                Xb[L0 & 1][i] = xv[it];
            }
        }
    }
    for (int c = L0; c >= 0; --c) {
        const FlowLayerDev& L = net.layer[c];
        const FlowLayerDev& Ln = net.layer[c > 0 ? c - 1 : 0];
        const int* am = masks + (c % 4) * 128;
        const double* X = Xb[c & 1];
        float* goT = pl.goT + uint64_t(c) * pl.g_stride;
        float* gpT = pl.gpT + uint64_t(c) * pl.g_stride;
        __bf16* hT = pl.hT + uint64_t(c) * pl.h_stride;
        __bf16* xaT = pl.xaT + uint64_t(c) * pl.xa_stride;
        __syncthreads();                             // G and X_c complete; xa, hs, go, gp free
        double xn[kTileRegs];                        // X_{c-1}, stored to the other buffer at the end
#pragma unroll
        for (int it = 0; it < kTileRegs; ++it) {
            const int i = t + it * kBlock;
            const uint64_t Pi = p0 + uint64_t(i % kTP);
            xn[it] = c > 0 && i < D * kTP && Pi < n ? Xg[uint64_t(c - 1) * plane + uint64_t(i / kTP) * ld + Pi] : 0.0;
        }
        train_xa(L, am, X, xa);
        __syncthreads();
        for (int i = t; i < kTP * kFlowK; i += kBlock) {
            const int Pi = i % kTP, k = i / kTP;
            if (p0 + uint64_t(Pi) < n) xaT[uint64_t(k) * pld + p0 + Pi] = xa[Pi * kTLdA + k];
        }
        floatx4 pre[2];
        train_hidden(F, xa, hs, pre);
        load_w1(F, Ln);
        __syncthreads();
        for (int i = t; i < kTP * kFlowH; i += kBlock) {
            const int Pi = i % kTP, k = i / kTP;
            if (p0 + uint64_t(Pi) < n) hT[uint64_t(k) * pld + p0 + Pi] = hs[Pi * kTLdH + k];
        }
        floatx4 os, ot;
        train_output(F, hs, os, ot);
        load_w2(F, Ln);
        // affine backward of coordinate k of path P (this lane's slots)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 16 * w + 4 * (l >> 4) + j;
            float gsh = 0.f, gt = 0.f;
            if (k < L.dB && valid) {
                const float th = tanh_fast(0.5f * os[j]);
                const float sv = 2.0f * th;
                const int a = am[64 + k] * kTP + P;
                const double es = exp_logscale(double(sv));
                const double gy = G[a];
                G[a] = gy * es;
                const double gs = gy * X[a] * es + al;
                gsh = float(gs * (1.0 - double(th) * double(th)));
                gt = float(gy);
            }
            go[P * kTLdG + k] = gsh;
            go[P * kTLdG + 64 + k] = gt;
            if (valid) {
                goT[uint64_t(k) * pld + p0 + P] = gsh;
                goT[uint64_t(64 + k) * pld + p0 + P] = gt;
            }
        }
        __syncthreads();
        // g_h = W2^T g_o, g_pre = g_h silu'(pre)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const floatx4 gh = fma16_f32(B.w2t[mb], go, kTLdG, floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int hid = 32 * w + 16 * mb + 4 * (l >> 4) + j;
                const float v = pre[mb][j];
                const float sg = sigmoid_fast(v);
                const float g = valid ? gh[j] * (sg * (1.0f + v * (1.0f - sg))) : 0.f;
                gp[P * kTLdG + hid] = g;
                if (valid) gpT[uint64_t(hid) * pld + p0 + P] = g;
            }
        }
        load_w2t(B, Ln);
        __syncthreads();
        // g_xa = W1^T g_pre into G of the conditioner coordinates
        {
            const floatx4 gx = fma16_f32(B.w1t, gp, kTLdG, floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * w + 4 * (l >> 4) + j;
                if (k < L.dA && valid) G[am[k] * kTP + P] += double(gx[j]);
            }
        }
        load_w1t(B, Ln);
        if (c > 0) {
            double* Xn = Xb[(c - 1) & 1];            // last read by layer c + 1
#pragma unroll
            for (int it = 0; it < kTileRegs; ++it) {
                const int i = t + it * kBlock;
                if (i < D * kTP) Xn[i] = xn[it];
            }
        }
    }
}

// Parameter gradients from the planes (leading dimension pl.ld, a multiple of kWgChunk, zero beyond
// the batch), split over batch slices and summed in a fixed order. k_flow_wgrad_part: grid (layer,
// output block, slice); output block b < 16 is the 32 x 32 block (b / 4, b % 4) of g_W2 (rows out,
// columns hid), b < 24 a block of g_W1 (rows hid, columns in); slice k takes the chunks of 128 paths
// [k nc / S, (k+1) nc / S). The workgroup stages a chunk of its 32 A rows (FP32) and 32 B rows (bf16)
// through LDS with 16-byte loads, the next chunk's loads in flight while the current one is
// multiplied; wave w accumulates the 16 x 16 sub-block (w / 2, w % 2) on FP32 MFMA. The blocks of
// column 0 also sum their A rows over the slice (FP64, fixed order): the b2 gradient from the output
// gradient rows, b1 from the pre-activation rows. k_flow_wgrad_sum adds the slices in slice order.
constexpr int kWgSlices = 8;                   // batch slices of the weight gradients (at most)
constexpr int kWgChunk = 128;                  // paths staged per step
constexpr int kWgLd = kWgChunk + 4;            // LDS row stride (floats)

__device__ __forceinline__ void wg_load(const float* A, const __bf16* B, uint64_t ld, uint64_t kc, floatx4 (&ra)[4],
                                        bf16x8 (&rb)[2]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int i = t + it * kBlock;                         // row i >> 5, 4 paths (i & 31)
        ra[it] = *reinterpret_cast<const floatx4*>(A + uint64_t(i >> 5) * ld + kc + 4 * (i & 31));
    }
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int i = t + it * kBlock;                         // row i >> 4, 8 paths (i & 15)
        rb[it] = *reinterpret_cast<const bf16x8*>(B + uint64_t(i >> 4) * ld + kc + 8 * (i & 15));
    }
}

__global__ void __launch_bounds__(kBlock) k_flow_wgrad_part(TrainPlanes pl, int slices, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) float As[32 * kWgLd];
    __shared__ __attribute__((aligned(16))) float Bs[32 * kWgLd];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int c = blockIdx.x, b = blockIdx.y, sl = blockIdx.z;
    const uint64_t ld = pl.ld;
    const bool w2 = b < 16;
    const int r0 = w2 ? 32 * (b / 4) : 32 * ((b - 16) / 2);
    const int c0 = w2 ? 32 * (b % 4) : 32 * ((b - 16) % 2);
    const bool bias = c0 == 0;
    const float* A = (w2 ? pl.goT : pl.gpT) + uint64_t(c) * pl.g_stride + uint64_t(r0) * ld;
    const __bf16* B = (w2 ? pl.hT + uint64_t(c) * pl.h_stride : pl.xaT + uint64_t(c) * pl.xa_stride) + uint64_t(c0) * ld;
    const uint64_t nc = ld / kWgChunk;
    const uint64_t q0 = uint64_t(sl) * nc / uint64_t(slices), q1 = uint64_t(sl + 1) * nc / uint64_t(slices);
    const int wr = 16 * (w >> 1), wc = 16 * (w & 1);
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    double bsum = 0.0;                               // row t >> 3, paths 16 (t & 7) .. of each chunk
    floatx4 ra[4];
    bf16x8 rb[2];
    if (q0 < q1) wg_load(A, B, ld, q0 * kWgChunk, ra, rb);
    for (uint64_t q = q0; q < q1; ++q) {
        __syncthreads();                             // the previous chunk's reads are done
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int i = t + it * kBlock;
            *reinterpret_cast<floatx4*>(As + (i >> 5) * kWgLd + 4 * (i & 31)) = ra[it];
        }
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int i = t + it * kBlock;
            float* d = Bs + (i >> 4) * kWgLd + 8 * (i & 15);
            *reinterpret_cast<floatx4*>(d) = floatx4{float(rb[it][0]), float(rb[it][1]), float(rb[it][2]), float(rb[it][3])};
            *reinterpret_cast<floatx4*>(d + 4) =
                floatx4{float(rb[it][4]), float(rb[it][5]), float(rb[it][6]), float(rb[it][7])};
        }
        __syncthreads();
        if (q + 1 < q1) wg_load(A, B, ld, (q + 1) * kWgChunk, ra, rb);
        const float* ar = As + (wr + (l & 15)) * kWgLd + 8 * (l >> 4);
        const float* br = Bs + (wc + (l & 15)) * kWgLd + 8 * (l >> 4);
#pragma unroll
        for (int kb = 0; kb < kWgChunk / 32; ++kb) {
            const floatx4 a0 = *reinterpret_cast<const floatx4*>(ar + 32 * kb);
            const floatx4 a1 = *reinterpret_cast<const floatx4*>(ar + 32 * kb + 4);
            const floatx4 b0 = *reinterpret_cast<const floatx4*>(br + 32 * kb);
            const floatx4 b1 = *reinterpret_cast<const floatx4*>(br + 32 * kb + 4);
#pragma unroll
            for (int j = 0; j < 4; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[j], b0[j], acc, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[j], b1[j], acc, 0, 0, 0);
        }
        if (bias) {
            const float* rr = As + (t >> 3) * kWgLd + 16 * (t & 7);
#pragma unroll
            for (int j = 0; j < 16; ++j) bsum += double(rr[j]);
        }
    }
    float* o = part + (uint64_t(sl) * gridDim.x + uint64_t(c)) * kFlowNP;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = r0 + wr + 4 * (l >> 4) + j, col = c0 + wc + (l & 15);
        if (w2)
            o[kFlowOffW2 + r * kFlowH + col] = acc[j];
        else
            o[r * kFlowK + col] = acc[j];
    }
    if (bias) {
        bsum += __shfl_xor(bsum, 1, 64);
        bsum += __shfl_xor(bsum, 2, 64);
        bsum += __shfl_xor(bsum, 4, 64);
        if ((t & 7) == 0) o[(w2 ? kFlowOffB2 : kFlowOffB1) + r0 + (t >> 3)] = float(bsum);
    }
}

__global__ void __launch_bounds__(kBlock) k_flow_wgrad_sum(const float* __restrict__ part, int slices, uint64_t total,
                                                           float* __restrict__ grad) {
    const uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= total) return;
    float v[kWgSlices];
#pragma unroll
    for (int k = 0; k < kWgSlices; ++k) v[k] = k < slices ? part[uint64_t(k) * total + i] : 0.f;
    float s = v[0];
#pragma unroll
    for (int k = 1; k < kWgSlices; ++k) s += v[k];
    grad[i] = s;
}

// ------------------------------------------------------------------------------------ action and its gradient
// A workgroup takes 16 paths, 16 threads per path (thread (P = t & 15, g = t >> 4)). The points
// of the level-s path (positions 0..N, Sec. 4.1 bisection with sigma_n^2 = T/2^(n+1)) are built
// level by level in LDS; S = sum_k eps W_p with each slice as sum_k dlt^(2k) P_k(v), v = mid^2
// (even potential) or mid, dlt = q_{k+1} - q_k, from the folded level table (P_k highest power
// first, consecutive in k); dS/dq from the slice derivatives, then the adjoint of the (linear)
// bisection map level by level from the finest. Writes l = -(S - shift) - |z|^2/2 + |u|^2/2 +
// log det and G = dl/dz = -dS/dz - z.
constexpr int kAgPaths = 16;
constexpr int kAgMaxN = 128;

__global__ void __launch_bounds__(kBlock) k_flow_action_grad(const double* __restrict__ tab, const int* __restrict__ deg,
                                                             int K, int even, const double* __restrict__ sig, double shift,
                                                             double a, double b, int s, const double* __restrict__ X,
                                                             uint64_t ld, uint64_t n, const double* __restrict__ hu2,
                                                             const double* __restrict__ logdet, double* __restrict__ ell,
                                                             double* __restrict__ G) {
    __shared__ double Q[(kAgMaxN + 1) * kAgPaths];      // points, then d S / d q, position-major
    __shared__ double SA[kAgMaxN * kAgPaths];           // slice k: d/dq_k
    __shared__ double SB[kAgMaxN * kAgPaths];           // slice k: d/dq_{k+1}
    __shared__ double red[2][16][kAgPaths];
    __shared__ double Z[(kAgMaxN - 1) * kAgPaths];      // the tile's normals z[(h-1)*16 + P]
    const int t = threadIdx.x, P = t & 15, g = t >> 4;
    const uint64_t path = uint64_t(blockIdx.x) * kAgPaths + uint64_t(P);
    const bool valid = path < n;
    const int N = 1 << s;
    {   // every load of the tile in flight at once: thread t takes node h - 1 = g + 16 it of path P
        constexpr int kRegs = (kAgMaxN - 1 + 15) / 16;
        double zv[kRegs];
#pragma unroll
        for (int it = 0; it < kRegs; ++it) {
            const int h1 = g + 16 * it;
            zv[it] = valid && h1 < N - 1 ? X[uint64_t(h1) * ld + path] : 0.0;
        }
#pragma unroll
        for (int it = 0; it < kRegs; ++it) {
            const int h1 = g + 16 * it;
            if (h1 < N - 1) Z[h1 * kAgPaths + P] = zv[it];
        }
    }
    if (g == 0) {
        Q[P] = a;
        Q[N * kAgPaths + P] = b;
    }
    __syncthreads();
    for (int lev = 1; lev <= s; ++lev) {
        const int step = 1 << (s - lev), cnt = 1 << (lev - 1);
        for (int i = g; i < cnt; i += 16) {
            const int h = cnt + i, pos = (2 * i + 1) * step;
            const double z = Z[(h - 1) * kAgPaths + P];
            Q[pos * kAgPaths + P] = sig[lev] * z + 0.5 * (Q[(pos - step) * kAgPaths + P] + Q[(pos + step) * kAgPaths + P]);
        }
        __syncthreads();
    }
    const const_ptr<double> tb = as_const(tab);
    const const_ptr<int> dg = as_const(deg);
    double Sp = 0.0;
    for (int k = g; k < N; k += 16) {
        const double q0 = Q[k * kAgPaths + P], q1 = Q[(k + 1) * kAgPaths + P];
        const double mid = 0.5 * (q0 + q1), dl = q1 - q0;
        const double y = even ? mid * mid : mid, zz = dl * dl;
        double val = 0.0, dmid = 0.0, ddl = 0.0, pw = 1.0, pwm1 = 0.0;
        int off = 0;
        for (int kk = 0; kk < K; ++kk) {
            const int d = dg[kk];
            double Pv = tb[off], dP = 0.0;
            for (int e = 1; e <= d; ++e) {
                dP = fma(dP, y, Pv);
                Pv = fma(Pv, y, tb[off + e]);
            }
            off += d + 1;
            val += pw * Pv;
            dmid += pw * dP;
            ddl += double(kk) * pwm1 * Pv;
            pwm1 = pw;
            pw *= zz;
        }
        Sp += val;
        const double gmid = even ? 2.0 * mid * dmid : dmid;   // d/dmid of sum_k dlt^(2k) P_k(v)
        const double gdl = 2.0 * dl * ddl;                    // d/ddlt of the same
        SA[k * kAgPaths + P] = 0.5 * gmid - gdl;
        SB[k * kAgPaths + P] = 0.5 * gmid + gdl;
    }
    __syncthreads();
    for (int pos = 1 + g; pos < N; pos += 16) Q[pos * kAgPaths + P] = SA[pos * kAgPaths + P] + SB[(pos - 1) * kAgPaths + P];
    __syncthreads();
    double z2p = 0.0;
    for (int lev = s; lev >= 1; --lev) {
        const int step = 1 << (s - lev), cnt = 1 << (lev - 1);
        for (int i = g; i < cnt; i += 16) {
            const int h = cnt + i, pos = (2 * i + 1) * step;
            if (valid) G[uint64_t(h - 1) * ld + path] = -sig[lev] * Q[pos * kAgPaths + P] - Z[(h - 1) * kAgPaths + P];
        }
        // the node points at this level depend on the two neighbouring coarser points
        for (int p2 = 2 * step * (1 + g); p2 < N; p2 += 2 * step * 16)
            Q[p2 * kAgPaths + P] = (Q[p2 * kAgPaths + P] + 0.5 * Q[(p2 + step) * kAgPaths + P]) +
                                   0.5 * Q[(p2 - step) * kAgPaths + P];
        __syncthreads();
    }
    for (int h = 1 + g; h < N; h += 16) {
        const double z = Z[(h - 1) * kAgPaths + P];
        z2p += z * z;
    }
    red[0][g][P] = Sp;
    red[1][g][P] = z2p;
    __syncthreads();
    if (g == 0 && valid) {
        double S = 0.0, z2 = 0.0;
        for (int q = 0; q < 16; ++q) {
            S += red[0][q][P];
            z2 += red[1][q][P];
        }
        ell[path] = -(S - shift) - 0.5 * z2 + hu2[path] + logdet[path];
    }
}

// One workgroup per canonical chunk (the order of the plain estimator, pimc_internal.hpp): wave w
// takes the groups of 64 paths g = w, w + 4, ... of the chunk, adds each group's wave sums of
// d = expm1(l), d^2 and the non-finite count to its slot in order, and the chunk sum is the slots
// added in slot order.
__global__ void __launch_bounds__(kBlock) k_flow_partials(const double* __restrict__ ell, uint64_t ell_first_path,
                                                          uint64_t n_total, uint64_t first_chunk,
                                                          double* __restrict__ partials) {
    static_assert(kBlock / 64 == kChunkSlots, "one wave per accumulator slot");
    __shared__ double red[kChunkSlots][3];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint64_t c = first_chunk + blockIdx.x;
    const uint64_t first = c * kChunkPaths;
    double s1 = 0.0, s2 = 0.0, nb = 0.0;
    for (int g = w; g < kChunkGroups; g += kChunkSlots) {
        const uint64_t path = first + uint64_t(g) * 64 + uint64_t(l);
        if (first + uint64_t(g) * 64 >= n_total) break;         // wave-uniform
        const bool valid = path < n_total;
        const double d = valid ? expm1(ell[path - ell_first_path]) : 0.0;
        const bool bad = valid && !isfinite(d);
        const double sd = wave_sum(d);
        const double sd2 = wave_sum(d * d);
        const unsigned long long badmask = __ballot(bad);
        s1 += sd;
        s2 += sd2;
        nb += double(__popcll(badmask));
    }
    if (l == 0) {
        red[w][0] = s1;
        red[w][1] = s2;
        red[w][2] = nb;
    }
    __syncthreads();
    if (t == 0) {
        double a = 0.0, b = 0.0, e = 0.0;
        for (int q = 0; q < kChunkSlots; ++q) {
            a += red[q][0];
            b += red[q][1];
            e += red[q][2];
        }
        const uint64_t rem = n_total - first;
        double* o = partials + c * 4;
        o[0] = double(rem < kChunkPaths ? rem : kChunkPaths);
        o[1] = a;
        o[2] = b;
        o[3] = e;
    }
}

// ------------------------------------------------------------------------------------ loss weights
// alpha_i = (1-beta) 2 exp(2 l_i) / sum_j exp(2 l_j) - beta/n; loss = (1-beta) log mean exp(2l) -
// beta mean l, stored at loss[*step] (loss[0] without step). One workgroup, fixed reduction order.
__global__ void __launch_bounds__(kBlock) k_flow_alpha(const double* __restrict__ ell, uint64_t n, double beta,
                                                       double* __restrict__ alpha, double* __restrict__ loss,
                                                       const int* __restrict__ step) {
    __shared__ double red[kBlock];
    const int t = threadIdx.x;
    double mx = -HUGE_VAL;
#pragma unroll 16
    for (uint64_t i = t; i < n; i += kBlock) mx = fmax(mx, 2.0 * ell[i]);
    red[t] = mx;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if (t < w) red[t] = fmax(red[t], red[t + w]);
        __syncthreads();
    }
    mx = red[0];
    __syncthreads();
    double se = 0.0, sl = 0.0;
#pragma unroll 16
    for (uint64_t i = t; i < n; i += kBlock) {
        se += exp(2.0 * ell[i] - mx);
        sl += ell[i];
    }
    red[t] = se;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    se = red[0];
    __syncthreads();
    red[t] = sl;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    sl = red[0];
#pragma unroll 16
    for (uint64_t i = t; i < n; i += kBlock)
        alpha[i] = (1.0 - beta) * 2.0 * exp(2.0 * ell[i] - mx) / se - beta / double(n);
    if (t == 0 && loss) loss[step ? *step : 0] = (1.0 - beta) * (mx + log(se / double(n))) - beta * sl / double(n);
}

// ------------------------------------------------------------------------------------ parameters
__device__ __forceinline__ void store_bf16_copies(int layer, int off, float v, __bf16* W1, __bf16* W2, __bf16* W1T,
                                                  __bf16* W2T) {
    const __bf16 b = (__bf16)v;
    if (off < kFlowOffB1) {
        const int hid = off / kFlowK, in = off % kFlowK;
        W1[size_t(layer) * kFlowH * kFlowK + off] = b;
        W1T[size_t(layer) * kFlowH * kFlowK + in * kFlowH + hid] = b;
    } else if (off >= kFlowOffW2 && off < kFlowOffB2) {
        const int o = off - kFlowOffW2;
        const int out = o / kFlowH, hid = o % kFlowH;
        W2[size_t(layer) * kFlowH * kFlowH + o] = b;
        W2T[size_t(layer) * kFlowH * kFlowH + hid * kFlowH + out] = b;
    }
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master parameters, then bfloat16 copies.
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, int layers, const int* __restrict__ step, float lr,
                       __bf16* W1, __bf16* W2, __bf16* W1T, __bf16* W2T) {
    const uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= uint64_t(layers) * kFlowNP) return;
    const float b1 = 0.9f, b2 = 0.999f;
    const int tstep = *step + 1;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(b1, float(tstep)));
    const float vh = vi / (1.0f - powf(b2, float(tstep)));
    const float th = theta[i] - lr * mh / (sqrtf(vh) + 1e-8f);
    theta[i] = th;
    store_bf16_copies(int(i / kFlowNP), int(i % kFlowNP), th, W1, W2, W1T, W2T);
}

__global__ void k_params_to_bf16(const float* __restrict__ theta, int layers, __bf16* W1, __bf16* W2, __bf16* W1T,
                                 __bf16* W2T) {
    const uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= uint64_t(layers) * kFlowNP) return;
    store_bf16_copies(int(i / kFlowNP), int(i % kFlowNP), theta[i], W1, W2, W1T, W2T);
}

__global__ void k_step_inc(int* step) { *step += 1; }

// ------------------------------------------------------------------------------------ fused estimation
// One workgroup carries 64 paths through the whole proposal: base normals (Philox, in LDS as FP64
// [node][path]), every coupling, the bisection and the level-s action, and writes log w (and,
// when asked, log det and z) per path. Only 8 bytes per path reach HBM.
//
// The products are oriented weights x activations: wave w computes hidden rows 32w..32w+31 and
// output rows {16w..16w+15} (s_hat) and {64+16w..64+16w+15} (t) for all 64 paths, so each wave
// reads a quarter of the weights and the workgroup reads each weight once per tile; the
// activations are shared through LDS. In the output layout a lane holds s_hat and t of the same
// (coordinate, path) in the same register slot.
constexpr int kFusedPaths = 64;
constexpr int kLdXa = kFlowK + 8;                 // x_A tile [path][in], padded rows

// Hidden tile [path][hidden] without padding: 16-byte chunk c of row P is stored at chunk
// c ^ (P & 15), so the 16 rows read by one operand fetch fall in 16 different bank groups.
__device__ __forceinline__ int hs_index(int P, int c) { return P * kFlowH + ((((c >> 3) ^ (P & 15)) << 3) | (c & 7)); }

__device__ __forceinline__ int node_of_position(int pos, int s) {
    const int tz = __builtin_ctz(pos);             // pos = (2i+1) 2^tz: level n = s - tz, offset i
    return (1 << (s - tz - 1)) + (pos >> (tz + 1));
}

__global__ void __launch_bounds__(kBlock, 2)
k_flow_fused(FlowNet net, RngKey key, uint64_t first_path, uint64_t n, int s, const double* __restrict__ tab,
             const int* __restrict__ deg, int K, int stride, int even, const double* __restrict__ sig, double shift, double a,
             double b, double* __restrict__ ell_out, double* __restrict__ logdet_out, double* __restrict__ z_out,
             uint64_t zld) {
    __shared__ double X[kFusedMaxD * kFusedPaths];                              // [h-1][P]
    __shared__ __attribute__((aligned(16))) __bf16 act[kFusedPaths * kFlowH];   // x_A or hidden tile; sums at the end
    const int t = threadIdx.x;
    const int l = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int P = t & 63;                           // path of this thread in the scalar phases
    const int N = 1 << s, D = N - 1;
    const uint64_t local = uint64_t(blockIdx.x) * kFusedPaths + uint64_t(P);
    const bool valid = local < n;
    // ---- base normals: group w takes node pairs j = w, w+4, ...; |u|^2 in that order
    double u2 = 0.0;
    {
        // the Box-Muller table lives in the activation tile until the first coupling needs it
        double* bm = reinterpret_cast<double*>(act);
        load_bm_table(bm, kBlock);
        __syncthreads();
        const PathRng pr = path_rng(key, first_path + local);
        for (int j = w; 2 * j <= D; j += 4) {
            double ze, zo;
            normal_pair(key, pr, uint32_t(j), bm, ze, zo);
            if (j > 0) {
                X[(2 * j - 1) * kFusedPaths + P] = ze;
                u2 += ze * ze;
            }
            if (2 * j + 1 <= D) {
                X[(2 * j) * kFusedPaths + P] = zo;
                u2 += zo * zo;
            }
        }
    }
    double ldet[4] = {0.0, 0.0, 0.0, 0.0};        // this wave's share of log det, path 16nb + (l & 15)
    for (int c = 0; c < net.n_layers; ++c) {
        const FlowLayerDev& L = net.layer[c];
        __syncthreads();                             // X complete, act free
        {   // x_A tile: thread (P, inputs 16w..16w+15)
            bf16x8 v0, v1;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int k0 = 16 * w + q, k1 = 16 * w + 8 + q;
                v0[q] = (__bf16)(float)(k0 < L.dA ? X[L.Aidx[k0] * kFusedPaths + P] : 0.0);
                v1[q] = (__bf16)(float)(k1 < L.dA ? X[L.Aidx[k1] * kFusedPaths + P] : 0.0);
            }
            *reinterpret_cast<bf16x8*>(act + P * kLdXa + 16 * w) = v0;
            *reinterpret_cast<bf16x8*>(act + P * kLdXa + 16 * w + 8) = v1;
        }
        __syncthreads();
        floatx4 acc[2][4];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[mb][nb] = mma16(L.W1 + (32 * w + 16 * mb) * kFlowK, kFlowK, act + 16 * nb * kLdXa, kLdXa, kFlowK,
                                    floatx4{0.f, 0.f, 0.f, 0.f});
        __syncthreads();                             // every wave has read x_A
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int h0 = 32 * w + 16 * mb + 4 * (l >> 4);
            float bias[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) bias[j] = L.b1[h0 + j];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const int Pn = 16 * nb + (l & 15);
                bf16x4 hv;
#pragma unroll
                for (int j = 0; j < 4; ++j) hv[j] = (__bf16)silu(acc[mb][nb][j] + bias[j]);
                *reinterpret_cast<bf16x4*>(act + hs_index(Pn, h0)) = hv;
            }
        }
        __syncthreads();
        floatx4 os[4], ot[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            os[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            ot[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            const int Pn = 16 * nb + (l & 15);
            for (int ks = 0; ks < kFlowH; ks += 32) {
                const bf16x8 hb = *reinterpret_cast<const bf16x8*>(act + hs_index(Pn, ks + 8 * (l >> 4)));
                const bf16x8 as = *reinterpret_cast<const bf16x8*>(L.W2 + (16 * w + (l & 15)) * kFlowH + ks + 8 * (l >> 4));
                const bf16x8 at = *reinterpret_cast<const bf16x8*>(L.W2 + (64 + 16 * w + (l & 15)) * kFlowH + ks +
                                                                  8 * (l >> 4));
                os[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as, hb, os[nb], 0, 0, 0);
                ot[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(at, hb, ot[nb], 0, 0, 0);
            }
        }
        // affine update of coordinates k = 16w + 4(l>>4) + j, paths 16nb + (l & 15)
        const int kb = 16 * w + 4 * (l >> 4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kb + j;
            if (k < L.dB) {
                const float bs = L.b2[k], bt = L.b2[64 + k];
                const int row = L.Bidx[k] * kFusedPaths;
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    const float sv = 2.0f * tanh_fast(0.5f * (os[nb][j] + bs));
                    const int Pn = 16 * nb + (l & 15);
                    X[row + Pn] = X[row + Pn] * exp_logscale(double(sv)) + double(ot[nb][j] + bt);
                    os[nb][j] = sv;
                }
            } else {
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) os[nb][j] = 0.f;
            }
        }
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            double v = double(os[nb][0]) + double(os[nb][1]) + double(os[nb][2]) + double(os[nb][3]);
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            ldet[nb] += v;
        }
    }
    __syncthreads();
    // ---- |z|^2 in the order of |u|^2, optional copy of z
    double z2 = 0.0;
    for (int j = w; 2 * j <= D; j += 4) {
        if (j > 0) {
            const double z = X[(2 * j - 1) * kFusedPaths + P];
            z2 += z * z;
            if (z_out && valid) z_out[uint64_t(2 * j - 1) * zld + local] = z;
        }
        if (2 * j + 1 <= D) {
            const double z = X[(2 * j) * kFusedPaths + P];
            z2 += z * z;
            if (z_out && valid) z_out[uint64_t(2 * j) * zld + local] = z;
        }
    }
    // ---- bisection in place, level by level: X[h-1] becomes the point of node h
    for (int lev = 1; lev <= s; ++lev) {
        const int step = 1 << (s - lev), cnt = 1 << (lev - 1);
        for (int i = w; i < cnt; i += 4) {
            const int h = cnt + i, pos = (2 * i + 1) * step;
            const int pl = pos - step, pr = pos + step;
            const double ql = pl == 0 ? a : X[(node_of_position(pl, s) - 1) * kFusedPaths + P];
            const double qr = pr == N ? b : X[(node_of_position(pr, s) - 1) * kFusedPaths + P];
            X[(h - 1) * kFusedPaths + P] = sig[lev] * X[(h - 1) * kFusedPaths + P] + 0.5 * (ql + qr);
        }
        __syncthreads();
    }
    // ---- level-s action: group w takes slices [w*per, (w+1)*per), 8 per coefficient pass
    double S = 0.0;
    {
        const int per = (N + 3) / 4;
        const int k0 = w * per, k1 = min(N, k0 + per);
        auto point = [&](int pos) -> double {
            return pos == 0 ? a : (pos >= N ? b : X[(node_of_position(pos, s) - 1) * kFusedPaths + P]);
        };
        if (per % 8 == 0) {
            for (int k = k0; k < k1; k += 8) {
                double qa[8], qb[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    qa[i] = point(k + i);
                    qb[i] = point(k + i + 1);
                }
                if (even)
                    GenericEval64<true>{tab, deg, K, stride}.eval<8>(0, qa, qb, S);
                else
                    GenericEval64<false>{tab, deg, K, stride}.eval<8>(0, qa, qb, S);
            }
        } else {
            for (int k = k0; k < k1; ++k) {
                double qa[1] = {point(k)}, qb[1] = {point(k + 1)};
                if (even)
                    GenericEval64<true>{tab, deg, K, stride}.eval<1>(0, qa, qb, S);
                else
                    GenericEval64<false>{tab, deg, K, stride}.eval<1>(0, qa, qb, S);
            }
        }
    }
    // ---- combine the four groups / waves in a fixed order
    double* red = reinterpret_cast<double*>(act);   // [4][4][64]: u2, z2, S, log det
    red[(0 * 4 + w) * kFusedPaths + P] = u2;
    red[(1 * 4 + w) * kFusedPaths + P] = z2;
    red[(2 * 4 + w) * kFusedPaths + P] = S;
    if (l < 16) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) red[(3 * 4 + w) * kFusedPaths + 16 * nb + l] = ldet[nb];
    }
    __syncthreads();
    if (t < kFusedPaths && valid) {
        double sum[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double* r = red + q * 4 * kFusedPaths + P;
            sum[q] = ((r[0] + r[kFusedPaths]) + r[2 * kFusedPaths]) + r[3 * kFusedPaths];
        }
        ell_out[local] = -(sum[2] - shift) - 0.5 * sum[1] + 0.5 * sum[0] + sum[3];
        if (logdet_out) logdet_out[local] = sum[3];
    }
}

// ------------------------------------------------------------------------------------ launchers
static inline uint32_t blocks_for(uint64_t n) { return uint32_t((n + kBlock - 1) / kBlock); }

hipError_t launch_train_fwd(const FlowNet& net, const RngKey& key, const int* step, uint64_t n, int D, double* Xg,
                            uint64_t ld, uint64_t plane, double* hu2, double* logdet, hipStream_t st) {
    const uint64_t tiles = (n + kTP - 1) / kTP;
    if (D > kFusedMaxD || tiles == 0 || tiles > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_train_fwd, dim3(uint32_t(tiles)), dim3(kBlock), 0, st, net, key, step, n, D, Xg, ld, plane, hu2,
                       logdet);
    return hipGetLastError();
}

hipError_t launch_train_bwd(const FlowNet& net, const double* Xg, const double* G, uint64_t ld, uint64_t plane, uint64_t n,
                            int D, const double* alpha, const TrainPlanes& planes, hipStream_t st) {
    const uint64_t tiles = (n + kTP - 1) / kTP;
    if (D > kFusedMaxD || tiles == 0 || tiles > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_train_bwd, dim3(uint32_t(tiles)), dim3(kBlock), 0, st, net, Xg, G, ld, plane, n, D, alpha,
                       planes);
    return hipGetLastError();
}

static int wgrad_slices(uint64_t ld) {
    const uint64_t nc = ld / kWgChunk;
    return int(nc < uint64_t(kWgSlices) ? nc : uint64_t(kWgSlices));
}

hipError_t launch_flow_wgrad(const TrainPlanes& planes, int layers, float* part, float* grad, hipStream_t st) {
    if (layers < 1 || layers > kFlowMaxLayers || planes.ld == 0 || planes.ld % kWgChunk) return hipErrorInvalidValue;
    const int slices = wgrad_slices(planes.ld);
    hipLaunchKernelGGL(k_flow_wgrad_part, dim3(uint32_t(layers), 24, uint32_t(slices)), dim3(kBlock), 0, st, planes,
                       slices, part);
    const uint64_t total = uint64_t(layers) * kFlowNP;
    hipLaunchKernelGGL(k_flow_wgrad_sum, dim3(uint32_t((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, part,
                       slices, total, grad);
    return hipGetLastError();
}

size_t flow_wgrad_part_floats(int layers) { return size_t(kWgSlices) * size_t(layers) * kFlowNP; }
uint64_t flow_plane_ld(uint64_t batch) { return (batch + kWgChunk - 1) / kWgChunk * kWgChunk; }

hipError_t launch_flow_action_grad(const double* tab, const int* deg, int K, int even, const double* sig, double shift,
                                   double a, double b, int s, const double* X, uint64_t ld, uint64_t n,
                                   const double* hu2, const double* logdet, double* ell, double* G, hipStream_t st) {
    if (s < 1 || (1 << s) > kAgMaxN || !G) return hipErrorInvalidValue;
    const uint32_t blocks = uint32_t((n + kAgPaths - 1) / kAgPaths);
    hipLaunchKernelGGL(k_flow_action_grad, dim3(blocks), dim3(kBlock), 0, st, tab, deg, K, even, sig, shift, a, b, s,
                       X, ld, n, hu2, logdet, ell, G);
    return hipGetLastError();
}

hipError_t launch_flow_partials(const double* ell, uint64_t ell_first_path, uint64_t n_total, uint64_t first_chunk,
                                uint64_t n_chunks, double* partials, hipStream_t st) {
    hipLaunchKernelGGL(k_flow_partials, dim3(uint32_t(n_chunks)), dim3(kBlock), 0, st, ell, ell_first_path, n_total,
                       first_chunk, partials);
    return hipGetLastError();
}

hipError_t launch_flow_fused(const FlowNet& net, const RngKey& key, uint64_t first_path, uint64_t n, int s,
                             const double* tab, const int* deg, int K, int stride, int even, const double* sig, double shift,
                             double a, double b, double* ell, double* logdet, double* z, uint64_t zld,
                             hipStream_t st) {
    if (s < 1 || (1 << s) - 1 > kFusedMaxD || net.n_layers < 0 || net.n_layers > kFlowMaxLayers)
        return hipErrorInvalidValue;
    const uint32_t tiles = uint32_t((n + kFusedPaths - 1) / kFusedPaths);
    hipLaunchKernelGGL(k_flow_fused, dim3(tiles), dim3(kBlock), 0, st, net, key, first_path, n, s, tab, deg, K, stride,
                       even, sig, shift, a, b, ell, logdet, z, zld);
    return hipGetLastError();
}

hipError_t launch_flow_alpha(const double* ell, uint64_t n, double beta, double* alpha, double* loss_out,
                             const int* step, hipStream_t st) {
    hipLaunchKernelGGL(k_flow_alpha, dim3(1), dim3(kBlock), 0, st, ell, n, beta, alpha, loss_out, step);
    return hipGetLastError();
}

hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int layers, const int* step, float lr,
                       __bf16* W1, __bf16* W2, __bf16* W1T, __bf16* W2T, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(uint64_t(layers) * kFlowNP)), dim3(kBlock), 0, st, theta, m, v, grad,
                       layers, step, lr, W1, W2, W1T, W2T);
    return hipGetLastError();
}

hipError_t launch_params_to_bf16(const float* theta, int layers, __bf16* W1, __bf16* W2, __bf16* W1T, __bf16* W2T,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_params_to_bf16, dim3(blocks_for(uint64_t(layers) * kFlowNP)), dim3(kBlock), 0, st, theta,
                       layers, W1, W2, W1T, W2T);
    return hipGetLastError();
}

hipError_t launch_step_inc(int* step, hipStream_t st) {
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(1), 0, st, step);
    return hipGetLastError();
}

}  // namespace pimc
