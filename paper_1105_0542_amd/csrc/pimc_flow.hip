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
// The training step works on tiles of kTP = 16 paths (256 workgroups at a batch of 4096, one per CU):
//  * k_train_fwd carries a tile through the base normals and every coupling in LDS -- the same
//    bf16 MFMA products and FP64 affine update as the fused estimation kernel -- and keeps each
//    layer's input X_c (FP64 planes [h-1][path]) for the backward;
//  * k_train_bwd recomputes each layer from X_c with the same products and back-propagates through
//    it on FP32 MFMA (v_mfma_f32_16x16x4f32): the bf16 weights and activations of the forward enter
//    as exact FP32 values, so the gradient is the derivative of the map the forward computes, up to
//    FP32 accumulation. It writes, per layer, the output and pre-activation gradients (FP32) and the
//    conditioner inputs and hidden activations (bf16) as [row][path] planes;
//  * k_flow_wgrad forms the parameter gradients from those planes: each 16 x 16 block of a weight
//    gradient and each bias row is summed over the batch by one workgroup in a fixed order.
constexpr int kTP = 16;                        // paths per training tile
constexpr int kFusedMaxD = 127;                // coordinates of a tile (N <= 128)
constexpr int kTLdA = kFlowK + 8;              // xa [P][in] row stride (bf16 elements)
constexpr int kTLdH = kFlowH + 8;              // hs [P][hid] row stride (bf16 elements)
constexpr int kTLdG = kFlowH + 4;              // go, gp [P][row] row stride (floats)

// C(16x16) += A(16 rows x K) * BT(16 rows x K)^T on FP32 MFMA: A rows bf16 in global memory
// (converted exactly), BT rows FP32; K a multiple of 32.
__device__ __forceinline__ floatx4 mma16_f32_bf16A(const __bf16* A, int lda, const float* BT, int ldb, int K, floatx4 c) {
    const int l = threadIdx.x & 63;
    const __bf16* ar = A + (l & 15) * lda + (l >> 4);
    const float* br = BT + (l & 15) * ldb + (l >> 4);
    for (int ks = 0; ks < K; ks += 32) {
        float a[8], bv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            a[q] = float(ar[ks + 4 * q]);
            bv[q] = br[ks + 4 * q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], bv[q], c, 0, 0, 0);
    }
    return c;
}

// x_A tile of layer L: bf16 [P][in] from the FP64 tile X[(h-1)*kTP + P] (inputs beyond dA are 0).
__device__ __forceinline__ void train_xa(const FlowLayerDev& L, const double* X, __bf16* xa) {
    for (int i = threadIdx.x; i < kTP * kFlowK; i += kBlock) {
        const int P = i % kTP, k = i / kTP;
        xa[P * kTLdA + k] = (__bf16)(float)(k < L.dA ? X[L.Aidx[k] * kTP + P] : 0.0);
    }
}

// Hidden layer of the tile: wave w computes hidden rows 32w..32w+31 for the 16 paths; pre-activation
// (with bias) returned in pre[mb][j] for hid = 32w + 16mb + 4(l>>4) + j, path l & 15; h = silu(pre)
// stored to hs [P][hid] as bf16.
__device__ __forceinline__ void train_hidden(const FlowLayerDev& L, const __bf16* xa, __bf16* hs, floatx4 (&pre)[2]) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const int h0 = 32 * w + 16 * mb;
        pre[mb] = mma16(L.W1 + h0 * kFlowK, kFlowK, xa, kTLdA, kFlowK, floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int hid = h0 + 4 * (l >> 4) + j;
            pre[mb][j] += L.b1[hid];
            hs[(l & 15) * kTLdH + hid] = (__bf16)silu(pre[mb][j]);
        }
    }
}

// Output layer: wave w computes s_hat rows 16w..16w+15 (os) and t rows 64+16w.. (ot) for the tile;
// lane l, slot j holds coordinate 16w + 4(l>>4) + j of path l & 15 (bias not added).
__device__ __forceinline__ void train_output(const FlowLayerDev& L, const __bf16* hs, floatx4& os, floatx4& ot) {
    const int w = threadIdx.x >> 6;
    os = mma16(L.W2 + (16 * w) * kFlowH, kFlowH, hs, kTLdH, kFlowH, floatx4{0.f, 0.f, 0.f, 0.f});
    ot = mma16(L.W2 + (64 + 16 * w) * kFlowH, kFlowH, hs, kTLdH, kFlowH, floatx4{0.f, 0.f, 0.f, 0.f});
}

// Base normals (the plain sampler's, stream key.stream + *step), every coupling; X_c (c = 0..L) to
// the planes Xg + c*plane ([h-1][path], ld), |u|^2/2 and log det per path.
__global__ void __launch_bounds__(kBlock) k_train_fwd(FlowNet net, RngKey key, const int* step, uint64_t n, int D,
                                                      double* __restrict__ Xg, uint64_t ld, uint64_t plane,
                                                      double* __restrict__ hu2, double* __restrict__ logdet) {
    __shared__ double X[kFusedMaxD * kTP];
    __shared__ __attribute__((aligned(16))) __bf16 xa[kTP * kTLdA];
    __shared__ __attribute__((aligned(16))) __bf16 hs[kTP * kTLdH];      // also the Box-Muller table at first
    __shared__ double red[kTP][kTP];
    __shared__ double redl[4][kTP];
    static_assert(sizeof(hs) >= kBoxMullerTable * sizeof(double), "table fits the hidden tile");
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const uint64_t p0 = uint64_t(blockIdx.x) * kTP;
    {   // base normals: thread (P = t & 15, g = t >> 4) takes node pairs j = g, g + 16, ...
        double* bm = reinterpret_cast<double*>(hs);
        load_bm_table(bm, kBlock);
        __syncthreads();
        RngKey k = key;
        if (step) k.stream += uint32_t(*step);
        const int P = t & 15, g = t >> 4;
        const PathRng pr = path_rng(k, p0 + uint64_t(P));
        double u2 = 0.0;
        for (int j = g; 2 * j <= D; j += 16) {
            double ze, zo;
            normal_pair(k, pr, uint32_t(j), bm, ze, zo);
            if (j > 0) {
                X[(2 * j - 1) * kTP + P] = ze;
                u2 += ze * ze;
            }
            if (2 * j + 1 <= D) {
                X[(2 * j) * kTP + P] = zo;
                u2 += zo * zo;
            }
        }
        red[g][P] = u2;
    }
    double ldet = 0.0;                               // this wave's share of log det of path l & 15
    for (int c = 0; c < net.n_layers; ++c) {
        const FlowLayerDev& L = net.layer[c];
        __syncthreads();                             // X complete; hs, xa free
        for (int i = t; i < D * kTP; i += kBlock) {
            const uint64_t P = p0 + uint64_t(i % kTP);
            if (P < n) Xg[uint64_t(c) * plane + uint64_t(i / kTP) * ld + P] = X[i];
        }
        train_xa(L, X, xa);
        __syncthreads();
        floatx4 pre[2];
        train_hidden(L, xa, hs, pre);
        __syncthreads();
        floatx4 os, ot;
        train_output(L, hs, os, ot);
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 16 * w + 4 * (l >> 4) + j;
            if (k < L.dB) {
                const float sv = 2.0f * tanh_fast(0.5f * (os[j] + L.b2[k]));
                const int a = L.Bidx[k] * kTP + (l & 15);
                X[a] = X[a] * exp_logscale(double(sv)) + double(ot[j] + L.b2[64 + k]);
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
        const uint64_t P = p0 + uint64_t(i % kTP);
        if (P < n) Xg[uint64_t(net.n_layers) * plane + uint64_t(i / kTP) * ld + P] = X[i];
    }
    if (t < kTP && p0 + t < n) {
        double u2 = 0.0, ld2 = 0.0;
        for (int g = 0; g < kTP; ++g) u2 += red[g][t];
        for (int q = 0; q < 4; ++q) ld2 += redl[q][t];
        hu2[p0 + t] = 0.5 * u2;
        logdet[p0 + t] = ld2;
    }
}

// Backward through every layer, last first: G (d sum_i alpha_i l_i / d layer output, [h-1][path])
// becomes the gradient for the layer input; the planes of TrainPlanes are written for k_flow_wgrad.
__global__ void __launch_bounds__(kBlock) k_train_bwd(FlowNet net, const double* __restrict__ Xg, double* __restrict__ Gg,
                                                      uint64_t ld, uint64_t plane, uint64_t n, int D,
                                                      const double* __restrict__ alpha, TrainPlanes pl) {
    __shared__ double G[kFusedMaxD * kTP];
    __shared__ double X[kFusedMaxD * kTP];
    __shared__ __attribute__((aligned(16))) __bf16 xa[kTP * kTLdA];
    __shared__ __attribute__((aligned(16))) __bf16 hs[kTP * kTLdH];
    __shared__ float go[kTP * kTLdG];
    __shared__ float gp[kTP * kTLdG];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int P = l & 15;
    const uint64_t p0 = uint64_t(blockIdx.x) * kTP;
    const bool valid = p0 + uint64_t(P) < n;
    const double al = valid ? alpha[p0 + P] : 0.0;
    for (int i = t; i < D * kTP; i += kBlock) {
        const uint64_t Pi = p0 + uint64_t(i % kTP);
        G[i] = Pi < n ? Gg[uint64_t(i / kTP) * ld + Pi] : 0.0;
    }
    for (int c = net.n_layers - 1; c >= 0; --c) {
        const FlowLayerDev& L = net.layer[c];
        float* goT = pl.goT + uint64_t(c) * pl.g_stride;
        float* gpT = pl.gpT + uint64_t(c) * pl.g_stride;
        __bf16* hT = pl.hT + uint64_t(c) * pl.h_stride;
        __bf16* xaT = pl.xaT + uint64_t(c) * pl.xa_stride;
        __syncthreads();                             // G complete; X, xa, hs, go, gp free
        for (int i = t; i < D * kTP; i += kBlock) {
            const uint64_t Pi = p0 + uint64_t(i % kTP);
            X[i] = Pi < n ? Xg[uint64_t(c) * plane + uint64_t(i / kTP) * ld + Pi] : 0.0;
        }
        __syncthreads();
        train_xa(L, X, xa);
        __syncthreads();
        for (int i = t; i < kTP * kFlowK; i += kBlock) {
            const int Pi = i % kTP, k = i / kTP;
            if (p0 + uint64_t(Pi) < n) xaT[uint64_t(k) * ld + p0 + Pi] = xa[Pi * kTLdA + k];
        }
        floatx4 pre[2];
        train_hidden(L, xa, hs, pre);
        __syncthreads();
        for (int i = t; i < kTP * kFlowH; i += kBlock) {
            const int Pi = i % kTP, k = i / kTP;
            if (p0 + uint64_t(Pi) < n) hT[uint64_t(k) * ld + p0 + Pi] = hs[Pi * kTLdH + k];
        }
        floatx4 os, ot;
        train_output(L, hs, os, ot);
        // affine backward of coordinate k of path P (this lane's slots)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 16 * w + 4 * (l >> 4) + j;
            float gsh = 0.f, gt = 0.f;
            if (k < L.dB && valid) {
                const float th = tanh_fast(0.5f * (os[j] + L.b2[k]));
                const float sv = 2.0f * th;
                const int a = L.Bidx[k] * kTP + P;
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
                goT[uint64_t(k) * ld + p0 + P] = gsh;
                goT[uint64_t(64 + k) * ld + p0 + P] = gt;
            }
        }
        __syncthreads();
        // g_h = W2^T g_o (A = W2T [hid][out]), g_pre = g_h silu'(pre)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int h0 = 32 * w + 16 * mb;
            const floatx4 gh = mma16_f32_bf16A(L.W2T + h0 * kFlowH, kFlowH, go, kTLdG, kFlowH, floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int hid = h0 + 4 * (l >> 4) + j;
                const float v = pre[mb][j];
                const float sg = sigmoid_fast(v);
                const float g = valid ? gh[j] * (sg * (1.0f + v * (1.0f - sg))) : 0.f;
                gp[P * kTLdG + hid] = g;
                if (valid) gpT[uint64_t(hid) * ld + p0 + P] = g;
            }
        }
        __syncthreads();
        // g_xa = W1^T g_pre (A = W1T [in][hid]) into G of the conditioner coordinates
        {
            const floatx4 gx = mma16_f32_bf16A(L.W1T + (16 * w) * kFlowH, kFlowH, gp, kTLdG, kFlowH,
                                               floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * w + 4 * (l >> 4) + j;
                if (k < L.dA && valid) G[L.Aidx[k] * kTP + P] += double(gx[j]);
            }
        }
    }
}

// Parameter gradients of every layer from the planes: blockIdx.y < 64 a 16 x 16 block of g_W2
// (rows out, columns hid), < 96 a block of g_W1 (rows hid, columns in), else 16 bias rows (b2 rows
// 0..127, b1 rows 128..255). A weight block: wave w sums paths [w q, (w+1) q) on FP32 MFMA, then the
// four partial blocks are added in wave order. A bias row: lane-strided sums in FP64, then a wave
// butterfly. grad: [layer][kFlowNP] FP32.
__global__ void __launch_bounds__(kBlock) k_flow_wgrad(TrainPlanes pl, uint64_t ld, uint64_t n, float* __restrict__ grad) {
    __shared__ float part[4][256];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int c = blockIdx.x, b = blockIdx.y;
    const float* goT = pl.goT + uint64_t(c) * pl.g_stride;
    const float* gpT = pl.gpT + uint64_t(c) * pl.g_stride;
    const __bf16* hT = pl.hT + uint64_t(c) * pl.h_stride;
    const __bf16* xaT = pl.xaT + uint64_t(c) * pl.xa_stride;
    float* gl = grad + uint64_t(c) * kFlowNP;
    if (b < 96) {
        const bool w2 = b < 64;
        const int r0 = w2 ? 16 * (b / 8) : 16 * ((b - 64) / 4);
        const int c0 = w2 ? 16 * (b % 8) : 16 * ((b - 64) % 4);
        const float* A = (w2 ? goT : gpT) + uint64_t(r0 + (l & 15)) * ld;
        const __bf16* B = (w2 ? hT : xaT) + uint64_t(c0 + (l & 15)) * ld;
        const uint64_t q = ((n + 15) / 16) * 4;      // paths per wave, a multiple of 4
        const uint64_t k0 = uint64_t(w) * q, k1 = k0 + q < n ? k0 + q : n;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        for (uint64_t k = k0; k < k1; k += 4) {
            const uint64_t kk = k + uint64_t(l >> 4);
            const float a = kk < k1 ? A[kk] : 0.f;
            const float bv = kk < k1 ? float(B[kk]) : 0.f;
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) part[w][(4 * (l >> 4) + j) * 16 + (l & 15)] = acc[j];
        __syncthreads();
        const int r = t >> 4, col = t & 15;
        const float v = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
        if (w2)
            gl[kFlowOffW2 + (r0 + r) * kFlowH + c0 + col] = v;
        else
            gl[(r0 + r) * kFlowK + c0 + col] = v;
    } else {
        const int rb = b - 96;
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * rb + 4 * w + i;
            const float* src = row < 128 ? goT + uint64_t(row) * ld : gpT + uint64_t(row - 128) * ld;
            double sacc = 0.0;
            for (uint64_t k = uint64_t(l); k < n; k += 64) sacc += double(src[k]);
            sacc = wave_sum(sacc);
            if (l == 0) {
                if (row < 128)
                    gl[kFlowOffB2 + row] = float(sacc);
                else
                    gl[kFlowOffB1 + row - 128] = float(sacc);
            }
        }
    }
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
    const int t = threadIdx.x, P = t & 15, g = t >> 4;
    const uint64_t path = uint64_t(blockIdx.x) * kAgPaths + uint64_t(P);
    const bool valid = path < n;
    const int N = 1 << s;
    if (g == 0) {
        Q[P] = a;
        Q[N * kAgPaths + P] = b;
    }
    __syncthreads();
    for (int lev = 1; lev <= s; ++lev) {
        const int step = 1 << (s - lev), cnt = 1 << (lev - 1);
        for (int i = g; i < cnt; i += 16) {
            const int h = cnt + i, pos = (2 * i + 1) * step;
            const double z = valid ? X[uint64_t(h - 1) * ld + path] : 0.0;
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
            if (valid) {
                const double z = X[uint64_t(h - 1) * ld + path];
                G[uint64_t(h - 1) * ld + path] = -sig[lev] * Q[pos * kAgPaths + P] - z;
            }
        }
        // the node points at this level depend on the two neighbouring coarser points
        for (int p2 = 2 * step * (1 + g); p2 < N; p2 += 2 * step * 16)
            Q[p2 * kAgPaths + P] = (Q[p2 * kAgPaths + P] + 0.5 * Q[(p2 + step) * kAgPaths + P]) +
                                   0.5 * Q[(p2 - step) * kAgPaths + P];
        __syncthreads();
    }
    for (int h = 1 + g; h < N; h += 16) {
        const double z = valid ? X[uint64_t(h - 1) * ld + path] : 0.0;
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
    for (uint64_t i = t; i < n; i += kBlock)
        alpha[i] = (1.0 - beta) * 2.0 * exp(2.0 * ell[i] - mx) / se - beta / double(n);
    if (t == 0 && loss) loss[step ? *step : 0] = (1.0 - beta) * (mx + log(se / double(n))) - beta * sl / double(n);
}

__global__ void k_flow_seed(double* __restrict__ G, const double* __restrict__ alpha, int D, uint64_t ld, uint64_t n) {
    const uint64_t g = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (g >= uint64_t(D) * n) return;
    const uint64_t h = g / n, i = g % n;
    G[h * ld + i] *= alpha[i];
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

hipError_t launch_train_bwd(const FlowNet& net, const double* Xg, double* G, uint64_t ld, uint64_t plane, uint64_t n,
                            int D, const double* alpha, const TrainPlanes& planes, hipStream_t st) {
    const uint64_t tiles = (n + kTP - 1) / kTP;
    if (D > kFusedMaxD || tiles == 0 || tiles > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_train_bwd, dim3(uint32_t(tiles)), dim3(kBlock), 0, st, net, Xg, G, ld, plane, n, D, alpha,
                       planes);
    return hipGetLastError();
}

hipError_t launch_flow_wgrad(const TrainPlanes& planes, int layers, uint64_t ld, uint64_t n, float* grad,
                             hipStream_t st) {
    if (layers < 1 || layers > kFlowMaxLayers) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_flow_wgrad, dim3(uint32_t(layers), 96 + 16), dim3(kBlock), 0, st, planes, ld, n, grad);
    return hipGetLastError();
}

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

hipError_t launch_flow_seed(double* G, const double* alpha, int D, uint64_t ld, uint64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_flow_seed, dim3(blocks_for(uint64_t(D) * n)), dim3(kBlock), 0, st, G, alpha, D, ld, n);
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
