// Learned proposal for the bisection normals: affine couplings whose conditioners are 2-layer MLPs
// (bfloat16 MFMA with FP32 accumulation), affine update, log-determinant, action and weights in
// FP64. Shared by the flow kernels (pimc_flow.hip) and the host code.
//
// The estimator stays the paper's (Sec. 4): A_N^(p) = K_0 E_phi[exp(-sum eps W_p)]; with z = f(u),
// u ~ N(0, I), it is K_0 E_u[w] with log w = -(S(z) - S_ref) - |z|^2/2 + |u|^2/2 + log det df/du.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pimc_device.hpp"

namespace pimc {

constexpr int kFlowH = 128;                       // hidden width
constexpr int kFlowK = 64;                        // padded conditioner width (|A| <= 64, |B| <= 64)
constexpr int kFlowNP = kFlowH * kFlowK + kFlowH + kFlowH * kFlowH + kFlowH;   // parameters per layer
constexpr int kFlowOffB1 = kFlowH * kFlowK;
constexpr int kFlowOffW2 = kFlowOffB1 + kFlowH;
constexpr int kFlowOffB2 = kFlowOffW2 + kFlowH * kFlowH;
constexpr int kFlowMaxLayers = 16;

// One coupling layer as the kernels read it.
struct FlowLayerDev {
    const __bf16* W1;      // [128][64]  row-major [hidden][in]
    const __bf16* W2;      // [128][128] row-major [out][hidden]
    const __bf16* W1T;     // [64][128]  [in][hidden]
    const __bf16* W2T;     // [128][128] [hidden][out]
    const float* b1;       // [128]
    const float* b2;       // [128]
    const int* Aidx;       // [64] conditioner coordinates (heap node - 1), ascending
    const int* Bidx;       // [64] transformed coordinates
    int dA, dB;
};

// Every layer of a proposal, passed by value (kernel arguments: scalar loads).
struct FlowNet {
    FlowLayerDev layer[kFlowMaxLayers];
    const int* masks;      // [4][128]: the Aidx and Bidx arrays of the four layer types, zero-padded
    int n_layers;
};

// Fused estimation: base normals, every coupling, the bisection and the level-s action in one
// kernel per 64 paths (N <= 128). Writes log w per path to ell; log det and z ([h-1]*zld + path)
// only when those pointers are not null.
hipError_t launch_flow_fused(const FlowNet& net, const RngKey& key, uint64_t first_path, uint64_t n, int s,
                             const double* tab, const int* deg, int K, int stride, int even, const double* sig, double shift,
                             double a, double b, double* ell, double* logdet, double* z, uint64_t zld,
                             hipStream_t st);

// Per-layer gradient planes of the training backward (ld paths per row, a multiple of 128 of at
// least the batch, zero beyond the batch): output gradients goT [128 out][ld] and pre-activation
// gradients gpT [128 hid][ld] in FP32, hidden activations hT [128 hid][ld] and conditioner inputs
// xaT [64 in][ld] in bf16; layer c starts at c * *_stride.
struct TrainPlanes {
    float* goT;
    float* gpT;
    __bf16* hT;
    __bf16* xaT;
    uint64_t ld;
    uint64_t g_stride, h_stride, xa_stride;
};
// Leading dimension of the planes for a batch.
uint64_t flow_plane_ld(uint64_t batch);

// Training forward on tiles of 16 paths: base normals (the plain sampler's, stream key.stream +
// *step when step is not null), every coupling; the input of layer c (c = 0..L, L = the output) in
// the plane Xg + c * plane ([h-1][path], ld), |u|^2/2 and log det per path.
hipError_t launch_train_fwd(const FlowNet& net, const RngKey& key, const int* step, uint64_t n, int D, double* Xg,
                            uint64_t ld, uint64_t plane, double* hu2, double* logdet, hipStream_t st);
// Training backward, last layer first, from G (d l / d z of the output, [h-1][path]; read only) and
// alpha (per-path loss weights); writes the gradient planes for launch_flow_wgrad.
hipError_t launch_train_bwd(const FlowNet& net, const double* Xg, const double* G, uint64_t ld, uint64_t plane,
                            uint64_t n, int D, const double* alpha, const TrainPlanes& planes, hipStream_t st);
// Parameter gradients [layer][kFlowNP] (FP32) from the planes, in a fixed order; part: scratch of
// flow_wgrad_part_floats(layers) floats (per-slice partial sums).
hipError_t launch_flow_wgrad(const TrainPlanes& planes, int layers, float* part, float* grad, hipStream_t st);
size_t flow_wgrad_part_floats(int layers);
// Level-s action of the paths in X (N <= 128), log weights ell and G = d ell / dz.
hipError_t launch_flow_action_grad(const double* tab, const int* deg, int K, int even, const double* sig, double shift,
                                   double a, double b, int s, const double* X, uint64_t ld, uint64_t n,
                                   const double* hu2, const double* logdet, double* ell, double* G, hipStream_t st);
// Canonical chunk sums (n, sum d, sum d^2, non-finite count), d = expm1(ell), of chunks
// first_chunk .. first_chunk + n_chunks - 1 of ell (canonical chunks of kChunkPaths paths, the last
// one may be short: n_total paths in all) into partials[chunk][4].
hipError_t launch_flow_partials(const double* ell, uint64_t ell_first_path, uint64_t n_total, uint64_t first_chunk,
                                uint64_t n_chunks, double* partials, hipStream_t st);
hipError_t launch_flow_alpha(const double* ell, uint64_t n, double beta, double* alpha, double* loss_out,
                             const int* step, hipStream_t st);
hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int layers, const int* step, float lr,
                       __bf16* W1, __bf16* W2, __bf16* W1T, __bf16* W2T, hipStream_t st);
hipError_t launch_params_to_bf16(const float* theta, int layers, __bf16* W1, __bf16* W2, __bf16* W1T, __bf16* W2T,
                                 hipStream_t st);
hipError_t launch_step_inc(int* step, hipStream_t st);

}  // namespace pimc
