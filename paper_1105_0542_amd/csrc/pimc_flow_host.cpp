// Host side of the learned proposal (pimc_flow_* in include/pimc.h): parameters and Adam state on
// the device, the training step captured as one HIP graph, and estimation in batches of base paths
// summed in the canonical chunks of the plain estimator (Sec. 4 estimator, reweighted exactly).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "pimc.h"
#include "pimc_flow.hpp"
#include "pimc_host_common.hpp"

using namespace pimc;
using namespace pimc_host;

static_assert(PIMC_FLOW_NPARAM == kFlowNP, "parameter count of the public header");
static_assert(PIMC_FLOW_MAX_LAYERS == kFlowMaxLayers, "layer limit of the public header");

struct pimc_flow {
    pimc_ctx* ctx = nullptr;
    Problem P;
    int L = 0, D = 0;
    uint32_t B = 0;                      // training batch
    float lr = 0.f;
    double beta = 0.0;
    int dA[4] = {0, 0, 0, 0}, dB[4] = {0, 0, 0, 0};
    // device: constants
    double* d_sig = nullptr;             // s+1
    double* d_tab = nullptr;             // level-s table
    int* d_deg = nullptr;                // K
    int* d_mask = nullptr;               // [4][128]: A indices (64), B indices (64)
    // device: parameters
    float* d_theta = nullptr;            // L * NP master
    float* d_m = nullptr;
    float* d_v = nullptr;
    float* d_grad = nullptr;
    void* d_planes = nullptr;            // gradient planes of the training backward (TrainPlanes)
    float* d_wpart = nullptr;            // per-slice partial weight gradients
    TrainPlanes planes{};
    __bf16* d_W1 = nullptr;              // L * 128 * 64
    __bf16* d_W2 = nullptr;              // L * 128 * 128
    __bf16* d_W1T = nullptr;
    __bf16* d_W2T = nullptr;
    int* d_step = nullptr;
    // device: training buffers (ld = B)
    double* d_X = nullptr;               // (L+1) * D * B
    double* d_G = nullptr;               // D * B
    double* d_hu2 = nullptr;
    double* d_logdet = nullptr;
    double* d_ell = nullptr;
    double* d_alpha = nullptr;
    double* d_loss = nullptr;            // loss history, indexed by the step counter
    double* d_gloss = nullptr;           // loss of pimc_flow_grad
    size_t loss_cap = 0;
    // device: estimation buffers (per path: log w, log det; z only for pimc_flow_log_weights)
    uint64_t EB = 0, ZB = 0;
    double* d_Eell = nullptr;
    double* d_Elogdet = nullptr;
    double* d_EX = nullptr;              // [h-1][ZB]
    FlowNet net{};
    // graph of one training step
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t graph_seed = 0;
    uint32_t graph_stream = 0;
    bool graph_valid = false;
    int steps_done = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

namespace {

void subtree_masks(int D, int type, std::vector<int>& A, std::vector<int>& Bv) {
    A.clear();
    Bv.clear();
    for (int h = 1; h <= D; ++h) {
        int side = -1;                   // node 1
        if (h > 1) {
            int bits = 0;
            while ((h >> bits) > 1) ++bits;      // h has bits+1 binary digits
            side = (h >> (bits - 1)) & 1;        // the digit after the leading one: 0 left, 1 right
        }
        bool inA = false;
        switch (type) {
            case 0: inA = side <= 0; break;
            case 1: inA = side != 0; break;
            case 2: inA = (h & 1) == 1; break;
            default: inA = (h & 1) == 0; break;
        }
        (inA ? A : Bv).push_back(h - 1);
    }
}

uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform_pm(uint64_t& x, double r) { return r * (2.0 * double(splitmix64(x) >> 11) * 0x1p-53 - 1.0); }

template <class T>
int dev_alloc(pimc_ctx* c, T** p, size_t count) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess)
        return ctx_fail(c, PIMC_ENOMEM, "hipMalloc(%zu) failed: %s", count * sizeof(T), hipGetErrorString(e));
    return PIMC_OK;
}

FlowLayerDev layer_dev(const pimc_flow* f, int c) {
    FlowLayerDev L;
    L.W1 = f->d_W1 + size_t(c) * kFlowH * kFlowK;
    L.W2 = f->d_W2 + size_t(c) * kFlowH * kFlowH;
    L.W1T = f->d_W1T + size_t(c) * kFlowH * kFlowK;
    L.W2T = f->d_W2T + size_t(c) * kFlowH * kFlowH;
    L.b1 = f->d_theta + size_t(c) * kFlowNP + kFlowOffB1;
    L.b2 = f->d_theta + size_t(c) * kFlowNP + kFlowOffB2;
    L.Aidx = f->d_mask + (c % 4) * 128;
    L.Bidx = f->d_mask + (c % 4) * 128 + 64;
    L.dA = f->dA[c % 4];
    L.dB = f->dB[c % 4];
    return L;
}

// Forward of every layer, the action, the loss weights, the backward and the parameter gradients
// into d_grad. With step != null (training) the base stream and the loss slot follow the device
// step counter.
hipError_t enqueue_grad(pimc_flow* f, const RngKey& key, const int* step, double* loss) {
    const Problem& P = f->P;
    const uint64_t B = f->B;
    const size_t plane = size_t(f->D) * B;
    hipStream_t st = f->ctx->stream;
    hipError_t e = launch_train_fwd(f->net, key, step, B, f->D, f->d_X, B, plane, f->d_hu2, f->d_logdet, st);
    if (e == hipSuccess)
        e = launch_flow_action_grad(f->d_tab, f->d_deg, int(P.deg.size()), P.even ? 1 : 0, f->d_sig,
                                    P.shift[size_t(P.s)], P.a, P.b, P.s, f->d_X + size_t(f->L) * plane, B, B,
                                    f->d_hu2, f->d_logdet, f->d_ell, f->d_G, st);
    if (e == hipSuccess) e = launch_flow_alpha(f->d_ell, B, f->beta, f->d_alpha, loss, step, st);
    if (e == hipSuccess) e = launch_train_bwd(f->net, f->d_X, f->d_G, B, plane, B, f->D, f->d_alpha, f->planes, st);
    if (e == hipSuccess) e = launch_flow_wgrad(f->planes, f->L, f->d_wpart, f->d_grad, st);
    return e;
}

void destroy_graph(pimc_flow* f) {
    if (f->exec) (void)hipGraphExecDestroy(f->exec);
    if (f->graph) (void)hipGraphDestroy(f->graph);
    f->exec = nullptr;
    f->graph = nullptr;
    f->graph_valid = false;
}

int capture_step(pimc_flow* f, uint64_t seed, uint32_t stream_base) {
    pimc_ctx* c = f->ctx;
    destroy_graph(f);
    const RngKey key{uint32_t(seed), uint32_t(seed >> 32), stream_base};
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_grad(f, key, f->d_step, f->d_loss);
    if (e == hipSuccess)
        e = launch_adam(f->d_theta, f->d_m, f->d_v, f->d_grad, f->L, f->d_step, f->lr, f->d_W1, f->d_W2, f->d_W1T,
                        f->d_W2T, c->stream);
    if (e == hipSuccess) e = launch_step_inc(f->d_step, c->stream);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return ctx_fail(c, PIMC_EDEVICE, "flow step capture failed: %s", hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return ctx_fail(c, PIMC_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e2));
    f->graph = g;
    HIP_TRY(c, hipGraphInstantiate(&f->exec, f->graph, nullptr, nullptr, 0));
    f->graph_seed = seed;
    f->graph_stream = stream_base;
    f->graph_valid = true;
    return PIMC_OK;
}

int reset_optimizer(pimc_flow* f) {
    pimc_ctx* c = f->ctx;
    const size_t np = size_t(f->L) * kFlowNP;
    HIP_TRY(c, hipMemsetAsync(f->d_m, 0, np * sizeof(float), c->stream));
    HIP_TRY(c, hipMemsetAsync(f->d_v, 0, np * sizeof(float), c->stream));
    HIP_TRY(c, hipMemsetAsync(f->d_step, 0, sizeof(int), c->stream));
    HIP_TRY(c, launch_params_to_bf16(f->d_theta, f->L, f->d_W1, f->d_W2, f->d_W1T, f->d_W2T, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    f->steps_done = 0;
    return PIMC_OK;
}

void free_flow(pimc_flow* f) {
    destroy_graph(f);
    void* ptrs[] = {f->d_sig, f->d_tab, f->d_deg, f->d_mask, f->d_theta, f->d_m, f->d_v, f->d_grad, f->d_planes, f->d_wpart,
                    f->d_W1, f->d_W2, f->d_W1T, f->d_W2T, f->d_step, f->d_X, f->d_G, f->d_hu2, f->d_logdet,
                    f->d_ell, f->d_alpha, f->d_loss, f->d_gloss, f->d_EX, f->d_Elogdet, f->d_Eell};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (f->e0) (void)hipEventDestroy(f->e0);
    if (f->e1) (void)hipEventDestroy(f->e1);
}

int ensure_estimation(pimc_flow* f, uint64_t eb, uint64_t zb) {
    pimc_ctx* c = f->ctx;
    int st;
    if (eb > f->EB) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (double** p : {&f->d_Eell, &f->d_Elogdet}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        f->EB = 0;
        if ((st = dev_alloc(c, &f->d_Eell, eb))) return st;
        if ((st = dev_alloc(c, &f->d_Elogdet, eb))) return st;
        f->EB = eb;
    }
    if (zb > f->ZB) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (f->d_EX) (void)hipFree(f->d_EX);
        f->d_EX = nullptr;
        f->ZB = 0;
        if ((st = dev_alloc(c, &f->d_EX, size_t(f->D) * zb))) return st;
        f->ZB = zb;
    }
    return PIMC_OK;
}

// Log weights (and log det, and z when want_z) of paths first..first+n-1 by the fused kernel.
hipError_t enqueue_log_weights(pimc_flow* f, const RngKey& key, uint64_t first, uint64_t n, bool want_z) {
    const Problem& P = f->P;
    return launch_flow_fused(f->net, key, first, n, P.s, f->d_tab, f->d_deg, int(P.deg.size()), P.stride, P.even ? 1 : 0,
                             f->d_sig, P.shift[size_t(P.s)], P.a, P.b, f->d_Eell, f->d_Elogdet,
                             want_z ? f->d_EX : nullptr, f->ZB, f->ctx->stream);
}

constexpr uint64_t kEstimationBatch = uint64_t(1) << 20;

}  // namespace

extern "C" {

int pimc_flow_create(pimc_ctx* c, const pimc_potential* V, double m, double a, double b, double T, uint32_t N, int p,
                     const pimc_flow_config* cfg, pimc_flow** out) {
    if (!out) { set_thread_error("out is NULL"); return PIMC_EINVAL; }
    *out = nullptr;
    int st = check_args(V, m, a, b, T, N, p, 2);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!cfg) return ctx_fail(c, PIMC_EINVAL, "config is NULL");
    if (cfg->layers < 1 || cfg->layers > kFlowMaxLayers)
        return ctx_fail(c, PIMC_EINVAL, "layers = %d outside 1..%d", cfg->layers, kFlowMaxLayers);
    if (cfg->batch < 2 || cfg->batch > 65536) return ctx_fail(c, PIMC_EINVAL, "batch = %u outside 2..65536", cfg->batch);
    if (!std::isfinite(cfg->lr) || cfg->lr < 0) return ctx_fail(c, PIMC_EINVAL, "lr must be finite and >= 0");
    if (!(cfg->beta >= 0.0 && cfg->beta <= 1.0)) return ctx_fail(c, PIMC_EINVAL, "beta outside 0..1");
    if (!std::isfinite(cfg->init_scale)) return ctx_fail(c, PIMC_EINVAL, "init_scale is not finite");
    if (N < 2 || N > 128)
        return ctx_fail(c, PIMC_EUNSUPPORTED, "the proposal needs 2 <= N <= 128 (every coupling part <= 64 nodes)");
    HIP_TRY(c, hipSetDevice(c->device));
    pimc_flow* f = new (std::nothrow) pimc_flow();
    if (!f) return ctx_fail(c, PIMC_ENOMEM, "out of host memory");
    f->ctx = c;
    char why[256] = "";
    st = build_problem(V, m, a, b, T, N, p, 0, f->P, why, sizeof(why));
    if (st) {
        delete f;
        return ctx_fail(c, st, "%s", why);
    }
    f->L = cfg->layers;
    f->D = int(N) - 1;
    f->B = cfg->batch;
    f->lr = float(cfg->lr);
    f->beta = cfg->beta;
    auto fail = [&](int s2) {
        free_flow(f);
        delete f;
        return s2;
    };
    const Problem& P = f->P;
    const size_t np = size_t(f->L) * kFlowNP;
    const size_t Bs = f->B;
    const size_t plane = size_t(f->D) * Bs;
    if ((st = dev_alloc(c, &f->d_sig, P.sig.size()))) return fail(st);
    if ((st = dev_alloc(c, &f->d_tab, size_t(P.stride)))) return fail(st);
    if ((st = dev_alloc(c, &f->d_deg, P.deg.size()))) return fail(st);
    if ((st = dev_alloc(c, &f->d_mask, 4 * 128))) return fail(st);
    if ((st = dev_alloc(c, &f->d_theta, np))) return fail(st);
    if ((st = dev_alloc(c, &f->d_m, np))) return fail(st);
    if ((st = dev_alloc(c, &f->d_v, np))) return fail(st);
    if ((st = dev_alloc(c, &f->d_grad, np))) return fail(st);
    {   // gradient planes: goT, gpT (FP32) and hT (bf16), 128 rows each, and xaT (bf16), 64 rows, per
        // layer; rows padded to a multiple of 128 paths and zeroed once (the padding is never written)
        const size_t L = size_t(f->L);
        const size_t ldp = flow_plane_ld(Bs);
        const size_t bytes = L * ldp * (128 * 4 + 128 * 4 + 128 * 2 + 64 * 2);
        unsigned char* base = nullptr;
        if ((st = dev_alloc(c, &base, bytes))) return fail(st);
        f->d_planes = base;
        if (hipMemsetAsync(base, 0, bytes, c->stream) != hipSuccess)
            return fail(ctx_fail(c, PIMC_EDEVICE, "clearing the gradient planes failed"));
        f->planes.goT = reinterpret_cast<float*>(base);
        f->planes.gpT = f->planes.goT + L * 128 * ldp;
        f->planes.hT = reinterpret_cast<__bf16*>(f->planes.gpT + L * 128 * ldp);
        f->planes.xaT = f->planes.hT + L * 128 * ldp;
        f->planes.ld = ldp;
        f->planes.g_stride = 128 * ldp;
        f->planes.h_stride = 128 * ldp;
        f->planes.xa_stride = 64 * ldp;
        if ((st = dev_alloc(c, &f->d_wpart, flow_wgrad_part_floats(f->L)))) return fail(st);
    }
    if ((st = dev_alloc(c, &f->d_W1, size_t(f->L) * kFlowH * kFlowK))) return fail(st);
    if ((st = dev_alloc(c, &f->d_W2, size_t(f->L) * kFlowH * kFlowH))) return fail(st);
    if ((st = dev_alloc(c, &f->d_W1T, size_t(f->L) * kFlowH * kFlowK))) return fail(st);
    if ((st = dev_alloc(c, &f->d_W2T, size_t(f->L) * kFlowH * kFlowH))) return fail(st);
    if ((st = dev_alloc(c, &f->d_step, 1))) return fail(st);
    if ((st = dev_alloc(c, &f->d_X, size_t(f->L + 1) * plane))) return fail(st);
    if ((st = dev_alloc(c, &f->d_G, plane))) return fail(st);
    if ((st = dev_alloc(c, &f->d_hu2, Bs))) return fail(st);
    if ((st = dev_alloc(c, &f->d_logdet, Bs))) return fail(st);
    if ((st = dev_alloc(c, &f->d_ell, Bs))) return fail(st);
    if ((st = dev_alloc(c, &f->d_alpha, Bs))) return fail(st);
    f->loss_cap = 1 << 16;
    if ((st = dev_alloc(c, &f->d_loss, f->loss_cap))) return fail(st);
    if ((st = dev_alloc(c, &f->d_gloss, 1))) return fail(st);
    if (hipEventCreate(&f->e0) != hipSuccess || hipEventCreate(&f->e1) != hipSuccess)
        return fail(ctx_fail(c, PIMC_EDEVICE, "hipEventCreate failed"));
    // masks
    std::vector<int> mask(4 * 128, 0);
    for (int t = 0; t < 4; ++t) {
        std::vector<int> A, Bv;
        subtree_masks(f->D, t, A, Bv);
        f->dA[t] = int(A.size());
        f->dB[t] = int(Bv.size());
        std::copy(A.begin(), A.end(), mask.begin() + t * 128);
        std::copy(Bv.begin(), Bv.end(), mask.begin() + t * 128 + 64);
    }
    // parameters
    std::vector<float> theta(np, 0.f);
    uint64_t x = cfg->init_seed;
    for (int l = 0; l < f->L; ++l) {
        float* th = theta.data() + size_t(l) * kFlowNP;
        for (int i = 0; i < kFlowH * kFlowK; ++i) th[i] = float(uniform_pm(x, 0.125));
        for (int i = 0; i < kFlowH * kFlowH; ++i) th[kFlowOffW2 + i] = float(cfg->init_scale * uniform_pm(x, 0.05));
    }
    hipStream_t s0 = c->stream;
    const double* tab_s = P.tab.data() + size_t(P.s) * size_t(P.stride);
    if (hipMemcpyAsync(f->d_sig, P.sig.data(), P.sig.size() * 8, hipMemcpyHostToDevice, s0) != hipSuccess ||
        hipMemcpyAsync(f->d_tab, tab_s, size_t(P.stride) * 8, hipMemcpyHostToDevice, s0) != hipSuccess ||
        hipMemcpyAsync(f->d_deg, P.deg.data(), P.deg.size() * 4, hipMemcpyHostToDevice, s0) != hipSuccess ||
        hipMemcpyAsync(f->d_mask, mask.data(), mask.size() * 4, hipMemcpyHostToDevice, s0) != hipSuccess ||
        hipMemcpyAsync(f->d_theta, theta.data(), np * 4, hipMemcpyHostToDevice, s0) != hipSuccess)
        return fail(ctx_fail(c, PIMC_EDEVICE, "upload of the proposal's constants failed"));
    if ((st = reset_optimizer(f))) return fail(st);     // synchronizes: the host vectors may go
    f->net.n_layers = f->L;
    f->net.masks = f->d_mask;
    for (int l = 0; l < f->L; ++l) f->net.layer[l] = layer_dev(f, l);
    *out = f;
    return PIMC_OK;
}

int pimc_flow_destroy(pimc_flow* f) {
    if (!f) return PIMC_OK;
    (void)hipSetDevice(f->ctx->device);
    (void)hipStreamSynchronize(f->ctx->stream);
    free_flow(f);
    delete f;
    return PIMC_OK;
}

int pimc_flow_get_params(pimc_flow* f, float* out, size_t cap, size_t* n_out) {
    if (!f) { set_thread_error("flow is NULL"); return PIMC_EINVAL; }
    pimc_ctx* c = f->ctx;
    const size_t np = size_t(f->L) * kFlowNP;
    if (n_out) *n_out = np;
    if (!out || cap < np) return ctx_fail(c, PIMC_EINVAL, "capacity %zu < %zu", cap, np);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(out, f->d_theta, np * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIMC_OK;
}

int pimc_flow_set_params(pimc_flow* f, const float* in, size_t n) {
    if (!f) { set_thread_error("flow is NULL"); return PIMC_EINVAL; }
    pimc_ctx* c = f->ctx;
    const size_t np = size_t(f->L) * kFlowNP;
    if (!in || n != np) return ctx_fail(c, PIMC_EINVAL, "expected %zu parameters, got %zu", np, n);
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(in[i])) return ctx_fail(c, PIMC_EINVAL, "parameter %zu is not finite", i);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(f->d_theta, in, np * 4, hipMemcpyHostToDevice, c->stream));
    return reset_optimizer(f);
}

// File: 8 bytes "PIMCFLW1", then int32 layers, N, p, parameters per layer, then the FP32 parameters
// (host byte order).
int pimc_flow_save(pimc_flow* f, const char* path) {
    if (!f) { set_thread_error("flow is NULL"); return PIMC_EINVAL; }
    pimc_ctx* c = f->ctx;
    if (!path) return ctx_fail(c, PIMC_EINVAL, "path is NULL");
    const size_t np = size_t(f->L) * kFlowNP;
    std::vector<float> th(np);
    int st = pimc_flow_get_params(f, th.data(), np, nullptr);
    if (st) return st;
    std::FILE* fp = std::fopen(path, "wb");
    if (!fp) return ctx_fail(c, PIMC_EINVAL, "cannot open %s for writing", path);
    const int32_t hdr[4] = {f->L, f->D + 1, f->P.p, kFlowNP};
    bool ok = std::fwrite("PIMCFLW1", 1, 8, fp) == 8 && std::fwrite(hdr, sizeof(hdr), 1, fp) == 1 &&
              std::fwrite(th.data(), sizeof(float), np, fp) == np;
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return ctx_fail(c, PIMC_EINVAL, "write to %s failed", path);
    return PIMC_OK;
}

int pimc_flow_load(pimc_flow* f, const char* path) {
    if (!f) { set_thread_error("flow is NULL"); return PIMC_EINVAL; }
    pimc_ctx* c = f->ctx;
    if (!path) return ctx_fail(c, PIMC_EINVAL, "path is NULL");
    std::FILE* fp = std::fopen(path, "rb");
    if (!fp) return ctx_fail(c, PIMC_EINVAL, "cannot open %s", path);
    char magic[8];
    int32_t hdr[4];
    const size_t np = size_t(f->L) * kFlowNP;
    std::vector<float> th(np);
    bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "PIMCFLW1", 8) == 0 &&
              std::fread(hdr, sizeof(hdr), 1, fp) == 1;
    if (ok && (hdr[0] != f->L || hdr[1] != f->D + 1 || hdr[3] != kFlowNP)) {
        std::fclose(fp);
        return ctx_fail(c, PIMC_EINVAL, "%s holds %d layers for N = %d; this proposal has %d layers, N = %d", path,
                        hdr[0], hdr[1], f->L, f->D + 1);
    }
    ok = ok && std::fread(th.data(), sizeof(float), np, fp) == np;
    std::fclose(fp);
    if (!ok) return ctx_fail(c, PIMC_EINVAL, "%s is not a proposal file", path);
    return pimc_flow_set_params(f, th.data(), np);
}

int pimc_flow_grad(pimc_flow* f, uint64_t seed, uint32_t stream, double* loss, double* ell, float* grad) {
    if (!f) { set_thread_error("flow is NULL"); return PIMC_EINVAL; }
    pimc_ctx* c = f->ctx;
    if (!loss) return ctx_fail(c, PIMC_EINVAL, "loss is NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    const RngKey key{uint32_t(seed), uint32_t(seed >> 32), stream};
    HIP_TRY(c, enqueue_grad(f, key, nullptr, f->d_gloss));
    HIP_TRY(c, hipMemcpyAsync(loss, f->d_gloss, 8, hipMemcpyDeviceToHost, c->stream));
    if (ell) HIP_TRY(c, hipMemcpyAsync(ell, f->d_ell, size_t(f->B) * 8, hipMemcpyDeviceToHost, c->stream));
    if (grad)
        HIP_TRY(c, hipMemcpyAsync(grad, f->d_grad, size_t(f->L) * kFlowNP * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIMC_OK;
}

int pimc_flow_train(pimc_flow* f, uint64_t seed, uint32_t stream_base, uint32_t steps, double* losses, double* ms) {
    if (!f) { set_thread_error("flow is NULL"); return PIMC_EINVAL; }
    pimc_ctx* c = f->ctx;
    if (steps == 0) return PIMC_OK;
    if (uint64_t(f->steps_done) + steps > 0x7fffffffull) return ctx_fail(c, PIMC_EINVAL, "too many steps");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t need = size_t(f->steps_done) + steps;
    if (need > f->loss_cap) {
        size_t cap = f->loss_cap;
        while (cap < need) cap *= 2;
        double* nl = nullptr;
        int st = dev_alloc(c, &nl, cap);
        if (st) return st;
        HIP_TRY(c, hipMemcpyAsync(nl, f->d_loss, size_t(f->steps_done) * 8, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        (void)hipFree(f->d_loss);
        f->d_loss = nl;
        f->loss_cap = cap;
        destroy_graph(f);
    }
    if (!f->graph_valid || f->graph_seed != seed || f->graph_stream != stream_base) {
        int st = capture_step(f, seed, stream_base);
        if (st) return st;
    }
    HIP_TRY(c, hipEventRecord(f->e0, c->stream));
    for (uint32_t i = 0; i < steps; ++i) HIP_TRY(c, hipGraphLaunch(f->exec, c->stream));
    HIP_TRY(c, hipEventRecord(f->e1, c->stream));
    if (losses)
        HIP_TRY(c, hipMemcpyAsync(losses, f->d_loss + f->steps_done, size_t(steps) * 8, hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    f->steps_done += int(steps);
    float t = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&t, f->e0, f->e1));
    if (ms) *ms = t;
    return PIMC_OK;
}

int pimc_flow_log_weights(pimc_flow* f, uint64_t seed, uint32_t stream, uint64_t first_path, uint64_t k_paths,
                          double* ell, double* z, double* logdet) {
    if (!f) { set_thread_error("flow is NULL"); return PIMC_EINVAL; }
    pimc_ctx* c = f->ctx;
    if (k_paths == 0) return PIMC_OK;
    if (k_paths > (uint64_t(1) << 32)) return ctx_fail(c, PIMC_EINVAL, "request too large");
    HIP_TRY(c, hipSetDevice(c->device));
    const uint64_t eb = std::min<uint64_t>(k_paths, kEstimationBatch);
    int st = ensure_estimation(f, eb, z ? eb : 0);
    if (st) return st;
    const RngKey key{uint32_t(seed), uint32_t(seed >> 32), stream};
    std::vector<double> zt;
    for (uint64_t off = 0; off < k_paths; off += eb) {
        const uint64_t n = std::min<uint64_t>(eb, k_paths - off);
        HIP_TRY(c, enqueue_log_weights(f, key, first_path + off, n, z != nullptr));
        if (ell) HIP_TRY(c, hipMemcpyAsync(ell + off, f->d_Eell, n * 8, hipMemcpyDeviceToHost, c->stream));
        if (logdet) HIP_TRY(c, hipMemcpyAsync(logdet + off, f->d_Elogdet, n * 8, hipMemcpyDeviceToHost, c->stream));
        if (z) {
            zt.resize(size_t(f->D) * n);
            for (int h = 0; h < f->D; ++h)
                HIP_TRY(c, hipMemcpyAsync(zt.data() + size_t(h) * n, f->d_EX + size_t(h) * f->ZB, n * 8,
                                          hipMemcpyDeviceToHost, c->stream));
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (z)
            for (uint64_t i = 0; i < n; ++i)
                for (int h = 0; h < f->D; ++h) z[(off + i) * size_t(f->D) + size_t(h)] = zt[size_t(h) * n + i];
    }
    return PIMC_OK;
}

int pimc_flow_amplitude(pimc_flow* f, uint64_t n_samples, uint64_t seed, uint32_t stream, pimc_level_result* out,
                        double* ms) {
    if (!f) { set_thread_error("flow is NULL"); return PIMC_EINVAL; }
    pimc_ctx* c = f->ctx;
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    if (n_samples < 2) return ctx_fail(c, PIMC_EINVAL, "need at least 2 samples");
    HIP_TRY(c, hipSetDevice(c->device));
    const Problem& P = f->P;
    const uint64_t CH = kChunkPaths;
    const uint64_t n_chunks = (n_samples + CH - 1) / CH;
    const uint64_t eb = std::min<uint64_t>(n_chunks * CH, kEstimationBatch);   // a multiple of CH
    int st = ensure_estimation(f, eb, 0);
    if (st) return st;
    st = ensure(c, reinterpret_cast<void**>(&c->d_partials), &c->partial_bytes, size_t(n_chunks) * 4 * 8);
    if (st) return st;
    st = ensure(c, reinterpret_cast<void**>(&c->d_red), &c->red_bytes, 4 * 8);
    if (st) return st;
    st = ensure(c, reinterpret_cast<void**>(&c->d_seg), &c->seg_bytes, 2 * 8);
    if (st) return st;
    c->h_seg.assign({0, n_chunks});
    HIP_TRY(c, hipMemcpyAsync(c->d_seg, c->h_seg.data(), 16, hipMemcpyHostToDevice, c->stream));
    const RngKey key{uint32_t(seed), uint32_t(seed >> 32), stream};
    const uint64_t step = f->EB - f->EB % CH;
    HIP_TRY(c, hipEventRecord(f->e0, c->stream));
    for (uint64_t first = 0; first < n_samples; first += step) {
        const uint64_t n = std::min<uint64_t>(step, n_samples - first);
        HIP_TRY(c, enqueue_log_weights(f, key, first, n, false));
        HIP_TRY(c, launch_flow_partials(f->d_Eell, first, n_samples, first / CH, (n + CH - 1) / CH, c->d_partials,
                                        c->stream));
    }
    HIP_TRY(c, launch_seg_reduce(c->d_partials, c->d_seg, c->d_seg + 1, 1, c->d_red, c->stream));
    HIP_TRY(c, hipEventRecord(f->e1, c->stream));
    double red[4];
    HIP_TRY(c, hipMemcpyAsync(red, c->d_red, 32, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float t = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&t, f->e0, f->e1));
    if (ms) *ms = t;
    c->last_ms = t;
    c->last_partials_ptr = c->d_partials;
    c->last_chunks = n_chunks;
    c->last_chunk_paths = CH;
    c->last_s = P.s;
    c->last_hier = false;
    c->last_shift = P.shift;
    *out = pimc_level_result{};
    const bool bad = assemble_level(red, std::log(P.pref * P.K0) - P.shift[size_t(P.s)], *out);
    return bad ? PIMC_WNONFINITE : PIMC_OK;
}

}  // extern "C"
