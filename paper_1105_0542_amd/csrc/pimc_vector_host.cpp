// Host side of the several-coordinate entry points (pimc_amplitude_radial, pimc_path_actions_radial,
// pimc_level_table_radial and the *_poly variants in include/pimc.h): eq.(MBrec)/(DIA) on polynomials
// in the invariants u = x.x, w = x.xbar, z = xbar.xbar (FP64) for rotation-invariant potentials, or
// in the 2d components of x and xbar for any polynomial potential; the per-level fold (the table
// layout of pimc_vector.hpp, or the records of the component evaluator), the straight-line reference
// actions, and the estimation through the vector kernels.
//
// Invariant forms of the operators in d dimensions (partial derivatives in u, w, z; chain rule with
// grad u = 2x, grad w = xbar, gradbar w = x, gradbar z = 2 xbar):
//     grad^2 f            = 2d f_u + 4u f_uu + 4w f_uw + z f_ww
//     gradbar^2 f         = 2d f_z + 4z f_zz + 4w f_wz + u f_ww
//     grad f . grad g     = 4u f_u g_u + 2w (f_u g_w + f_w g_u) + z f_w g_w
//     gradbar f . gradbar g = u f_w g_w + 2w (f_w g_z + f_z g_w) + 4z f_z g_z
//     xbar . grad f       = 2w f_u + z f_w
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pimc.h"
#include "pimc_host_common.hpp"
#include "pimc_vector.hpp"

using namespace pimc;
using namespace pimc_host;

static_assert(PIMC_MAX_DIM == kVecMaxDim, "dimension limit of the public header");
static_assert(PIMC_MAX_RADIAL_DEGREE == 2, "the table shape bound covers u-degree <= 2");

namespace {

constexpr double kPi = 3.14159265358979323846;

using IKey = std::array<int, 3>;                 // exponents of u, w, z
using IPoly = std::map<IKey, double>;

void axpy(IPoly& y, double a, const IPoly& x) {
    for (const auto& kv : x) y[kv.first] += a * kv.second;
}

IPoly der(const IPoly& f, int var) {
    IPoly out;
    for (const auto& kv : f)
        if (kv.first[size_t(var)]) {
            IKey k = kv.first;
            k[size_t(var)] -= 1;
            out[k] += kv.second * double(kv.first[size_t(var)]);
        }
    return out;
}

IPoly times(const IPoly& f, int var, double s) {
    IPoly out;
    for (const auto& kv : f) {
        IKey k = kv.first;
        k[size_t(var)] += 1;
        out[k] = kv.second * s;
    }
    return out;
}

IPoly mul(const IPoly& a, const IPoly& b) {
    IPoly out;
    for (const auto& ka : a)
        for (const auto& kb : b)
            out[IKey{ka.first[0] + kb.first[0], ka.first[1] + kb.first[1], ka.first[2] + kb.first[2]}] +=
                ka.second * kb.second;
    return out;
}

constexpr int U_ = 0, W_ = 1, Z_ = 2;

IPoly lap(const IPoly& f, int d) {
    const IPoly fu = der(f, U_), fw = der(f, W_);
    IPoly out;
    axpy(out, 2.0 * d, fu);
    axpy(out, 1.0, times(der(fu, U_), U_, 4.0));
    axpy(out, 1.0, times(der(fu, W_), W_, 4.0));
    axpy(out, 1.0, times(der(fw, W_), Z_, 1.0));
    return out;
}

IPoly lapbar(const IPoly& f, int d) {
    const IPoly fz = der(f, Z_), fw = der(f, W_);
    IPoly out;
    axpy(out, 2.0 * d, fz);
    axpy(out, 1.0, times(der(fz, Z_), Z_, 4.0));
    axpy(out, 1.0, times(der(fz, W_), W_, 4.0));
    axpy(out, 1.0, times(der(fw, W_), U_, 1.0));
    return out;
}

IPoly gdot(const IPoly& f, const IPoly& g) {
    const IPoly fu = der(f, U_), fw = der(f, W_), gu = der(g, U_), gw = der(g, W_);
    IPoly out = times(mul(fu, gu), U_, 4.0);
    IPoly cross = mul(fu, gw);
    axpy(cross, 1.0, mul(fw, gu));
    axpy(out, 1.0, times(cross, W_, 2.0));
    axpy(out, 1.0, times(mul(fw, gw), Z_, 1.0));
    return out;
}

IPoly gbdot(const IPoly& f, const IPoly& g) {
    const IPoly fz = der(f, Z_), fw = der(f, W_), gz = der(g, Z_), gw = der(g, W_);
    IPoly out = times(mul(fw, gw), U_, 1.0);
    IPoly cross = mul(fw, gz);
    axpy(cross, 1.0, mul(fz, gw));
    axpy(out, 1.0, times(cross, W_, 2.0));
    axpy(out, 1.0, times(mul(fz, gz), Z_, 4.0));
    return out;
}

IPoly xbar_grad(const IPoly& f) {
    IPoly out = times(der(f, U_), W_, 2.0);
    axpy(out, 1.0, times(der(f, W_), Z_, 1.0));
    return out;
}

void prune(IPoly& f) {
    for (auto it = f.begin(); it != f.end();)
        it = (it->second == 0.0) ? f.erase(it) : std::next(it);
}

// W[m][k], 0 <= k <= m <= p-1: eq.(DIA) on the diagonal, then eq.(MBrec) for k = m-1..0 (Fig. 1).
std::vector<std::vector<IPoly>> radial_coefficients(const std::vector<double>& a, int d, int p) {
    std::vector<std::vector<IPoly>> W(static_cast<size_t>(p), std::vector<IPoly>(static_cast<size_t>(p)));
    IPoly V;
    for (size_t n = 0; n < a.size(); ++n)
        if (a[n] != 0.0) V[IKey{int(n), 0, 0}] = a[n];
    W[0][0] = V;
    double fact = 1.0;
    for (int m = 1; m < p; ++m) {
        fact *= double(2 * m) * double(2 * m + 1);
        IPoly t = V;
        for (int i = 0; i < 2 * m; ++i) t = xbar_grad(t);
        IPoly diag;
        axpy(diag, 1.0 / fact, t);
        prune(diag);
        W[size_t(m)][size_t(m)] = diag;
        for (int k = m - 1; k >= 0; --k) {
            IPoly rhs = lap(W[size_t(m - 1)][size_t(k)], d);
            axpy(rhs, 1.0, lapbar(W[size_t(m)][size_t(k + 1)], d));
            for (int l = 0; l <= m - 2; ++l)
                for (int r = std::max(0, k - m + l + 2); r <= std::min(k, l); ++r)
                    axpy(rhs, -1.0, gdot(W[size_t(l)][size_t(r)], W[size_t(m - l - 2)][size_t(k - r)]));
            for (int l = 1; l <= m - 2; ++l)
                for (int r = std::max(0, k - m + l + 2); r <= std::min(k, l); ++r)
                    axpy(rhs, -1.0, gbdot(W[size_t(l)][size_t(r)], W[size_t(m - l - 1)][size_t(k - r + 1)]));
            IPoly out;
            axpy(out, 1.0 / double(8 * (m + k + 1)), rhs);
            prune(out);
            W[size_t(m)][size_t(k)] = out;
        }
    }
    return W;
}

struct Group {
    int j, l, len, off;
};

// Groups of the layout in consumption order.
std::vector<Group> layout_groups(int p) {
    std::vector<Group> g;
    int off = 0;
    for (int j = radial_nj(p) - 1; j >= 0; --j)
        for (int l = radial_nl(p, j) - 1; l >= 0; --l) {
            const int len = radial_len(p, j + l, j);
            g.push_back(Group{j, l, len, off});
            off += len;
        }
    return g;
}

// The level table at eps (unscaled, consumption order, highest power of u first); false if a
// coefficient falls outside the shape bound.
bool fold_radial(const std::vector<std::vector<IPoly>>& W, int p, double eps, std::vector<double>& tab) {
    const std::vector<Group> groups = layout_groups(p);
    tab.assign(size_t(radial_size(p)), 0.0);
    std::map<std::pair<int, int>, const Group*> where;
    for (const Group& g : groups) where[{g.j + g.l, g.j}] = &g;
    for (int m = 0; m < p; ++m)
        for (int k = 0; k <= m; ++k) {
            const double f = std::pow(eps, double(m - k + 1));
            for (const auto& kv : W[size_t(m)][size_t(k)]) {
                const int i = kv.first[0], jw = kv.first[1], lz = kv.first[2];
                if (jw % 2 != 0 || jw / 2 + lz != k) return false;
                auto it = where.find({k, jw / 2});
                if (it == where.end() || i >= it->second->len) return false;
                const Group& g = *it->second;
                tab[size_t(g.off + g.len - 1 - i)] += kv.second * f;
            }
        }
    return true;
}

// eps W_p of one slice from an unscaled table (the kernels' order: Horner in u, z, w^2).
double eval_slice(const std::vector<double>& tab, int p, const double* x, const double* xb, int d) {
    double u = 0.0, w = 0.0, z = 0.0;
    for (int c = 0; c < d; ++c) {
        u = std::fma(x[c], x[c], u);
        w = std::fma(x[c], xb[c], w);
        z = std::fma(xb[c], xb[c], z);
    }
    const double w2 = w * w;
    const int nj = radial_nj(p);
    size_t off = 0;
    double acc = 0.0;
    for (int j = nj - 1; j >= 0; --j) {
        const int nl = radial_nl(p, j);
        double zs = 0.0;
        for (int l = nl - 1; l >= 0; --l) {
            const int len = radial_len(p, j + l, j);
            double v = 0.0;
            if (len > 0) {
                v = tab[off];
                for (int e = 1; e < len; ++e) v = std::fma(v, u, tab[off + size_t(e)]);
            }
            off += size_t(len);
            zs = (l == nl - 1) ? v : std::fma(zs, z, v);
        }
        acc = (j == nj - 1) ? zs : std::fma(acc, w2, zs);
    }
    return acc;
}

// Device copy: coefficient of u^i (w^2)^j z^l times 4^-(i + 2j + l).
std::vector<double> scale_for_sums(const std::vector<double>& tab, int p) {
    std::vector<double> out = tab;
    for (const Group& g : layout_groups(p))
        for (int e = 0; e < g.len; ++e) {
            const int i = g.len - 1 - e;
            out[size_t(g.off + e)] = std::ldexp(tab[size_t(g.off + e)], -2 * (i + 2 * g.j + g.l));
        }
    return out;
}

std::vector<int> shape_array(int p) {
    const int nj = radial_nj(p);
    std::vector<int> sh{nj};
    for (int j = 0; j < nj; ++j) sh.push_back(radial_nl(p, j));
    for (const Group& g : layout_groups(p)) sh.push_back(g.len);
    return sh;
}

struct VecProblem {
    int dim = 1, s = 0, p = 1, U = 0, D = 0;
    bool specialized = false;
    bool poly = false;                           // component evaluator (tab: records per level)
    double a[kVecMaxDim] = {0, 0, 0}, b[kVecMaxDim] = {0, 0, 0};
    double T = 0, pref = 1.0, K0 = 0.0;
    int stride = 0;
    std::vector<double> tab, tab_dev;            // (s+1) * stride
    std::vector<int> shape;
    std::vector<double> sig, shift;
    double level0_action = 0.0;
};

int check_radial(const pimc_radial_potential* V, double m, const double* a, const double* b, double T, uint32_t N,
                 int p, uint64_t n_samples) {
    if (!V) { set_thread_error("potential is NULL"); return PIMC_EINVAL; }
    if (V->dim < 1 || V->dim > PIMC_MAX_DIM) {
        set_thread_error("dim = %d outside 1..%d", V->dim, PIMC_MAX_DIM);
        return PIMC_EINVAL;
    }
    if (V->degree < 0 || V->degree > PIMC_MAX_RADIAL_DEGREE) {
        set_thread_error("radial degree %d outside 0..%d", V->degree, PIMC_MAX_RADIAL_DEGREE);
        return PIMC_EINVAL;
    }
    for (int n = 0; n <= V->degree; ++n)
        if (!std::isfinite(V->coef[n])) { set_thread_error("coefficient %d is not finite", n); return PIMC_EINVAL; }
    if (!a || !b) { set_thread_error("endpoint array is NULL"); return PIMC_EINVAL; }
    for (int c = 0; c < V->dim; ++c)
        if (!std::isfinite(a[c]) || !std::isfinite(b[c])) { set_thread_error("endpoints must be finite"); return PIMC_EINVAL; }
    pimc_potential zero{};
    return check_args(&zero, m, 0.0, 0.0, T, N, p, n_samples);
}

std::vector<double> rescaled(const pimc_radial_potential* V, double m) {
    std::vector<double> a(size_t(V->degree) + 1);
    for (int n = 0; n <= V->degree; ++n) a[size_t(n)] = V->coef[n] * std::pow(1.0 / m, double(n));
    return a;
}

int build_vector_problem(const pimc_radial_potential* V, double m, const double* a, const double* b, double T,
                         uint32_t N, int p, uint32_t flags, VecProblem& P, char* why, size_t whylen) {
    if (flags & PIMC_FP32_POLY) {
        std::snprintf(why, whylen, "the several-coordinate kernels evaluate in FP64 only");
        return PIMC_EUNSUPPORTED;
    }
    P.dim = V->dim;
    P.s = log2_exact(N);
    P.p = p;
    P.T = T;
    const double sm = std::sqrt(m);
    double r2 = 0.0;
    for (int c = 0; c < P.dim; ++c) {
        P.a[c] = a[c] * sm;
        P.b[c] = b[c] * sm;
        r2 += (P.b[c] - P.a[c]) * (P.b[c] - P.a[c]);
    }
    P.pref = std::pow(sm, double(P.dim));
    P.K0 = std::exp(-r2 / (2.0 * T)) / std::pow(2.0 * kPi * T, 0.5 * double(P.dim));
    P.U = std::min(P.s, kVecU);
    P.D = P.s - P.U;
    P.specialized = (P.dim >= 2 && P.U == kVecU);
    const auto W = radial_coefficients(rescaled(V, m), P.dim, p);
    P.stride = radial_size(p);
    P.tab.assign(size_t(P.s + 1) * size_t(P.stride), 0.0);
    P.tab_dev.assign(P.tab.size(), 0.0);
    P.shift.assign(size_t(P.s + 1), 0.0);
    std::vector<double> lt;
    for (int n = 0; n <= P.s; ++n) {
        if (!fold_radial(W, p, std::ldexp(T, -n), lt)) {
            std::snprintf(why, whylen, "internal: a coefficient falls outside the radial table shape");
            return PIMC_EUNSUPPORTED;
        }
        std::copy(lt.begin(), lt.end(), P.tab.begin() + size_t(n) * size_t(P.stride));
        const std::vector<double> sc = scale_for_sums(lt, p);
        std::copy(sc.begin(), sc.end(), P.tab_dev.begin() + size_t(n) * size_t(P.stride));
        // straight line q_k = a + (b - a) k / 2^n
        const int M = 1 << n;
        double S = 0.0;
        for (int k = 0; k < M; ++k) {
            double x[kVecMaxDim], xb[kVecMaxDim];
            for (int c = 0; c < P.dim; ++c) {
                const double q0 = P.a[c] + (P.b[c] - P.a[c]) * double(k) / double(M);
                const double q1 = P.a[c] + (P.b[c] - P.a[c]) * double(k + 1) / double(M);
                x[c] = 0.5 * (q0 + q1);
                xb[c] = 0.5 * (q1 - q0);
            }
            S += eval_slice(lt, p, x, xb, P.dim);
        }
        P.shift[size_t(n)] = S;
    }
    P.level0_action = P.shift[0];
    P.shape = shape_array(p);
    P.sig.assign(size_t(P.s + 1), 0.0);
    for (int n = 1; n <= P.s; ++n) P.sig[size_t(n)] = std::sqrt(T / std::ldexp(1.0, n + 1));
    return PIMC_OK;
}

int stage_vector(pimc_ctx* c, const VecProblem& P, uint64_t seed, uint32_t stream, VecArgs& A) {
    const size_t nlev = size_t(P.s + 1);
    const size_t n_tab = P.tab_dev.size();
    const size_t off_shift = nlev * 8;
    const size_t off_tab = 2 * nlev * 8;
    const size_t off_shape = off_tab + n_tab * 8;
    const size_t total = off_shape + P.shape.size() * 4 + 16;
    std::vector<unsigned char> host(total, 0);
    std::memcpy(host.data(), P.sig.data(), nlev * 8);
    std::memcpy(host.data() + off_shift, P.shift.data(), nlev * 8);
    std::memcpy(host.data() + off_tab, P.tab_dev.data(), n_tab * 8);
    std::memcpy(host.data() + off_shape, P.shape.data(), P.shape.size() * 4);
    int st = ensure(c, &c->d_prm, &c->prm_bytes, total);
    if (st) return st;
    HIP_TRY(c, hipMemcpyAsync(c->d_prm, host.data(), total, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));     // the host vector must outlive the copy
    unsigned char* base = static_cast<unsigned char*>(c->d_prm);
    std::memset(&A, 0, sizeof(A));
    A.sig = reinterpret_cast<const double*>(base);
    A.shift = reinterpret_cast<const double*>(base + off_shift);
    A.tab = reinterpret_cast<const double*>(base + off_tab);
    A.shape = reinterpret_cast<const int*>(base + off_shape);
    A.stride = P.stride;
    for (int k = 0; k < kVecMaxDim; ++k) {
        A.a[k] = k < P.dim ? P.a[k] : 0.0;
        A.b[k] = k < P.dim ? P.b[k] : 0.0;
    }
    A.key.seed_lo = uint32_t(seed);
    A.key.seed_hi = uint32_t(seed >> 32);
    A.key.stream = stream;
    A.s = P.s;
    A.D = P.D;
    return PIMC_OK;
}

// The walk keeps vec_top_slots(dim, D) doubles per lane in LDS: refuse a launch the device cannot hold.
int check_lds(pimc_ctx* c, const VecProblem& P) {
    int max_lds = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    const size_t need = vec_lds_bytes(P.dim, P.D, P.s);
    if (need > size_t(max_lds))
        return ctx_fail(c, PIMC_EUNSUPPORTED, "N = 2^%d in %d coordinates needs %zu bytes of LDS per workgroup (device limit %d)",
                        P.s, P.dim, need, max_lds);
    return PIMC_OK;
}

int vector_grid(pimc_ctx* c, const VecProblem& P, uint64_t n_chunks) {
    const size_t lds = vec_lds_bytes(P.dim, P.D, P.s);
    const int resident = P.poly ? vector_poly_resident(P.dim, P.U, lds, c->device)
                                : vector_resident_blocks(P.dim, P.p, P.U, P.specialized, lds, c->device);
    const uint64_t g = std::min<uint64_t>(n_chunks, uint64_t(std::max(resident, 1)));
    return int(std::max<uint64_t>(g, 1));
}

int vector_amplitude_core(pimc_ctx* c, const VecProblem& P, uint64_t n_samples, uint64_t seed, uint32_t stream,
                          uint32_t flags, pimc_level_result* out) {
    const int nlev = P.s + 1;
    const bool hier = (flags & PIMC_HIERARCHY) != 0;
    for (int n = 0; n < nlev; ++n) out[n] = pimc_level_result{};
    out[0].log_amp = std::log(P.pref * P.K0) - P.level0_action;
    out[0].amp = std::exp(out[0].log_amp);
    out[0].n = n_samples;
    out[0].ess = double(n_samples);
    c->last_s = P.s;
    c->last_shift = P.shift;
    if (P.s == 0) return PIMC_OK;
    int st = check_lds(c, P);
    if (st) return st;
    VecArgs A;
    st = stage_vector(c, P, seed, stream, A);
    if (st) return st;
    const uint64_t chunk_paths = kChunkPaths;
    const uint64_t n_chunks = (n_samples + chunk_paths - 1) / chunk_paths;
    const int slots = hier ? nlev : 1;
    st = ensure(c, reinterpret_cast<void**>(&c->d_partials), &c->partial_bytes, size_t(slots) * n_chunks * 4 * 8);
    if (st) return st;
    st = ensure(c, reinterpret_cast<void**>(&c->d_red), &c->red_bytes, size_t(slots) * 4 * 8);
    if (st) return st;
    st = ensure(c, reinterpret_cast<void**>(&c->d_seg), &c->seg_bytes, size_t(slots) * 2 * 8);
    if (st) return st;
    c->h_seg.assign(size_t(slots) * 2, 0);
    for (int k = 0; k < slots; ++k) {
        c->h_seg[size_t(k)] = uint64_t(k) * n_chunks * 4;
        c->h_seg[size_t(slots + k)] = n_chunks;
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_seg, c->h_seg.data(), c->h_seg.size() * 8, hipMemcpyHostToDevice, c->stream));
    A.first_path = 0;
    A.n_paths = n_samples;
    A.n_chunks = n_chunks;
    A.hier = hier ? 1 : 0;
    A.partials = c->d_partials;
    A.dump = nullptr;
    const int grid = vector_grid(c, P, n_chunks);
    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    HIP_TRY(c, P.poly ? launch_vector_poly(A, P.dim, P.U, grid, c->stream)
                      : launch_vector(A, P.dim, P.p, P.U, P.specialized, grid, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
    HIP_TRY(c, launch_seg_reduce(c->d_partials, c->d_seg, c->d_seg + slots, uint64_t(slots), c->d_red, c->stream));
    std::vector<double> red(size_t(slots) * 4);
    HIP_TRY(c, hipMemcpyAsync(red.data(), c->d_red, red.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms = ms;
    c->last_partials_ptr = c->d_partials;
    c->last_chunks = n_chunks;
    c->last_chunk_paths = chunk_paths;
    c->last_hier = hier;
    bool nonfinite = false;
    for (int n = 1; n < nlev; ++n) {
        if (!hier && n != P.s) continue;
        const size_t k = size_t(hier ? n : 0);
        if (assemble_level(&red[k * 4], std::log(P.pref * P.K0) - P.shift[size_t(n)], out[n])) nonfinite = true;
    }
    return nonfinite ? PIMC_WNONFINITE : PIMC_OK;
}

int vector_path_actions_core(pimc_ctx* c, const VecProblem& P, uint64_t seed, uint32_t stream, uint32_t flags,
                             uint64_t first_path, uint64_t k_paths, double* S_out) {
    const size_t nlev = size_t(P.s + 1);
    if (P.s == 0) {
        for (uint64_t i = 0; i < k_paths; ++i) S_out[i] = P.level0_action;
        return PIMC_OK;
    }
    int st = check_lds(c, P);
    if (st) return st;
    VecArgs A;
    st = stage_vector(c, P, seed, stream, A);
    if (st) return st;
    st = ensure(c, reinterpret_cast<void**>(&c->d_dump), &c->dump_bytes, size_t(k_paths) * nlev * 8);
    if (st) return st;
    const uint64_t chunk_paths = kChunkPaths;
    A.first_path = first_path;
    A.n_paths = k_paths;
    A.n_chunks = (k_paths + chunk_paths - 1) / chunk_paths;
    A.hier = (flags & PIMC_HIERARCHY) ? 1 : 0;
    A.partials = nullptr;
    A.dump = c->d_dump;
    const int grid = vector_grid(c, P, A.n_chunks);
    HIP_TRY(c, P.poly ? launch_vector_poly(A, P.dim, P.U, grid, c->stream)
                      : launch_vector(A, P.dim, P.p, P.U, P.specialized, grid, c->stream));
    HIP_TRY(c, hipMemcpyAsync(S_out, c->d_dump, size_t(k_paths) * nlev * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIMC_OK;
}

// ============================================================================ component route
// eq.(MBrec)/(DIA) with W_{m,k} as polynomials in the components x_1..x_4 (slots 0..3) and
// xbar_1..xbar_4 (slots 4..7); every derivative is taken component by component, so any polynomial V.
using MKey = std::array<uint8_t, 2 * kVecMaxDim>;
using MPoly = std::map<MKey, double>;
constexpr int kXb = kVecMaxDim;                   // slot of xbar_1

void maxpy(MPoly& y, double a, const MPoly& x) {
    for (const auto& kv : x) y[kv.first] += a * kv.second;
}

MPoly mder(const MPoly& f, int var) {
    MPoly out;
    for (const auto& kv : f)
        if (kv.first[size_t(var)]) {
            MKey k = kv.first;
            k[size_t(var)] -= 1;
            out[k] += kv.second * double(kv.first[size_t(var)]);
        }
    return out;
}

MPoly mtimes(const MPoly& f, int var) {
    MPoly out;
    for (const auto& kv : f) {
        MKey k = kv.first;
        k[size_t(var)] += 1;
        out[k] += kv.second;
    }
    return out;
}

MPoly mmul(const MPoly& a, const MPoly& b) {
    MPoly out;
    for (const auto& ka : a)
        for (const auto& kb : b) {
            MKey k;
            for (size_t i = 0; i < k.size(); ++i) k[i] = uint8_t(ka.first[i] + kb.first[i]);
            out[k] += ka.second * kb.second;
        }
    return out;
}

void mprune(MPoly& f) {
    for (auto it = f.begin(); it != f.end();)
        it = (it->second == 0.0) ? f.erase(it) : std::next(it);
}

// grad^2 (off = 0) or gradbar^2 (off = kXb)
MPoly mlap(const MPoly& f, int d, int off) {
    MPoly out;
    for (int i = 0; i < d; ++i) maxpy(out, 1.0, mder(mder(f, off + i), off + i));
    return out;
}

// grad f . grad g (off = 0) or gradbar f . gradbar g (off = kXb)
MPoly mgdot(const MPoly& f, const MPoly& g, int d, int off) {
    MPoly out;
    for (int i = 0; i < d; ++i) maxpy(out, 1.0, mmul(mder(f, off + i), mder(g, off + i)));
    return out;
}

// xbar . grad f
MPoly mxbar_grad(const MPoly& f, int d) {
    MPoly out;
    for (int i = 0; i < d; ++i) maxpy(out, 1.0, mtimes(mder(f, i), kXb + i));
    return out;
}

// W[m][k], 0 <= k <= m <= p-1, in components: eq.(DIA), then eq.(MBrec) for k = m-1..0 (Fig. 1).
std::vector<std::vector<MPoly>> component_coefficients(const MPoly& V, int d, int p) {
    std::vector<std::vector<MPoly>> W(static_cast<size_t>(p), std::vector<MPoly>(static_cast<size_t>(p)));
    W[0][0] = V;
    double fact = 1.0;
    for (int m = 1; m < p; ++m) {
        fact *= double(2 * m) * double(2 * m + 1);
        MPoly t = V;
        for (int i = 0; i < 2 * m; ++i) t = mxbar_grad(t, d);
        MPoly diag;
        maxpy(diag, 1.0 / fact, t);
        mprune(diag);
        W[size_t(m)][size_t(m)] = diag;
        for (int k = m - 1; k >= 0; --k) {
            MPoly rhs = mlap(W[size_t(m - 1)][size_t(k)], d, 0);
            maxpy(rhs, 1.0, mlap(W[size_t(m)][size_t(k + 1)], d, kXb));
            for (int l = 0; l <= m - 2; ++l)
                for (int r = std::max(0, k - m + l + 2); r <= std::min(k, l); ++r)
                    maxpy(rhs, -1.0, mgdot(W[size_t(l)][size_t(r)], W[size_t(m - l - 2)][size_t(k - r)], d, 0));
            for (int l = 1; l <= m - 2; ++l)
                for (int r = std::max(0, k - m + l + 2); r <= std::min(k, l); ++r)
                    maxpy(rhs, -1.0, mgdot(W[size_t(l)][size_t(r)], W[size_t(m - l - 1)][size_t(k - r + 1)], d, kXb));
            MPoly out;
            maxpy(out, 1.0 / double(8 * (m + k + 1)), rhs);
            mprune(out);
            W[size_t(m)][size_t(k)] = out;
        }
    }
    return W;
}

// The recursion of one (V after the mass rescaling, d, p), computed once per process.
struct PolyCoefficients {
    int d = 1, p = 1;
    std::vector<std::vector<MPoly>> W;
    std::vector<MKey> keys;                      // every monomial of any W_{m,k}, in consumption order
};

// Device variables of a slice: y_c = qb_c - qa_c = 2 xbar_c (c < d), y_{d+c} = qa_c + qb_c = 2 x_c.
// Exponent of device variable v in a monomial.
int var_exp(const MKey& k, int d, int v) { return v < d ? k[size_t(kXb + v)] : k[size_t(v - d)]; }

// Structure stream and coefficient slots of the component evaluator (pimc_vector_impl.hpp,
// PolyEvalRT): the prefix tree of the monomials ordered by the exponents of y_0, y_1, ... from high
// to low, in pre-order; the last variable's chains are dense (absent exponents get a zero slot).
struct PolyCode {
    std::vector<int> code;                       // structure stream
    std::vector<int> slot;                       // per coefficient slot: index into keys, or -1 (zero)
};

// Emit the node over keys[r0, r1) at depth v; returns its lowest exponent of y_v (the tail its
// parent applies).
int emit_poly_node(const std::vector<MKey>& keys, size_t r0, size_t r1, int v, int nv, int d, PolyCode& P, bool& ok) {
    if (v == nv - 1) {
        const int hi = var_exp(keys[r0], d, v), lo = var_exp(keys[r1 - 1], d, v);
        P.code.push_back(hi - lo + 1);
        size_t g = r0;
        for (int e = hi; e >= lo; --e) {
            if (g < r1 && var_exp(keys[g], d, v) == e) {
                P.slot.push_back(int(g));
                ++g;
            } else {
                P.slot.push_back(-1);
            }
        }
        if (g != r1) ok = false;                 // two monomials with one exponent vector
        return lo;
    }
    int groups = 0;
    for (size_t g0 = r0; g0 < r1; ++groups) {
        const int k = var_exp(keys[g0], d, v);
        while (g0 < r1 && var_exp(keys[g0], d, v) == k) ++g0;
    }
    P.code.push_back(groups);
    int prev = -1;
    for (size_t g0 = r0; g0 < r1;) {
        const int k = var_exp(keys[g0], d, v);
        size_t g1 = g0;
        while (g1 < r1 && var_exp(keys[g1], d, v) == k) ++g1;
        const size_t h = P.code.size();
        P.code.push_back(0);
        const int tail = emit_poly_node(keys, g0, g1, v + 1, nv, d, P, ok);
        const int gap = prev < 0 ? 1 : prev - k;
        if (gap < 1 || gap > 255 || tail > 255) ok = false;
        P.code[h] = gap | (tail << 8);
        prev = k;
        g0 = g1;
    }
    return prev;
}

// keys must not be empty (a polynomial without monomials is given the constant monomial, whose
// coefficient is then 0): every node has a child and every chain a coefficient.
bool build_poly_code(const std::vector<MKey>& keys, int d, PolyCode& P) {
    P.code.assign(1, 0);
    P.slot.clear();
    if (keys.empty()) return false;
    bool ok = true;
    P.code[0] = emit_poly_node(keys, 0, keys.size(), 0, 2 * d, d, P, ok);
    return ok;
}

// The same arithmetic as PolyEvalRT on one slice (y as defined above), for the reference actions.
double eval_poly_node(const std::vector<int>& code, size_t& s, const double* coef, size_t& c, const double* y, int v,
                      int nv) {
    if (v == nv - 1) {
        const int L = code[s++];
        double a = coef[c];
        for (int j = 1; j < L; ++j) a = std::fma(a, y[v], coef[c + size_t(j)]);
        c += size_t(L);
        return a;
    }
    const int n = code[s++];
    const int h0 = code[s++];
    double a = eval_poly_node(code, s, coef, c, y, v + 1, nv);
    for (int e = 0; e < (h0 >> 8); ++e) a *= y[v + 1];
    for (int k = 1; k < n; ++k) {
        const int h = code[s++];
        for (int e = 1; e < (h & 255); ++e) a *= y[v];
        double t = eval_poly_node(code, s, coef, c, y, v + 1, nv);
        for (int e = 0; e < (h >> 8); ++e) t *= y[v + 1];
        a = std::fma(a, y[v], t);
    }
    return a;
}

double eval_poly_code(const std::vector<int>& code, const double* coef, const double* y, int nv) {
    size_t s = 1, c = 0;
    double x = eval_poly_node(code, s, coef, c, y, 0, nv);
    for (int e = 0; e < code[0]; ++e) x *= y[0];
    return x;
}

std::string poly_cache_key(const pimc_poly_potential* V, double m, int p) {
    std::string k;
    auto put = [&k](const void* q, size_t n) { k.append(static_cast<const char*>(q), n); };
    put(&V->dim, sizeof(int));
    put(&V->n_terms, sizeof(int));
    put(&m, sizeof(double));
    put(&p, sizeof(int));
    for (int t = 0; t < V->n_terms; ++t) {
        put(&V->coef[t], sizeof(double));
        put(V->exps[t], sizeof(int) * PIMC_MAX_DIM);
    }
    return k;
}

const PolyCoefficients& cached_poly(const pimc_poly_potential* V, double m, int p) {
    static std::mutex mu;
    static std::map<std::string, std::unique_ptr<PolyCoefficients>> cache;
    const std::string key = poly_cache_key(V, m, p);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return *it->second;
    auto C = std::make_unique<PolyCoefficients>();
    C->d = V->dim;
    C->p = p;
    MPoly Vm;                                    // V(y / sqrt(m)): coef times m^(-degree/2)
    for (int t = 0; t < V->n_terms; ++t) {
        MKey k{};
        int deg = 0;
        for (int c = 0; c < V->dim; ++c) {
            k[size_t(c)] = uint8_t(V->exps[t][c]);
            deg += V->exps[t][c];
        }
        Vm[k] += V->coef[t] * std::pow(m, -0.5 * double(deg));
    }
    mprune(Vm);
    C->W = component_coefficients(Vm, V->dim, p);
    MPoly all;
    for (const auto& row : C->W)
        for (const MPoly& f : row)
            for (const auto& kv : f) all[kv.first] = 1.0;
    for (const auto& kv : all) C->keys.push_back(kv.first);
    const int d = V->dim;
    std::sort(C->keys.begin(), C->keys.end(), [d](const MKey& x, const MKey& y) {
        for (int v = 0; v < 2 * d; ++v) {
            const int ex = var_exp(x, d, v), ey = var_exp(y, d, v);
            if (ex != ey) return ex > ey;
        }
        return false;
    });
    return *cache.emplace(key, std::move(C)).first->second;
}

// eps W_p at level eps: the coefficient of each monomial of keys (unscaled).
std::vector<double> fold_poly(const PolyCoefficients& C, double eps) {
    std::map<MKey, double> f;
    for (int m = 0; m < C.p; ++m)
        for (int k = 0; k <= m; ++k) {
            const double e = std::pow(eps, double(m - k + 1));
            for (const auto& kv : C.W[size_t(m)][size_t(k)]) f[kv.first] += kv.second * e;
        }
    std::vector<double> out(C.keys.size());
    for (size_t i = 0; i < C.keys.size(); ++i) out[i] = f[C.keys[i]];
    return out;
}

int check_poly(const pimc_poly_potential* V, double m, const double* a, const double* b, double T, uint32_t N, int p,
               uint64_t n_samples) {
    if (!V) { set_thread_error("potential is NULL"); return PIMC_EINVAL; }
    if (V->dim < 1 || V->dim > PIMC_MAX_DIM) {
        set_thread_error("dim = %d outside 1..%d", V->dim, PIMC_MAX_DIM);
        return PIMC_EINVAL;
    }
    if (V->n_terms < 0 || V->n_terms > PIMC_POLY_MAX_TERMS) {
        set_thread_error("n_terms = %d outside 0..%d", V->n_terms, PIMC_POLY_MAX_TERMS);
        return PIMC_EINVAL;
    }
    for (int t = 0; t < V->n_terms; ++t) {
        if (!std::isfinite(V->coef[t])) { set_thread_error("coefficient %d is not finite", t); return PIMC_EINVAL; }
        int deg = 0;
        for (int c = 0; c < PIMC_MAX_DIM; ++c) {
            const int e = V->exps[t][c];
            if (e < 0 || (c >= V->dim && e != 0)) {
                set_thread_error("term %d: exponent %d of coordinate %d (dim %d)", t, e, c + 1, V->dim);
                return PIMC_EINVAL;
            }
            deg += e;
        }
        if (deg > PIMC_POLY_MAX_DEGREE) {
            set_thread_error("term %d has total degree %d > %d", t, deg, PIMC_POLY_MAX_DEGREE);
            return PIMC_EINVAL;
        }
    }
    if (!a || !b) { set_thread_error("endpoint array is NULL"); return PIMC_EINVAL; }
    for (int c = 0; c < V->dim; ++c)
        if (!std::isfinite(a[c]) || !std::isfinite(b[c])) { set_thread_error("endpoints must be finite"); return PIMC_EINVAL; }
    pimc_potential zero{};
    return check_args(&zero, m, 0.0, 0.0, T, N, p, n_samples);
}

int build_poly_problem(const pimc_poly_potential* V, double m, const double* a, const double* b, double T, uint32_t N,
                       int p, uint32_t flags, VecProblem& P, char* why, size_t whylen) {
    if (flags & PIMC_FP32_POLY) {
        std::snprintf(why, whylen, "the several-coordinate kernels evaluate in FP64 only");
        return PIMC_EUNSUPPORTED;
    }
    P.poly = true;
    P.dim = V->dim;
    P.s = log2_exact(N);
    P.p = p;
    P.T = T;
    const double sm = std::sqrt(m);
    double r2 = 0.0;
    for (int c = 0; c < P.dim; ++c) {
        P.a[c] = a[c] * sm;
        P.b[c] = b[c] * sm;
        r2 += (P.b[c] - P.a[c]) * (P.b[c] - P.a[c]);
    }
    P.pref = std::pow(sm, double(P.dim));
    P.K0 = std::exp(-r2 / (2.0 * T)) / std::pow(2.0 * kPi * T, 0.5 * double(P.dim));
    P.U = std::min(P.s, poly_subtree_levels(P.dim));
    P.D = P.s - P.U;
    P.specialized = false;
    const PolyCoefficients& C = cached_poly(V, m, p);
    if (C.keys.size() > size_t(PIMC_POLY_MAX_MONOMIALS)) {
        std::snprintf(why, whylen, "eps W_p has %zu monomials (limit %d)", C.keys.size(), PIMC_POLY_MAX_MONOMIALS);
        return PIMC_EUNSUPPORTED;
    }
    const std::vector<MKey> keys = C.keys.empty() ? std::vector<MKey>(1, MKey{}) : C.keys;
    PolyCode R;
    if (!build_poly_code(keys, P.dim, R) || R.slot.size() > size_t(kPolyMaxSlots)) {
        std::snprintf(why, whylen, "internal: the monomials do not fit the component evaluator");
        return PIMC_EUNSUPPORTED;
    }
    const size_t nslot = R.slot.size();
    P.stride = int(nslot);                       // coefficient slots per level
    P.tab.assign(size_t(P.s + 1) * nslot, 0.0);
    P.shift.assign(size_t(P.s + 1), 0.0);
    const int nv = 2 * P.dim;
    for (int n = 0; n <= P.s; ++n) {
        const std::vector<double> f = fold_poly(C, std::ldexp(T, -n));
        double* coef = P.tab.data() + size_t(n) * nslot;
        for (size_t o = 0; o < nslot; ++o) {
            if (R.slot[o] < 0 || C.keys.empty()) continue;          // no monomials: the one slot is 0
            const MKey& k = C.keys[size_t(R.slot[o])];
            int deg = 0;
            for (int c = 0; c < 2 * kVecMaxDim; ++c) deg += k[size_t(c)];
            coef[o] = std::ldexp(f[size_t(R.slot[o])], -deg);   // y = 2 x, 2 xbar
        }
        const int M = 1 << n;
        double S = 0.0;
        for (int k = 0; k < M; ++k) {
            double y[2 * kVecMaxDim] = {0, 0, 0, 0, 0, 0};
            for (int c = 0; c < P.dim; ++c) {
                const double q0 = P.a[c] + (P.b[c] - P.a[c]) * double(k) / double(M);
                const double q1 = P.a[c] + (P.b[c] - P.a[c]) * double(k + 1) / double(M);
                y[c] = q1 - q0;
                y[P.dim + c] = q0 + q1;
            }
            S += eval_poly_code(R.code, coef, y, nv);
        }
        P.shift[size_t(n)] = S;
    }
    P.tab_dev = P.tab;
    P.level0_action = P.shift[0];
    P.shape = R.code;
    P.sig.assign(size_t(P.s + 1), 0.0);
    for (int n = 1; n <= P.s; ++n) P.sig[size_t(n)] = std::sqrt(T / std::ldexp(1.0, n + 1));
    return PIMC_OK;
}

}  // namespace

namespace pimc {

hipError_t launch_vector(const VecArgs& A, int dim, int p, int U, bool specialized, int grid, hipStream_t st) {
    switch (dim) {
        case 1: return launch_vector_d1(A, p, U, specialized, grid, st);
        case 2: return launch_vector_d2(A, p, U, specialized, grid, st);
        case 3: return launch_vector_d3(A, p, U, specialized, grid, st);
        case 4: return launch_vector_d4(A, p, U, specialized, grid, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vector_poly(const VecArgs& A, int dim, int U, int grid, hipStream_t st) {
    switch (dim) {
        case 1: return launch_vector_poly_dim<1>(A, U, grid, st);
        case 2: return launch_vector_poly_dim<2>(A, U, grid, st);
        case 3: return launch_vector_poly_dim<3>(A, U, grid, st);
        case 4: return launch_vector_poly_dim<4>(A, U, grid, st);
        default: return hipErrorInvalidValue;
    }
}

int vector_poly_resident(int dim, int U, size_t lds_bytes, int device) {
    switch (dim) {
        case 1: return vector_poly_resident_dim<1>(U, lds_bytes, device);
        case 2: return vector_poly_resident_dim<2>(U, lds_bytes, device);
        case 3: return vector_poly_resident_dim<3>(U, lds_bytes, device);
        case 4: return vector_poly_resident_dim<4>(U, lds_bytes, device);
        default: return 256;
    }
}

int vector_resident_blocks(int dim, int p, int U, bool specialized, size_t lds_bytes, int device) {
    switch (dim) {
        case 1: return vector_resident_d1(p, U, specialized, lds_bytes, device);
        case 2: return vector_resident_d2(p, U, specialized, lds_bytes, device);
        case 3: return vector_resident_d3(p, U, specialized, lds_bytes, device);
        case 4: return vector_resident_d4(p, U, specialized, lds_bytes, device);
        default: return 256;
    }
}

}  // namespace pimc

// ============================================================================================ C ABI
extern "C" {

int pimc_amplitude_radial(pimc_ctx* c, const pimc_radial_potential* V, double m, const double* a, const double* b,
                          double T, uint32_t N, int p, uint64_t n_samples, uint64_t seed, uint32_t stream,
                          uint32_t flags, pimc_level_result* out) {
    int st = check_radial(V, m, a, b, T, N, p, n_samples);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    HIP_TRY(c, hipSetDevice(c->device));
    VecProblem P;
    char why[256] = "";
    st = build_vector_problem(V, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return vector_amplitude_core(c, P, n_samples, seed, stream, flags, out);
}

int pimc_path_actions_radial(pimc_ctx* c, const pimc_radial_potential* V, double m, const double* a, const double* b,
                             double T, uint32_t N, int p, uint64_t seed, uint32_t stream, uint32_t flags,
                             uint64_t first_path, uint64_t k_paths, double* S_out) {
    int st = check_radial(V, m, a, b, T, N, p, 2);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!S_out && k_paths) return ctx_fail(c, PIMC_EINVAL, "S_out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    if (k_paths == 0) return PIMC_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    VecProblem P;
    char why[256] = "";
    st = build_vector_problem(V, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return vector_path_actions_core(c, P, seed, stream, flags, first_path, k_paths, S_out);
}

int pimc_level_table_radial(const pimc_radial_potential* V, double m, double T, int p, uint32_t level, double* out,
                            size_t cap, size_t* n_out, int* shape, size_t shape_cap, int* n_groups) {
    const double zero[PIMC_MAX_DIM] = {0.0, 0.0, 0.0};
    int st = check_radial(V, m, zero, zero, T, 1u, p, 2);
    if (st) return st;
    if (level > PIMC_MAX_S) { set_thread_error("level > %d", PIMC_MAX_S); return PIMC_EINVAL; }
    const auto W = radial_coefficients(rescaled(V, m), V->dim, p);
    std::vector<double> tab;
    if (!fold_radial(W, p, std::ldexp(T, -int(level)), tab)) {
        set_thread_error("internal: a coefficient falls outside the radial table shape");
        return PIMC_EUNSUPPORTED;
    }
    const std::vector<Group> groups = layout_groups(p);
    if (n_out) *n_out = tab.size();
    if (n_groups) *n_groups = int(groups.size());
    if (!out || cap < tab.size()) {
        set_thread_error("output capacity %zu < %zu", cap, tab.size());
        return PIMC_EINVAL;
    }
    if (!shape || shape_cap < 3 * groups.size()) {
        set_thread_error("shape capacity %zu < %zu", shape_cap, 3 * groups.size());
        return PIMC_EINVAL;
    }
    std::copy(tab.begin(), tab.end(), out);
    for (size_t g = 0; g < groups.size(); ++g) {
        shape[3 * g] = groups[g].j + groups[g].l;
        shape[3 * g + 1] = groups[g].j;
        shape[3 * g + 2] = groups[g].len;
    }
    return PIMC_OK;
}

int pimc_amplitude_poly(pimc_ctx* c, const pimc_poly_potential* V, double m, const double* a, const double* b, double T,
                        uint32_t N, int p, uint64_t n_samples, uint64_t seed, uint32_t stream, uint32_t flags,
                        pimc_level_result* out) {
    int st = check_poly(V, m, a, b, T, N, p, n_samples);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!out) return ctx_fail(c, PIMC_EINVAL, "out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    HIP_TRY(c, hipSetDevice(c->device));
    VecProblem P;
    char why[256] = "";
    st = build_poly_problem(V, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return vector_amplitude_core(c, P, n_samples, seed, stream, flags, out);
}

int pimc_path_actions_poly(pimc_ctx* c, const pimc_poly_potential* V, double m, const double* a, const double* b,
                           double T, uint32_t N, int p, uint64_t seed, uint32_t stream, uint32_t flags,
                           uint64_t first_path, uint64_t k_paths, double* S_out) {
    int st = check_poly(V, m, a, b, T, N, p, 2);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (!S_out && k_paths) return ctx_fail(c, PIMC_EINVAL, "S_out is NULL");
    if (flags & ~kKnownFlags) return ctx_fail(c, PIMC_EINVAL, "unknown flags 0x%x", flags & ~kKnownFlags);
    if (k_paths == 0) return PIMC_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    VecProblem P;
    char why[256] = "";
    st = build_poly_problem(V, m, a, b, T, N, p, flags, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    return vector_path_actions_core(c, P, seed, stream, flags, first_path, k_paths, S_out);
}

int pimc_level_table_poly(const pimc_poly_potential* V, double m, double T, int p, uint32_t level, double* coef,
                          size_t cap, int* exps, size_t exps_cap, size_t* n_out) {
    const double zero[PIMC_MAX_DIM] = {0.0, 0.0, 0.0};
    int st = check_poly(V, m, zero, zero, T, 1u, p, 2);
    if (st) return st;
    if (level > PIMC_MAX_S) { set_thread_error("level > %d", PIMC_MAX_S); return PIMC_EINVAL; }
    if (!n_out) { set_thread_error("n_out is NULL"); return PIMC_EINVAL; }
    const PolyCoefficients& C = cached_poly(V, m, p);
    PolyCode R;
    if (C.keys.empty()) {
        *n_out = 0;
        return PIMC_OK;
    }
    if (!build_poly_code(C.keys, V->dim, R)) {
        set_thread_error("internal: the monomials do not fit the component evaluator");
        return PIMC_EUNSUPPORTED;
    }
    const std::vector<double> f = fold_poly(C, std::ldexp(T, -int(level)));
    size_t n = 0;
    for (int l : R.slot) n += l >= 0 ? 1 : 0;
    *n_out = n;
    const size_t nv = size_t(2 * V->dim);
    if (cap < n || exps_cap < n * nv || !coef || !exps) {
        set_thread_error("need %zu doubles and %zu ints", n, n * nv);
        return PIMC_EINVAL;
    }
    size_t i = 0;
    for (int l : R.slot) {
        if (l < 0) continue;
        const MKey& k = C.keys[size_t(l)];
        coef[i] = f[size_t(l)];
        for (int c = 0; c < V->dim; ++c) {
            exps[i * nv + size_t(c)] = k[size_t(c)];
            exps[i * nv + size_t(V->dim + c)] = k[size_t(kXb + c)];
        }
        ++i;
    }
    return PIMC_OK;
}

}  // extern "C"
