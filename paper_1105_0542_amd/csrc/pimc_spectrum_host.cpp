// Host side of the spectrum entry points (pimc_evolution_matrix, pimc_spectrum in include/pimc.h).
//
// The paper computes energy eigenvalues and eigenfunctions by diagonalizing the space-discretized
// matrix of short-time transition amplitudes (Sec. 2; Sec. 4.2 with Fig. 3): on the grid
// x_i = -L + (i + 1/2) D, D = 2L/n, M_ij = D A_1^(p)(x_i, x_j; t) approximates exp(-t H), so its
// largest eigenvalues are exp(-t E_n). The matrix is built on the device from the level-p table at
// eps = t (for the eigenvalue iteration only its upper tiles: the matrix is exactly symmetric); its
// largest eigenpairs come from a Lanczos iteration with full reorthogonalization (classical
// Gram-Schmidt applied twice) run on the device, with the small tridiagonal problem solved on the
// host by Sturm-sequence bisection (eigenvalues) and inverse iteration (vectors).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "pimc.h"
#include "pimc_host_common.hpp"
#include "pimc_spectrum.hpp"

using namespace pimc;
using namespace pimc_host;

namespace {

// ------------------------------------------------------------------------------ tridiagonal T
// T has diagonal a[0..m) and off-diagonal b[0..m-1).

// Number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots).
int sturm_below(const std::vector<double>& a, const std::vector<double>& b, int m, double x, double pivmin) {
    int cnt = 0;
    double d = a[0] - x;
    if (std::fabs(d) < pivmin) d = -pivmin;
    if (d < 0) ++cnt;
    for (int i = 1; i < m; ++i) {
        d = (a[i] - x) - b[i - 1] * b[i - 1] / d;
        if (std::fabs(d) < pivmin) d = -pivmin;
        if (d < 0) ++cnt;
    }
    return cnt;
}

// Eigenvalue number r (ascending, 0-based) by bisection on [lo, hi].
double tri_eigenvalue(const std::vector<double>& a, const std::vector<double>& b, int m, int r, double lo, double hi,
                      double pivmin) {
    for (int it = 0; it < 256; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_below(a, b, m, mid, pivmin) > r)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Eigenvector of T for the eigenvalue theta by inverse iteration: Gaussian elimination with
// partial pivoting of T - theta I (tridiagonal, one extra superdiagonal from row swaps), three
// solves from a fixed start vector, each followed by orthogonalization against `prev` (vectors of
// nearby eigenvalues) and normalization.
std::vector<double> tri_eigenvector(const std::vector<double>& a, const std::vector<double>& b, int m, double theta,
                                    double tiny, const std::vector<std::vector<double>>& prev) {
    std::vector<double> D(m), DU(m, 0.0), DU2(m, 0.0), DL(m, 0.0);
    std::vector<char> swapped(m, 0);
    for (int i = 0; i < m; ++i) D[i] = a[i] - theta;
    for (int i = 0; i + 1 < m; ++i) {
        DU[i] = b[i];
        DL[i] = b[i];
    }
    for (int i = 0; i + 1 < m; ++i) {
        if (std::fabs(D[i]) >= std::fabs(DL[i])) {
            if (D[i] == 0.0) D[i] = tiny;
            const double f = DL[i] / D[i];
            DL[i] = f;
            D[i + 1] -= f * DU[i];
        } else {
            const double f = D[i] / DL[i];
            D[i] = DL[i];
            DL[i] = f;
            const double u = DU[i];
            DU[i] = D[i + 1];
            D[i + 1] = u - f * D[i + 1];
            if (i + 2 < m) {
                DU2[i] = DU[i + 1];
                DU[i + 1] = -f * DU[i + 1];
            }
            swapped[i] = 1;
        }
    }
    if (D[m - 1] == 0.0) D[m - 1] = tiny;
    std::vector<double> x(m);
    for (int i = 0; i < m; ++i) x[i] = 1.0 + 0.5 * std::sin(1.0 + 0.7 * i);   // fixed, generic start
    for (int it = 0; it < 3; ++it) {
        for (int i = 0; i + 1 < m; ++i) {
            if (!swapped[i]) {
                x[i + 1] -= DL[i] * x[i];
            } else {
                const double tmp = x[i];
                x[i] = x[i + 1];
                x[i + 1] = tmp - DL[i] * x[i];
            }
        }
        x[m - 1] /= D[m - 1];
        if (m > 1) x[m - 2] = (x[m - 2] - DU[m - 2] * x[m - 1]) / D[m - 2];
        for (int i = m - 3; i >= 0; --i) x[i] = (x[i] - DU[i] * x[i + 1] - DU2[i] * x[i + 2]) / D[i];
        for (const auto& v : prev) {
            double dot = 0.0;
            for (int i = 0; i < m; ++i) dot += v[i] * x[i];
            for (int i = 0; i < m; ++i) x[i] -= dot * v[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += x[i] * x[i];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) break;
        for (int i = 0; i < m; ++i) x[i] /= nrm;
    }
    return x;
}

struct Ritz {
    std::vector<double> theta;                 // descending
    std::vector<std::vector<double>> s;        // eigenvectors of T
    std::vector<double> resid;                 // |beta_m s[m-1]|
};

// The k largest eigenpairs of T_m and their Lanczos residual norms (beta_last = beta[m-1]).
Ritz top_ritz(const std::vector<double>& a, const std::vector<double>& b, int m, int k, double beta_last) {
    double lo = std::numeric_limits<double>::infinity(), hi = -lo, bmax = 0.0;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
        if (i + 1 < m) bmax = std::max(bmax, std::fabs(b[i]));
    }
    const double scale = std::max(std::fabs(lo), std::fabs(hi));
    const double pivmin = std::numeric_limits<double>::min() * std::max(1.0, bmax * bmax);
    const double span = hi - lo;
    lo -= 1e-12 * (span + scale) + pivmin;
    hi += 1e-12 * (span + scale) + pivmin;
    Ritz R;
    const int kk = std::min(k, m);
    for (int q = 0; q < kk; ++q) R.theta.push_back(tri_eigenvalue(a, b, m, m - 1 - q, lo, hi, pivmin));
    const double tiny = std::numeric_limits<double>::epsilon() * std::max(scale, std::numeric_limits<double>::min());
    for (int q = 0; q < kk; ++q) {
        std::vector<std::vector<double>> near;
        for (int r = 0; r < q; ++r)
            if (std::fabs(R.theta[r] - R.theta[q]) <= 1e-3 * scale) near.push_back(R.s[r]);
        R.s.push_back(tri_eigenvector(a, b, m, R.theta[q], tiny, near));
        R.resid.push_back(std::fabs(beta_last * R.s.back()[m - 1]));
    }
    return R;
}

int validate(pimc_ctx* c, const pimc_potential* V, double m, double t, int p, double L, uint32_t n) {
    int st = check_args(V, m, 0.0, 0.0, t, 1, 1, 2);
    if (st) return c ? ctx_fail(c, st, "%s", g_thread_error) : st;
    if (!c) { set_thread_error("context is NULL"); return PIMC_EINVAL; }
    if (p < 1 || p > PIMC_MAX_P_SHORT_TIME)
        return ctx_fail(c, PIMC_EINVAL, "p = %d outside 1..%d", p, PIMC_MAX_P_SHORT_TIME);
    if (!std::isfinite(L) || L <= 0) return ctx_fail(c, PIMC_EINVAL, "L must be finite and > 0");
    if (n < 2 || n > PIMC_MAX_GRID) return ctx_fail(c, PIMC_EINVAL, "n = %u outside 2..%d", n, PIMC_MAX_GRID);
    return PIMC_OK;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

int dev_alloc(pimc_ctx* c, DevBuf& b, size_t bytes) {
    const hipError_t e = hipMalloc(&b.p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
        b.p = nullptr;
        return ctx_fail(c, PIMC_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return PIMC_OK;
}

// Problem, table upload and launch of the matrix kernel on the context stream: the full matrix
// (M, ld) or, with map != nullptr, the packed upper tiles.
int build_matrix(pimc_ctx* c, const pimc_potential* V, double m, double t, int p, double L, uint32_t n, double* M,
                 uint64_t ld, DevBuf& tabbuf, const uint32_t* map = nullptr, uint32_t ntiles = 0) {
    Problem P;
    char why[256] = "";
    int st = build_problem(V, m, 0.0, 0.0, t, 1, p, 0, P, why, sizeof(why));
    if (st) return ctx_fail(c, st, "%s", why);
    const size_t nt = size_t(P.stride), nk = P.deg.size();
    if ((st = dev_alloc(c, tabbuf, nt * 8 + nk * 4 + 16))) return st;
    std::vector<unsigned char> blob(nt * 8 + nk * 4);
    std::memcpy(blob.data(), P.tab.data(), nt * 8);                   // level 0: eps = t
    std::memcpy(blob.data() + nt * 8, P.deg.data(), nk * 4);
    HIP_TRY(c, hipMemcpyAsync(tabbuf.p, blob.data(), blob.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    SpecTable tb;
    tb.tab = static_cast<const double*>(tabbuf.p);
    tb.deg = reinterpret_cast<const int*>(static_cast<const unsigned char*>(tabbuf.p) + nt * 8);
    tb.K = int(nk);
    tb.stride = P.stride;
    tb.even = P.even ? 1 : 0;
    const double D = 2.0 * L / double(n);
    const double sm = std::sqrt(m);
    const double pref = D * sm / std::sqrt(2.0 * M_PI * t);
    if (map)
        HIP_TRY(c, launch_evolution_tiles(tb, L, D, sm, t, pref, n, map, ntiles, M, c->stream));
    else
        HIP_TRY(c, launch_evolution_matrix(tb, L, D, sm, t, pref, n, M, ld, c->stream));
    return PIMC_OK;
}

uint64_t splitmix(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int pimc_evolution_matrix(pimc_ctx* c, const pimc_potential* V, double m, double t, int p, double L, uint32_t n,
                          double* M, uint64_t ld) {
    int st = validate(c, V, m, t, p, L, n);
    if (st) return st;
    if (!M) return ctx_fail(c, PIMC_EINVAL, "M is NULL");
    if (ld < n) return ctx_fail(c, PIMC_EINVAL, "ld = %llu < n = %u", (unsigned long long)ld, n);
    HIP_TRY(c, hipSetDevice(c->device));
    DevBuf tab;
    if ((st = build_matrix(c, V, m, t, p, L, n, M, ld, tab))) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIMC_OK;
}

int pimc_spectrum(pimc_ctx* c, const pimc_potential* V, double m, double t, int p, double L, uint32_t n, uint32_t k,
                  uint32_t max_iter, double tol, double* E, double* psi, pimc_spectrum_info* info) {
    int st = validate(c, V, m, t, p, L, n);
    if (st) return st;
    if (!E) return ctx_fail(c, PIMC_EINVAL, "E is NULL");
    if (k < 1 || k > PIMC_MAX_STATES || k > n) return ctx_fail(c, PIMC_EINVAL, "k = %u outside 1..min(n, %d)", k, PIMC_MAX_STATES);
    if (max_iter < k + 1 || max_iter > PIMC_MAX_LANCZOS || max_iter > n)
        return ctx_fail(c, PIMC_EINVAL, "max_iter = %u outside %u..min(n, %d)", max_iter, k + 1, PIMC_MAX_LANCZOS);
    if (!(tol > 0.0 && tol < 1.0)) return ctx_fail(c, PIMC_EINVAL, "tol outside (0, 1)");
    HIP_TRY(c, hipSetDevice(c->device));
    const uint64_t ld = (uint64_t(n) + 63) / 64 * 64;
    // the matrix as packed upper tiles (it is exactly symmetric): half the bytes per product
    const uint32_t nb = (n + kTile - 1) / kTile;
    const uint32_t ntiles = nb * (nb + 1) / 2;
    std::vector<uint32_t> map(ntiles);
    for (uint32_t I = 0, q = 0; I < nb; ++I)
        for (uint32_t J = I; J < nb; ++J) map[q++] = (I << 16) | J;
    DevBuf Mb, Qb, wb, ab, bb, hb, tab, mapb, prb, pcb;
    if ((st = dev_alloc(c, Mb, size_t(ntiles) * kTile * kTile * 8))) return st;
    if ((st = dev_alloc(c, mapb, size_t(ntiles) * 4))) return st;
    if ((st = dev_alloc(c, prb, size_t(ntiles) * kTile * 8))) return st;
    if ((st = dev_alloc(c, pcb, size_t(ntiles) * kTile * 8))) return st;
    if ((st = dev_alloc(c, Qb, size_t(ld) * (max_iter + 1) * 8))) return st;
    if ((st = dev_alloc(c, wb, size_t(ld) * 8))) return st;
    if ((st = dev_alloc(c, ab, size_t(max_iter) * 8))) return st;
    if ((st = dev_alloc(c, bb, size_t(max_iter) * 8))) return st;
    if ((st = dev_alloc(c, hb, size_t(max_iter + 1) * 8))) return st;
    double* M = static_cast<double*>(Mb.p);
    double* Q = static_cast<double*>(Qb.p);
    double* w = static_cast<double*>(wb.p);
    double* alpha = static_cast<double*>(ab.p);
    double* beta = static_cast<double*>(bb.p);
    double* h = static_cast<double*>(hb.p);
    const uint32_t* dmap = static_cast<const uint32_t*>(mapb.p);
    double* prow = static_cast<double*>(prb.p);
    double* pcol = static_cast<double*>(pcb.p);
    HIP_TRY(c, hipMemcpyAsync(mapb.p, map.data(), map.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    if ((st = build_matrix(c, V, m, t, p, L, n, M, ld, tab, dmap, ntiles))) return st;
    HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
    // start vector: fixed pseudo-random, normalized on the host
    std::vector<double> q0(n);
    uint64_t sx = 0x5eedULL;
    double nrm = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        q0[i] = 2.0 * double(splitmix(sx) >> 11) * 0x1p-53 - 1.0;
        nrm += q0[i] * q0[i];
    }
    nrm = std::sqrt(nrm);
    for (auto& v : q0) v /= nrm;
    HIP_TRY(c, hipMemcpyAsync(Q, q0.data(), size_t(n) * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float mat_ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&mat_ms, c->ev0, c->ev1));
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> ha, hbv;
    Ritz R;
    uint32_t used = 0;
    bool converged = false;
    const uint32_t check_every = 16;
    for (uint32_t j = 0; j < max_iter; ++j) {
        double* qj = Q + uint64_t(j) * ld;
        HIP_TRY(c, launch_symv_tiles(M, dmap, ntiles, nb, n, qj, prow, pcol, w, c->stream));
        // w = (1 - Q Q^T) M q_j by classical Gram-Schmidt, twice: in exact arithmetic the first pass
        // removes alpha_j q_j + beta_{j-1} q_{j-1} (the three-term recurrence) and nothing else, so
        // alpha_j = <q_j, M q_j> is its coefficient of q_j, and beta_j = |w| afterwards
        for (int pass = 0; pass < 2; ++pass) {
            HIP_TRY(c, launch_col_dots(Q, ld, n, j + 1, w, h, c->stream, pass == 0 ? alpha + j : nullptr, j));
            HIP_TRY(c, launch_combine_cols(Q, ld, n, j + 1, h, w, 1, c->stream));
        }
        HIP_TRY(c, launch_normalize(w, n, beta, j, Q + uint64_t(j + 1) * ld, c->stream));
        const uint32_t mm = j + 1;
        if (mm >= k + 1 && (mm % check_every == 0 || mm == max_iter)) {
            ha.resize(mm);
            hbv.resize(mm);
            HIP_TRY(c, hipMemcpyAsync(ha.data(), alpha, size_t(mm) * 8, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipMemcpyAsync(hbv.data(), beta, size_t(mm) * 8, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            R = top_ritz(ha, hbv, int(mm), int(k), hbv[mm - 1]);
            used = mm;
            converged = true;
            for (uint32_t q = 0; q < k; ++q)
                if (!(R.resid[q] <= tol * std::fabs(R.theta[0]))) converged = false;
            if (converged) break;
        }
    }
    if (used == 0) return ctx_fail(c, PIMC_EINVAL, "no Lanczos step taken");
    for (uint32_t q = 0; q < k; ++q) {
        if (!(R.theta[q] > 0.0)) return ctx_fail(c, PIMC_EUNSUPPORTED, "eigenvalue %u of the matrix is not positive", q);
        E[q] = -std::log(R.theta[q]) / t;
    }
    if (psi) {
        const double D = 2.0 * L / double(n);
        std::vector<double> y(n);
        for (uint32_t q = 0; q < k; ++q) {
            HIP_TRY(c, hipMemcpyAsync(h, R.s[q].data(), size_t(used) * 8, hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, launch_combine_cols(Q, ld, n, used, h, w, 0, c->stream));
            HIP_TRY(c, hipMemcpyAsync(y.data(), w, size_t(n) * 8, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            double s2 = 0.0, big = 0.0;
            uint32_t ibig = 0;
            for (uint32_t i = 0; i < n; ++i) {
                s2 += y[i] * y[i];
                if (std::fabs(y[i]) > big) {
                    big = std::fabs(y[i]);
                    ibig = i;
                }
            }
            const double sc = (y[ibig] < 0 ? -1.0 : 1.0) / std::sqrt(s2 * D);
            for (uint32_t i = 0; i < n; ++i) psi[size_t(q) * n + i] = y[i] * sc;
        }
    }
    const auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->iterations = used;
        double mr = 0.0;
        for (uint32_t q = 0; q < k; ++q) mr = std::max(mr, R.resid[q] / std::fabs(R.theta[0]));
        info->max_residual = mr;
        info->matrix_ms = mat_ms;
        info->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        info->converged = converged ? 1 : 0;
    }
    return converged ? PIMC_OK : PIMC_WNOTCONVERGED;
}

}  // extern "C"
