/*
 * pimc.h -- C ABI of the MI355X (gfx950) Path Integral Monte Carlo amplitude library.
 *
 * The library estimates the imaginary-time transition amplitude A(a,b;T) = <b|exp(-T H)|a> of a
 * particle of mass m in a 1D polynomial potential V, H = p^2/(2m) + V(q), hbar = 1, following
 * Balaz et al., "SPEEDUP Code for Calculation of Transition Amplitudes via the Effective Action
 * Approach":
 *   - time slicing, eq.(AMC), into N = 2^s steps of eps = T/N;
 *   - the level-p short-time effective action, eq.(ansatz) truncated at m <= p-1, with the
 *     coefficients c_{m,k}(x) from eq.(1Drec) and eq.(diagonal) (Sec. 2.1);
 *   - the discretized amplitude A_N^(p) and action eq.(SNp) (Sec. 4);
 *   - trajectories by bisection with Gaussian offsets, every coarser level 2^n, n = 0..s, read off
 *     the same level-s trajectory, amplitude and Monte Carlo error per level (Sec. 4.1).
 *
 * Conventions (shared by every entry point):
 *   - Status: 0 = PIMC_OK, < 0 error (nothing written to outputs unless stated), > 0 warning
 *     (outputs written).
 *   - All pointers are plain host pointers unless the argument says "device". The caller owns every
 *     input and output array; the context owns its device buffers, streams and graphs.
 *   - Offsets of the bisection are standard normals from Philox4x32-10 (Salmon et al., SC'11) with
 *     counter (h>>1, path_lo32, path_hi32, stream) and key (seed_lo32, seed_hi32) for heap node h of a
 *     path; Box-Muller cosine for even h, sine for odd h; the offset of a level-n node has
 *     variance T/2^(n+1) (the Brownian-bridge width), so the estimator of A_N^(p) is
 *     K_0(a,b;T) * E[exp(-sum_k eps W_p(x_k, xbar_k; eps))] with K_0 the free kernel.
 *   - Mass: A_m(a,b;T) = sqrt(m) A_1(sqrt(m) a, sqrt(m) b; T) with V(y/sqrt(m)).
 *   - Level 0 (N = 1) is the analytic short-time amplitude with error 0 (Sec. 4.2).
 *   - A context is used by one host thread at a time; calls on one context are serialized on its
 *     stream.
 */
#ifndef PIMC_H
#define PIMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------------- */
enum {
    PIMC_OK = 0,
    PIMC_EINVAL = -1,          /* argument out of range or non-finite                              */
    PIMC_EUNSUPPORTED = -2,    /* valid request outside what the library implements                */
    PIMC_ENOMEM = -3,          /* host or device allocation failed                                 */
    PIMC_EDEVICE = -4,         /* a HIP call failed; text via pimc_last_error                       */
    PIMC_WNONFINITE = 1,       /* some weights were inf/nan; they are kept in the sums (never dropped) */
    PIMC_WNOTCONVERGED = 2     /* an iteration stopped at its limit before its tolerance; outputs written */
};

/* ---- flags ---------------------------------------------------------------------------------- */
enum {
    PIMC_FP64 = 0,             /* slice polynomials in FP64 (default)                              */
    PIMC_FP32_POLY = 1,        /* slice polynomials in FP32; mid-point/deviation, per-path action
                                  sums and weights stay FP64                                        */
    PIMC_HIERARCHY = 2         /* also estimate every coarser level n < s from the same paths       */
};

#define PIMC_MAX_DEGREE 8      /* highest power of q in a potential                                 */
#define PIMC_MAX_P 18          /* highest effective-action level                                    */
#define PIMC_MAX_S 20          /* N <= 2^20                                                         */
#define PIMC_CHUNK_PATHS 4096  /* paths per canonical chunk of the estimators' sums                 */

/* V(q) = sum_{j=0..degree} coef[j] q^j. The paper's anharmonic oscillator (Sec. 3.3)
 * V = A q^2/2 + g q^4/24 is coef[2] = A/2, coef[4] = g/24. */
typedef struct {
    int degree;                /* 0..PIMC_MAX_DEGREE; coef[j] for j > degree are ignored            */
    double coef[PIMC_MAX_DEGREE + 1];
} pimc_potential;

/* Per bisection level n (N = 2^n): the amplitude estimate and its Monte Carlo error (standard
 * deviation of the mean, unbiased sample variance), as printed per level by the paper's program. */
typedef struct {
    double amp;                /* A_{2^n}^(p)(a,b;T)                                               */
    double err;                /* Monte Carlo error of amp; 0 at n = 0                              */
    double log_amp;            /* log(amp) (finite where amp underflows)                             */
    double relvar;             /* var(w)/mean(w)^2 of the weights                                   */
    double ess;                /* (sum w)^2 / sum w^2                                                */
    uint64_t n;                /* samples used                                                      */
    uint64_t n_nonfinite;      /* weights that were inf or nan                                      */
} pimc_level_result;

typedef struct pimc_ctx pimc_ctx;

/* Message for a status code (static string). */
const char *pimc_strerror(int status);

/* Detail of the last failure on this context (HIP error text, which argument was invalid).
 * ctx may be NULL: then the last failure of this host thread outside any context. */
const char *pimc_last_error(const pimc_ctx *ctx);

/* Validate a problem (Sec. 2.1/4 problem statement) without touching any device.
 * EINVAL: N not a power of two or N > 2^PIMC_MAX_S, p outside 1..PIMC_MAX_P, T <= 0, m <= 0,
 * n_samples < 2, non-finite a/b/T/m/coefficients, degree outside 0..PIMC_MAX_DEGREE. */
int pimc_check_problem(const pimc_potential *V, double m, double a, double b, double T,
                       uint32_t N, int p, uint64_t n_samples);

/* Host-side effective-action table of one level (no device needed).
 * Writes the folded polynomials of  eps W_p(x, xbar; eps) = sum_k dlt^(2k) P_k(u),  with
 * dlt = 2 xbar the full slice deviation, eps = T/2^level, and u = x^2 if V is even (all odd
 * coefficients zero) else u = x, after the mass rescaling: P_k = eps 4^-k sum_{m=k}^{p-1}
 * eps^(m-k) c_{m,k} (eq.(ansatz) and eq.(1Drec)/(diagonal) evaluated in FP64).
 * Layout of out: for k = 0..*n_k-1, the coefficients of P_k from the highest power deg[k] down to
 * power 0 (deg[k]+1 doubles each). deg must hold p ints; *is_even reports the variable.
 * p in 1..PIMC_MAX_P_SHORT_TIME (the tables of the spectrum entry points go beyond PIMC_MAX_P).
 * cap = capacity of out in doubles; EINVAL if too small (*n_out then holds the size needed). */
int pimc_level_table(const pimc_potential *V, double m, double T, int p, uint32_t level,
                     double *out, size_t cap, size_t *n_out, int *n_k, int *deg, int *is_even);

/* Create a context on HIP device `device`. hip_stream: a hipStream_t to launch on (for example
 * torch's current stream), or NULL for a stream owned by the context. */
int pimc_create(pimc_ctx **out, int device, void *hip_stream);
/* Batches and proposals keep a pointer to the context they were created on: destroy them first. */
int pimc_destroy(pimc_ctx *ctx);

/* Estimate A_{2^n}^(p)(a,b;T) +- err for every level n = 0..s (N = 2^s) from n_samples paths with
 * path indices 0..n_samples-1 (Sec. 4.1: trajectories by bisection, action eq.(SNp), e^{-S}
 * averaged, error per level). Without PIMC_HIERARCHY only levels 0 and s are estimated (entries
 * 1..s-1 have n = 0). out: caller-owned host array of log2(N)+1 entries.
 * The sums over paths are taken in canonical chunks of PIMC_CHUNK_PATHS consecutive path indices
 * (groups of 64 paths in a fixed order, then the chunks in index order), so results are bitwise
 * reproducible, independent of the launch, and level n of an s-run equals the n-run bitwise.
 * Returns PIMC_WNONFINITE (> 0) if any weight was not finite. */
int pimc_amplitude(pimc_ctx *ctx, const pimc_potential *V, double m, double a, double b, double T,
                   uint32_t N, int p, uint64_t n_samples, uint64_t seed, uint32_t stream,
                   uint32_t flags, pimc_level_result *out);

/* pimc_amplitude for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same computation, kernels and results
 * (bit for bit), with every device buffer -- tables, chunk sums, segment list, reduced sums -- in a
 * static workspace of PIMC_NOALLOC_BYTES that the library holds on each GPU it runs on until the
 * process ends. No hipMalloc, hipFree or other device or pinned allocation is made (host-side
 * temporaries of the table construction use the C++ heap). Limit: the chunk sums need
 * 32 * (levels) * ceil(n_samples / PIMC_CHUNK_PATHS) bytes, levels = log2(N)+1 with
 * PIMC_HIERARCHY, else 1; at most 16,513,792 bytes (the workspace less 263,424 bytes of tables,
 * segment list and sums: about 2.1e9 samples for one level, 1.9e8 with every level of N = 1024);
 * larger requests return PIMC_EINVAL with the
 * sizes in pimc_last_error, as do tables beyond 256 KiB. All calls on one GPU share the workspace:
 * calls that overlap on one GPU (several host threads or streams) race, and pimc_last_partials
 * after this call reads the workspace, so it is valid until the next such call on that GPU. */
#define PIMC_NOALLOC_BYTES (16u << 20)
int pimc_amplitude_noalloc(pimc_ctx *ctx, const pimc_potential *V, double m, double a, double b, double T,
                           uint32_t N, int p, uint64_t n_samples, uint64_t seed, uint32_t stream,
                           uint32_t flags, pimc_level_result *out);

/* Per-path level actions sum_k eps_n W_p(x_k, xbar_k; eps_n) (the potential part of eq.(SNp); the
 * kinetic part is absorbed by the bisection sampling) of paths first_path..first_path+k_paths-1,
 * computed by the same kernels as pimc_amplitude.  S_out: caller-owned host array
 * [k_paths][log2(N)+1]; levels not evaluated (no PIMC_HIERARCHY: 1..s-1) are written as 0. */
int pimc_path_actions(pimc_ctx *ctx, const pimc_potential *V, double m, double a, double b,
                      double T, uint32_t N, int p, uint64_t seed, uint32_t stream, uint32_t flags,
                      uint64_t first_path, uint64_t k_paths, double *S_out);

/* Canonical-chunk partial sums of the last pimc_amplitude call on this context: for level
 * `level`, chunks first_chunk..first_chunk+n_chunks-1, four doubles per chunk:
 * (paths, sum d, sum d^2, non-finite count) with d = exp(-(S - S_ref)) - 1 and S_ref the level
 * action of the straight line from a to b (written to *shift). A chunk holds paths
 * [c*chunk_paths, (c+1)*chunk_paths). Lets any chunk of a large run be checked independently. */
int pimc_last_partials(pimc_ctx *ctx, uint32_t level, uint64_t first_chunk, uint64_t n_chunks,
                       double *out, uint64_t *chunk_paths, uint64_t *total_chunks, double *shift);

/* Standard normals of the bisection (Sec. 4.1 offsets before scaling by sigma_n): for paths
 * first_path..first_path+k_paths-1 and heap nodes h = 1..n_nodes, out[path][h-1] = z_h from the
 * Philox4x32-10 / Box-Muller map stated at the top of this header. out: caller-owned host array
 * of k_paths*n_nodes doubles. EINVAL if n_nodes == 0 or n_nodes > 2^PIMC_MAX_S - 1. */
int pimc_normals(pimc_ctx *ctx, uint64_t seed, uint32_t stream, uint64_t first_path, uint64_t k_paths,
                 uint32_t n_nodes, double *out);

/* ---- the modified Poeschl-Teller potential ----------------------------------------------------
 *
 * V(q) = -lambda / cosh^2(alpha q) (eq.(1D-MPT)), by the model-specific ansatz of the paper
 * (eq.(1D-MPTansatz)): with y = tanh(alpha q), 1/cosh^2 = 1 - y^2 and d/dq = alpha (1 - y^2) d/dy,
 * so eq.(1Drec)/(diagonal) run on polynomials in y and every c_{m,k} is an even polynomial in y.
 * The slice action is eps W_p = sum_k dlt^(2k) P_k(tanh^2(alpha mid)) with the same folding as the
 * polynomial tables (mass: alpha -> alpha/sqrt(m), coordinates times sqrt(m), as above). FP64 only
 * (PIMC_FP32_POLY returns EUNSUPPORTED). Outputs, errors and the Philox/bisection conventions are
 * those of pimc_amplitude / pimc_path_actions / pimc_level_table. */
typedef struct {
    double lambda;             /* depth (any finite value; > 0 is attractive)                       */
    double alpha;              /* inverse width, finite and > 0                                     */
} pimc_mpt;

int pimc_amplitude_mpt(pimc_ctx *ctx, const pimc_mpt *V, double m, double a, double b, double T, uint32_t N, int p,
                       uint64_t n_samples, uint64_t seed, uint32_t stream, uint32_t flags, pimc_level_result *out);
int pimc_path_actions_mpt(pimc_ctx *ctx, const pimc_mpt *V, double m, double a, double b, double T, uint32_t N,
                          int p, uint64_t seed, uint32_t stream, uint32_t flags, uint64_t first_path,
                          uint64_t k_paths, double *S_out);
/* Table of one level in the variable u = tanh^2(alpha' q'), layout as pimc_level_table (p up to
 * PIMC_MAX_P_SHORT_TIME; deg must hold p ints). */
int pimc_level_table_mpt(const pimc_mpt *V, double m, double T, int p, uint32_t level, double *out, size_t cap,
                         size_t *n_out, int *n_k, int *deg);

/* ---- general potentials: the effective potential in the derivatives of V ----------------------
 *
 * For a general V the coefficients of eq.(ansatz) are expressions in V and its derivatives up to
 * order 2p-2 (Sec. 3.1/3.2). Here eq.(1Drec)/(diagonal) run once per p on polynomials in the
 * symbols v_j = V^(j)(x) (d v_j/dx = v_{j+1}); each slice evaluates the monomials (in a dimensionless
 * form whose coefficients are the same at every bisection level) from the derivatives of V at its
 * mid-point. The potentials of this mode are
 *     V(q) = sum_{j <= degree} coef[j] q^j + sum_i A_i / cosh^2(alpha_i q) + sum_i B_i exp(-beta_i q^2)
 * (derivatives from closed-form recurrences). p in 1..PIMC_GEN_MAX_P, FP64 only; everything else
 * (mass rescaling, Philox/bisection, outputs, errors) as pimc_amplitude / pimc_path_actions. */
#define PIMC_GEN_MAX_P 18
#define PIMC_GEN_MAX_TERMS 4

typedef struct {
    int degree;                           /* polynomial part, 0..PIMC_MAX_DEGREE                   */
    double coef[PIMC_MAX_DEGREE + 1];
    int n_sech2;                          /* 0..PIMC_GEN_MAX_TERMS terms A / cosh^2(alpha q)        */
    double sech2_A[PIMC_GEN_MAX_TERMS], sech2_alpha[PIMC_GEN_MAX_TERMS];   /* alpha > 0              */
    int n_gauss;                          /* 0..PIMC_GEN_MAX_TERMS terms B exp(-beta q^2)           */
    double gauss_B[PIMC_GEN_MAX_TERMS], gauss_beta[PIMC_GEN_MAX_TERMS];    /* beta > 0               */
} pimc_general_potential;

int pimc_amplitude_general(pimc_ctx *ctx, const pimc_general_potential *V, double m, double a, double b, double T,
                           uint32_t N, int p, uint64_t n_samples, uint64_t seed, uint32_t stream, uint32_t flags,
                           pimc_level_result *out);
int pimc_path_actions_general(pimc_ctx *ctx, const pimc_general_potential *V, double m, double a, double b,
                              double T, uint32_t N, int p, uint64_t seed, uint32_t stream, uint32_t flags,
                              uint64_t first_path, uint64_t k_paths, double *S_out);

/* ---- several coordinates: rotation-invariant potentials (Sec. 2.2) ----------------------------
 *
 * d = D*M coordinates (D dimensions, M particles, no quantum statistics) with
 *     V(q) = sum_{n <= degree} coef[n] (q.q)^n,   q in R^d
 * (the 2D anharmonic oscillator of Sec. 3.3 is d = 2, coef = {0, A/2, g/24}). The short-time
 * amplitude is (2 pi eps)^(-d/2) exp(-(2/eps) xbar.xbar - eps W) with W = sum_{m<p} sum_k eps^(m-k)
 * W_{m,k}, the full contractions of eq.(EXP); W_{m,k} follow from eq.(MBrec) and eq.(DIA), run on
 * polynomials in the invariants u = x.x, w = x.xbar, z = xbar.xbar. Paths: d independent bisection
 * bridges; coordinate c of heap node h takes the normal of Philox call (h >> 1) + c * 2^20 (so
 * coordinate 0 is the one-dimensional path of the same seed, stream and index). Mass m: coordinates
 * times sqrt(m), coef[n] times m^(-n), amplitude times m^(d/2).
 * a and b: host arrays of dim doubles. FP64 only (PIMC_FP32_POLY returns EUNSUPPORTED); outputs,
 * flags and errors as pimc_amplitude / pimc_path_actions. EUNSUPPORTED also when the walk's
 * per-workgroup LDS (the pending right endpoints of its upper levels) exceeds the device's limit:
 * with 160 KB, N = 2^20 in four coordinates. EINVAL: dim outside 1..PIMC_MAX_DIM,
 * degree outside 0..PIMC_MAX_RADIAL_DEGREE, non-finite coefficients or endpoints, and the conditions
 * of pimc_amplitude. */
#define PIMC_MAX_DIM 4             /* d = D*M <= 4: e.g. two particles in two dimensions        */
#define PIMC_MAX_RADIAL_DEGREE 2   /* up to (q.q)^2: the anharmonic-oscillator family               */

typedef struct {
    int dim;                               /* d = D*M, 1..PIMC_MAX_DIM                              */
    int degree;                            /* 0..PIMC_MAX_RADIAL_DEGREE                             */
    double coef[PIMC_MAX_RADIAL_DEGREE + 1];
} pimc_radial_potential;

int pimc_amplitude_radial(pimc_ctx *ctx, const pimc_radial_potential *V, double m, const double *a,
                          const double *b, double T, uint32_t N, int p, uint64_t n_samples, uint64_t seed,
                          uint32_t stream, uint32_t flags, pimc_level_result *out);
int pimc_path_actions_radial(pimc_ctx *ctx, const pimc_radial_potential *V, double m, const double *a,
                             const double *b, double T, uint32_t N, int p, uint64_t seed, uint32_t stream,
                             uint32_t flags, uint64_t first_path, uint64_t k_paths, double *S_out);
/* Folded table of one level (eps = T/2^level, after the mass rescaling), unscaled: with
 * eps W_p = sum_{k,j} (x.xbar)^(2j) (xbar.xbar)^(k-j) Q_{k,j}(x.x), group g holds Q_{k,j} for
 * k = shape[3g], j = shape[3g+1], with shape[3g+2] coefficients (highest power of x.x first), stored
 * consecutively in out. Groups are listed for j from high to low and, within j, k from high to low
 * (the order in which the kernels consume them). *n_groups and *n_out are set; EINVAL if cap or
 * shape_cap (ints) is too small. No device work. */
int pimc_level_table_radial(const pimc_radial_potential *V, double m, double T, int p, uint32_t level,
                            double *out, size_t cap, size_t *n_out, int *shape, size_t shape_cap,
                            int *n_groups);

/* ---- several coordinates: any polynomial potential (Sec. 2.2) ---------------------------------
 *
 * The same as the radial entry points for a potential without rotational symmetry (anisotropic
 * traps, pair interactions such as (q_1 - q_2)^4 of two particles on a line):
 *     V(q) = sum_t coef[t] prod_c q_c^exps[t][c - 1],   q in R^dim
 * (exponents of coordinates beyond dim must be 0). eq.(MBrec) and eq.(DIA) run on polynomials in
 * the 2 dim components of x and xbar (FP64); each level's eps W_p is a polynomial in those
 * components, evaluated by a multivariate Horner scheme over the prefix tree of its monomials.
 * Paths, mass rescaling (coef[t] times m^(-total degree / 2)), outputs, flags and errors as
 * pimc_amplitude_radial. EINVAL: dim outside 1..PIMC_MAX_DIM, n_terms outside 0..PIMC_POLY_MAX_TERMS,
 * a term of total degree above PIMC_POLY_MAX_DEGREE or with a negative exponent, non-finite
 * coefficients or endpoints, and the conditions of pimc_amplitude. EUNSUPPORTED: a level polynomial
 * with more than PIMC_POLY_MAX_MONOMIALS monomials. The recursion for one (V, m, p) is computed once
 * per process and cached. */
#define PIMC_POLY_MAX_TERMS 70      /* every monomial of total degree <= 4 in 4 coordinates         */
#define PIMC_POLY_MAX_DEGREE 4
#define PIMC_POLY_MAX_MONOMIALS 65536

typedef struct {
    int dim;                               /* 1..PIMC_MAX_DIM                                       */
    int n_terms;                           /* 0..PIMC_POLY_MAX_TERMS                                */
    double coef[PIMC_POLY_MAX_TERMS];
    int exps[PIMC_POLY_MAX_TERMS][PIMC_MAX_DIM];
} pimc_poly_potential;

int pimc_amplitude_poly(pimc_ctx *ctx, const pimc_poly_potential *V, double m, const double *a, const double *b,
                        double T, uint32_t N, int p, uint64_t n_samples, uint64_t seed, uint32_t stream,
                        uint32_t flags, pimc_level_result *out);
int pimc_path_actions_poly(pimc_ctx *ctx, const pimc_poly_potential *V, double m, const double *a,
                           const double *b, double T, uint32_t N, int p, uint64_t seed, uint32_t stream,
                           uint32_t flags, uint64_t first_path, uint64_t k_paths, double *S_out);
/* eps W_p at one level (eps = T/2^level, after the mass rescaling) as monomials in the components:
 * term i is coef[i] * prod_c x_c^exps[2 dim i + c] * prod_c xbar_c^exps[2 dim i + dim + c] (x the
 * mid-point, xbar the half-deviation of a slice), in the order the kernels consume them. *n_out is
 * set to the number of terms; EINVAL if cap (doubles) or exps_cap (ints, 2 dim per term) is too
 * small. No device work. */
int pimc_level_table_poly(const pimc_poly_potential *V, double m, double T, int p, uint32_t level, double *coef,
                          size_t cap, int *exps, size_t exps_cap, size_t *n_out);

/* ---- batches: whole grids of endpoints with mixed N, p, T in one graph launch ------------------- */

/* One amplitude of a batch: potential systems[system] with mass m, A_N^(p)(a, b; T) estimated from
 * n_samples paths with path indices 0..n_samples-1 on Philox stream `stream` (the batch's seed).
 * Batches use the specialized kernels: the potential must be even with degree <= 4 (the paper's
 * anharmonic oscillator family, Sec. 3.3) and N >= 16. */
typedef struct {
    uint32_t system;
    double m, a, b, T;
    uint32_t N;
    int p;
    uint64_t n_samples;
    uint32_t stream;
} pimc_task;

typedef struct pimc_batch pimc_batch;

/* Plan a batch: validates every task, builds one table set per (system, m, p, T), numbers every
 * task's canonical chunks (the same chunks as a single pimc_amplitude call, so a task's result is
 * bitwise the single-call result), uploads everything and captures one HIP graph: queue reset, one
 * persistent launch per kernel class (the tasks of one p with N = 16, or with N >= 32), the
 * canonical reduction and the copy of the sums to pinned host memory. flags: 0 or PIMC_HIERARCHY
 * (FP64 only). The batch owns its device memory and stream. Each class starts with its default
 * launch shape. */
int pimc_batch_create(pimc_ctx *ctx, const pimc_potential *systems, int n_systems, const pimc_task *tasks,
                      size_t n_tasks, uint64_t seed, uint32_t flags, pimc_batch **out);

/* Replay the graph once and assemble every task: out[task * (s_max+1) + n] for level n (s_max the
 * largest s of the batch; levels a task does not estimate have n = 0). *ms (may be NULL): device
 * time of the replay. Returns PIMC_WNONFINITE if any task had non-finite weights. */
int pimc_batch_run(pimc_batch *batch, pimc_level_result *out, double *ms);

/* The same with the results written to device memory when out_on_device is nonzero: out is then a
 * caller-owned device buffer of n_tasks * (s_max+1) records (for example a torch tensor), filled by
 * a copy on the context's stream that has completed when the call returns. */
int pimc_batch_run_to(pimc_batch *batch, pimc_level_result *out, int out_on_device, double *ms);

/* Scheduling of the persistent kernels: grid = resident workgroups * grid_mult_x2 / 2
 * (grid_mult_x2 in 1..8), each queue grab takes `grab` consecutive chunks (1..64). Changes only
 * scheduling: results are bitwise identical for every setting. Re-captures the graph. */
int pimc_batch_set_tuning(pimc_batch *batch, int grid_mult_x2, uint32_t grab);

/* A kernel class of a batch and its launch shape: subtree levels held in registers, workgroup
 * size, occupancy target (waves per SIMD) and slices evaluated together. Levels p = 8, 12 and 18
 * have several compiled shapes (8 for tasks with N >= 32, 5 for N = 16), every other level one.
 * tuned_ms / default_ms: the autotuner's device time of the class alone with the chosen and with
 * the default shape (0 before tuning). */
typedef struct {
    int p;
    int n16;                     /* 1: the tasks with N = 16; 0: the tasks with N >= 32 */
    uint64_t n_tasks, n_items;   /* tasks, canonical chunks */
    int shape, n_shapes;         /* chosen shape index (0 = default), number of candidates */
    int subtree_levels, block, waves_per_eu, slice_batch;
    double tuned_ms, default_ms;
} pimc_batch_class;
int pimc_batch_n_classes(const pimc_batch *batch);
int pimc_batch_class_info(const pimc_batch *batch, int k, pimc_batch_class *out);

/* Select launch shape `shape` (0..n_shapes-1) for class k. Every shape gives the same bits: the
 * canonical chunks fix the order of every sum. Re-captures the graph. */
int pimc_batch_set_shape(pimc_batch *batch, int k, int shape);

/* Autotuner: for every class, time each candidate launch shape on the class alone (one launch
 * each) and keep the fastest; then time grid_mult_x2 in {1, 2, 4} x grab in {1, 4, 16} on whole
 * replays. The choice is appended to the text cache file cache_path (may be NULL) under a key of
 * (GPU architecture, the classes, largest s, flags); a later call with a matching key -- for
 * example on a batch of the same tasks with more samples each -- applies the cached choice without
 * timing. */
int pimc_batch_autotune(pimc_batch *batch, const char *cache_path, int *grid_mult_x2, uint32_t *grab);

int pimc_batch_destroy(pimc_batch *batch);
const char *pimc_batch_last_error(const pimc_batch *batch);

/* Create, run once and destroy: out as in pimc_batch_run_to (host memory, or a caller-owned device
 * buffer when out_on_device is nonzero). */
int pimc_amplitude_batch(pimc_ctx *ctx, const pimc_potential *systems, int n_systems, const pimc_task *tasks,
                         size_t n_tasks, uint64_t seed, uint32_t flags, pimc_level_result *out, int out_on_device);

/* ---- learned proposal: affine couplings over the bisection normals -------------------------------
 *
 * The estimator is the paper's A_N^(p) = K_0 E[exp(-sum_k eps W_p)] (Sec. 4) with the bisection
 * normals z (heap nodes h = 1..N-1, z_h scaled by the bridge width of its level as in Sec. 4.1)
 * drawn from a learned density q instead of N(0, I) and reweighted exactly: with z = f(u),
 * u ~ N(0, I) the plain sampler's normals,
 *     log w = -(S(z) - S_ref) - |z|^2/2 + |u|^2/2 + log|det df/du|,   A = sqrt(m) K_0 e^{-S_ref} E[w].
 * f is `layers` affine couplings; layer c splits the heap nodes by mask type c mod 4
 * (0: node 1 + left subtree | right subtree, 1: node 1 + right subtree | left subtree, 2: odd h | even h,
 * 3: even h | odd h; first part conditions, second is transformed) and maps x_B -> x_B e^s + t with
 * (s_hat, t) = W2 silu(W1 x_A + b1) + b2 and s = 2 tanh(s_hat/2) (hidden width 128, x_A zero-padded
 * to 64, s_hat = rows 0..|B|-1, t = rows 64..64+|B|-1). The two products run on bfloat16 matrix
 * cores with FP32 accumulation (x_A, W1, the hidden layer and W2 rounded to bfloat16, round to
 * nearest even); the affine map, log-determinant, action and weights are FP64.
 * Parameters per layer, one flat float vector of PIMC_FLOW_NPARAM: W1 [128][64] row-major, b1 [128],
 * W2 [128][128] row-major [out][hidden], b2 [128].
 * Training minimizes (1-beta) log mean_i w_i^2 + beta (-mean_i log w_i) over batches of fresh base
 * samples with Adam; any parameters give an unbiased estimate, training only lowers its variance.
 * Supported: 2 <= N <= 128 (every coupling part fits 64 inputs); any potential pimc_amplitude takes,
 * FP64 polynomials.
 */
#define PIMC_FLOW_NPARAM 24832
#define PIMC_FLOW_MAX_LAYERS 16

typedef struct {
    int layers;                /* coupling layers, 1..PIMC_FLOW_MAX_LAYERS                           */
    uint32_t batch;            /* training paths per step, 2..65536                                 */
    double lr;                 /* Adam learning rate (beta1 0.9, beta2 0.999, eps 1e-8)             */
    double beta;               /* weight of the reverse-KL term, 0..1                               */
    uint64_t init_seed;        /* W1 ~ U(-1/8, 1/8), W2 ~ init_scale U(-1/20, 1/20), b1 = b2 = 0     */
    double init_scale;         /* 0: the initial map is the identity (the plain sampler)            */
} pimc_flow_config;

typedef struct pimc_flow pimc_flow;

/* Plan a proposal for one problem (validated as in pimc_check_problem with N <= 128): builds the
 * level-s table, allocates parameters, Adam state and training buffers on the context's device.
 * EUNSUPPORTED for N = 1 or N > 128. The flow uses the context's stream and records errors on it. */
int pimc_flow_create(pimc_ctx *ctx, const pimc_potential *V, double m, double a, double b, double T,
                     uint32_t N, int p, const pimc_flow_config *cfg, pimc_flow **out);
int pimc_flow_destroy(pimc_flow *flow);

/* Copy the FP32 master parameters out (layers * PIMC_FLOW_NPARAM floats; *n_out = that count;
 * EINVAL if cap is smaller) or in (n must equal that count; resets the Adam moments and step). */
int pimc_flow_get_params(pimc_flow *flow, float *out, size_t cap, size_t *n_out);
int pimc_flow_set_params(pimc_flow *flow, const float *in, size_t n);

/* Write the parameters to a file (8-byte tag, layer count, N, p, parameters per layer, FP32 values)
 * or read them back into a proposal with the same layer count and N (then as pimc_flow_set_params).
 * EINVAL when the file cannot be opened, is not such a file, or has another shape. */
int pimc_flow_save(pimc_flow *flow, const char *path);
int pimc_flow_load(pimc_flow *flow, const char *path);

/* Loss and gradient of one batch without updating: base normals of paths 0..batch-1 on Philox
 * stream `stream` with the context seed convention (seed, stream) of pimc_normals. loss: host
 * double; ell: host [batch] log weights (may be NULL); grad: host [layers * PIMC_FLOW_NPARAM]
 * floats (may be NULL). The gradient of every tile of 64 paths is added in a fixed order. */
int pimc_flow_grad(pimc_flow *flow, uint64_t seed, uint32_t stream, double *loss, double *ell, float *grad);

/* `steps` Adam steps, step j on paths 0..batch-1 of Philox stream stream_base + (number of steps
 * taken before it), replayed as one captured HIP graph per step. losses: host [steps] or NULL;
 * *ms (may be NULL): device time of all steps. */
int pimc_flow_train(pimc_flow *flow, uint64_t seed, uint32_t stream_base, uint32_t steps, double *losses,
                    double *ms);

/* Log weights, proposal samples and log-determinants of paths first_path..first_path+k_paths-1
 * (base normals as in pimc_normals). ell, logdet: host [k_paths] (may be NULL); z: host
 * [k_paths][N-1] (may be NULL). */
int pimc_flow_log_weights(pimc_flow *flow, uint64_t seed, uint32_t stream, uint64_t first_path, uint64_t k_paths,
                          double *ell, double *z, double *logdet);

/* Estimate A_N^(p)(a,b;T) +- err from n_samples proposal paths 0..n_samples-1 with the current
 * parameters: one level result for level s, summed in the canonical chunks of pimc_amplitude (so
 * pimc_last_partials on the context reads them afterwards). *ms (may be NULL): device time.
 * Returns PIMC_WNONFINITE if any weight was not finite. */
int pimc_flow_amplitude(pimc_flow *flow, uint64_t n_samples, uint64_t seed, uint32_t stream,
                        pimc_level_result *out, double *ms);

/* ---- spectrum from the space-discretized evolution operator ----------------------------------
 *
 * The paper's application of short-time amplitudes (Sec. 2; Sec. 4.2 with Fig. 3): on the grid
 * x_i = -L + (i + 1/2) D, D = 2L/n (symmetric about 0), the matrix
 *     M_ij = D A_1^(p)(x_i, x_j; t),  A_1^(p)(a,b;t) = sqrt(m) (2 pi t)^(-1/2)
 *            exp(-m (b-a)^2/(2t) - t W~_p(sqrt(m)(a+b)/2, sqrt(m)(b-a)/2; t))
 * with W~_p the level-p effective potential of V(y/sqrt(m)) (the mass rescaling above; the N = 1
 * amplitude of Sec. 4.2 at T = t)
 * approximates exp(-t H) on the grid; its largest eigenvalues are exp(-t E_n) and its eigenvectors
 * sample the eigenfunctions. No Monte Carlo is involved (N = 1 at level p). Elements whose
 * free-particle exponent m (x_j - x_i)^2 / (2t) exceeds 40 are exactly zero: the expansion of W_p in
 * the half-deviation has a finite radius (Sec. 4), so there the truncated exponent may grow without
 * bound while the true element is below exp(-40) of the free one. */
#define PIMC_MAX_P_SHORT_TIME 21   /* highest level p for the short-time matrix                       */
#define PIMC_MAX_GRID 65536        /* n <= 65536                                                      */
#define PIMC_MAX_STATES 256        /* eigenpairs per call                                             */
#define PIMC_MAX_LANCZOS 4096      /* Lanczos steps per call                                          */

typedef struct {
    uint32_t iterations;       /* Lanczos steps taken                                               */
    int converged;             /* 1 if every requested residual met the tolerance                   */
    double max_residual;       /* max |M y - theta y| over the returned pairs, relative to theta_0  */
    double matrix_ms;          /* device time of the matrix build                                   */
    double solve_ms;           /* wall time of the eigenvalue iteration (device work + host checks) */
} pimc_spectrum_info;

/* Fill the n x n matrix M_ij above (row-major, leading dimension ld >= n) into DEVICE memory M
 * owned by the caller. p in 1..PIMC_MAX_P_SHORT_TIME, 2 <= n <= PIMC_MAX_GRID, t > 0, L > 0.
 * The matrix is exactly symmetric (every element depends on (x_i - x_j)^2 and x_i + x_j only). */
int pimc_evolution_matrix(pimc_ctx *ctx, const pimc_potential *V, double m, double t, int p, double L,
                          uint32_t n, double *M, uint64_t ld);

/* Lowest k energies E_n = -ln(lambda_n)/t of that matrix (host array E[k], ascending) and, if psi
 * is not NULL, the eigenfunctions on the grid (host psi[k][n], sum_i psi(x_i)^2 D = 1, the largest
 * |psi| positive). Lanczos with full reorthogonalization on the device (the matrix as its upper
 * 64 x 64 tiles, about n^2/2 doubles since it is exactly symmetric, and max_iter + 1 Lanczos vectors
 * are allocated for the call), checked every 16 steps; stops when
 * every requested pair has |M y - theta y| <= tol * theta_0 (returns PIMC_OK) or after max_iter
 * steps (returns PIMC_WNOTCONVERGED with the best values). k in 1..min(n, PIMC_MAX_STATES),
 * max_iter in k+1..min(n, PIMC_MAX_LANCZOS), 0 < tol < 1. info may be NULL. */
int pimc_spectrum(pimc_ctx *ctx, const pimc_potential *V, double m, double t, int p, double L, uint32_t n,
                  uint32_t k, uint32_t max_iter, double tol, double *E, double *psi, pimc_spectrum_info *info);

/* Device time of the last estimation kernel on this context, in milliseconds (HIP events on the
 * context's stream around that launch). */
int pimc_last_kernel_ms(pimc_ctx *ctx, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* PIMC_H */
