/*
 * dhtrace: deflated Hutchinson / hierarchical-probing estimation of Tr(D^-1)
 * for the Wilson-Dirac matrix on one AMD Instinct MI355X (gfx950).
 *
 * Method: Gambhir, Stathopoulos and Orginos, "Deflation as a Method of
 * Variance Reduction for Estimating the Trace of a Matrix Inverse"
 * (arXiv:1603.05988), Algorithm 1 ("deflatedHP").  Each probe z is Z4 noise
 * (Section 1) or a Z4 base vector times a hierarchical-probing Hadamard
 * vector (Section 5.2); the library solves D y = z, forms z^H y, subtracts the
 * deflated quadrature z^H P z with P = W M W^H g5 built from eigenvectors W of
 * Q = g5 D (Section 5.2's z^H V Lambda^-1 V^H (A^H z) in g5 form), and keeps
 * the running trace T_R / j + T_D with its sample variances.
 *
 * Conventions (all entry points):
 *  - Lattice L = {Lx, Ly, Lz, Lt}, every extent even; site
 *    n = x + Lx (y + Ly (z + Lz t)); V = Lx Ly Lz Lt; N = 12 V.
 *  - Canonical spinor: complex128 (interleaved re, im doubles), layout
 *    [rhs][t][z][y][x][spin 4][colour 3]; rhs stride N complex.
 *  - Canonical links: complex128 [4][t][z][y][x][3][3], direction 0..3 =
 *    x, y, z, t; U_mu(x) couples x to x + mu-hat.
 *  - Operator: D psi(x) = (4+m) psi(x) - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu)
 *    + (1 + g_mu) U_mu(x-mu)^H psi(x-mu)], -1 on hops across the t boundary
 *    if t_antiperiodic; chiral basis with g5 = diag(1, 1, -1, -1).
 *  - Pointers named *_dev are device pointers on the context's device; all
 *    other pointers are host pointers.  The caller owns every buffer it
 *    passes; the library never frees caller memory and keeps no pointer to it
 *    after the call returns (except a workspace handed over with
 *    dht_set_workspace).  The library owns its internal copies (links in
 *    three precisions, the deflation basis) and, unless the caller provides
 *    one, its workspace, allocated with hipMalloc on first use and released by
 *    dht_destroy or dht_workspace_trim.
 *  - Streams: all device work is enqueued on the stream given to dht_create,
 *    except dht_trace_batch's per-batch projection, which runs on a second
 *    stream of the library's own (default priority) after the probes are made
 *    and is joined before the call returns.  Calls that return host values
 *    synchronise the context stream before returning.
 *  - Errors: every int-returning call returns DHT_OK (0) or a negative code;
 *    dht_last_error() gives a message for the calling thread.  No C++
 *    exception crosses the interface.
 *  - Threads: a context must not be used by two threads at once.
 */
#ifndef DHTRACE_H
#define DHTRACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dht_ctx dht_ctx;

/* Largest batch (right-hand sides per call) of dht_make_probes, dht_solve,
 * dht_project*, dht_trace_batch; batches are padded internally to the next
 * power of two with zero right-hand sides.  dht_apply takes any count. */
#define DHT_MAX_BATCH 256

enum {
    DHT_OK = 0,
    DHT_ERR_INVALID_ARG = -1,
    DHT_ERR_HIP = -2,
    DHT_ERR_OOM = -3,
    DHT_ERR_STATE = -4,        /* call order violated (e.g. no gauge field yet)  */
    DHT_ERR_BREAKDOWN = -5,    /* Krylov breakdown that no fallback could repair */
    DHT_ERR_NOT_CONVERGED = -6 /* some right-hand side missed the tolerance      */
};

/* Storage precision of fields on the device.  FP32 and BF16 accumulate in FP32. */
typedef enum { DHT_FP64 = 0, DHT_FP32 = 1, DHT_BF16 = 2 } dht_prec;

/* Operators for dht_apply: D, D^H = g5 D g5, g5, and the Hermitian Q = g5 D. */
typedef enum { DHT_OP_D = 0, DHT_OP_DDAG = 1, DHT_OP_G5 = 2, DHT_OP_Q = 3 } dht_op;

typedef struct {
    int L[4];            /* Lx, Ly, Lz, Lt: each even and >= 2                */
    double mass;         /* bare mass m; the diagonal is 4 + m (must be != 0) */
    int t_antiperiodic;  /* 1: -1 phase on hops across the t boundary         */
} dht_lattice;

/* Probe vectors (Algorithm 1: Z4 base vector, Hadamard vector, product).
 * hp = 0: plain Z4 noise, a fresh vector per probe index j.
 * hp = 1: one Z4 base vector z0 per (seed, run), times the hierarchical-
 *         probing Hadamard vector h_j; probe indices j < 2^63.
 * Noise index generator: SplitMix64 (Steele, Lea, Flood 2014).  With
 * out(s, i) = mix(s + (i+1) * 0x9E3779B97F4A7C15):  K_run = out(seed, run);
 * key = K_run (hp) or out(K_run, j) (plain); component n takes the 2 bits at
 * 2 (n mod 32) of out(key, n / 32), value k -> i^k.  HP colour of a site:
 * for level l, bit 4l = parity of sum_mu floor(x_mu / 2^l), bits 4l+1..4l+3 =
 * floor(x_mu / 2^l) mod 2 for mu = x, y, z; h_j(x) = (-1)^popcount(c(x) & j). */
typedef struct {
    uint64_t seed;
    uint64_t run;
    int hp;
} dht_probe_spec;

/* Solver methods (the paper leaves the linear solver open: Algorithm 1, "Solve Ay = z"). */
enum {
    DHT_SOLVER_BICGSTAB_FP64 = 0, /* plain FP64 BiCGStab on the even/odd Schur system          */
    DHT_SOLVER_DC_BICGSTAB = 1,   /* FP64 defect correction around an FP32/BF16 BiCGStab      */
    DHT_SOLVER_DC_FGMRES_NN = 2,  /* FP64 defect correction, one FP32 FGMRES(restart) cycle
                                     per correction, the learned network as right
                                     preconditioner (needs dht_nn_init / _set_weights);
                                     falls back to DC_BICGSTAB if maxiter is exhausted      */
    DHT_SOLVER_DC_FGMRES = 3      /* the same with the identity preconditioner              */
};

enum { /* dht_solve_stats.status */
    DHT_STATUS_CONVERGED = 0,
    DHT_STATUS_NOT_CONVERGED = 1,
    DHT_STATUS_FALLBACK_FP32 = 2,     /* converged after escalating the inner precision   */
    DHT_STATUS_FALLBACK_FP64 = 3,     /* converged on the FP64 inner solve                 */
    DHT_STATUS_FALLBACK_BICGSTAB = 4  /* FGMRES missed the target; BiCGStab finished      */
};

typedef struct {
    int method;        /* DHT_SOLVER_*                                          */
    int inner;         /* dht_prec of the inner solve (DC methods)              */
    double tol;        /* target relative true residual ||z - D x|| / ||z||     */
    int maxiter;       /* cap on inner iterations summed over outer cycles      */
    int restart;       /* FGMRES restart length (<= 64)                         */
    double inner_tol;  /* relative reduction per inner solve (0: 1e-2 BF16, 1e-5 FP32) */
    int max_outer;     /* cap on defect-correction cycles (0: default 50)       */
    uint32_t fault_inject; /* testing only, conditions forced from the host:
                              bit 0: the first inner right-hand side is NaN;
                              bit 1: one full-residual check after a predicted
                                     convergence is treated as failed;
                              bit 2: one in-place residual update reports
                                     norms 1e-12 of the true ones (the loop
                                     must then catch the miss in FP64)      */
    int history;       /* BF16 inner solves: iterations whose p and s are kept
                          before x is rebuilt from them (0: automatic, up to 16
                          within a 12 GB budget; else 2..16)                   */
} dht_solver_params;

typedef struct {
    int iters;          /* inner Krylov iterations (all cycles)        */
    int outer;          /* defect-correction cycles                    */
    double true_resid;  /* final ||z - D x|| / ||z|| in FP64            */
    int status;         /* DHT_STATUS_*                                 */
} dht_solve_stats;

/* Per-probe record of dht_trace_batch: q = z^H D^-1 z (as solved), and the
 * deflated quadrature q_defl = q - z^H P z. */
typedef struct {
    double q_re, q_im;
    double qd_re, qd_im;
    dht_solve_stats s;
} dht_record;

/* Running estimates (Algorithm 1, the trace update): mean = T_R / n, mean_defl =
 * T_D + (mean of q_defl).  Variances are unbiased sample variances
 * (1/(n-1)): var = mean |q - qbar|^2 (the Z4 variance of Section 1),
 * var_re / var_im of the real / imaginary parts. */
typedef struct {
    int64_t n;
    double mean_re, mean_im;
    double mean_defl_re, mean_defl_im;
    double TD_re, TD_im;
    double var, var_re, var_im;
    double var_defl, var_defl_re, var_defl_im;
} dht_estimate;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  Validates the lattice. */
int dht_create(const dht_lattice* lat, int device, void* hip_stream, dht_ctx** out);
int dht_destroy(dht_ctx* ctx);
const char* dht_last_error(void);
/* Library version string (static storage). */
const char* dht_version(void);

/* Caller-owned workspace.  dht_workspace_size plans the device scratch of
 * dht_trace_batch and dht_solve for batches of up to max_nrhs right-hand
 * sides with the parameters prm (its method, inner precision and history,
 * with every precision fallback they can reach), the current deflation basis
 * and projection window, and returns the bytes needed.  dht_set_workspace then
 * hands over a device buffer of at least that size (256-byte aligned, e.g. a
 * torch.empty uint8 tensor; the caller keeps it alive and owns it): those
 * calls take all their device scratch from it and allocate none -- a request
 * beyond the plan (a larger batch, another method, a basis or window changed
 * afterwards) fails with DHT_ERR_OOM instead.  Other calls (dht_apply,
 * dht_project*, the eigensolver, the autotuner, the network's training) use
 * the buffer where the plan covers their request and library workspace
 * otherwise.  The library-owned device workspace is released when the buffer
 * is set; ptr = NULL returns to library-owned workspace.  A small pinned host
 * buffer of the solver's per-RHS states stays library-owned.  The buffer is
 * scratch except for the projection window's probe codes and coefficients,
 * which later batches of the window read: the caller must leave it untouched
 * while it is set. */
int dht_workspace_size(dht_ctx* ctx, int max_nrhs, const dht_solver_params* prm, size_t* bytes);
int dht_set_workspace(dht_ctx* ctx, void* dev_ptr, size_t bytes);

/* Release the library-owned workspace (solver fields, reduction partials,
 * projection window, network activations); links, the deflation basis, the
 * network weights and the running estimates stay.  Later calls allocate again
 * what they need.  For callers that run methods of very different footprint
 * one after another on one context. */
int dht_workspace_trim(dht_ctx* ctx);

/* Upload links (device pointer, canonical layout).  Packs them into the
 * internal even/odd layout in FP64, FP32 and BF16 (round to nearest even). */
int dht_set_gauge(dht_ctx* ctx, const double* U_dev);

/* Y = op(X) for nrhs canonical spinors (device pointers, complex128), with the
 * operator evaluated in storage precision `prec` (X is rounded to `prec` on
 * entry; Y is returned in complex128).  X and Y must not overlap. */
int dht_apply(dht_ctx* ctx, int op, int prec, const double* X_dev, double* Y_dev, int nrhs);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same Y = op(X) as dht_apply, with the library's internal even/odd
 * copies of each chunk of up to 64 right-hand sides held in a fixed
 * device-resident scratch array of DHT_NOALLOC_SCRATCH_BYTES per GPU instead
 * of allocated workspace.  The call makes no hipMalloc / hipFree and does not
 * synchronise: the work is enqueued on the context stream and Y is complete
 * when that stream reaches it (launches are not counted by dht_profile_*).
 * Limit: 2 * 12 * V * pad(min(nrhs, 64)) * s bytes must not exceed
 * DHT_NOALLOC_SCRATCH_BYTES (pad = next power of two, s = 16 / 8 / 4 bytes
 * per complex for FP64 / FP32 / BF16), else DHT_ERR_INVALID_ARG and nothing
 * is enqueued.  Every call on one GPU (any context) shares that GPU's array,
 * and the last call's contents stay in it: calls that may overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller. */
#define DHT_NOALLOC_SCRATCH_BYTES (32u << 20)
int dht_apply_noalloc(dht_ctx* ctx, int op, int prec, const double* X_dev, double* Y_dev, int nrhs);

/* Write probes j = first .. first+nrhs-1 to Z_dev (canonical complex128). */
int dht_make_probes(dht_ctx* ctx, const dht_probe_spec* spec, int64_t first, int nrhs, double* Z_dev);

/* Same probes as dht_make_probes, returned as the 2-bit Z4 indices k(n) of
 * the base noise (uint8, [rhs][N]) and the Hadamard sign per site (int8,
 * [rhs][V], all +1 when hp = 0).  For bit-exact checks of the generator. */
int dht_probe_indices(dht_ctx* ctx, const dht_probe_spec* spec, int64_t first, int nrhs,
                      uint8_t* k_dev, int8_t* sign_dev);

/* Solve D X = Z for nrhs right-hand sides (device, canonical complex128).
 * stats (host, nrhs entries, may be NULL) receives per-RHS results.  Returns
 * DHT_ERR_NOT_CONVERGED if any RHS missed the tolerance (stats still filled). */
int dht_solve(dht_ctx* ctx, const dht_solver_params* prm, const double* Z_dev, double* X_dev,
              int nrhs, dht_solve_stats* stats);

/* ---- deflation (Section 5.2; Algorithm 1, the deflation space and T_D) ---- */

/* Start a deflation basis of k vectors stored in precision `prec`. */
int dht_deflation_begin(dht_ctx* ctx, int k, int prec);
/* Copy columns first .. first+count-1 of W from W_dev (canonical complex128,
 * [count][N]) into the stored basis, rounding to the storage precision. */
int dht_deflation_set(dht_ctx* ctx, int first, int count, const double* W_dev);
/* Eigensolver for the basis (Section 5.1: the smallest singular triplets of D
 * follow from the eigenpairs of Q = g5 D of smallest |lambda|).  FP64
 * Chebyshev-filtered subspace iteration: a polynomial of `degree` in Q^2,
 * bounded on [a, ||Q||^2] with a = the block's largest Ritz value of Q^2,
 * amplifies the bottom of the spectrum of Q^2; each cycle orthonormalises the
 * block (Cholesky QR, twice) and takes a Rayleigh-Ritz step with Q.
 *   tol       relative residual target ||Q w - lambda w|| / B_Q with the norm
 *             bound B_Q = |4 + m| + 4 >= ||Q||;
 *   max_iter  filter cycles;  guard  extra block vectors beyond k (0: max(16, k/4));
 *   seed      Z4 start block.
 * The block (k + guard rounded up to a power of two >= 32) must not exceed
 * 256 vectors; it takes four FP64 full fields of that many RHS of workspace. */
typedef struct dht_eig_params {
    double tol;
    int max_iter;
    int degree;
    int guard;
    uint64_t seed;
} dht_eig_params;
typedef struct dht_eig_stats {
    int iters;          /* filter cycles run */
    int converged;      /* leading Ritz pairs (by |lambda|) within tol */
    int block;          /* block size used */
    int64_t matvecs;    /* applications of Q to the whole block */
} dht_eig_stats;
/* Fill the k columns set up by dht_deflation_begin with the k Ritz vectors of
 * smallest |lambda| (rounded to the storage precision); call
 * dht_deflation_finalize afterwards for M and T_D.  lambda_host and
 * resid_host (k doubles each, may be NULL) receive the Ritz values, ordered
 * by |lambda|, and their relative residuals; stats may be NULL.  Returns
 * DHT_ERR_NOT_CONVERGED (basis still filled) if some pair missed tol within
 * max_iter cycles. */
int dht_deflation_eigensolve(dht_ctx* ctx, const dht_eig_params* prm, double* lambda_host, double* resid_host,
                             dht_eig_stats* stats);
/* Preconditioned block eigensolver with locking (Section 5.1: the paper
 * computes its deflation space with a preconditioned Davidson-type method,
 * a window of block vectors and locking).  LOBPCG on Q^2 = D^H D for its k
 * smallest eigenvalues sigma^2 (sigma: the smallest singular values of D):
 * a window of `block` (32 or 64) vectors, the preconditioned residuals and
 * the previous directions, a Rayleigh-Ritz step on the three blocks per
 * iteration; a leading Ritz vector is locked once ||Q^2 x - sigma^2 x|| <=
 * tol ||Q||^2 (||Q|| taken as |4 + m| + 4), and its window slot refilled with
 * Z4 noise.  precond != 0 applies (Q^2)^-1 = D^-1 g5 D^-1 g5 approximately by
 * two mixed-precision (BF16) BiCGStab solves to the relative residual
 * precond_tol each; precond = 0 runs plain LOBPCG.  The k locked vectors fill
 * the columns set up by dht_deflation_begin (rounded to the storage
 * precision; any basis of the space serves the Galerkin finalize that must
 * follow).  sigma_host and resid_host (k doubles each, may be NULL) receive
 * sigma and the relative residual of each locked vector in locking order.
 * Returns DHT_ERR_NOT_CONVERGED (basis filled with the best Ritz vectors) if
 * fewer than k converged within max_iter iterations.  Its working fields
 * (13 FP64 blocks of N x block complex, and the locked vectors in FP64,
 * ceil(k / block) more) are library-owned workspace outside the plan of
 * dht_workspace_size.  Errors: DHT_ERR_INVALID_ARG for bad parameters,
 * DHT_ERR_STATE without gauge field or dht_deflation_begin,
 * DHT_ERR_BREAKDOWN if a block loses rank, DHT_ERR_OOM if the fields do not
 * fit. */
typedef struct dht_lobpcg_params {
    double tol;          /* locking threshold, relative to ||Q||^2          */
    int max_iter;        /* cap on block iterations                         */
    int block;           /* window size: 32 or 64                           */
    int precond;         /* 1: two loose solves with D; 0: none             */
    double precond_tol;  /* relative residual of each preconditioner solve  */
    uint64_t seed;       /* Z4 noise of the start and refill vectors        */
} dht_lobpcg_params;
typedef struct dht_lobpcg_stats {
    int iters;                /* block iterations                            */
    int converged;            /* locked vectors within tol                   */
    int64_t q_applications;   /* applications of Q to a whole block          */
    int64_t precond_solves;   /* right-hand sides solved by the preconditioner */
} dht_lobpcg_stats;
int dht_deflation_lobpcg(dht_ctx* ctx, const dht_lobpcg_params* prm, double* sigma_host, double* resid_host,
                         dht_lobpcg_stats* stats);
/* Copy columns first .. first+count-1 of the stored basis, as rounded to its
 * storage precision, to W_dev (device, canonical complex128, [count][N]). */
int dht_deflation_get(dht_ctx* ctx, int first, int count, double* W_dev);
/* Finish: H = W^H Q W accumulated in FP64 from the stored basis, M = H^-1,
 * T_D = Tr(M W^H g5 W).  TD_host (2 doubles: re, im) may be NULL. */
int dht_deflation_finalize(dht_ctx* ctx, double* TD_host);
/* Finish with the diagonal Galerkin inverse M = diag(1 / w_i^H Q w_i) and
 * T_D = sum_i M_ii w_i^H g5 w_i: k FP64 dot products instead of k^2.  Exact
 * when W holds orthonormal eigenvectors of Q; for any W the estimator stays
 * unbiased (T_D is the trace of the same P), only its variance changes. */
int dht_deflation_finalize_diag(dht_ctx* ctx, double* TD_host);
/* Host copy of M (k x k complex128, row-major) for checks and playback. */
int dht_deflation_get_M(dht_ctx* ctx, double* M_host);
/* Drop the deflation basis (later batches are undeflated, T_D = 0). */
int dht_deflation_clear(dht_ctx* ctx);

/* c1 = W^H Z and c2 = W^H g5 Z for nrhs canonical spinors Z_dev; results on
 * the host, complex128 row-major [k][nrhs]. */
int dht_project(dht_ctx* ctx, const double* Z_dev, int nrhs, double* c1_host, double* c2_host);

/* c1 = W^H z and c2 = W^H g5 z for the probes j = first .. first+nrhs-1 of
 * `spec`, generated on the device.  With a BF16 basis (nrhs <= 64) this is
 * the MFMA projection used inside dht_trace_batch: probes enter as exact
 * 2-bit codes, products accumulate in FP32 inside the matrix cores and are
 * summed in FP64 every 64 complex entries; otherwise FP64 accumulation.
 * Results on the host, complex128 row-major [k][nrhs]. */
int dht_project_probes(dht_ctx* ctx, const dht_probe_spec* spec, int64_t first, int nrhs, double* c1_host,
                       double* c2_host);

/* ---- Algorithm 1 ---------------------------------------------------------- */

/* The loop body of Algorithm 1 for probes j = first .. first+nrhs-1: generate the
 * probes on the device, solve, form q = z^H x in FP64, project on the
 * deflation basis (when set) and accumulate the running estimates.  With a
 * BiCGStab method the probes are generated in BF16 storage (their values
 * i^k * (+-1) are exact there) and the FP64 hops that read them widen them
 * exactly, so results equal those of FP64 probes.  records
 * (host, nrhs entries, may be NULL) receives per-probe results; coef_host
 * (may be NULL) receives the projection coefficients c1, c2 as complex128
 * [2][k][nrhs] for playback with other k (Section 6.3).  Only probes whose
 * solve met the tolerance (status != DHT_STATUS_NOT_CONVERGED) enter the
 * running estimates; the others are still reported in records, and the call
 * then returns DHT_ERR_NOT_CONVERGED, so a batch that is retried is counted
 * once. */
int dht_trace_batch(dht_ctx* ctx, const dht_probe_spec* spec, int64_t first, int nrhs,
                    const dht_solver_params* prm, dht_record* records, double* coef_host);

/* Projection window for dht_trace_batch (Section 5.2: the coefficients
 * V^H z and V^H g5 z of each probe).  nprobes = 0 (the default) projects each
 * batch on its own.  With 0 < nrhs < nprobes <= 64 and a BF16 basis, a batch
 * whose probes are not covered by the last window starts a new window
 * j = first .. first+nprobes-1: the coefficients of all its probes come out
 * of one pass over the basis (the basis read is shared by up to 64 probes)
 * and later batches inside the window reuse them.  Each coefficient has the
 * same FP32 partial sums over 64-entry chunks as in a per-batch projection;
 * only the FP64 order in which the chunk sums are added may differ (the split
 * of the basis over workgroups depends on the column count).  Changing the
 * basis, or calling this function, drops the window.  The window's 2-bit
 * probe codes (N x pad(nprobes) bytes) and coefficients stay allocated in
 * the context.  Errors: DHT_ERR_INVALID_ARG outside 0..64. */
int dht_set_projection_window(dht_ctx* ctx, int nprobes);
int dht_estimate_get(dht_ctx* ctx, dht_estimate* est);
int dht_estimate_reset(dht_ctx* ctx);

/* ---- Traces Tr(Gamma D^-1) over one deflation space ----------------------- */

/* End of Section 5.2: the deflated split Tr(Gamma D^-1) = Tr(Gamma P) +
 * Tr(Gamma (D^-1 - P)) holds for any inexpensive matrix Gamma, the estimator
 * takes one Gamma product per probe, and the deflation space is shared.  Here
 * Gamma is a 4 x 4 complex spin matrix acting alike on every site and colour,
 * (Gamma psi)(x, s, c) = sum_t Gamma[s][t] psi(x, t, c) -- the Dirac matrices
 * and their products, or any other; P = W M W^H g5 is the current deflated
 * part (T_D(Gamma) = Tr(M W^H g5 Gamma W)).
 *
 * dht_gamma_set registers ng matrices (host, complex128 [ng][4][4], row-major),
 * resets their running estimates and, when TD_host is not NULL, writes
 * T_D(Gamma) for each (complex128 [ng]; 0 without a basis).  T_D(Gamma) comes
 * from the 16 spin-pair traces sum_ab M_ab W_b,s^H W_a,t, accumulated in FP64
 * from the stored basis once per basis: k spin-pair self products for a
 * diagonal M, and for a full M four times the FP64 basis products of
 * dht_deflation_finalize.  Errors: DHT_ERR_INVALID_ARG for ng outside
 * 1..DHT_MAX_GAMMA or a non-finite entry, DHT_ERR_STATE for a basis set but
 * not finalized. */
#define DHT_MAX_GAMMA 64
int dht_gamma_set(dht_ctx* ctx, const double* gamma_host, int ng, double* TD_host);
/* Algorithm 1's loop body for every registered matrix at once, on the probes
 * j = first .. first+nrhs-1 of spec (generated in FP64 storage).  One solve
 * x = D^-1 z per probe serves all matrices: z^H Gamma x = sum_st Gamma[s][t]
 * z_s^H x_t from the 16 spin-pair forms of (z, x) (one pass over both), and
 * with a basis z^H Gamma P z = (W^H Gamma^H z)^H M (W^H g5 z) from the 16
 * spin-pair projections W_s^H z_t (v_s: the spin-s entries of v) -- one pass
 * over the basis per 16 probes with a BF16 basis (MFMA over the probes' exact
 * 2-bit codes, FP32 sums flushed to FP64 every 64 entries, as in
 * dht_project_probes), one FP64 pass per batch otherwise.  records (host, may
 * be NULL) receives [ng][nrhs] entries: q = z^H Gamma x, qd = q - z^H Gamma P z
 * and the probe's solve stats.  The running estimates per matrix take only
 * converged probes; the call then returns DHT_ERR_NOT_CONVERGED if a probe
 * missed the tolerance.  The estimates are not reset when the basis changes
 * (dht_gamma_set resets them).  This call is outside the workspace plan of
 * dht_workspace_size: slots it needs beyond the plan are allocated by the
 * library.  Errors: DHT_ERR_STATE without registered matrices or gauge field,
 * or with a basis set but not finalized. */
int dht_trace_gamma_batch(dht_ctx* ctx, const dht_probe_spec* spec, int64_t first, int nrhs,
                          const dht_solver_params* prm, dht_record* records);
/* Running estimate of Tr(Gamma_g D^-1), g = 0..ng-1, with the fields of
 * dht_estimate_get (TD = T_D(Gamma_g)). */
int dht_gamma_estimate_get(dht_ctx* ctx, int g, dht_estimate* est);
/* Checkpoint / resume of the running estimates (Algorithm 1 accumulates over
 * probes; a long run can be split across processes).  save writes a small text
 * file at `path` (exact round trip of the moments); load restores them into a
 * context of the same lattice and mass, and of the same deflation space when
 * one is set (T_D must agree to 1e-12 relative).  Errors: DHT_ERR_INVALID_ARG
 * for an unreadable or foreign file, DHT_ERR_STATE for a mismatched context. */
int dht_state_save(dht_ctx* ctx, const char* path);
int dht_state_load(dht_ctx* ctx, const char* path);

/* ---- learned preconditioner ----------------------------------------------- */
/* A 3-layer 4D convolutional network (3^4 taps, 24 -> 48 -> 48 -> 24 real
 * channels = real and imaginary parts of the 12 spin-colour components,
 * ReLU after layers 1 and 2, no bias, periodic padding) approximating
 * r -> D^-1 r, used as the right preconditioner of FGMRES.  Weights:
 * float [3 layers][81 taps][Cout][Cin] concatenated (dht_nn_num_weights()
 * floats); tap t = (dx+1) + 3 (dy+1) + 9 (dz+1) + 27 (dt+1) and
 * out[x] = sum_t W[t] in[x + d_t].  Inference and training run on BF16
 * matrix cores with FP32 accumulation and an FP32 master copy of the
 * weights.  R and E are canonical complex128 spinors (device), read as
 * [n][V][24] reals. */
int64_t dht_nn_num_weights(void);
/* He-normal initial weights (std sqrt(2 / (81 Cin)), the last layer scaled
 * by 0.1) from a seeded SplitMix64/Box-Muller generator; resets the optimiser. */
int dht_nn_init(dht_ctx* ctx, uint64_t seed);
/* Skip coefficient s of the preconditioner M(r) = net(r) + s r (default 0).
 * s = 1 / (4 + m) makes M the point-Jacobi inverse of D plus the learned
 * correction; it enters forward, loss, training and the FGMRES application. */
int dht_nn_set_skip(dht_ctx* ctx, double s);
int dht_nn_set_weights(dht_ctx* ctx, const float* w_host);
int dht_nn_get_weights(dht_ctx* ctx, float* w_host);
/* E = M(R) for n spinors. */
int dht_nn_forward(dht_ctx* ctx, const double* R_dev, double* E_dev, int n);
/* Loss sum_b ||M(R_b) - E_b||^2 / ||E_b||^2 / n and its weight gradient
 * (grad_host: dht_nn_num_weights() floats, may be NULL); n <= 64. */
int dht_nn_grad(dht_ctx* ctx, const double* R_dev, const double* E_dev, int n, float* grad_host, double* loss);
/* Adam (beta 0.9 / 0.999, eps 1e-8) over npairs pairs in minibatches of
 * `batch` (<= 64) for `epochs` passes; final_loss (may be NULL) receives the
 * mean loss of the last epoch. */
int dht_nn_train(dht_ctx* ctx, const double* R_dev, const double* E_dev, int npairs, int epochs, int batch, float lr,
                 double* final_loss);
/* Training pairs from FGMRES restarts: for probes j = first .. first+nrhs-1
 * of `spec`, x* is solved to 1e-12 (FP64 BiCGStab), then FGMRES(restart)
 * cycles with the identity preconditioner run to 1e-8; at every restart k the
 * pair (r_k / ||r_k||, (x* - x_k) / ||r_k||) is written to R_dev / E_dev
 * (capacity `cap` spinors each).  *count receives the number written. */
int dht_nn_make_pairs(dht_ctx* ctx, const dht_probe_spec* spec, int64_t first, int nrhs, int restart, double* R_dev,
                      double* E_dev, int cap, int* count);

/* ---- instrumentation ------------------------------------------------------ */

/* Counts of defect-correction branches taken since dht_create, out[0..3]:
 * full-residual checks after an inner solve predicted convergence; such
 * checks that missed (the loop continued from the stored FP64 residual);
 * in-place residual updates (r -= sigma Dhat e, Dhat e in FP32); loops that
 * stopped on in-place norms whose FP64 residual then missed the tolerance
 * and were resumed from it.  n must be >= 4. */
int dht_solver_counters(dht_ctx* ctx, int64_t* out, int n);

/* Timing of the last dht_trace_batch / dht_solve, from HIP events, in
 * milliseconds: [0] probes, [1] solve, [2] projection (a batch's own pass
 * runs on a second stream concurrently with the solve; a projection window's
 * pass runs on the context stream before it; 0 when the batch reused a
 * window), [3] quadratic forms, [4] whole call.  n must be >= 5. */
int dht_last_timings(dht_ctx* ctx, double* ms_host, int n);

/* Per-kernel-class timing: when enabled, every launch of an instrumented
 * kernel is bracketed by HIP events on the context stream; totals are
 * accumulated at the next synchronising call.  Classes: 0/1/2 = hop kernel
 * in FP64/FP32/BF16, 3 = MFMA projection, 4 = generic projection (also its
 * spin-pair form), 5 = the network's convolutions (BF16 matrix cores), 6 =
 * spin-pair MFMA projection (dht_trace_gamma_batch).  total_bytes is the
 * algorithmic byte count of those launches (input and output fields once,
 * links once); for class 5 it is the flop count (2 per multiply-add). */
int dht_profile_enable(dht_ctx* ctx, int on);
int dht_profile_reset(dht_ctx* ctx);
int dht_profile_get(dht_ctx* ctx, int cls, int64_t* count, double* total_ms, double* total_bytes);

/* Benchmark helper: time `reps` back-to-back applications of the even/odd
 * hopping kernel (out parity 0 from parity 1) on nrhs internal fields in
 * precision prec, after `warmup` untimed ones; returns the mean kernel time
 * in ms measured with HIP events on the context stream. */
int dht_bench_hop(dht_ctx* ctx, int prec, int nrhs, int warmup, int reps, double* ms_per_call);

/* ---- launch-shape autotuning ---------------------------------------------- */

/* Form of the even/odd hopping kernel (the stencil of Section 1 applied on one
 * parity); all forms compute the same sums in a different order of
 * accumulation (results agree to rounding).
 *   DHT_HOP_SITE      one lane per (site, RHS), links read per lane;
 *   DHT_HOP_SITE_LDS  as SITE, the workgroup's links copied once into LDS
 *                     (needs 256 / nrhs <= 32, i.e. nrhs >= 8);
 *   DHT_HOP_TMARCH    one lane per (x, y, z column, RHS) walking t_chunk
 *                     slices in t, the backward t-neighbour kept in registers
 *                     (t_chunk even, divides Lt; 0 = automatic);
 *   DHT_HOP_SITE_ROWL, DHT_HOP_TMARCH_ROWL  as SITE / TMARCH, with each
 *                     site's links loaded once per 16-lane row (the row's 16
 *                     right-hand sides) and broadcast within the row; BF16
 *                     sweeps of >= 16 right-hand sides only (other precisions
 *                     and smaller sweeps run the plain form);
 *   DHT_HOP_TSKEW, DHT_HOP_TSKEW_ROWL  as TMARCH / TMARCH_ROWL, skewed so that
 *                     each step reads one input slice: step t completes
 *                     output t and starts output t + 1, whose accumulator is
 *                     carried to the next step (same t_chunk rules).
 * streaming_stores = 1 writes the output with non-temporal stores.
 * rhs_group = G (a power of two dividing nrhs; 0 = nrhs): the lattice is swept
 * once per group of G right-hand sides, the groups side by side on the chip,
 * so fewer bytes per site share the caches while the links are read once per
 * group (the LDS form needs G >= 8).
 * z_block = Z (t-marching forms; a power of two dividing Lz, 0 or 1 = none):
 * the x-rows of a chunk are walked in blocks of Z consecutive z planes, y
 * next, so that the workgroups resident together hold the z neighbours of
 * their rows as well as the y neighbours. */
enum {
    DHT_HOP_SITE = 0,
    DHT_HOP_SITE_LDS = 1,
    DHT_HOP_TMARCH = 2,
    DHT_HOP_SITE_ROWL = 3,
    DHT_HOP_TMARCH_ROWL = 4,
    DHT_HOP_TSKEW = 5,
    DHT_HOP_TSKEW_ROWL = 6
};
typedef struct dht_hop_config {
    int form;
    int streaming_stores;
    int t_chunk;
    int rhs_group;
    int z_block;
} dht_hop_config;

/* Epilogue classes, tuned separately: DHT_HOP_PLAIN launches compute
 * out = b Hop(in); DHT_HOP_FUSED launches also read an x-pay operand (and a
 * second axpy operand or fused sums of the output with its own operands);
 * DHT_HOP_FUSED_A launches read an x-pay operand and sum (a, out) with a
 * third operand a (BiCGStab's (rhat, v)). */
enum { DHT_HOP_PLAIN = 0, DHT_HOP_FUSED = 1, DHT_HOP_FUSED_A = 2 };

/* Set the hopping-kernel shape used for (prec, nrhs, epilogue class) on this
 * context; cfg = NULL restores the built-in default.  Errors:
 * DHT_ERR_INVALID_ARG for a shape that does not fit the lattice or batch
 * (nrhs: power of two <= 256) or a bad class. */
int dht_hop_config_set(dht_ctx* ctx, int prec, int nrhs, int epilogue, const dht_hop_config* cfg);
/* The shape in effect for (prec, nrhs, epilogue class) (t_chunk resolved). */
int dht_hop_config_get(dht_ctx* ctx, int prec, int nrhs, int epilogue, dht_hop_config* out);

typedef struct dht_tune_result {
    dht_hop_config best[3];  /* per epilogue class: fastest candidate that passed the parity check */
    double best_ms[3];       /* its mean time per hop application */
    double default_ms[3];    /* the built-in default's time */
    int candidates;          /* shapes of the grid timed per class (z blocks excluded) */
    int rejected;            /* shapes whose output differed from the default's beyond rounding */
    double max_rel_diff;     /* largest max|out - out_default| / max|out_default| among accepted shapes */
} dht_tune_result;

/* Autotuner: for each epilogue class, time every hopping-kernel shape valid
 * for (prec, nrhs) on this lattice (reps applications each, HIP events on the
 * context stream, after warm-up; the fused class with an x-pay operand and the
 * fused (out, x), (out, out) sums), check each output against the default
 * shape's (relative max-norm difference <= 1e-12 FP64, 1e-5 FP32, 1.6e-2 BF16,
 * i.e. a few units in the last place of the storage format), then time the
 * fastest shape of each t-marching form again with z blocks of 2, 4 and 8
 * (those dividing Lz), and install the fastest accepted shape per class on
 * the context.  Needs the gauge field;
 * uses the context workspace (four half fields of nrhs RHS). */
int dht_autotune_hop(dht_ctx* ctx, int prec, int nrhs, int reps, dht_tune_result* out);
/* The autotuner with a cache file: if `cache_path` (may be NULL) holds shapes
 * for this lattice, prec and nrhs they are installed without timing
 * (out->candidates = 0); otherwise dht_autotune_hop runs and its shapes are
 * appended to the file (one text line per epilogue class; lines written in
 * another layout are skipped). */
int dht_autotune(dht_ctx* ctx, int prec, int nrhs, int reps, const char* cache_path, dht_tune_result* out);

/* ---- variance analysis (Sections 6.1-6.3; host arrays, no device) -------- */

/* Run-to-run statistics of the hierarchical-probing estimate.  q holds, for R
 * independent runs of Algorithm 1 (different base vectors z0), the quadratic
 * forms of their first S probes (complex128 [R][S]; deflated or not).  For
 * each s of s_list the run estimates t_r(s) = (1/s) sum_{j<s} q[r][j] give:
 * mean (over runs) and its standard error sqrt(var / R); var = V_hp(s), the
 * unbiased variance over runs of t_r(s), with its Jackknife error (leave one
 * run out); and, when v_stoc > 0 (the variance per probe of plain Z4 noise),
 * the speedup over Monte Carlo R_s = v_stoc / (V_hp(s) s) with its Jackknife
 * error.  Needs R >= 3. */
typedef struct dht_hp_var {
    int s;
    double mean_re, mean_im, mean_err;
    double var, var_err;
    double rs, rs_err;
} dht_hp_var;
int dht_hp_variance(const double* q_host, int R, int S, const int* s_list, int ns, double v_stoc, dht_hp_var* out);

/* Playback with fewer deflation vectors (Section 6.3: the stored inner
 * products replayed with a smaller subspace).  From the Galerkin matrices
 * H = W^H Q W and G5 = W^H g5 W of a basis of k vectors (complex128 k x k
 * row-major, as dht_deflation_get_galerkin returns them; diagonal = 1 uses
 * their diagonals only, as dht_deflation_finalize_diag does), the projection
 * coefficients of n probes (complex128 [2][k][n]: c1 = W^H z, c2 = W^H g5 z,
 * as dht_trace_batch returns them) and their quadratic forms q (complex128
 * [n]), computes for each kk of k_list (0..k) the deflated quadratures
 * q - c1'^H M' c2' with M' = (H[:kk, :kk])^-1 over the leading kk vectors
 * (qd_out, complex128 [nk][n]) and T_D' = Tr(M' G5[:kk, :kk]) (TD_out,
 * complex128 [nk]): the estimator of Algorithm 1 with a basis of kk vectors. */
int dht_playback(const double* H, const double* G5, int k, int diagonal, const double* coef, const double* q, int n,
                 const int* k_list, int nk, double* qd_out, double* TD_out);
/* The Galerkin matrices of the finalized basis (H, G5: 2 k^2 doubles each). */
int dht_deflation_get_galerkin(dht_ctx* ctx, double* H, double* G5, int* diagonal);

/* Theorem 2 (Section 2.1): the expected Z4 variance of the deflated estimator
 * when the singular vectors are random unitary, from the mean mu_k and the
 * variance V_k of the N - k values left after deflating the k of largest
 * modulus: (N - k)(1 - 1/N)(V_k + mu_k^2) for a non-Hermitian matrix, and
 * (N - k)(V_k N / (N + 1) + mu_k^2 k / (N + 1)) for a Hermitian one; var_0
 * is Remark 4's undeflated value and `reduces` the Corollary's verdict
 * (always 1 for non-Hermitian matrices).  Inputs (host): sumsq_all = the sum
 * of the squares of all N values (||A||_F^2; for A = D^-1 the mean of
 * ||D^-1 z||^2 over probes, or N times the mean squared row norm that
 * dht_distance_profile samples); sum_all = the sum of all N values (needed
 * for Hermitian matrices; for non-Hermitian ones only mu_k and V_k use it,
 * NaN allowed); top = the k deflated values (for D^-1 = Q^-1 g5 these are
 * 1 / |lambda| of the deflated eigenvalues of Q = g5 D).  For Hermitian
 * matrices the values are the eigenvalues with their signs (equal to the
 * singular values when positive definite).  Errors: DHT_ERR_INVALID_ARG for
 * N < 1, k outside 0..N, non-finite input, or deflated squares above
 * sumsq_all. */
typedef struct dht_thm2 {
    double var_k;     /* E(Var(t(A_R)))                                      */
    double var_0;     /* E(Var(t(A))) (k = 0)                                */
    double ratio;     /* var_k / var_0                                       */
    double mu_k, V_k; /* mean and variance of the N - k remaining values     */
    int reduces;      /* 1 if var_k < var_0                                  */
} dht_thm2;
int dht_theorem2(int64_t N, int k, int hermitian, double sum_all, double sumsq_all, const double* top, dht_thm2* out);

/* The distance profile W_d of Section 6.2, for nrows sampled rows (matrix
 * indices n = 12 site + 3 spin + colour, host array) of B = D^-1, or of the
 * deflated remainder D^-1 - P (deflate != 0, current finalized basis), each
 * optionally masked to the entries that the first hp_vectors
 * hierarchical-probing vectors leave in the variance (hp_vectors = 2^m: the
 * entries whose sites' colours agree on the low m bits; 0 = no mask).
 * W_host[r][d] (host, nrows x (dmax + 1), dmax = sum_mu L_mu / 2) receives the
 * sum of |B_ij|^2 over the entries j whose site lies at torus Manhattan
 * distance d from the site of row i = rows[r], divided by m_d, the number of
 * such entries (12 per site); m_host (host, dmax + 1, may be NULL) receives
 * m_d.  The paper's W_d is the mean of W_host over the rows.  Each row is
 * obtained as a column (|B_ij| = |B_ji| by g5-hermiticity of D and P): one
 * point-source solve with prm per row, batched by 16, minus W M (W^H g5 e_i)
 * when deflated.  Returns DHT_ERR_NOT_CONVERGED (with every row filled) if
 * a solve missed the tolerance.  Errors: DHT_ERR_INVALID_ARG for a row
 * outside 0..N-1 or hp_vectors not 0 or a power of two <= 65536;
 * DHT_ERR_STATE without gauge field, or with deflate and no finalized basis. */
int dht_distance_profile(dht_ctx* ctx, const int64_t* rows, int nrows, int deflate, int hp_vectors,
                         const dht_solver_params* prm, double* W_host, int64_t* m_host);

/* Batch-size tuner (the right-hand sides per dht_trace_batch call): for each
 * candidate batch whose planned workspace (dht_workspace_size with prm) fits
 * mem_budget bytes (0: 90% of the device memory free now plus the workspace
 * the library holds), the hop shapes of the solve's precisions are tuned if
 * they are not set, and reps Algorithm-1 batches of the probes of spec
 * (j = 0 .. reps*B - 1, after one untimed batch) are timed by the host clock
 * (the host's convergence polls are part of a batch's cost);
 * best_nrhs is the candidate of most right-hand sides per second.  The
 * running estimates and the projection window are left as they were.  The
 * caller then passes best_nrhs to dht_trace_batch. */
#define DHT_TUNE_MAX_BATCHES 8
enum { DHT_BATCH_INVALID = 0, DHT_BATCH_TIMED = 1, DHT_BATCH_OVER_BUDGET = 2, DHT_BATCH_FAILED = 3 };
typedef struct dht_batch_tune {
    int best_nrhs;
    int candidates;
    int nrhs[DHT_TUNE_MAX_BATCHES];
    int status[DHT_TUNE_MAX_BATCHES];         /* DHT_BATCH_* */
    double rhs_per_s[DHT_TUNE_MAX_BATCHES];
    size_t workspace[DHT_TUNE_MAX_BATCHES];   /* planned workspace bytes */
} dht_batch_tune;
int dht_autotune_batch(dht_ctx* ctx, const dht_probe_spec* spec, const dht_solver_params* prm, const int* cand,
                       int ncand, size_t mem_budget, int reps, dht_batch_tune* out);

/* Split of the MFMA projection (BF16 basis, nrhs <= 64 probes): the basis
 * entries are divided over about 256 .. 4096 workgroups of split-K partial
 * sums; each split is timed (reps passes) and checked against the default
 * split (max difference <= 1e-12 of the largest coefficient: only the FP64
 * order of adding the FP32 chunk sums differs), and the fastest is installed
 * on the context.  best_ms (may be NULL) receives its time per pass. */
int dht_autotune_projection(dht_ctx* ctx, int nrhs, int reps, int* best_wgs, double* best_ms);

#ifdef __cplusplus
}
#endif
#endif /* DHTRACE_H */
