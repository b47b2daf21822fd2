// Batched Krylov solvers: shared declarations.
//
// Every internal batch size `nrhs` below is a power of two (<= 256); the
// interface pads callers' batches with zero right-hand sides.
#pragma once

#include "internal.h"

namespace dht {

enum { RS_RUNNING = 0, RS_CONVERGED = 1, RS_BREAKDOWN = 2, RS_NAN = 3 };
enum { FIN_INIT = 0, FIN_ALPHA = 1, FIN_OMEGA = 2, FIN_RHO = 3, FIN_SUM = 4 };

// Per-RHS BiCGStab state, resident on the device.
struct RhsState {
    Cx<double> rho, alpha, omega, beta;
    double rnorm2;    // current recurrence residual norm^2
    double rhat2;     // ||rhat||^2 (shadow residual)
    double target2;   // stop when rnorm2 <= target2
    int active;       // 1 while iterating
    int status;       // RS_*
    int iters;
    int pad;
};

struct DotArgs {
    const void* a[3];
    const void* b[3];
    size_t nvec;        // 16-byte vectors per operand
    int B;
    Cx<double>* partial;
    int nblocks;
};

// workspace bytes for reduction partials (generic dots and fused hop epilogues)
size_t partial_bytes(const dht_ctx* c, int nrhs);
int launch_dot_partials(dht_ctx* c, int prec, int np, const void* const* a, const void* const* b, size_t nvec,
                        int nrhs, Cx<double>* partial, int* nblocks_out);
// sum partials per (pair, RHS) into sums[pair][r] (if non-null) and apply the
// BiCGStab scalar update `op` to st (unless op == FIN_SUM)
int finalize(dht_ctx* c, const Cx<double>* partial, int nblocks, int np, int nrhs, RhsState* st, int op,
             double bd_eps, Cx<double>* sums = nullptr);
// out_dev[pair][r] = sum conj(a_pair) b_pair over nvec vectors
int dots(dht_ctx* c, int prec, int np, const void* const* a, const void* const* b, size_t nvec, int nrhs,
         Cx<double>* out_dev);
// p = r + beta (p_in - omega v) (p_in = null: in place)
int p_update(dht_ctx* c, int prec, void* p, const void* r, const void* v, const RhsState* st, size_t nvec, int B,
             const void* p_in = nullptr);
int s_update(dht_ctx* c, int prec, void* s, const void* r, const void* v, const RhsState* st, size_t nvec, int B);
int xr_update_dots(dht_ctx* c, int prec, void* x, void* r, const void* p, const void* s, const void* t, const void* rh,
                   const RhsState* st, size_t nvec, int B, Cx<double>* partial, int* nblocks,
                   bool x_zero = false,
                   bool x32 = false);
// half fields: out_low = scale[r] * in_fp64 ; x_fp64 += scale[r] * e_low
int scale_down(dht_ctx* c, const void* in, void* out, int pout, const double* scale, int nrhs);
int accum_up(dht_ctx* c, void* x, const void* e, int pin, const double* scale, int nrhs, bool assign = false);
// r = s - omega t, (rhat, r), (r, r); (alpha, omega) of the iteration to hist [2][B]
int r_update_dots(dht_ctx* c, int prec, void* r, const void* s, const void* t, const void* rh, const RhsState* st,
                  size_t nvec, int B, Cx<double>* partial, int* nblocks, Cx<double>* hist);
// X (FP64) = [X +] scale * sum over n stored iterations of (alpha_j p_j + omega_j s_j)
// (P0 non-null: p_0 is read from P0 instead of slot 0)
// (E32 non-null: the sum is also accumulated into that FP32 field, assigned when e_assign)
int accum_hist(dht_ctx* c, int prec, void* X, const void* P, const void* Sv, const Cx<double>* hist, int n, int nrhs,
               const double* scale, bool assign, const void* P0 = nullptr, void* E32 = nullptr, bool e_assign = false);
// r = r_in - scale * w (r, r_in FP64, may alias; w FP32), with the (r, r) partials of the new r;
// rh16 non-null: also writes s16 * r (device scales per RHS) as a BF16 half field
int residual_step(dht_ctx* c, void* r, const void* r_in, const void* w32, const double* scale, int nrhs,
                  Cx<double>* partial, int* nblocks, void* rh16 = nullptr, const double* s16 = nullptr);
int sub(dht_ctx* c, const void* a, const void* b, void* y, size_t ncomplex);
int zero(dht_ctx* c, void* p, size_t bytes);

inline size_t half_vecs(const dht_ctx* c, int nrhs, int prec) { return half_elems(c, nrhs) / vec_width(prec); }
inline size_t full_vecs(const dht_ctx* c, int nrhs, int prec) { return full_elems(c, nrhs) / vec_width(prec); }

// Schur operator on even sites: out = (4+m) in - Hop_eo Hop_oe in / (4 (4+m)),
// optionally with a fused reduction in the second hop.
int apply_schur(dht_ctx* c, int prec, const void* in_e, void* out_e, void* tmp_o, int nrhs, HopDot* dot = nullptr);

// Batched BiCGStab on the Schur system in storage precision `prec`:
//   solves  Dhat x = b  for nrhs columns (half fields), x overwritten (starts at 0),
//   stops each RHS when ||r||^2 <= target2[r] (host array).
// Returns per-RHS iteration counts and status (host arrays).
struct BicgResult {
    std::vector<int> iters, status;
    std::vector<double> rnorm2;
};
// r = rhat = p = round(scale * in) (in: FP64 half field), partials of (r, r)
int solve_init(dht_ctx* c, const void* in, int pout, const double* scale, void* r, void* rh, void* p, int nrhs,
               Cx<double>* partial, int* nblocks);
// BiCGStab on the Schur system from x = 0 for the right-hand side scale * src
// (src: FP64 half field, scale: device, per RHS), in storage precision prec
// Solution by history: instead of updating x every iteration, keep the
// iterations' p and s (rings of up to 16) with their (alpha, omega) and add
// scale_r * x to the FP64 field X when a ring is full and at the end (an RHS
// whose solve ended in NaN contributes nothing from then on).
struct XAccum {
    int ring = 0;                  // iterations kept before a rebuild (0: automatic)
    void* X = nullptr;             // FP64 half field
    std::vector<double> scale;     // per RHS (0: leave the RHS alone)
    bool assign = false;           // the first contribution assigns X
    void* E32 = nullptr;           // optional FP32 half field that receives x itself
    // with E32: the outer targets (units of the caller's residual); E32 is left
    // unwritten when every RHS's predicted residual scale^2 ||r_inner||^2 meets
    // them (the caller then checks the full residual and never reads E32)
    const std::vector<double>* predict_t2 = nullptr;
};
// x32: the solution x is kept in FP32 storage (BF16 vectors only); xa: see XAccum (x unused);
// r0n2 (host, nrhs; with xa only): the right-hand side is already in rhat (the BF16
// copy written by residual_step), with these squared norms; src and scale are unused
int bicgstab(dht_ctx* c, int prec, const void* src, const double* scale, void* x, int nrhs,
             const std::vector<double>& target2, int maxiter, BicgResult* res, bool x32 = false,
             XAccum* xa = nullptr, const double* r0n2 = nullptr);

// Top-level solve of D X = Z on internal full FP64 fields (Z, X: [2][12][Vh][B]);
// stats has nrhs entries (the padded batch).
// zn2_known (host, nrhs, may be null): ||Z||^2 per RHS when the caller knows it exactly;
// zx_out (host, nrhs, may be null; BiCGStab methods only): z^H x per RHS, summed in
// the epilogues of the final full-lattice residual.
// zprec DHT_BF16: Z is in the BF16 layout ([2][3][Vh][B][4]) and holds values exact
// in BF16 (probes); needs zn2_known and a BiCGStab method; results equal those of the
// same Z in FP64
int solve_fields(dht_ctx* c, const dht_solver_params* prm, const void* Z, void* X, int nrhs, dht_solve_stats* stats,
                 const double* zn2_known = nullptr, Cx<double>* zx_out = nullptr, int zprec = DHT_FP64);

// workspace plans (bytes per slot, maxima over the call's code paths, with
// the precision fallbacks) of solve_fields, the FGMRES solver, the network's
// inference and the two projections, for a padded batch nrhs
void ws_plan_solve(const dht_ctx* c, const dht_solver_params* prm, int nrhs, size_t* plan);
void ws_plan_fgmres(const dht_ctx* c, const dht_solver_params* prm, int nrhs, bool use_nn, size_t* plan);
size_t nn_infer_bytes(const dht_ctx* c, int nrhs);
void ws_plan_project_codes(const dht_ctx* c, int nrhs, size_t* plan);
void ws_plan_project_field(const dht_ctx* c, int nrhs, size_t* plan);
void ws_plan_dots(const dht_ctx* c, int nrhs, size_t* plan);

// fgmres.hip: FP64 defect correction around FGMRES(m) cycles (FP32) on the
// full lattice with the network (use_nn) or the identity as right
// preconditioner.  A PairSink, if given, records (r_k / ||r_k||,
// (x* - x_k) / ||r_k||) at every restart k for the first n real RHS.
struct PairSink {
    const void* xstar = nullptr;   // full FP64 field of reference solutions
    double* R = nullptr;           // canonical complex128 outputs [cap][V][12]
    double* E = nullptr;
    int cap = 0, count = 0, nreal = 0;
    int take(dht_ctx* c, const void* r, const void* x, const std::vector<bool>& act, const std::vector<double>& rn2);
};
int solve_fgmres(dht_ctx* c, const dht_solver_params* prm, const void* Z, void* X, int B, dht_solve_stats* stats,
                 bool use_nn, PairSink* sink);

// nn.hip
static constexpr int NN_MAX_BATCH = 64;
int nn_alloc(dht_ctx* c);
int nn_set_weights(dht_ctx* c, const float* host);
int nn_get_weights(dht_ctx* c, float* host, bool grads);
int64_t nn_num_weights();
int nn_forward_canon(dht_ctx* c, const double* R, double* E, int n);
int nn_grad_canon(dht_ctx* c, const double* R, const double* E, int n, double* loss);
int nn_train_canon(dht_ctx* c, const double* R, const double* E, int npairs, int epochs, int batch, float lr,
                   double* final_loss);
int nn_apply_field(dht_ctx* c, const void* in, void* out, int nrhs);   // FP32 full fields

// deflation.hip
int project_field(dht_ctx* c, const void* Z, int zprec, int nrhs, Cx<double>* c1, Cx<double>* c2);
int deflation_begin(dht_ctx* c, int k, int prec);
int deflation_set(dht_ctx* c, int first, int count, const double* W_dev);
int deflation_finalize(dht_ctx* c, bool diagonal);
// eigenvectors of Q of smallest |lambda| into the begun basis (eig.hip)
int eigensolve(dht_ctx* c, const dht_eig_params* prm, double* lambda_host, double* resid_host, dht_eig_stats* st);
// LOBPCG with locking for the same space (eig.hip)
int lobpcg(dht_ctx* c, const dht_lobpcg_params* prm, double* sigma_host, double* resid_host, dht_lobpcg_stats* st);
void deflation_corrections(const dht_ctx* c, const Cx<double>* c1, const Cx<double>* c2, int B, int nuse,
                           double* dre, double* dim);
int gather_columns(dht_ctx* c, int j0, int n, int bp, void* out);
int project_codes(dht_ctx* c, const uint8_t* zc, int nrhs, Cx<double>* c1, Cx<double>* c2);
// spin-pair projections P[4 s + t][k][nrhs] = W_s^H z_t (traces with a spin
// matrix): MFMA form over probe codes (BF16 basis, nrhs <= 16), generic form
// over FP64 probe fields (any basis precision)
int project_codes_sp(dht_ctx* c, const uint8_t* zc, int nrhs, Cx<double>* P);
int project_field_sp(dht_ctx* c, const void* Z, int nrhs, Cx<double>* P);
// X -= W v for an FP64 full field X of bp columns (v: device [k][bp])
int basis_subtract(dht_ctx* c, const Cx<double>* v, int bp, void* X);

}  // namespace dht
