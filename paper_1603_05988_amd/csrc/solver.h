// Batched Krylov solvers: shared declarations.
#pragma once

#include "internal.h"

namespace dht {

enum { RS_RUNNING = 0, RS_CONVERGED = 1, RS_BREAKDOWN = 2, RS_NAN = 3 };
enum { FIN_INIT = 0, FIN_ALPHA = 1, FIN_OMEGA = 2, FIN_RHO = 3 };

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
    int64_t nsite;
    int B, Bp;
    Cx<double>* partial;
    int nblocks;
};

int launch_dot_partials(dht_ctx* c, int prec, int np, const void* const* a, const void* const* b, int64_t nsite,
                        int nrhs, Cx<double>* partial, int* nblocks_out);
int finalize(dht_ctx* c, const Cx<double>* partial, int nblocks, int np, int nrhs, RhsState* st, int op,
             double bd_eps);
int dots(dht_ctx* c, int prec, int np, const void* const* a, const void* const* b, int64_t nsite, int nrhs,
         Cx<double>* out_dev);
int p_update(dht_ctx* c, int prec, void* p, const void* r, const void* v, const RhsState* st, size_t n, int B);
int s_update(dht_ctx* c, int prec, void* s, const void* r, const void* v, const RhsState* st, size_t n, int B);
int xr_update(dht_ctx* c, int prec, void* x, void* r, const void* p, const void* s, const void* t,
              const RhsState* st, size_t n, int B);
int scale_down(dht_ctx* c, const void* in, void* out, int pout, const double* scale, size_t n, int B);
int accum_up(dht_ctx* c, void* x, const void* e, int pin, const double* scale, size_t n, int B);
int sub(dht_ctx* c, const void* a, const void* b, void* y, size_t n);
int zero(dht_ctx* c, void* p, size_t bytes);

// Schur operator on even sites: out = (4+m) in - Hop_eo Hop_oe in / (4 (4+m)).
int apply_schur(dht_ctx* c, int prec, const void* in_e, void* out_e, void* tmp_o, int nrhs);

// Batched BiCGStab on the Schur system in storage precision `prec`:
//   solves  Dhat x = b  for nrhs columns (half fields), x overwritten (starts at 0),
//   stops each RHS when ||r||^2 <= target2[r] (host array).
// Returns per-RHS iteration counts and status (host arrays).
struct BicgResult {
    std::vector<int> iters, status;
    std::vector<double> rnorm2;
};
int bicgstab(dht_ctx* c, int prec, const void* b, void* x, int nrhs, const std::vector<double>& target2, int maxiter,
             BicgResult* res);

// Top-level solve of D X = Z on internal full FP64 fields (Z, X: [2][12][Vh][B]).
int solve_fields(dht_ctx* c, const dht_solver_params* prm, const void* Z, void* X, int nrhs, dht_solve_stats* stats);

// deflation.hip
int project_field(dht_ctx* c, const void* Z, int zprec, int nrhs, Cx<double>* c1, Cx<double>* c2);
int deflation_begin(dht_ctx* c, int k, int prec);
int deflation_set(dht_ctx* c, int first, int count, const double* W_dev);
int deflation_finalize(dht_ctx* c, bool diagonal);
void deflation_corrections(const dht_ctx* c, const Cx<double>* c1, const Cx<double>* c2, int B, double* dre,
                           double* dim);
int gather_columns(dht_ctx* c, int j0, int n, void* out);
int project_codes(dht_ctx* c, const uint8_t* zc, int nrhs, Cx<double>* c1, Cx<double>* c2);

}  // namespace dht
