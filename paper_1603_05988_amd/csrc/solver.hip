// Batched solves of D X = Z (Algorithm 1, "Solve Ay = z"; the paper leaves
// the solver open).
//
// Structure:
//  * even/odd reduction: with a = 4 + m and Hop_pq the hop from parity q to p,
//      Dhat x_e = b_e + Hop_eo b_o / (2a),  Dhat = a - Hop_eo Hop_oe / (4a),
//      x_o = (b_o + Hop_oe x_e / 2) / a,
//    and the Schur residual equals the full-lattice residual (odd part zero);
//  * batched BiCGStab (van der Vorst 1992) with per-RHS scalars on the device;
//    its five reductions per iteration ride on the epilogues of the second
//    hop of each operator application and of the x/r update, so an iteration
//    is 4 hop launches + 3 vector passes + 3 one-workgroup-per-RHS finalises;
//  * FP64 defect correction: r = b - Dhat x in FP64, inner solve of
//    Dhat e = r / ||r|| in FP32 or BF16 storage, x += ||r|| e in FP64, until
//    the FP64 residual meets the target.  The plain FP64 method is the same
//    loop with an FP64 inner solve.
//  * fallback: an inner breakdown or NaN, or a cycle that fails to reduce the
//    residual, escalates the inner precision BF16 -> FP32 -> FP64.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "solver.h"

namespace dht {

// relative ||r||^2 / ||z||^2 below which the Schur residual is updated in place
static constexpr double INC_REL2 = 1e-4;

int apply_schur(dht_ctx* c, int prec, const void* in_e, void* out_e, void* tmp_o, int nrhs, HopDot* dot) {
    const double a = 4.0 + c->mass;
    DHT_TRY(hop(c, prec, 1, in_e, tmp_o, nullptr, 0.0, 1.0, nrhs, false, false));
    DHT_TRY(hop(c, prec, 0, tmp_o, out_e, in_e, a, -1.0 / (4.0 * a), nrhs, false, false, dot));
    return DHT_OK;
}

static int slot_base(int prec) { return prec == DHT_FP64 ? WS_K64 : WS_KLO; }

// the rings of stored iterations of a BF16 inner solve (see bicgstab)
static int ring_slots(int history, size_t bytes) {
    const size_t budget = (size_t)12 << 30;   // bytes for both rings
    return history > 0 ? history : (int)std::min<size_t>(16, std::max<size_t>(2, budget / (2 * bytes)));
}


int bicgstab(dht_ctx* c, int prec, const void* src, const double* scale, void* x, int nrhs,
             const std::vector<double>& target2, int maxiter, BicgResult* res, bool x32, XAccum* xa,
             const double* r0n2) {
    if (r0n2 && !xa) return set_error(DHT_ERR_INVALID_ARG, "a prepared right-hand side needs the stored iterations");
    const size_t nvec = half_vecs(c, nrhs, prec);
    const size_t bytes = nvec * 16;
    const int base = slot_base(prec);
    void *r, *rh, *p, *v, *s, *t, *tmp, *stv, *part, *hostv;
    DHT_TRY(ws_get(c, base + 0, bytes, &r));
    DHT_TRY(ws_get(c, base + 1, bytes, &rh));
    DHT_TRY(ws_get(c, base + 3, bytes, &v));
    DHT_TRY(ws_get(c, base + 5, bytes, &t));
    DHT_TRY(ws_get(c, base + 6, bytes, &tmp));
    // p and s: one vector each, or with XAccum rings of K slots
    int K = 1;
    char *ringP, *ringS;
    Cx<double>* hist = nullptr;
    double* hscale = nullptr;
    if (xa) {
        K = ring_slots(xa->ring, bytes);
        void *pp, *ss, *hh, *sc;
        DHT_TRY(ws_get(c, WS_RING_P, (size_t)K * bytes, &pp));
        DHT_TRY(ws_get(c, WS_RING_S, (size_t)K * bytes, &ss));
        DHT_TRY(ws_get(c, WS_HIST, sizeof(Cx<double>) * 2 * (size_t)K * nrhs, &hh));
        DHT_TRY(ws_get(c, WS_HIST_SCALE, sizeof(double) * nrhs, &sc));
        ringP = (char*)pp;
        ringS = (char*)ss;
        hist = (Cx<double>*)hh;
        hscale = (double*)sc;
    } else {
        DHT_TRY(ws_get(c, base + 2, bytes, &p));
        DHT_TRY(ws_get(c, base + 4, bytes, &s));
        ringP = (char*)p;
        ringS = (char*)s;
    }
    DHT_TRY(ws_get(c, WS_SCAL, sizeof(RhsState) * nrhs, &stv));
    DHT_TRY(ws_get(c, WS_PARTIAL, partial_bytes(c, nrhs), &part));
    DHT_TRY(ws_get(c, WS_HOSTPIN, sizeof(RhsState) * nrhs, &hostv));   // pinned host buffer
    RhsState* st = (RhsState*)stv;
    RhsState* hs = (RhsState*)hostv;
    Cx<double>* partial = (Cx<double>*)part;

    for (int i = 0; i < nrhs; i++) {
        memset(&hs[i], 0, sizeof(RhsState));
        hs[i].target2 = target2[i];
    }
    DHT_HIP(hipMemcpyAsync(st, hs, sizeof(RhsState) * nrhs, hipMemcpyHostToDevice, c->stream));
    // x = 0 is never materialised: the first x update writes x; r, rhat and
    // p = r come out of one pass over the FP64 source with the (r, r) sums,
    // unless the caller's residual pass has already written rhat (r0n2)
    const double bd_eps = prec == DHT_FP64 ? 1e-14 : 1e-6;
    int nb;
    // with XAccum, r_0 and the first direction p_0 = r_0 are rhat itself (not
    // copied): iteration 0 reads rhat for both, and r is first written by its
    // residual update
    std::vector<Cx<double>> h0;   // alive until the copy below has run (the polls synchronise)
    if (r0n2) {   // rhat was written by the residual update, with norms known on the host
        h0.resize(nrhs);
        for (int i = 0; i < nrhs; i++) h0[i] = cmake(r0n2[i], 0.0);
        DHT_HIP(hipMemcpyAsync(partial, h0.data(), sizeof(Cx<double>) * nrhs, hipMemcpyHostToDevice, c->stream));
        nb = 1;
    } else {
        DHT_TRY(solve_init(c, src, prec, scale, xa ? nullptr : r, rh, xa ? nullptr : ringP, nrhs, partial, &nb));
    }
    DHT_TRY(finalize(c, partial, nb, 1, nrhs, st, FIN_INIT, bd_eps));
    // add the stored iterations [0, n) to X (after a synchronisation, so hs
    // holds the current states)
    bool first_flush = true;
    std::vector<double> fs(nrhs);
    auto flush = [&](int n, bool last) -> int {
        for (int i = 0; i < nrhs; i++) fs[i] = hs[i].status == RS_NAN ? 0.0 : xa->scale[i];
        void* e32 = xa->E32;
        if (e32 && last && first_flush && xa->predict_t2) {   // a single flush: E32 may be skipped whole
            bool pred = true;
            for (int i = 0; i < nrhs; i++)
                if (fs[i] > 0 && !(fs[i] * fs[i] * hs[i].rnorm2 <= (*xa->predict_t2)[i])) pred = false;
            if (pred) e32 = nullptr;
        }
        DHT_HIP(hipMemcpyAsync(hscale, fs.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
        DHT_TRY(accum_hist(c, prec, xa->X, ringP, ringS, hist, n, nrhs, hscale, xa->assign && first_flush,
                           first_flush ? rh : nullptr, e32, first_flush));
        first_flush = false;
        return DHT_OK;
    };
    // the host reads the per-RHS states after every iteration: a batch that
    // converges stops at once (a skipped check costs a whole iteration of 4
    // hops, a check only a short stream synchronisation)
    int stored = 0;
    for (int it = 0; it < maxiter; it++) {
        const int slot = xa ? it % K : 0;
        char* pc = (xa && it == 0) ? (char*)rh : ringP + (size_t)slot * bytes;
        char* sc = ringS + (size_t)slot * bytes;
        if (it > 0) {
            const void* pin = nullptr;   // in place
            if (xa) pin = it == 1 ? rh : (const void*)(ringP + (size_t)((it - 1) % K) * bytes);
            DHT_TRY(p_update(c, prec, pc, r, v, st, nvec, nrhs, pin));
        }
        HopDot d1;
        d1.kind = HOPDOT_A_OUT;   // (rhat, v)
        d1.a = rh;
        d1.partial = partial;
        DHT_TRY(apply_schur(c, prec, pc, v, tmp, nrhs, &d1));
        DHT_TRY(finalize(c, partial, d1.nblocks, 1, nrhs, st, FIN_ALPHA, bd_eps));
        DHT_TRY(s_update(c, prec, sc, (xa && it == 0) ? rh : r, v, st, nvec, nrhs));
        HopDot d2;
        d2.kind = HOPDOT_OUT_X;   // (t, s), (t, t)
        d2.partial = partial;
        DHT_TRY(apply_schur(c, prec, sc, t, tmp, nrhs, &d2));
        DHT_TRY(finalize(c, partial, d2.nblocks, 2, nrhs, st, FIN_OMEGA, bd_eps));
        if (xa) {
            DHT_TRY(r_update_dots(c, prec, r, sc, t, rh, st, nvec, nrhs, partial, &nb, hist + (size_t)slot * 2 * nrhs));
        } else {
            DHT_TRY(xr_update_dots(c, prec, x, r, pc, sc, t, rh, st, nvec, nrhs, partial, &nb, it == 0, x32));
        }
        DHT_TRY(finalize(c, partial, nb, 2, nrhs, st, FIN_RHO, bd_eps));
        stored++;
        DHT_HIP(hipMemcpyAsync(hs, st, sizeof(RhsState) * nrhs, hipMemcpyDeviceToHost, c->stream));
        DHT_HIP(hipStreamSynchronize(c->stream));
        DHT_TRY(prof_harvest(c));
        bool any = false;
        for (int i = 0; i < nrhs; i++) any |= hs[i].active != 0;
        if (!any) break;
        if (xa && stored == K) {   // the rings are full
            DHT_TRY(flush(K, false));
            stored = 0;
        }
    }
    if (xa && (stored > 0 || first_flush)) DHT_TRY(flush(stored, true));
    DHT_HIP(hipMemcpyAsync(hs, st, sizeof(RhsState) * nrhs, hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    res->iters.assign(nrhs, 0);
    res->status.assign(nrhs, 0);
    res->rnorm2.assign(nrhs, 0);
    for (int i = 0; i < nrhs; i++) {
        res->iters[i] = hs[i].iters;
        res->status[i] = hs[i].status;
        res->rnorm2[i] = hs[i].rnorm2;
    }
    return DHT_OK;
}

// residual of a parity, out = z + ca x + cb Hop(in), with its per-RHS squared
// norms reduced from the hop's fused epilogue sums; `slot` selects where the
// sums are kept so that two residuals can be summed on the host.  With zx
// non-null the same epilogue also sums z^H x per RHS (z and x are the
// epilogue's operands) into *zx.  mix marks operands held in BF16 (see hop).
static int residual_hop(dht_ctx* c, int parity, const void* in, void* out, const void* x, double ca, double cb,
                        const void* z, int nrhs, int slot, std::vector<double>& n2,
                        std::vector<Cx<double>>* zx = nullptr, int mix = 0, void* out16 = nullptr,
                        const double* s16 = nullptr) {
    void *part, *sums;
    DHT_TRY(ws_get(c, WS_PARTIAL, partial_bytes(c, nrhs), &part));
    DHT_TRY(ws_get(c, WS_NORMS, sizeof(Cx<double>) * 6 * nrhs, &sums));
    const int np = zx ? 2 : 1;
    HopDot d;
    d.kind = zx ? HOPDOT_NORM_ZX : HOPDOT_NORM;
    d.partial = (Cx<double>*)part;
    DHT_TRY(hop(c, DHT_FP64, parity, in, out, x, ca, cb, nrhs, false, false, &d, z, z ? 1.0 : 0.0,
                mix | (out16 ? HOP_OUT16 : 0), out16, s16));
    Cx<double>* s = (Cx<double>*)sums + (size_t)slot * 2 * nrhs;
    DHT_TRY(finalize(c, d.partial, d.nblocks, np, nrhs, nullptr, FIN_SUM, 0.0, s));
    std::vector<Cx<double>> h((size_t)np * nrhs);
    DHT_HIP(hipMemcpyAsync(h.data(), s, sizeof(Cx<double>) * h.size(), hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    n2.resize(nrhs);
    for (int i = 0; i < nrhs; i++) n2[i] = h[i].re;
    if (zx) zx->assign(h.begin() + nrhs, h.end());
    return DHT_OK;
}

// odd sites from the even ones, x_o = (z_o + Hop_oe x_e / 2) / a; with zx
// non-null the epilogue also sums z_o^H x_o per RHS into *zx; z16: z_o is
// held in BF16
static int odd_from_even(dht_ctx* c, const void* X_e, void* X_o, const void* Z_o, int nrhs,
                         std::vector<Cx<double>>* zx, bool z16) {
    const double a = 4.0 + c->mass;
    const int mix = z16 ? HOP_X16 : 0;
    if (!zx) return hop(c, DHT_FP64, 1, X_e, X_o, Z_o, 1.0 / a, 1.0 / (2.0 * a), nrhs, false, false, nullptr, nullptr,
                        0.0, mix);
    void *part, *sums;
    DHT_TRY(ws_get(c, WS_PARTIAL, partial_bytes(c, nrhs), &part));
    DHT_TRY(ws_get(c, WS_NORMS, sizeof(Cx<double>) * 6 * nrhs, &sums));
    HopDot d;
    d.kind = HOPDOT_OUT_X;   // (x_o, z_o) and (x_o, x_o)
    d.partial = (Cx<double>*)part;
    DHT_TRY(hop(c, DHT_FP64, 1, X_e, X_o, Z_o, 1.0 / a, 1.0 / (2.0 * a), nrhs, false, false, &d, nullptr, 0.0, mix));
    Cx<double>* s = (Cx<double>*)sums + (size_t)2 * 2 * nrhs;
    DHT_TRY(finalize(c, d.partial, d.nblocks, 2, nrhs, nullptr, FIN_SUM, 0.0, s));
    std::vector<Cx<double>> h(nrhs);
    DHT_HIP(hipMemcpyAsync(h.data(), s, sizeof(Cx<double>) * nrhs, hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    zx->resize(nrhs);
    for (int i = 0; i < nrhs; i++) (*zx)[i] = cmake(h[i].re, -h[i].im);   // z^H x = conj(x^H z)
    return DHT_OK;
}

// per-RHS FP64 norms^2 of an FP64 field of nvec vectors (host result)
static int norms2(dht_ctx* c, const void* f, size_t nvec, int nrhs, std::vector<double>& out) {
    void* d;
    DHT_TRY(ws_get(c, WS_SCAL2, sizeof(Cx<double>) * 3 * nrhs, &d));
    const void* aa[1] = {f};
    DHT_TRY(dots(c, DHT_FP64, 1, aa, aa, nvec, nrhs, (Cx<double>*)d));
    std::vector<Cx<double>> h(nrhs);
    DHT_HIP(hipMemcpyAsync(h.data(), d, sizeof(Cx<double>) * nrhs, hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    out.resize(nrhs);
    for (int i = 0; i < nrhs; i++) out[i] = h[i].re;
    return DHT_OK;
}

// 1 / (the residual norm a finished inner solve predicts) per RHS taking part
// (sup > 0; 0 for the others); false if a prediction is not positive and finite
static bool predict_scales(const std::vector<double>& sup, const BicgResult& br, std::vector<double>& sdn) {
    for (size_t i = 0; i < sup.size(); i++) {
        sdn[i] = 0.0;
        if (!(sup[i] > 0)) continue;
        const double pr = sup[i] * sup[i] * br.rnorm2[i];
        if (!(pr > 0 && isfinite(pr))) return false;
        sdn[i] = 1.0 / sqrt(pr);
    }
    return true;
}

// workspace of one inner BiCGStab in storage precision prec (see bicgstab)
static void ws_plan_bicgstab(const dht_ctx* c, int prec, int nrhs, bool hist, int history, size_t* plan) {
    const size_t bytes = half_vecs(c, nrhs, prec) * 16;
    const int base = slot_base(prec);
    for (int i : {0, 1, 3, 5, 6}) plan_max(plan, base + i, bytes);
    if (hist) {
        const int K = ring_slots(history, bytes);
        plan_max(plan, WS_RING_P, (size_t)K * bytes);
        plan_max(plan, WS_RING_S, (size_t)K * bytes);
        plan_max(plan, WS_HIST, sizeof(Cx<double>) * 2 * (size_t)K * nrhs);
        plan_max(plan, WS_HIST_SCALE, sizeof(double) * nrhs);
    } else {
        plan_max(plan, base + 2, bytes);
        plan_max(plan, base + 4, bytes);
        plan_max(plan, base + 8, bytes);   // the inner solution of a defect-correction cycle
    }
    plan_max(plan, WS_SCAL, sizeof(RhsState) * nrhs);
    ws_plan_dots(c, nrhs, plan);
}

void ws_plan_solve(const dht_ctx* c, const dht_solver_params* prm, int nrhs, size_t* plan) {
    if (prm->method == DHT_SOLVER_DC_FGMRES_NN || prm->method == DHT_SOLVER_DC_FGMRES) {
        ws_plan_fgmres(c, prm, nrhs, prm->method == DHT_SOLVER_DC_FGMRES_NN, plan);
        dht_solver_params p2 = *prm;   // the BiCGStab fallback
        p2.method = DHT_SOLVER_DC_BICGSTAB;
        p2.inner = DHT_FP32;
        ws_plan_solve(c, &p2, nrhs, plan);
        return;
    }
    const size_t nh = half_elems(c, nrhs), bh = nh * 16;
    for (int s : {WS_B, WS_RE, WS_TMPO}) plan_max(plan, s, bh);
    plan_max(plan, WS_FLAGS, sizeof(double) * nrhs);
    plan_max(plan, WS_SCAL2, sizeof(Cx<double>) * 3 * nrhs);
    plan_max(plan, WS_NORMS, sizeof(Cx<double>) * 6 * nrhs);
    ws_plan_dots(c, nrhs, plan);
    // every inner precision the escalation BF16 -> FP32 -> FP64 can reach
    const int start = prm->method == DHT_SOLVER_DC_BICGSTAB ? prm->inner : DHT_FP64;
    for (int prec = start; prec >= DHT_FP64; prec--) ws_plan_bicgstab(c, prec, nrhs, prec == DHT_BF16, prm->history, plan);
    if (start == DHT_BF16) {
        plan_max(plan, slot_base(DHT_BF16) + 1, half_vecs(c, nrhs, DHT_BF16) * 16);   // prepared right-hand side
        plan_max(plan, WS_S16, sizeof(double) * nrhs);
        for (int s : {WS_E32, WS_W32, WS_T32}) plan_max(plan, s, nh * elem_bytes(DHT_FP32));
    }
}

int solve_fields(dht_ctx* c, const dht_solver_params* prm, const void* Z, void* X, int nrhs, dht_solve_stats* stats,
                 const double* zn2_known, Cx<double>* zx_out, int zprec) {
    const double a = 4.0 + c->mass;
    const size_t nh = half_elems(c, nrhs);   // complex entries (= FP64 vectors) per half field
    const size_t bh = nh * 16;
    // Z in the BF16 layout (values exact in BF16, as probes are): the FP64
    // hops that read it widen it exactly, so every result is the one of an
    // FP64 Z
    const bool z16 = zprec == DHT_BF16;
    if (zprec != DHT_FP64 && !z16) return set_error(DHT_ERR_INVALID_ARG, "bad right-hand side precision");
    if (z16 && (!zn2_known || prm->method == DHT_SOLVER_DC_FGMRES_NN || prm->method == DHT_SOLVER_DC_FGMRES))
        return set_error(DHT_ERR_INVALID_ARG, "a BF16 right-hand side needs its norms and a BiCGStab method");
    const char* Zc = (const char*)Z;
    char* Xc = (char*)X;
    const void* Z_e = Zc;
    const void* Z_o = Zc + (z16 ? nh * elem_bytes(DHT_BF16) : bh);
    void* X_e = Xc;
    void* X_o = Xc + bh;
    void *bhat, *r_e, *scl, *tmp_o;
    DHT_TRY(ws_get(c, WS_B, bh, &bhat));
    DHT_TRY(ws_get(c, WS_RE, bh, &r_e));
    DHT_TRY(ws_get(c, WS_TMPO, bh, &tmp_o));
    DHT_TRY(ws_get(c, WS_FLAGS, sizeof(double) * nrhs, &scl));

    if (prm->tol <= 0.0 || prm->maxiter <= 0) return set_error(DHT_ERR_INVALID_ARG, "tol and maxiter must be positive");
    if (prm->history != 0 && (prm->history < 2 || prm->history > 16))
        return set_error(DHT_ERR_INVALID_ARG, "history must be 0 or 2..16");
    if (prm->method == DHT_SOLVER_DC_FGMRES_NN || prm->method == DHT_SOLVER_DC_FGMRES) {
        const bool use_nn = prm->method == DHT_SOLVER_DC_FGMRES_NN;
        if (zx_out) return set_error(DHT_ERR_INVALID_ARG, "z^H x is fused only into the BiCGStab paths");
        int rc = solve_fgmres(c, prm, Z, X, nrhs, stats, use_nn, nullptr);
        if (rc != DHT_ERR_NOT_CONVERGED) return rc;
        // fallback: plain BiCGStab (FP32 inner, FP64 defect correction) for the whole batch
        dht_solver_params p2 = *prm;
        p2.method = DHT_SOLVER_DC_BICGSTAB;
        p2.inner = DHT_FP32;
        std::vector<dht_solve_stats> st2(nrhs);
        std::vector<dht_solve_stats> st1(stats ? stats : st2.data(), (stats ? stats : st2.data()) + nrhs);
        rc = solve_fields(c, &p2, Z, X, nrhs, st2.data(), zn2_known, nullptr, zprec);
        if (stats)
            for (int i = 0; i < nrhs; i++) {
                stats[i] = st2[i];
                stats[i].iters += st1[i].iters;
                stats[i].outer += st1[i].outer;
                if (st2[i].status != DHT_STATUS_NOT_CONVERGED) stats[i].status = DHT_STATUS_FALLBACK_BICGSTAB;
            }
        return rc;
    }
    if (prm->method != DHT_SOLVER_BICGSTAB_FP64 && prm->method != DHT_SOLVER_DC_BICGSTAB)
        return set_error(DHT_ERR_INVALID_ARG, "unknown solver method");
    int inner = DHT_FP64;
    if (prm->method == DHT_SOLVER_DC_BICGSTAB) inner = prm->inner;
    if (inner < DHT_FP64 || inner > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad inner precision");
    const int max_outer = prm->max_outer > 0 ? prm->max_outer : 50;

    // ||Z||^2, and the right-hand side of the Schur system with its norms
    std::vector<double> zn2, rn2;
    if (zn2_known) zn2.assign(zn2_known, zn2_known + nrhs);
    else DHT_TRY(norms2(c, Z, 2 * nh, nrhs, zn2));
    // A residual pass that precedes a BF16 inner solve also writes that
    // solve's right-hand side in BF16, scaled per RHS by sdp (any positive
    // scale serves; the inner solve is told ||rhat||^2 = ||r||^2 sdp^2 and
    // scales its correction back by 1 / sdp), so that the solve need not read
    // the FP64 residual once more.  prep: the last residual pass did so.
    bool prep = false;
    std::vector<double> sdp(nrhs, 0.0), sdn(nrhs, 0.0);   // sdn: host source of the device scales
    void *rh16 = nullptr, *s16 = nullptr;
    auto want16 = [&]() -> int {
        DHT_TRY(ws_get(c, slot_base(DHT_BF16) + 1, half_vecs(c, nrhs, DHT_BF16) * 16, &rh16));
        DHT_TRY(ws_get(c, WS_S16, sizeof(double) * nrhs, &s16));
        DHT_HIP(hipMemcpyAsync(s16, sdn.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
        return DHT_OK;
    };
    // the first cycle's: bhat itself, scaled by 1 / ||z||
    const bool first16 = inner == DHT_BF16 && !(prm->fault_inject & 1u);
    if (first16) {
        for (int i = 0; i < nrhs; i++) sdn[i] = zn2[i] > 0 && isfinite(zn2[i]) ? 1.0 / sqrt(zn2[i]) : 0.0;
        DHT_TRY(want16());
    }
    DHT_TRY(residual_hop(c, 0, Z_o, bhat, Z_e, 1.0, 1.0 / (2.0 * a), nullptr, nrhs, 0, rn2, nullptr,
                         z16 ? HOP_IN16 | HOP_X16 : 0, first16 ? rh16 : nullptr, (const double*)s16));
    if (first16) {
        prep = true;
        sdp = sdn;
    }
    std::vector<double> target2(nrhs);
    // the Schur loop aims 10% below the tolerance so that the reconstructed
    // full-lattice residual, checked last, is not lost to rounding
    for (int i = 0; i < nrhs; i++) target2[i] = 0.81 * prm->tol * prm->tol * zn2[i];

    std::vector<int> iters(nrhs, 0), escalated(nrhs, DHT_STATUS_CONVERGED);
    std::vector<double> last_rn2(nrhs, INFINITY);
    int outer = 0, total_iters = 0;
    const int start_inner = inner;
    bool last_bad = false;
    bool have_full = false;        // the loop ended on a verified full-lattice residual
    std::vector<double> full2;     // its squared norms
    std::vector<Cx<double>> zx_e, zx_o;   // z^H x per parity from the same epilogues
    bool x_written = false;        // X_e holds the solution so far (else it is 0)
    // rn2 comes from the in-place update (FP32 arithmetic on D e): a loop that
    // stops on it must confirm it with an FP64 residual from X
    bool rn2_inplace = false;
    bool forced_predict = false, forced_drift = false;   // host-forced test conditions, once each
    std::vector<double> fr2;
    void* e;
    for (;;) {
        for (; outer < max_outer; outer++) {
            bool any = false, stalled = false;
            std::vector<double> sdown(nrhs), sup(nrhs), itarget(nrhs);
            for (int i = 0; i < nrhs; i++) {
                bool act = rn2[i] > target2[i] && isfinite(rn2[i]);
                any |= act;
                if (act && rn2[i] > 0.25 * last_rn2[i] && outer > 0 && !last_bad) stalled = true;
                sdown[i] = act ? 1.0 / sqrt(rn2[i]) : 0.0;
                sup[i] = act ? sqrt(rn2[i]) : 0.0;
                last_rn2[i] = act ? rn2[i] : last_rn2[i];
            }
            if (!any) break;
            if (stalled && inner != DHT_FP64) inner = inner == DHT_BF16 ? DHT_FP32 : DHT_FP64;
            if (total_iters >= prm->maxiter) break;
            for (int i = 0; i < nrhs; i++) {
                double itol = prm->inner_tol > 0 ? prm->inner_tol
                                                 : (inner == DHT_BF16 ? 1e-2 : (inner == DHT_FP32 ? 1e-5 : 0.0));
                double need = sup[i] > 0 ? 0.25 * target2[i] / rn2[i] : 1.0;
                itarget[i] = std::max(itol * itol, need);
            }
            // a BF16 solve adds its solution to X_e itself, rebuilt in FP64 from its
            // stored iterations; the others return it in their storage precision
            const bool hist = inner == DHT_BF16;
            // A prepared BF16 right-hand side (see prep): RHS that take no part
            // get a negative target (their rhat need not be zero).
            bool use_prep = prep && hist && !((prm->fault_inject & 1u) && outer == 0);
            for (int i = 0; i < nrhs && use_prep; i++)
                if (sup[i] > 0 && !(sdp[i] > 0 && isfinite(sdp[i]))) use_prep = false;
            std::vector<double> r0n2;
            if (use_prep) {
                r0n2.assign(nrhs, 0.0);
                for (int i = 0; i < nrhs; i++) {
                    if (sup[i] > 0) {
                        sdown[i] = sdp[i];
                        sup[i] = 1.0 / sdp[i];
                        r0n2[i] = rn2[i] * sdp[i] * sdp[i];
                        itarget[i] *= r0n2[i];
                    } else {
                        itarget[i] = -1.0;
                    }
                }
            }
            prep = false;
            const size_t lbytes = nh * elem_bytes(inner);
            const int base = slot_base(inner);
            e = nullptr;
            if (!hist) DHT_TRY(ws_get(c, base + 8, lbytes, &e));     // inner solution
            if ((prm->fault_inject & 1u) && outer == 0 && inner != DHT_FP64) {
                // testing hook: poison the first inner right-hand side to exercise the fallback
                for (int i = 0; i < nrhs; i++) sdown[i] = NAN;
            }
            DHT_HIP(hipMemcpyAsync(scl, sdown.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
            // the inner right-hand side is the scaled Schur residual (normalised
            // by the one-pass start, or prepared as above); in the first cycle
            // that is bhat itself
            // After the first cycle, once every active residual is below
            // 1e-2 ||z||, the Schur residual of a BF16 cycle is updated instead of
            // recomputed: r_new = r_old - sigma Dhat e, with the cycle's correction
            // e kept in FP32 (X moves by exactly sigma e) and Dhat e applied in
            // FP32 arithmetic.  Its rounding is of the order of 1e-7 of the old
            // residual (measured at 32^3x64: final residuals unchanged; from the
            // first cycle on, where the old residual is ||bhat||, the drift stalls
            // the loop).  The final residual is recomputed in FP64 from X, and the
            // loop goes on from it if it misses the tolerance.
            bool inc = hist && x_written;
            for (int i = 0; i < nrhs && inc; i++)
                if (sup[i] > 0 && !(rn2[i] <= INC_REL2 * zn2[i])) inc = false;
            void *E32 = nullptr, *W32 = nullptr, *T32 = nullptr;
            if (inc) {
                DHT_TRY(ws_get(c, WS_E32, nh * elem_bytes(DHT_FP32), &E32));
                DHT_TRY(ws_get(c, WS_W32, nh * elem_bytes(DHT_FP32), &W32));
                DHT_TRY(ws_get(c, WS_T32, nh * elem_bytes(DHT_FP32), &T32));
            }
            BicgResult br;
            XAccum xa;
            if (hist) {
                xa.ring = prm->history;
                xa.X = X_e;
                xa.scale = sup;
                xa.assign = !x_written;
                xa.E32 = E32;
                xa.predict_t2 = &target2;
            }
            DHT_TRY(bicgstab(c, inner, outer == 0 ? bhat : r_e, (const double*)scl, e, nrhs, itarget,
                             prm->maxiter - total_iters, &br, false, hist ? &xa : nullptr,
                             use_prep ? r0n2.data() : nullptr));
            int maxit = 0;
            bool bad = false;
            for (int i = 0; i < nrhs; i++) {
                iters[i] += br.iters[i];
                maxit = std::max(maxit, br.iters[i]);
                if (br.status[i] == RS_NAN || br.status[i] == RS_BREAKDOWN) {
                    if (br.status[i] == RS_NAN) sup[i] = 0.0;   // discard a poisoned correction
                    bad = true;
                }
            }
            total_iters += std::max(maxit, 1);
            if (!hist) {
                DHT_HIP(hipMemcpyAsync(scl, sup.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
                // the first correction is x itself: X_e = 0 is never materialised
                DHT_TRY(accum_up(c, X_e, e, inner, (const double*)scl, nrhs, !x_written));
            }
            x_written = true;
            // When the inner solver's own residual says this correction finishes
            // every RHS, go straight to the full-lattice check: its even residual
            // z_e - a x_e + Hop_eo x_o / 2 is the Schur residual (x_o reconstructed
            // from x_e), so a wrong guess costs one hop (x_o) and the loop continues
            // from it, while a right one saves a hop of the Schur residual.  The odd
            // residual z_o - a x_o + Hop_oe x_e / 2 vanishes by the construction of
            // x_o (to FP64 rounding), so the even one is the full residual.
            // the inner residual in units of r: ||r_new||^2 ~ sup^2 ||r_inner||^2
            bool predict = true;
            for (int i = 0; i < nrhs; i++)
                if (sup[i] > 0 && !(sup[i] * sup[i] * br.rnorm2[i] <= target2[i])) predict = false;
            if (predict) {
                // with the fused z^H x the even residual itself is not stored
                // (only its norms and z^H x are wanted if it meets the tolerance)
                const int nofield = zx_out ? HOP_NOOUT : 0;
                c->solver_count[SC_PREDICT]++;
                DHT_TRY(odd_from_even(c, X_e, X_o, Z_o, nrhs, zx_out ? &zx_o : nullptr, z16));
                DHT_TRY(residual_hop(c, 0, X_o, r_e, X_e, -a, 0.5, Z_e, nrhs, 0, rn2, zx_out ? &zx_e : nullptr,
                                     (z16 ? HOP_Z16 : 0) | nofield));
                rn2_inplace = false;
                bool done = true;
                full2 = rn2;
                for (int i = 0; i < nrhs; i++)
                    if (zn2[i] > 0 && !(full2[i] <= prm->tol * prm->tol * zn2[i])) done = false;
                if ((prm->fault_inject & 2u) && !forced_predict) {   // testing hook: reject one good prediction
                    forced_predict = true;
                    done = false;
                }
                if (done) {
                    have_full = true;
                    outer++;
                    break;
                }
                c->solver_count[SC_PREDICT_FAILED]++;
                if (nofield)   // the loop goes on from this residual: store it
                    DHT_TRY(residual_hop(c, 0, X_o, r_e, X_e, -a, 0.5, Z_e, nrhs, 0, rn2, &zx_e, z16 ? HOP_Z16 : 0));
            } else if (inc && !bad) {
                // r -= sigma Dhat e: Dhat e in FP32, the update and its norms in FP64
                // (after a NaN the discarded RHS's x may hold part of the
                // correction: that cycle recomputes the residual from x instead)
                DHT_TRY(apply_schur(c, DHT_FP32, E32, W32, T32, nrhs, nullptr));
                DHT_HIP(hipMemcpyAsync(scl, sup.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
                void *part, *sums;
                DHT_TRY(ws_get(c, WS_PARTIAL, partial_bytes(c, nrhs), &part));
                DHT_TRY(ws_get(c, WS_NORMS, sizeof(Cx<double>) * 6 * nrhs, &sums));
                // the next cycle's BF16 right-hand side in the same pass, scaled
                // by the inverse of each residual norm that this cycle predicts
                const bool can = predict_scales(sup, br, sdn);
                if (can) DHT_TRY(want16());
                int nbr;
                DHT_TRY(residual_step(c, r_e, r_e, W32, (const double*)scl, nrhs, (Cx<double>*)part, &nbr,
                                      can ? rh16 : nullptr, (const double*)s16));
                DHT_TRY(finalize(c, (const Cx<double>*)part, nbr, 1, nrhs, nullptr, FIN_SUM, 0.0, (Cx<double>*)sums));
                std::vector<Cx<double>> h(nrhs);
                DHT_HIP(hipMemcpyAsync(h.data(), sums, sizeof(Cx<double>) * nrhs, hipMemcpyDeviceToHost, c->stream));
                DHT_HIP(hipStreamSynchronize(c->stream));
                for (int i = 0; i < nrhs; i++) rn2[i] = h[i].re;
                c->solver_count[SC_INPLACE]++;
                rn2_inplace = true;
                if ((prm->fault_inject & 4u) && !forced_drift) {
                    // testing hook: the in-place norms understate the residual once, as
                    // an FP32 drift past the margin of the target would
                    forced_drift = true;
                    for (int i = 0; i < nrhs; i++) rn2[i] *= 1e-12;
                }
                if (can) {
                    prep = true;
                    sdp = sdn;
                }
            } else {
                // FP64 true residual of the Schur system, r = bhat - (a x - Hop_eo Hop_oe x / (4a)),
                // and its norms, in the second hop's epilogue (after a BF16 cycle
                // with the next BF16 right-hand side, scaled as predicted)
                const bool can = hist && !bad && predict_scales(sup, br, sdn);
                if (can) DHT_TRY(want16());
                DHT_TRY(hop(c, DHT_FP64, 1, X_e, tmp_o, nullptr, 0.0, 1.0, nrhs, false, false));
                DHT_TRY(residual_hop(c, 0, tmp_o, r_e, X_e, -a, 1.0 / (4.0 * a), bhat, nrhs, 0, rn2, nullptr, 0,
                                     can ? rh16 : nullptr, (const double*)s16));
                rn2_inplace = false;
                if (can) {
                    prep = true;
                    sdp = sdn;
                }
            }
            if (bad && inner != DHT_FP64) inner = inner == DHT_BF16 ? DHT_FP32 : DHT_FP64;
            last_bad = bad;
            for (int i = 0; i < nrhs; i++)
                if (inner != start_inner && rn2[i] > target2[i])
                    escalated[i] = inner == DHT_FP32 ? DHT_STATUS_FALLBACK_FP32 : DHT_STATUS_FALLBACK_FP64;
        }
        if (!x_written) DHT_TRY(zero(c, X_e, bh));
        if (have_full) {
            fr2 = full2;
            break;
        }
        // odd sites and the FP64 full-lattice true residual: its even half
        // r_e = z_e - (a x_e - Hop_eo x_o / 2) with norms fused (the odd half
        // vanishes by the construction of x_o)
        DHT_TRY(odd_from_even(c, X_e, X_o, Z_o, nrhs, zx_out ? &zx_o : nullptr, z16));
        DHT_TRY(residual_hop(c, 0, X_o, r_e, X_e, -a, 0.5, Z_e, nrhs, 0, fr2, zx_out ? &zx_e : nullptr,
                             (z16 ? HOP_Z16 : 0) | (zx_out ? HOP_NOOUT : 0)));
        bool met = true;
        for (int i = 0; i < nrhs; i++)
            if (zn2[i] > 0 && !(fr2[i] <= prm->tol * prm->tol * zn2[i])) met = false;
        // The loop stopped on residual norms from the in-place update, and the
        // FP64 residual of X misses the tolerance: go on from that residual while
        // cycles and iterations remain (it is the Schur residual of X_e, which the
        // next cycle needs stored)
        if (met || !rn2_inplace || outer >= max_outer || total_iters >= prm->maxiter) break;
        c->solver_count[SC_REENTRY]++;
        if (zx_out)
            DHT_TRY(residual_hop(c, 0, X_o, r_e, X_e, -a, 0.5, Z_e, nrhs, 0, fr2, &zx_e, z16 ? HOP_Z16 : 0));
        rn2 = fr2;
        rn2_inplace = false;
        prep = false;
        std::fill(last_rn2.begin(), last_rn2.end(), INFINITY);   // not a stall of the inner solves
    }
    if (zx_out)
        for (int i = 0; i < nrhs; i++) zx_out[i] = zx_e[i] + zx_o[i];
    bool all_ok = true;
    for (int i = 0; i < nrhs; i++) {
        double rr = zn2[i] > 0 ? sqrt(fr2[i] / zn2[i]) : 0.0;
        bool ok = rr <= prm->tol || zn2[i] == 0.0;
        all_ok &= ok;
        if (stats) {
            stats[i].iters = iters[i];
            stats[i].outer = outer;
            stats[i].true_resid = rr;
            stats[i].status = ok ? escalated[i] : DHT_STATUS_NOT_CONVERGED;
        }
    }
    return all_ok ? DHT_OK : set_error(DHT_ERR_NOT_CONVERGED, "some right-hand sides did not reach the tolerance");
}

}  // namespace dht
