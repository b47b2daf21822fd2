// Launch-shape autotuner for the even/odd hopping kernel.
//
// Every form of the kernel computes the same nearest-neighbour sums (the
// stencil of Section 1) in a different order, so the candidates are checked
// against the default form's output to rounding before they are timed; the
// fastest accepted shape is installed on the context for its (precision,
// batch, epilogue class) and used by every later hop launch of that kind.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"
#include "solver.h"

namespace dht {

static constexpr int TUNE_THREADS = 256;
static constexpr int TUNE_BLOCKS = 1024;

// per-block maxima of |a - b| and |b| over the real components of n 16-byte vectors
template <typename S>
__global__ __launch_bounds__(TUNE_THREADS) void maxdiff_kernel(const void* a, const void* b, size_t nvec,
                                                               Cx<double>* part) {
    constexpr int VW = Store<S>::VW;
    double dm = 0.0, rm = 0.0;
    for (size_t v = (size_t)blockIdx.x * TUNE_THREADS + threadIdx.x; v < nvec; v += (size_t)gridDim.x * TUNE_THREADS) {
        Cx<typename Store<S>::acc> x[VW], y[VW];
        Store<S>::ldv(a, (int64_t)v, x);
        Store<S>::ldv(b, (int64_t)v, y);
#pragma unroll
        for (int j = 0; j < VW; j++) {
            dm = fmax(dm, fmax(fabs((double)x[j].re - (double)y[j].re), fabs((double)x[j].im - (double)y[j].im)));
            rm = fmax(rm, fmax(fabs((double)y[j].re), fabs((double)y[j].im)));
        }
    }
    __shared__ double sd[TUNE_THREADS], sr[TUNE_THREADS];
    sd[threadIdx.x] = dm;
    sr[threadIdx.x] = rm;
    __syncthreads();
    for (int w = TUNE_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + w]);
            sr[threadIdx.x] = fmax(sr[threadIdx.x], sr[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = cmake(sd[0], sr[0]);
}

// max|a - b| / max|b| over one half field of nrhs RHS
static int rel_maxdiff(dht_ctx* c, int prec, const void* a, const void* b, int nrhs, Cx<double>* part, double* out) {
    const size_t nvec = half_elems(c, nrhs) / vec_width(prec);
    const int nb = (int)std::min<size_t>(TUNE_BLOCKS, (nvec + TUNE_THREADS - 1) / TUNE_THREADS);
    switch (prec) {
        case DHT_FP64: hipLaunchKernelGGL(maxdiff_kernel<double>, dim3(nb), dim3(TUNE_THREADS), 0, c->stream, a, b, nvec, part); break;
        case DHT_FP32: hipLaunchKernelGGL(maxdiff_kernel<float>, dim3(nb), dim3(TUNE_THREADS), 0, c->stream, a, b, nvec, part); break;
        default: hipLaunchKernelGGL(maxdiff_kernel<bf16x2>, dim3(nb), dim3(TUNE_THREADS), 0, c->stream, a, b, nvec, part); break;
    }
    DHT_HIP(hipGetLastError());
    std::vector<Cx<double>> h(nb);
    DHT_HIP(hipMemcpyAsync(h.data(), part, sizeof(Cx<double>) * nb, hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    double dm = 0.0, rm = 0.0;
    for (const auto& e : h) {
        dm = std::max(dm, e.re);
        rm = std::max(rm, e.im);
    }
    *out = rm > 0.0 ? dm / rm : dm;
    return DHT_OK;
}

// one hop of the class being tuned: plain out = Hop(in); fused out = 0.5 x +
// Hop(in) with the (out, x), (out, out) sums of BiCGStab's second product
struct TuneLaunch {
    int cls;
    const void* in;
    void* out;
    const void* x;
    Cx<double>* partial;
    const void* a;   // third operand of the (a, out) class: a field of its own, as in the solver
};

// one launch of the class's representative: plain; x-pay with (out, x) and
// (out, out); x-pay with (a, out)
static int tune_hop(dht_ctx* c, int prec, int nrhs, const TuneLaunch& L) {
    if (L.cls == HOP_PLAIN) return hop(c, prec, 0, L.in, L.out, nullptr, 0.0, 1.0, nrhs, false, false);
    HopDot d;
    d.kind = L.cls == HOP_FUSED_A ? HOPDOT_A_OUT : HOPDOT_OUT_X;
    d.a = L.cls == HOP_FUSED_A ? L.a : nullptr;
    d.partial = L.partial;
    return hop(c, prec, 0, L.in, L.out, L.x, 0.5, 1.0, nrhs, false, false, &d);
}

// mean time of `reps` launches in the shape in effect
static int time_hop(dht_ctx* c, int prec, int nrhs, const TuneLaunch& L, int reps, hipEvent_t e0, hipEvent_t e1,
                    double* ms) {
    for (int i = 0; i < 2; i++) DHT_TRY(tune_hop(c, prec, nrhs, L));
    DHT_HIP(hipEventRecord(e0, c->stream));
    for (int i = 0; i < reps; i++) DHT_TRY(tune_hop(c, prec, nrhs, L));
    DHT_HIP(hipEventRecord(e1, c->stream));
    DHT_HIP(hipEventSynchronize(e1));
    float f = 0.f;
    DHT_HIP(hipEventElapsedTime(&f, e0, e1));
    *ms = (double)f / reps;
    return DHT_OK;
}

static double tune_tolerance(int prec) { return prec == DHT_FP64 ? 1e-12 : (prec == DHT_FP32 ? 1e-5 : 1.6e-2); }

static int log2_pow2(int n) {
    for (int b = 0; b < 9; b++)
        if ((1 << b) == n) return b;
    return -1;
}

static int autotune(dht_ctx* c, int prec, int nrhs, int reps, dht_tune_result* res, hipEvent_t e0, hipEvent_t e1) {
    const int b = log2_pow2(nrhs);
    const size_t full = full_elems(c, nrhs) * elem_bytes(prec), half = full / 2;
    void *fi, *fo, *fr, *pp, *part;
    DHT_TRY(ws_get(c, WS_PACK_IN, full, &fi));
    DHT_TRY(ws_get(c, WS_PACK_OUT, half, &fo));
    DHT_TRY(ws_get(c, WS_TUNE_REF, half, &fr));
    void* fa;
    DHT_TRY(ws_get(c, WS_TUNE_A, half, &fa));
    DHT_TRY(zero(c, fa, half));
    DHT_TRY(ws_get(c, WS_TUNE_RED, sizeof(Cx<double>) * TUNE_BLOCKS, &pp));
    DHT_TRY(ws_get(c, WS_PARTIAL, partial_bytes(c, nrhs), &part));
    Cx<double>* red = (Cx<double>*)pp;
    dht_probe_spec sp = {2718281u, 0u, 0};
    DHT_TRY(probes_gen(c, &sp, 0, nrhs, nrhs, fi, prec, nullptr, nullptr));
    // in = the odd half of the probe field, x = its even half
    TuneLaunch L{HOP_PLAIN, (const char*)fi + half, fo, fi, (Cx<double>*)part, fa};

    // every form and t chunk, with streaming stores on and off, sweeping the
    // lattice once for all RHS or once per group of nrhs / 2 or nrhs / 4
    std::vector<HopConfig> cand;
    for (int gdiv = 1; gdiv <= 4 && gdiv <= nrhs; gdiv *= 2)
        for (int nt = 0; nt < 2; nt++) {
            HopConfig h;
            h.rg = gdiv == 1 ? 0 : nrhs / gdiv;
            const int G = nrhs / gdiv;
            h.nt = nt;
            h.form = DHT_HOP_SITE;
            cand.push_back(h);
            if (HOP_LANES / G <= 32) {
                h.form = DHT_HOP_SITE_LDS;
                cand.push_back(h);
            }
            for (int f : {DHT_HOP_TMARCH, DHT_HOP_TSKEW}) {
                h.form = f;
                for (int tc = 2; tc <= c->g.L[3]; tc += 2)
                    if (c->g.L[3] % tc == 0) {
                        h.tc = tc;
                        cand.push_back(h);
                    }
            }
            if (prec == DHT_BF16 && G >= 16) {   // links shared across each site's row of 16 lanes
                h.tc = 0;
                h.form = DHT_HOP_SITE_ROWL;
                cand.push_back(h);
                for (int f : {DHT_HOP_TMARCH_ROWL, DHT_HOP_TSKEW_ROWL}) {
                    h.form = f;
                    for (int tc = 2; tc <= c->g.L[3]; tc += 2)
                        if (c->g.L[3] % tc == 0) {
                            h.tc = tc;
                            cand.push_back(h);
                        }
                }
            }
        }
    int rejected = 0;
    double worst_ok = 0.0;
    for (int cls = 0; cls < HOP_NCLASS; cls++) {
        L.cls = cls;
        // reference: the built-in default shape
        c->hop_force = true;
        c->hop_forced = hop_default_config(c, prec, nrhs);
        const HopConfig def = c->hop_forced;
        L.out = fr;
        DHT_TRY(tune_hop(c, prec, nrhs, L));
        L.out = fo;
        double def_ms = 0.0;
        DHT_TRY(time_hop(c, prec, nrhs, L, reps, e0, e1, &def_ms));
        HopConfig best = def;
        double best_ms = def_ms;
        // the fastest shape of each t-marching form, then tried with z blocks
        HopConfig form_best[8];
        double form_ms[8];
        for (int f = 0; f < 8; f++) form_ms[f] = -1.0;
        auto try_shape = [&](const HopConfig& h, double* ms_out) -> int {
            *ms_out = -1.0;
            c->hop_forced = h;
            DHT_TRY(tune_hop(c, prec, nrhs, L));
            double rd = 0.0;
            DHT_TRY(rel_maxdiff(c, prec, fo, fr, nrhs, red, &rd));
            if (!(rd <= tune_tolerance(prec))) {
                rejected++;
                return DHT_OK;
            }
            worst_ok = std::max(worst_ok, rd);
            double ms = 0.0;
            DHT_TRY(time_hop(c, prec, nrhs, L, reps, e0, e1, &ms));
            *ms_out = ms;
            if (ms < best_ms) {
                best_ms = ms;
                best = h;
            }
            return DHT_OK;
        };
        for (const HopConfig& h : cand) {
            double ms;
            DHT_TRY(try_shape(h, &ms));
            if (ms >= 0.0 && hop_form_tmarch(h.form) && (form_ms[h.form] < 0.0 || ms < form_ms[h.form])) {
                form_ms[h.form] = ms;
                form_best[h.form] = h;
            }
        }
        for (int f = 0; f < 8; f++) {
            if (form_ms[f] < 0.0) continue;
            for (int zb = 1; zb <= 3 && c->g.L[2] % (1 << zb) == 0; zb++) {
                HopConfig h = form_best[f];
                h.zb = zb;
                double ms;
                DHT_TRY(try_shape(h, &ms));
            }
        }
        c->hop_force = false;
        if (hop_form_tmarch(best.form) && best.tc == 0) best.tc = hop_config(c, prec, nrhs, cls).tc;
        c->hop_cfg[prec][b][cls] = best;
        res->best[cls].form = best.form;
        res->best[cls].streaming_stores = best.nt;
        res->best[cls].t_chunk = hop_form_tmarch(best.form) ? best.tc : 0;
        res->best[cls].rhs_group = best.rg > 0 ? best.rg : nrhs;
        res->best[cls].z_block = 1 << best.zb;
        res->best_ms[cls] = best_ms;
        res->default_ms[cls] = def_ms;
    }
    res->candidates = (int)cand.size();
    res->rejected = rejected;
    res->max_rel_diff = worst_ok;
    return DHT_OK;
}

}  // namespace dht

using namespace dht;

extern "C" {

int dht_autotune_batch(dht_ctx* c, const dht_probe_spec* spec, const dht_solver_params* prm, const int* cand,
                       int ncand, size_t mem_budget, int reps, dht_batch_tune* out) {
    if (!c || !spec || !prm || !cand || !out || ncand <= 0 || ncand > DHT_TUNE_MAX_BATCHES || reps <= 0)
        return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    DHT_HIP(hipSetDevice(c->device));
    if (mem_budget == 0) {   // what the device has free now, plus the workspace the library holds
        size_t fr = 0, tot = 0;
        DHT_HIP(hipMemGetInfo(&fr, &tot));
        size_t held = 0;
        for (int i = 0; i < (int)c->ws.size(); i++)
            if (i != WS_HOSTPIN) held += c->ws[i].bytes;
        mem_budget = (size_t)(0.9 * (double)(fr + held));
    }
    memset(out, 0, sizeof(*out));
    out->candidates = ncand;
    // the timed batches must not change the running estimates or the projection window
    const Welford q0 = c->est_q, qd0 = c->est_qd;
    const int pin = DHT_HOP_PLAIN;
    (void)pin;
    double best = -1.0;
    int rc_all = DHT_OK;
    for (int i = 0; i < ncand; i++) {
        const int B = cand[i];
        out->nrhs[i] = B;
        if (B <= 0 || B > DHT_MAX_BATCH) {
            out->status[i] = DHT_BATCH_INVALID;
            continue;
        }
        size_t need = 0;
        DHT_TRY(dht_workspace_size(c, B, prm, &need));
        out->workspace[i] = need;
        if (need > mem_budget) {
            out->status[i] = DHT_BATCH_OVER_BUDGET;
            continue;
        }
        // hop shapes of every precision the solve runs at this batch
        const int bp = pad_rhs(B), lb = log2_pow2(bp);
        const int precs[3] = {DHT_FP64, DHT_FP32, DHT_BF16};
        for (int prec : precs) {
            if (c->hop_cfg[prec][lb][0].form >= 0) continue;
            if (prm->method == DHT_SOLVER_BICGSTAB_FP64 && prec != DHT_FP64) continue;
            dht_tune_result tr;
            DHT_TRY(dht_autotune_hop(c, prec, bp, 3, &tr));
        }
        c->pw_valid = false;
        int rc = dht_trace_batch(c, spec, 0, B, prm, nullptr, nullptr);   // warm-up (workspace, window)
        if (rc == DHT_OK) {   // wall clock: the host's per-iteration polls are part of a batch's cost
            c->pw_valid = false;
            DHT_HIP(hipStreamSynchronize(c->stream));
            const auto t0 = std::chrono::steady_clock::now();
            for (int r = 0; r < reps && rc == DHT_OK; r++) rc = dht_trace_batch(c, spec, (int64_t)r * B, B, prm, nullptr, nullptr);
            DHT_HIP(hipStreamSynchronize(c->stream));
            const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (rc == DHT_OK && s > 0) out->rhs_per_s[i] = reps * B / s;
        }
        if (rc != DHT_OK) {
            out->status[i] = DHT_BATCH_FAILED;
            rc_all = rc;
            continue;
        }
        out->status[i] = DHT_BATCH_TIMED;
        if (out->rhs_per_s[i] > best) {
            best = out->rhs_per_s[i];
            out->best_nrhs = B;
        }
    }
    c->est_q = q0;
    c->est_qd = qd0;
    c->pw_valid = false;
    if (out->best_nrhs == 0)
        return rc_all != DHT_OK ? rc_all : set_error(DHT_ERR_OOM, "no candidate batch fits the memory budget");
    return DHT_OK;
}

int dht_autotune_projection(dht_ctx* c, int nrhs, int reps, int* best_wgs, double* best_ms) {
    if (!c || !best_wgs || nrhs <= 0 || nrhs > 64 || reps <= 0) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    DHT_HIP(hipSetDevice(c->device));
    if (!c->defl_ready || c->wprec != DHT_BF16) return set_error(DHT_ERR_STATE, "needs a finalized BF16 basis");
    const int bp = pad_rhs(nrhs), k = c->k;
    void *zc, *cc, *pp;
    DHT_TRY(ws_get(c, WS_ZCODE, full_elems(c, bp), &zc));
    DHT_TRY(ws_get(c, WS_SCAL2, sizeof(Cx<double>) * 4 * (size_t)k * bp, &cc));
    DHT_TRY(ws_get(c, WS_TUNE_RED, sizeof(Cx<double>) * TUNE_BLOCKS, &pp));
    dht_probe_spec sp = {1414213u, 0u, 1};
    DHT_TRY(probes_gen(c, &sp, 0, nrhs, bp, nullptr, DHT_FP64, nullptr, nullptr, (uint8_t*)zc));
    Cx<double>* ref = (Cx<double>*)cc;
    Cx<double>* got = ref + 2 * (size_t)k * bp;
    const int saved = c->proj_wgs;
    c->proj_wgs = 0;
    DHT_TRY(project_codes(c, (const uint8_t*)zc, bp, ref, ref + (size_t)k * bp));
    std::vector<Cx<double>> hr(2 * (size_t)k * bp), hg(hr.size());
    DHT_HIP(hipMemcpyAsync(hr.data(), ref, sizeof(Cx<double>) * hr.size(), hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    double rmax = 0.0;
    for (auto& v : hr) rmax = std::max(rmax, std::max(std::fabs(v.re), std::fabs(v.im)));
    const int targets[5] = {256, 512, 1024, 2048, 4096};
    double bms = 1e300;
    int bw = 512;
    for (int t : targets) {
        c->proj_wgs = t;
        for (int i = 0; i < 1; i++) DHT_TRY(project_codes(c, (const uint8_t*)zc, bp, got, got + (size_t)k * bp));
        DHT_HIP(hipEventRecord(c->ev[0], c->stream));
        for (int i = 0; i < reps; i++) DHT_TRY(project_codes(c, (const uint8_t*)zc, bp, got, got + (size_t)k * bp));
        DHT_HIP(hipEventRecord(c->ev[1], c->stream));
        DHT_HIP(hipEventSynchronize(c->ev[1]));
        float ms = 0.f;
        DHT_HIP(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        // the FP32 chunk sums are the same in every split; only the FP64 order of adding them moves
        DHT_HIP(hipMemcpyAsync(hg.data(), got, sizeof(Cx<double>) * hg.size(), hipMemcpyDeviceToHost, c->stream));
        DHT_HIP(hipStreamSynchronize(c->stream));
        double dmax = 0.0;
        for (size_t i = 0; i < hg.size(); i++)
            dmax = std::max(dmax, std::max(std::fabs(hg[i].re - hr[i].re), std::fabs(hg[i].im - hr[i].im)));
        if (!(dmax <= 1e-12 * std::max(rmax, 1e-300))) continue;
        if (ms / reps < bms) {
            bms = ms / reps;
            bw = t;
        }
    }
    (void)pp;
    c->proj_wgs = bw;
    c->pw_valid = false;
    *best_wgs = bw;
    if (best_ms) *best_ms = bms;
    (void)saved;
    return DHT_OK;
}


int dht_hop_config_set(dht_ctx* c, int prec, int nrhs, int epilogue, const dht_hop_config* cfg) {
    if (!c) return set_error(DHT_ERR_INVALID_ARG, "null context");
    if (prec < DHT_FP64 || prec > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    if (epilogue < 0 || epilogue >= HOP_NCLASS) return set_error(DHT_ERR_INVALID_ARG, "bad epilogue class");
    const int b = log2_pow2(nrhs);
    if (b < 0) return set_error(DHT_ERR_INVALID_ARG, "batch must be a power of two <= 256");
    if (!cfg) {
        c->hop_cfg[prec][b][epilogue] = HopConfig();
        return DHT_OK;
    }
    HopConfig h;
    h.form = cfg->form;
    h.nt = cfg->streaming_stores;
    h.tc = hop_form_tmarch(cfg->form) ? cfg->t_chunk : 0;
    h.rg = cfg->rhs_group == nrhs ? 0 : cfg->rhs_group;
    if (cfg->z_block < 0 || (cfg->z_block & (cfg->z_block - 1)))
        return set_error(DHT_ERR_INVALID_ARG, "z block must be 0 or a power of two");
    h.zb = 0;
    while ((2 << h.zb) <= cfg->z_block) h.zb++;
    DHT_TRY(hop_config_check(c, nrhs, h));
    c->hop_cfg[prec][b][epilogue] = h;
    return DHT_OK;
}

int dht_hop_config_get(dht_ctx* c, int prec, int nrhs, int epilogue, dht_hop_config* out) {
    if (!c || !out) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    if (prec < DHT_FP64 || prec > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    if (epilogue < 0 || epilogue >= HOP_NCLASS) return set_error(DHT_ERR_INVALID_ARG, "bad epilogue class");
    if (log2_pow2(nrhs) < 0) return set_error(DHT_ERR_INVALID_ARG, "batch must be a power of two <= 256");
    HopConfig h = hop_config(c, prec, nrhs, epilogue);
    out->form = h.form;
    out->streaming_stores = h.nt;
    out->t_chunk = hop_form_tmarch(h.form) ? h.tc : 0;
    out->rhs_group = h.rg > 0 ? h.rg : nrhs;
    out->z_block = 1 << h.zb;
    return DHT_OK;
}

int dht_autotune_hop(dht_ctx* c, int prec, int nrhs, int reps, dht_tune_result* out) {
    if (!c || !out) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    if (prec < DHT_FP64 || prec > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    if (log2_pow2(nrhs) < 0) return set_error(DHT_ERR_INVALID_ARG, "batch must be a power of two <= 256");
    if (reps <= 0) return set_error(DHT_ERR_INVALID_ARG, "reps must be positive");
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    DHT_HIP(hipSetDevice(c->device));
    hipEvent_t e0, e1;
    DHT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(DHT_ERR_HIP, "hipEventCreate failed");
    }
    int rc = autotune(c, prec, nrhs, reps, out, e0, e1);
    c->hop_force = false;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int dht_autotune(dht_ctx* c, int prec, int nrhs, int reps, const char* cache_path, dht_tune_result* out) {
    if (!c || !out) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    if (prec < DHT_FP64 || prec > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    if (log2_pow2(nrhs) < 0) return set_error(DHT_ERR_INVALID_ARG, "batch must be a power of two <= 256");
    // cache lines: "hop2 Lx Ly Lz Lt prec nrhs class form streaming_stores t_chunk rhs_group z_block ms"
    // (lines of any other form are skipped)
    if (cache_path) {
        FILE* f = fopen(cache_path, "r");
        if (f) {
            dht_hop_config found[HOP_NCLASS];
            double ms[HOP_NCLASS] = {0, 0, 0};
            bool have[HOP_NCLASS] = {false, false, false};
            char line[512], tag[8];
            int L[4], p, n, cls, form, nt, tc, rg, zb;
            double t;
            while (fgets(line, sizeof(line), f)) {
                if (sscanf(line, "%7s %d %d %d %d %d %d %d %d %d %d %d %d %lf", tag, &L[0], &L[1], &L[2], &L[3], &p, &n,
                           &cls, &form, &nt, &tc, &rg, &zb, &t) != 14)
                    continue;
                if (strcmp(tag, "hop2") != 0 || p != prec || n != nrhs || cls < 0 || cls >= HOP_NCLASS) continue;
                if (L[0] != c->g.L[0] || L[1] != c->g.L[1] || L[2] != c->g.L[2] || L[3] != c->g.L[3]) continue;
                found[cls] = dht_hop_config{form, nt, tc, rg, zb};
                ms[cls] = t;
                have[cls] = true;
            }
            fclose(f);
            if (have[0] && have[1] && have[2]) {
                for (int cls2 = 0; cls2 < HOP_NCLASS; cls2++) {
                    DHT_TRY(dht_hop_config_set(c, prec, nrhs, cls2, &found[cls2]));
                    out->best[cls2] = found[cls2];
                    out->best_ms[cls2] = ms[cls2];
                    out->default_ms[cls2] = 0.0;
                }
                out->candidates = 0;
                out->rejected = 0;
                out->max_rel_diff = 0.0;
                return DHT_OK;
            }
        }
    }
    DHT_TRY(dht_autotune_hop(c, prec, nrhs, reps, out));
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (!f) return set_error(DHT_ERR_INVALID_ARG, std::string("cannot write ") + cache_path);
        for (int cls = 0; cls < HOP_NCLASS; cls++)
            fprintf(f, "hop2 %d %d %d %d %d %d %d %d %d %d %d %d %.6g\n", c->g.L[0], c->g.L[1], c->g.L[2], c->g.L[3],
                    prec, nrhs, cls, out->best[cls].form, out->best[cls].streaming_stores, out->best[cls].t_chunk,
                    out->best[cls].rhs_group, out->best[cls].z_block, out->best_ms[cls]);
        if (fclose(f) != 0) return set_error(DHT_ERR_INVALID_ARG, std::string("cannot write ") + cache_path);
    }
    return DHT_OK;
}

}  // extern "C"
