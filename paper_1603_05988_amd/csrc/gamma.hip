// Traces Tr(Gamma D^-1) for several spin matrices Gamma over one deflation
// space (end of Section 5.2: the deflated split of the trace holds with an
// inexpensive Gamma multiplied in, one Gamma product enters per probe, and the
// deflation space is shared by every Gamma).
//
// Everything is carried by the 16 spin pairs (s, t).  With a spin matrix
// Gamma acting alike on every site and colour:
//   z^H Gamma x        = sum_st Gamma_st Q_st,        Q_st = z_s^H x_t,
//   W^H Gamma^H z      = sum_st conj(Gamma_ts) P_st,  P_st = W_s^H z_t,
//   z^H Gamma P z      = sum_st Gamma_ts (P_st^H M c2),   c2 = W^H g5 z,
//   T_D(Gamma) = Tr(M W^H g5 Gamma W) = sum_st Gamma_st g5_s T_st,
//                T_st = sum_ab M_ab W_b,s^H W_a,t,
// where v_s is the spin-s part of v (its 3 V colour-site entries).  One
// solve, one pass over (z, x) and one pass over the basis per probe serve
// any number of matrices; the per-matrix work is O(16) per probe on the host
// (plus O(k) for the P_st^H M c2 contractions shared by all matrices).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <vector>

#include "solver.h"

namespace dht {

typedef std::complex<double> cplx;

static constexpr int SPF_THREADS = 256;
static constexpr int SPF_MAX_BLOCKS = 1024;

// partial[blk][st][r] = sum over this block's (parity, site) items of
// sum_c conj(a(s, c)) b(t, c) for RHS r, on FP64 full fields [2][12][Vh][B]
// (B a power of two <= 256, so a thread's RHS stays fixed over its grid-stride loop)
__global__ __launch_bounds__(SPF_THREADS) void spin_pair_forms_kernel(const Cx<double>* A, const Cx<double>* Bf,
                                                                      int64_t Vh, int B, Cx<double>* partial) {
    __shared__ Cx<double> red[16][SPF_THREADS];
    Cx<double> acc[16];
#pragma unroll
    for (int st = 0; st < 16; st++) acc[st] = cmake(0.0, 0.0);
    const int64_t n = 2 * Vh * B;
    const int64_t cstride = Vh * B;   // between colour-spin components
    for (int64_t it = (int64_t)blockIdx.x * SPF_THREADS + threadIdx.x; it < n; it += (int64_t)gridDim.x * SPF_THREADS) {
        const int64_t par = it / cstride;
        const int64_t base = it + 11 * cstride * par;   // component 0 of this (parity, site, RHS)
        Cx<double> a[12], b[12];
#pragma unroll
        for (int q = 0; q < 12; q++) {
            a[q] = A[base + q * cstride];
            b[q] = Bf[base + q * cstride];
        }
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int t = 0; t < 4; t++)
#pragma unroll
                for (int col = 0; col < 3; col++)
                    acc[s * 4 + t] = acc[s * 4 + t] + conjmul(a[3 * s + col], b[3 * t + col]);
    }
#pragma unroll
    for (int st = 0; st < 16; st++) red[st][threadIdx.x] = acc[st];
    __syncthreads();
    for (int half = SPF_THREADS / 2; half >= B; half >>= 1) {
        if (threadIdx.x < half) {
#pragma unroll
            for (int st = 0; st < 16; st++) red[st][threadIdx.x] = red[st][threadIdx.x] + red[st][threadIdx.x + half];
        }
        __syncthreads();
    }
    if (threadIdx.x < B) {
#pragma unroll
        for (int st = 0; st < 16; st++) partial[((int64_t)blockIdx.x * 16 + st) * B + threadIdx.x] = red[st][threadIdx.x];
    }
}

__global__ void spin_pair_sum_kernel(const Cx<double>* partial, int nblk, int n, Cx<double>* out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    Cx<double> s = cmake(0.0, 0.0);
    for (int b = 0; b < nblk; b++) s = s + partial[(int64_t)b * n + idx];
    out[idx] = s;
}

static int spf_blocks(const dht_ctx* c, int nrhs) {
    const int64_t n = 2 * c->g.Vh * nrhs;
    return (int)std::min<int64_t>(SPF_MAX_BLOCKS, (n + SPF_THREADS - 1) / SPF_THREADS);
}

// out[st][r] = a_s^H b_t for every RHS r < nrhs (FP64 full fields; nrhs a power of two <= 256)
static int spin_pair_forms(dht_ctx* c, const void* a, const void* b, int nrhs, Cx<double>* part, Cx<double>* out) {
    if (nrhs <= 0 || nrhs > SPF_THREADS || (nrhs & (nrhs - 1)))
        return set_error(DHT_ERR_INVALID_ARG, "spin-pair forms need a power-of-two batch <= 256");
    const int nblk = spf_blocks(c, nrhs);
    hipLaunchKernelGGL(spin_pair_forms_kernel, dim3(nblk), dim3(SPF_THREADS), 0, c->stream, (const Cx<double>*)a,
                       (const Cx<double>*)b, c->g.Vh, nrhs, part);
    DHT_HIP(hipGetLastError());
    hipLaunchKernelGGL(spin_pair_sum_kernel, dim3((16 * nrhs + 127) / 128), dim3(128), 0, c->stream,
                       (const Cx<double>*)part, nblk, 16 * nrhs, out);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

static const double G5_SIGN[4] = {1.0, 1.0, -1.0, -1.0};   // chiral basis

static cplx gam_at(const dht_ctx* c, int g, int s, int t) {
    const size_t o = 2 * ((size_t)g * 16 + s * 4 + t);
    return cplx(c->gam[o], c->gam[o + 1]);
}

// T_st = sum_ab M_ab W_b,s^H W_a,t, from the stored basis in FP64, once per basis
static int gamma_td_setup(dht_ctx* c) {
    if (c->gamT_valid && c->gam_gen == c->defl_gen) return DHT_OK;
    cplx T[16];
    for (int st = 0; st < 16; st++) T[st] = 0.0;
    const int k = c->defl_ready ? c->k : 0;
    if (k > 0) {
        const cplx* M = (const cplx*)c->M.data();
        const int nb = std::min(k, 32);
        const int bp = pad_rhs(nb);
        void *wb, *part, *outb;
        DHT_TRY(ws_get(c, WS_QW, full_elems(c, bp) * 16, &wb));
        std::vector<Cx<double>> h;
        if (c->M_diag) {   // only the diagonal W_a,s^H W_a,t enters
            DHT_TRY(ws_get(c, WS_GAM_FPART, (size_t)spf_blocks(c, bp) * 16 * bp * sizeof(Cx<double>), &part));
            DHT_TRY(ws_get(c, WS_GAM_OUT, (size_t)16 * bp * sizeof(Cx<double>), &outb));
            h.resize((size_t)16 * bp);
        } else {
            DHT_TRY(ws_get(c, WS_GAM_OUT, (size_t)16 * k * bp * sizeof(Cx<double>), &outb));
            h.resize((size_t)16 * k * bp);
        }
        for (int j0 = 0; j0 < k; j0 += nb) {
            const int n = std::min(nb, k - j0);
            DHT_TRY(gather_columns(c, j0, n, bp, wb));
            if (c->M_diag) {
                DHT_TRY(spin_pair_forms(c, wb, wb, bp, (Cx<double>*)part, (Cx<double>*)outb));
            } else {
                DHT_TRY(project_field_sp(c, wb, bp, (Cx<double>*)outb));   // [st][b][a - j0]
            }
            DHT_HIP(hipMemcpyAsync(h.data(), outb, sizeof(Cx<double>) * h.size(), hipMemcpyDeviceToHost, c->stream));
            DHT_HIP(hipStreamSynchronize(c->stream));
            for (int st = 0; st < 16; st++)
                for (int jj = 0; jj < n; jj++) {
                    const int a = j0 + jj;
                    if (c->M_diag) {
                        const Cx<double> v = h[(size_t)st * bp + jj];
                        T[st] += M[(size_t)a * k + a] * cplx(v.re, v.im);
                    } else {
                        cplx acc = 0.0;
                        for (int b = 0; b < k; b++) {
                            const Cx<double> v = h[((size_t)st * k + b) * bp + jj];
                            acc += M[(size_t)a * k + b] * cplx(v.re, v.im);
                        }
                        T[st] += acc;
                    }
                }
        }
        DHT_TRY(prof_harvest(c));
    }
    for (int st = 0; st < 16; st++) {
        c->gamT[2 * st] = T[st].real();
        c->gamT[2 * st + 1] = T[st].imag();
    }
    c->gamT_valid = true;
    c->gam_gen = c->defl_gen;
    return DHT_OK;
}

static cplx gamma_td(const dht_ctx* c, int g) {
    if (!c->defl_ready || c->k <= 0) return 0.0;
    cplx td = 0.0;
    for (int s = 0; s < 4; s++)
        for (int t = 0; t < 4; t++)
            td += gam_at(c, g, s, t) * G5_SIGN[s] * cplx(c->gamT[2 * (s * 4 + t)], c->gamT[2 * (s * 4 + t) + 1]);
    return td;
}

}  // namespace dht

using namespace dht;

extern "C" {

int dht_gamma_set(dht_ctx* c, const double* gamma_host, int ng, double* TD_host) {
    if (!c || !gamma_host) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    if (ng <= 0 || ng > DHT_MAX_GAMMA) return set_error(DHT_ERR_INVALID_ARG, "number of matrices outside 1..DHT_MAX_GAMMA");
    for (int i = 0; i < 32 * ng; i++)
        if (!isfinite(gamma_host[i])) return set_error(DHT_ERR_INVALID_ARG, "non-finite matrix entry");
    if (c->W && !c->defl_ready) return set_error(DHT_ERR_STATE, "deflation basis set but not finalized");
    DHT_HIP(hipSetDevice(c->device));
    c->gam.assign(gamma_host, gamma_host + 32 * (size_t)ng);
    c->ng = ng;
    c->gest_q.assign(ng, Welford());
    c->gest_qd.assign(ng, Welford());
    c->gamT_valid = false;
    DHT_TRY(gamma_td_setup(c));
    if (TD_host)
        for (int g = 0; g < ng; g++) {
            const cplx td = gamma_td(c, g);
            TD_host[2 * g] = td.real();
            TD_host[2 * g + 1] = td.imag();
        }
    return DHT_OK;
}

int dht_trace_gamma_batch(dht_ctx* c, const dht_probe_spec* spec, int64_t first, int nrhs, const dht_solver_params* prm,
                          dht_record* records) {
    if (!c || !spec || !prm || nrhs <= 0 || nrhs > DHT_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    DHT_HIP(hipSetDevice(c->device));
    if (c->ng <= 0) return set_error(DHT_ERR_STATE, "no matrices registered (dht_gamma_set)");
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    if (c->W && !c->defl_ready) return set_error(DHT_ERR_STATE, "deflation basis set but not finalized");
    DHT_TRY(gamma_td_setup(c));
    const int bp = pad_rhs(nrhs);
    const int k = c->defl_ready ? c->k : 0;
    const size_t fb = full_elems(c, bp) * 16;
    void *fz, *fx, *part, *outb;
    DHT_TRY(ws_get(c, WS_Z, fb, &fz));
    DHT_TRY(ws_get(c, WS_PACK_OUT, fb, &fx));
    const bool mfma = k > 0 && c->wprec == DHT_BF16;
    const int slice = mfma ? std::min(bp, 16) : bp;   // probes per pass over the basis
    const size_t pq = (size_t)16 * bp;                 // Q_st, then P_st [16][k][slice] per slice
    const size_t pn = (size_t)16 * k * slice;
    const int nslice = (nrhs + slice - 1) / slice;
    DHT_TRY(ws_get(c, WS_GAM_OUT, sizeof(Cx<double>) * (pq + pn * nslice), &outb));
    DHT_TRY(ws_get(c, WS_GAM_FPART, (size_t)spf_blocks(c, bp) * 16 * bp * sizeof(Cx<double>), &part));
    Cx<double>* dQ = (Cx<double>*)outb;
    Cx<double>* dP = dQ + pq;
    DHT_TRY(probes_gen(c, spec, first, nrhs, bp, fz, DHT_FP64, nullptr, nullptr, nullptr));
    // The 16 spin-pair projections of every probe run on the side stream while
    // the main stream solves: with a BF16 basis they regenerate the probes as
    // codes of their own; otherwise they read fz, which the solve only reads.
    const bool side = k > 0;
    if (side) {
        DHT_TRY(side_stream(c));
        DHT_HIP(hipEventRecord(c->side_ev[0], c->stream));
        DHT_HIP(hipStreamWaitEvent(c->side, c->side_ev[0], 0));
        hipStream_t main_stream = c->stream;
        c->stream = c->side;
        int prc = DHT_OK;
        if (mfma) {
            void* zc = nullptr;
            prc = ws_get(c, WS_GAM_CODE, full_elems(c, slice), &zc);
            for (int sl = 0; sl < nslice && prc == DHT_OK; sl++) {
                const int n0 = sl * slice, n = std::min(slice, nrhs - n0);
                prc = probes_gen(c, spec, first + n0, n, n, nullptr, DHT_FP64, nullptr, nullptr, (uint8_t*)zc);
                if (prc == DHT_OK) prc = project_codes_sp(c, (const uint8_t*)zc, n, dP + pn * sl);
            }
        } else {
            prc = project_field_sp(c, fz, bp, dP);
        }
        if (prc == DHT_OK && hipEventRecord(c->side_ev[2], c->side) != hipSuccess) prc = set_error(DHT_ERR_HIP, "event");
        c->stream = main_stream;
        if (prc != DHT_OK) {
            (void)hipStreamSynchronize(c->side);
            return prc;
        }
    }
    std::vector<dht_solve_stats> st(bp);
    std::vector<double> zn2(bp, 0.0);
    for (int r = 0; r < nrhs; r++) zn2[r] = (double)(12 * c->g.V);
    int rc = solve_fields(c, prm, fz, fx, bp, st.data(), zn2.data(), nullptr, DHT_FP64);
    if (rc != DHT_OK && rc != DHT_ERR_NOT_CONVERGED) {
        if (side) (void)hipStreamSynchronize(c->side);   // the next call rewrites its inputs
        return rc;
    }
    if (side) DHT_HIP(hipStreamWaitEvent(c->stream, c->side_ev[2], 0));
    const std::string msg = dht_last_error();   // the solve's message, if it missed the tolerance
    DHT_TRY(spin_pair_forms(c, fz, fx, bp, (Cx<double>*)part, dQ));
    std::vector<Cx<double>> h(pq + pn * nslice);
    DHT_HIP(hipMemcpyAsync(h.data(), outb, sizeof(Cx<double>) * h.size(), hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    DHT_TRY(prof_harvest(c));
    if (rc == DHT_ERR_NOT_CONVERGED) {
        bool any = false;
        for (int r = 0; r < nrhs; r++) any |= st[r].status == DHT_STATUS_NOT_CONVERGED;
        if (!any) rc = DHT_OK;
    }
    const cplx* M = (const cplx*)c->M.data();
    std::vector<cplx> c2(k), v(k);
    for (int r = 0; r < nrhs; r++) {
        cplx Q[16], E[16];
        for (int s = 0; s < 16; s++) {
            Q[s] = cplx(h[(size_t)s * bp + r].re, h[(size_t)s * bp + r].im);
            E[s] = 0.0;
        }
        if (k > 0) {
            // P_st of probe r: column r - n0 of its slice's [16][k][width] block,
            // width = the slice's probe count (MFMA passes) or bp (one field pass)
            const int sl = r / slice, n0 = sl * slice;
            const int width = mfma ? std::min(slice, nrhs - n0) : bp;
            const Cx<double>* Pr = h.data() + pq + pn * sl;
            const int col = r - n0;
            auto P = [&](int stp, int i) {
                const Cx<double> x = Pr[((size_t)stp * k + i) * width + col];
                return cplx(x.re, x.im);
            };
            for (int i = 0; i < k; i++) {
                cplx a = 0.0;
                for (int s = 0; s < 4; s++) a += G5_SIGN[s] * P(5 * s, i);
                c2[i] = a;
            }
            for (int a = 0; a < k; a++) {
                cplx acc = 0.0;
                if (c->M_diag) acc = M[(size_t)a * k + a] * c2[a];
                else
                    for (int b = 0; b < k; b++) acc += M[(size_t)a * k + b] * c2[b];
                v[a] = acc;
            }
            for (int stp = 0; stp < 16; stp++) {
                cplx acc = 0.0;
                for (int i = 0; i < k; i++) acc += std::conj(P(stp, i)) * v[i];
                E[stp] = acc;   // P_st^H M c2
            }
        }
        for (int g = 0; g < c->ng; g++) {
            cplx q = 0.0, d = 0.0;
            for (int s = 0; s < 4; s++)
                for (int t = 0; t < 4; t++) {
                    q += gam_at(c, g, s, t) * Q[s * 4 + t];
                    d += gam_at(c, g, t, s) * E[s * 4 + t];
                }
            const cplx qd = q - d;
            if (st[r].status != DHT_STATUS_NOT_CONVERGED) {
                c->gest_q[g].add(q.real(), q.imag());
                c->gest_qd[g].add(qd.real(), qd.imag());
            }
            if (records) {
                dht_record& rec = records[(size_t)g * nrhs + r];
                rec.q_re = q.real();
                rec.q_im = q.imag();
                rec.qd_re = qd.real();
                rec.qd_im = qd.imag();
                rec.s = st[r];
            }
        }
    }
    if (rc != DHT_OK) return set_error(rc, msg);
    return DHT_OK;
}

int dht_gamma_estimate_get(dht_ctx* c, int g, dht_estimate* e) {
    if (!c || !e) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    if (g < 0 || g >= c->ng) return set_error(DHT_ERR_INVALID_ARG, "no such matrix");
    if (c->W && !c->defl_ready) return set_error(DHT_ERR_STATE, "deflation basis set but not finalized");
    DHT_HIP(hipSetDevice(c->device));
    DHT_TRY(gamma_td_setup(c));
    const cplx td = gamma_td(c, g);
    const Welford& wq = c->gest_q[g];
    const Welford& wd = c->gest_qd[g];
    memset(e, 0, sizeof(*e));
    e->n = wq.n;
    e->mean_re = wq.mre;
    e->mean_im = wq.mim;
    e->TD_re = td.real();
    e->TD_im = td.imag();
    e->mean_defl_re = wd.mre + td.real();
    e->mean_defl_im = wd.mim + td.imag();
    if (e->n >= 2) {
        const double dn = (double)(e->n - 1);
        e->var_re = wq.m2re / dn;
        e->var_im = wq.m2im / dn;
        e->var = e->var_re + e->var_im;
        e->var_defl_re = wd.m2re / dn;
        e->var_defl_im = wd.m2im / dn;
        e->var_defl = e->var_defl_re + e->var_defl_im;
    } else {
        e->var = e->var_re = e->var_im = NAN;
        e->var_defl = e->var_defl_re = e->var_defl_im = NAN;
    }
    return DHT_OK;
}

}  // extern "C"
