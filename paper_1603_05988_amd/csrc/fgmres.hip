// Batched flexible GMRES (Saad 1993) with a right preconditioner, inside
// FP64 defect correction, on the full-lattice Wilson matrix.
//
// Each outer cycle: r = z - D x in FP64; one FGMRES(m) cycle in FP32 on
// D e = r / ||r|| with preconditioner M (the learned network, or the
// identity); x += ||r|| e in FP64.  A restart is therefore an outer cycle,
// which is where the (residual, error) training pairs of the network are
// taken.  Arnoldi uses classical Gram-Schmidt applied twice (CGS2) with
// FP64-accumulated reductions; the (m+1) x m Hessenberg matrices and their
// Givens rotations are kept per RHS on the host in FP64.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>

#include "solver.h"

namespace dht {

static constexpr int FG_THREADS = 256;
static constexpr int FG_CHUNK = 8;   // basis vectors per reduction pass

// partial[blk][q][r] = sum conj(V_{i0+q}) w over the blocks' vectors (FP32 storage)
__global__ __launch_bounds__(FG_THREADS) void basis_dots_kernel(const float4* V, size_t vstride, int i0, int nq,
                                                                const float4* w, size_t nvec, int B,
                                                                Cx<double>* partial) {
    __shared__ Cx<double> red[FG_CHUNK][FG_THREADS];
    Cx<double> acc[FG_CHUNK];
#pragma unroll
    for (int q = 0; q < FG_CHUNK; q++) acc[q] = cmake(0.0, 0.0);
    const size_t stride = (size_t)gridDim.x * FG_THREADS;
    for (size_t v = (size_t)blockIdx.x * FG_THREADS + threadIdx.x; v < nvec; v += stride) {
        float4 wv = w[v];
#pragma unroll
        for (int q = 0; q < FG_CHUNK; q++) {
            if (q < nq) {
                float4 b = V[(size_t)(i0 + q) * vstride + v];
                acc[q].re += (double)b.x * wv.x + (double)b.y * wv.y + (double)b.z * wv.z + (double)b.w * wv.w;
                acc[q].im += (double)b.x * wv.y - (double)b.y * wv.x + (double)b.z * wv.w - (double)b.w * wv.z;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < FG_CHUNK; q++) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int st = FG_THREADS / 2; st >= B; st >>= 1) {
        if ((int)threadIdx.x < st) {
#pragma unroll
            for (int q = 0; q < FG_CHUNK; q++) red[q][threadIdx.x] = red[q][threadIdx.x] + red[q][threadIdx.x + st];
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < B) {
        for (int q = 0; q < nq; q++) partial[((int64_t)blockIdx.x * nq + q) * B + threadIdx.x] = red[q][threadIdx.x];
    }
}

// w += sign * sum_{i < n} coef[i][r] V_i   (coef complex FP64 on the device)
__global__ void basis_axpy_kernel(float4* w, const float4* V, size_t vstride, int n, const Cx<double>* coef, int B,
                                  size_t nvec, float sign) {
    size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvec) return;
    const int r = (int)(v & (B - 1));
    float4 acc = w[v];
    for (int i = 0; i < n; i++) {
        Cx<double> c = coef[(size_t)i * B + r];
        float cr = sign * (float)c.re, ci = sign * (float)c.im;
        float4 b = V[(size_t)i * vstride + v];
        acc.x += cr * b.x - ci * b.y;
        acc.y += cr * b.y + ci * b.x;
        acc.z += cr * b.z - ci * b.w;
        acc.w += cr * b.w + ci * b.z;
    }
    w[v] = acc;
}

// out = scale[r] * in
__global__ void scale_kernel(float4* out, const float4* in, const double* scale, int B, size_t nvec) {
    size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvec) return;
    float s = (float)scale[v & (B - 1)];
    float4 a = in[v];
    out[v] = make_float4(s * a.x, s * a.y, s * a.z, s * a.w);
}

static dim3 gridv(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

// h[i][r] = V_i^H w for i < n (device result, [n][B])
static int basis_dots(dht_ctx* c, const float4* V, size_t vstride, int n, const float4* w, size_t nvec, int B,
                      Cx<double>* out) {
    void* part;
    DHT_TRY(ws_get(c, WS_PARTIAL, partial_bytes(c, B) * 4, &part));
    const int nb = (int)std::max<size_t>(1, std::min<size_t>((nvec + FG_THREADS - 1) / FG_THREADS, 512));
    for (int i0 = 0; i0 < n; i0 += FG_CHUNK) {
        const int nq = std::min(FG_CHUNK, n - i0);
        hipLaunchKernelGGL(basis_dots_kernel, dim3(nb), dim3(FG_THREADS), 0, c->stream, V, vstride, i0, nq, w, nvec, B,
                           (Cx<double>*)part);
        DHT_HIP(hipGetLastError());
        DHT_TRY(finalize(c, (const Cx<double>*)part, nb, nq, B, nullptr, FIN_SUM, 0.0, out + (size_t)i0 * B));
    }
    return DHT_OK;
}

static int fp32_full_copy_nn(dht_ctx* c, const void* in, void* out, int B, bool use_nn) {
    if (use_nn) return nn_apply_field(c, in, out, B);
    DHT_HIP(hipMemcpyAsync(out, in, full_elems(c, B) * 8, hipMemcpyDeviceToDevice, c->stream));
    return DHT_OK;
}

// One FGMRES(m) cycle in FP32 on D e = b (b has unit norm per active RHS,
// zero otherwise).  e is written; iters receives the Arnoldi steps taken.
static int fgmres_cycle(dht_ctx* c, const void* b, void* e, int B, int m, double tol, bool use_nn,
                        const std::vector<bool>& active, std::vector<int>& iters) {
    const size_t nvec = full_elems(c, B) / 2;   // FP32 vectors (2 complex) per full field
    const size_t fbytes = nvec * 16;
    void *Vb, *Zb, *w, *coef;
    DHT_TRY(ws_get(c, WS_FG_V, fbytes * (m + 1), &Vb));
    DHT_TRY(ws_get(c, WS_FG_Z, fbytes * m, &Zb));
    DHT_TRY(ws_get(c, WS_FG_W, fbytes, &w));
    DHT_TRY(ws_get(c, WS_FG_COEF, sizeof(Cx<double>) * (m + 2) * B * 2, &coef));
    float4* V = (float4*)Vb;
    float4* Z = (float4*)Zb;
    Cx<double>* h1 = (Cx<double>*)coef;
    Cx<double>* h2 = h1 + (size_t)(m + 2) * B;
    typedef std::complex<double> cd;
    std::vector<cd> H((size_t)B * (m + 1) * m, 0.0), gvec((size_t)B * (m + 1), 0.0), cs((size_t)B * m), sn((size_t)B * m);
    std::vector<double> betas(B, 0.0);
    std::vector<bool> live(active);
    for (int r = 0; r < B; r++) {
        gvec[(size_t)r * (m + 1)] = live[r] ? 1.0 : 0.0;
        betas[r] = live[r] ? 1.0 : 0.0;
        iters[r] = 0;
    }
    // v_0 = b (unit norm already)
    DHT_HIP(hipMemcpyAsync(V, b, fbytes, hipMemcpyDeviceToDevice, c->stream));
    std::vector<Cx<double>> hh((size_t)(m + 2) * B * 2);
    int j = 0;
    for (; j < m; j++) {
        bool any = false;
        for (int r = 0; r < B; r++) any |= live[r];
        if (!any) break;
        DHT_TRY(fp32_full_copy_nn(c, V + (size_t)j * nvec, Z + (size_t)j * nvec, B, use_nn));
        DHT_TRY(apply_full(c, DHT_OP_D, DHT_FP32, Z + (size_t)j * nvec, w, B));
        // CGS2
        DHT_TRY(basis_dots(c, V, nvec, j + 1, (const float4*)w, nvec, B, h1));
        hipLaunchKernelGGL(basis_axpy_kernel, gridv(nvec), dim3(256), 0, c->stream, (float4*)w, (const float4*)V, nvec,
                           j + 1, (const Cx<double>*)h1, B, nvec, -1.0f);
        DHT_HIP(hipGetLastError());
        DHT_TRY(basis_dots(c, V, nvec, j + 1, (const float4*)w, nvec, B, h2));
        hipLaunchKernelGGL(basis_axpy_kernel, gridv(nvec), dim3(256), 0, c->stream, (float4*)w, (const float4*)V, nvec,
                           j + 1, (const Cx<double>*)h2, B, nvec, -1.0f);
        DHT_HIP(hipGetLastError());
        // ||w|| (FP64 accumulation)
        DHT_TRY(basis_dots(c, (const float4*)w, 0, 1, (const float4*)w, nvec, B, h2 + (size_t)(j + 1) * B));
        DHT_HIP(hipMemcpyAsync(hh.data(), coef, sizeof(Cx<double>) * (m + 2) * B * 2, hipMemcpyDeviceToHost, c->stream));
        DHT_HIP(hipStreamSynchronize(c->stream));
        std::vector<double> inv(B, 0.0);
        for (int r = 0; r < B; r++) {
            if (!live[r]) continue;
            cd* Hc = &H[((size_t)r * (m + 1)) * m];   // H[row][col] at Hc[row * m + col]
            for (int i = 0; i <= j; i++) {
                Cx<double> a1 = hh[(size_t)i * B + r], a2 = hh[(size_t)(m + 2) * B + (size_t)i * B + r];
                Hc[(size_t)i * m + j] = cd(a1.re + a2.re, a1.im + a2.im);
            }
            double hn = sqrt(std::max(0.0, hh[(size_t)(m + 2) * B + (size_t)(j + 1) * B + r].re));
            Hc[(size_t)(j + 1) * m + j] = hn;
            inv[r] = hn > 0 ? 1.0 / hn : 0.0;
            // apply the previous rotations, then a new one to zero H[j+1][j]
            for (int i = 0; i < j; i++) {
                cd a = Hc[(size_t)i * m + j], bb = Hc[(size_t)(i + 1) * m + j];
                cd C = cs[(size_t)r * m + i], S = sn[(size_t)r * m + i];
                Hc[(size_t)i * m + j] = C * a + S * bb;
                Hc[(size_t)(i + 1) * m + j] = -std::conj(S) * a + std::conj(C) * bb;
            }
            cd a = Hc[(size_t)j * m + j];
            double bn = hn, an = std::abs(a);
            double den = sqrt(an * an + bn * bn);
            cd C = den > 0 ? a / den : 1.0, S = den > 0 ? cd(bn / den, 0.0) : 0.0;
            // rotation [[conj(C), conj(S)], [-S, C]] applied as rows: r1 = conj? use unitary G = [[C*, S*],[-S, C]]
            C = std::conj(C);
            cs[(size_t)r * m + j] = C;
            sn[(size_t)r * m + j] = S;
            Hc[(size_t)j * m + j] = C * a + S * bn;
            Hc[(size_t)(j + 1) * m + j] = 0.0;
            cd gj = gvec[(size_t)r * (m + 1) + j];
            gvec[(size_t)r * (m + 1) + j] = C * gj;
            gvec[(size_t)r * (m + 1) + j + 1] = -std::conj(S) * gj;
            iters[r] = j + 1;
            if (std::abs(gvec[(size_t)r * (m + 1) + j + 1]) <= tol || hn == 0.0) live[r] = false;
        }
        // v_{j+1} = w / ||w||
        DHT_HIP(hipMemcpyAsync(h1, inv.data(), sizeof(double) * B, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(scale_kernel, gridv(nvec), dim3(256), 0, c->stream, V + (size_t)(j + 1) * nvec,
                           (const float4*)w, (const double*)h1, B, nvec);
        DHT_HIP(hipGetLastError());
    }
    // back substitution per RHS: R y = g, then e = Z y
    std::vector<Cx<double>> ycoef((size_t)m * B, cmake(0.0, 0.0));
    for (int r = 0; r < B; r++) {
        const int k = iters[r];
        cd* Hc = &H[((size_t)r * (m + 1)) * m];
        std::vector<cd> y(k);
        for (int i = k - 1; i >= 0; i--) {
            cd s = gvec[(size_t)r * (m + 1) + i];
            for (int l = i + 1; l < k; l++) s -= Hc[(size_t)i * m + l] * y[l];
            y[i] = Hc[(size_t)i * m + i] != 0.0 ? s / Hc[(size_t)i * m + i] : 0.0;
        }
        for (int i = 0; i < k; i++) ycoef[(size_t)i * B + r] = cmake(y[i].real(), y[i].imag());
    }
    DHT_TRY(zero(c, e, fbytes));
    const int kmax = j;
    if (kmax > 0) {
        DHT_HIP(hipMemcpyAsync(coef, ycoef.data(), sizeof(Cx<double>) * kmax * B, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(basis_axpy_kernel, gridv(nvec), dim3(256), 0, c->stream, (float4*)e, (const float4*)Z, nvec,
                           kmax, (const Cx<double>*)coef, B, nvec, 1.0f);
        DHT_HIP(hipGetLastError());
    }
    return DHT_OK;
}

// FP64 full-field helpers built from the generic kernels
static int full_norms2(dht_ctx* c, const void* f, int B, std::vector<double>& out) {
    void* d;
    DHT_TRY(ws_get(c, WS_SCAL2, sizeof(Cx<double>) * 3 * B, &d));
    const void* aa[1] = {f};
    DHT_TRY(dots(c, DHT_FP64, 1, aa, aa, full_elems(c, B), B, (Cx<double>*)d));
    std::vector<Cx<double>> h(B);
    DHT_HIP(hipMemcpyAsync(h.data(), d, sizeof(Cx<double>) * B, hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    out.resize(B);
    for (int i = 0; i < B; i++) out[i] = h[i].re;
    return DHT_OK;
}

// full FP64 field <-> full FP32 field (scaled per RHS), through the half-field helpers
static int full_scale_down(dht_ctx* c, const void* in64, void* out32, const double* scale, int B) {
    const size_t h64 = half_elems(c, B) * 16, h32 = half_elems(c, B) * 8;
    DHT_TRY(scale_down(c, in64, out32, DHT_FP32, scale, B));
    DHT_TRY(scale_down(c, (const char*)in64 + h64, (char*)out32 + h32, DHT_FP32, scale, B));
    return DHT_OK;
}
static int full_accum_up(dht_ctx* c, void* x64, const void* e32, const double* scale, int B) {
    const size_t h64 = half_elems(c, B) * 16, h32 = half_elems(c, B) * 8;
    DHT_TRY(accum_up(c, x64, e32, DHT_FP32, scale, B));
    DHT_TRY(accum_up(c, (char*)x64 + h64, (const char*)e32 + h32, DHT_FP32, scale, B));
    return DHT_OK;
}

// one RHS slot of full FP64 fields -> canonical: R = sr * r, E = sr * (xs - x)
__global__ void pair_kernel(const Cx<double>* r, const Cx<double>* xs, const Cx<double>* x, int B, int slot, double sr,
                            Geom g, Cx<double>* R, Cx<double>* E) {
    int64_t ps = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (p, s)
    if (ps >= g.V) return;
    int p = (int)(ps / g.Vh);
    int64_t s = ps - (int64_t)p * g.Vh;
    int cc[4];
    cb_coords(g, s, p, cc);
    int64_t site = lex_index(g, cc);
    for (int comp = 0; comp < 12; comp++) {
        int64_t v = (((int64_t)p * 12 + comp) * g.Vh + s) * B + slot;
        Cx<double> rv = r[v], d = xs[v] - x[v];
        R[site * 12 + comp] = cmake(sr * rv.re, sr * rv.im);
        E[site * 12 + comp] = cmake(sr * d.re, sr * d.im);
    }
}

int PairSink::take(dht_ctx* c, const void* r, const void* x, const std::vector<bool>& act,
                   const std::vector<double>& rn2) {
    const int B = (int)act.size();
    const int64_t N = 12 * c->g.V;
    for (int i = 0; i < nreal && i < B; i++) {
        if (!act[i] || count >= cap || !(rn2[i] > 0)) continue;
        hipLaunchKernelGGL(pair_kernel, dim3((unsigned)((c->g.V + 255) / 256)), dim3(256), 0, c->stream,
                           (const Cx<double>*)r, (const Cx<double>*)xstar, (const Cx<double>*)x, B, i,
                           1.0 / sqrt(rn2[i]), c->g, (Cx<double>*)R + (int64_t)count * N,
                           (Cx<double>*)E + (int64_t)count * N);
        DHT_HIP(hipGetLastError());
        count++;
    }
    return DHT_OK;
}

void ws_plan_fgmres(const dht_ctx* c, const dht_solver_params* prm, int B, bool use_nn, size_t* plan) {
    const int m = prm->restart > 0 ? std::min(prm->restart, 64) : 32;
    const size_t fb = full_elems(c, B) * 16, fbytes = full_elems(c, B) / 2 * 16;
    plan_max(plan, WS_RE, fb);
    plan_max(plan, WS_XF, fb);
    plan_max(plan, WS_FLAGS, sizeof(double) * B);
    plan_max(plan, WS_FG_R, fb / 2);
    plan_max(plan, WS_FG_E, fb / 2);
    plan_max(plan, WS_SCAL2, sizeof(Cx<double>) * 3 * B);
    plan_max(plan, WS_FG_V, fbytes * (m + 1));
    plan_max(plan, WS_FG_Z, fbytes * m);
    plan_max(plan, WS_FG_W, fbytes);
    plan_max(plan, WS_FG_COEF, sizeof(Cx<double>) * (m + 2) * B * 2);
    ws_plan_dots(c, B, plan);
    plan_max(plan, WS_PARTIAL, partial_bytes(c, B) * 4);   // the basis dots
    if (use_nn) plan_max(plan, WS_NN_ACT, nn_infer_bytes(c, B));
}

int solve_fgmres(dht_ctx* c, const dht_solver_params* prm, const void* Z, void* X, int B, dht_solve_stats* stats,
                 bool use_nn, PairSink* sink) {
    if (use_nn && !c->nn.ready) return set_error(DHT_ERR_STATE, "network not initialised");
    const int m = prm->restart > 0 ? std::min(prm->restart, 64) : 32;
    const size_t fb = full_elems(c, B) * 16;
    void *r, *tmp, *scl, *rlo, *elo;
    DHT_TRY(ws_get(c, WS_RE, fb, &r));
    DHT_TRY(ws_get(c, WS_XF, fb, &tmp));
    DHT_TRY(ws_get(c, WS_FLAGS, sizeof(double) * B, &scl));
    DHT_TRY(ws_get(c, WS_FG_R, fb / 2, &rlo));
    DHT_TRY(ws_get(c, WS_FG_E, fb / 2, &elo));
    std::vector<double> zn2, rn2;
    DHT_TRY(full_norms2(c, Z, B, zn2));
    DHT_TRY(zero(c, X, fb));
    DHT_HIP(hipMemcpyAsync(r, Z, fb, hipMemcpyDeviceToDevice, c->stream));
    const int max_outer = prm->max_outer > 0 ? prm->max_outer : 200;
    const double itol = prm->inner_tol > 0 ? prm->inner_tol : 1e-5;
    std::vector<int> iters(B, 0), it(B, 0);
    int outer = 0, total = 0;
    for (; outer < max_outer; outer++) {
        DHT_TRY(full_norms2(c, r, B, rn2));
        std::vector<bool> act(B);
        std::vector<double> sdown(B), sup(B);
        bool any = false;
        for (int i = 0; i < B; i++) {
            act[i] = rn2[i] > prm->tol * prm->tol * zn2[i] * 0.81 && std::isfinite(rn2[i]);
            any |= act[i];
            sdown[i] = act[i] ? 1.0 / sqrt(rn2[i]) : 0.0;
            sup[i] = act[i] ? sqrt(rn2[i]) : 0.0;
        }
        if (!any || total >= prm->maxiter) break;
        if (sink) DHT_TRY(sink->take(c, r, X, act, rn2));
        DHT_HIP(hipMemcpyAsync(scl, sdown.data(), sizeof(double) * B, hipMemcpyHostToDevice, c->stream));
        DHT_TRY(full_scale_down(c, r, rlo, (const double*)scl, B));
        DHT_TRY(fgmres_cycle(c, rlo, elo, B, m, itol, use_nn, act, it));
        int mx = 0;
        for (int i = 0; i < B; i++) {
            iters[i] += it[i];
            mx = std::max(mx, it[i]);
        }
        total += std::max(mx, 1);
        DHT_HIP(hipMemcpyAsync(scl, sup.data(), sizeof(double) * B, hipMemcpyHostToDevice, c->stream));
        DHT_TRY(full_accum_up(c, X, elo, (const double*)scl, B));
        DHT_TRY(apply_full(c, DHT_OP_D, DHT_FP64, X, tmp, B));
        DHT_TRY(sub(c, Z, tmp, r, full_elems(c, B)));
    }
    DHT_TRY(full_norms2(c, r, B, rn2));
    bool ok_all = true;
    for (int i = 0; i < B; i++) {
        double rr = zn2[i] > 0 ? sqrt(rn2[i] / zn2[i]) : 0.0;
        bool ok = rr <= prm->tol || zn2[i] == 0.0;
        ok_all &= ok;
        if (stats) {
            stats[i].iters = iters[i];
            stats[i].outer = outer;
            stats[i].true_resid = rr;
            stats[i].status = ok ? DHT_STATUS_CONVERGED : DHT_STATUS_NOT_CONVERGED;
        }
    }
    return ok_all ? DHT_OK : set_error(DHT_ERR_NOT_CONVERGED, "some right-hand sides did not reach the tolerance");
}

}  // namespace dht
