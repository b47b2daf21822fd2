// Deflation of the trace estimator (Section 5.2; Algorithm 1, lines 1-2 and 8).
//
// With k eigenvectors W of the Hermitian Q = g5 D (stored rounded to FP64,
// FP32 or BF16), the deflated part of D^-1 = Q^-1 g5 is P = W M W^H g5 with
// M = (W^H Q W)^-1, the Galerkin inverse of Q on span(W) (equal to Lambda^-1
// for exact orthonormal eigenvectors, i.e. V Sigma^-1 U^H of Section 5.2).
// H = W^H Q W and the trace T_D = Tr(P) = Tr(M W^H g5 W) are accumulated in
// FP64 from the stored vectors, so the estimator stays unbiased whatever the
// storage precision: only its variance depends on how good W is.
//
// Per probe: c1 = W^H z and c2 = W^H g5 z (g5 = +1 on spins 0, 1 and -1 on
// spins 2, 3 in the chiral basis, so both come from one pass over W), and
// z^H P z = c1^H M c2.
//
// Storage: W is k full internal fields with one RHS each, column after
// column: [k][2 parity][12][Vh] complex in the storage precision.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>

#include "solver.h"

namespace dht {

static constexpr int PROJ_THREADS = 256;
static constexpr int PROJ_RT = 4;    // right-hand sides per pass

// partial[(chunk * k + i) * B + r] for c1 and c2 (two arrays)
template <typename SW, typename SZ>
__global__ __launch_bounds__(PROJ_THREADS) void proj_generic_kernel(const typename Store<SW>::elem* W,
                                                                    const typename Store<SZ>::elem* Z, int64_t Kn,
                                                                    int64_t per_comp_w, int B, int r0, int nr,
                                                                    int64_t chunk, Cx<double>* p1, Cx<double>* p2,
                                                                    int k) {
    __shared__ Cx<double> red[2 * PROJ_RT][PROJ_THREADS];
    const int i = blockIdx.y;
    const int64_t cbeg = (int64_t)blockIdx.x * chunk;
    const int64_t cend = cbeg + chunk < Kn ? cbeg + chunk : Kn;
    const typename Store<SW>::elem* w = W + (int64_t)i * Kn;
    Cx<double> a1[PROJ_RT], a2[PROJ_RT];
#pragma unroll
    for (int q = 0; q < PROJ_RT; q++) a1[q] = a2[q] = cmake(0.0, 0.0);
    for (int64_t K = cbeg + threadIdx.x; K < cend; K += PROJ_THREADS) {
        auto wv = Store<SW>::ld(w + K);
        Cx<double> wd = cmake<double>(wv.re, wv.im);
        // component index of K within its parity block [12][Vh]
        int comp = (int)((K / per_comp_w) % 12);
        double sg = comp < 6 ? 1.0 : -1.0;
        const typename Store<SZ>::elem* zp = Z + K * B + r0;
#pragma unroll
        for (int q = 0; q < PROJ_RT; q++) {
            if (q < nr) {
                auto zv = Store<SZ>::ld(zp + q);
                Cx<double> pr = conjmul(wd, cmake<double>(zv.re, zv.im));
                a1[q] = a1[q] + pr;
                a2[q] = a2[q] + sg * pr;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PROJ_RT; q++) {
        red[q][threadIdx.x] = a1[q];
        red[PROJ_RT + q][threadIdx.x] = a2[q];
    }
    __syncthreads();
    for (int st = PROJ_THREADS / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
#pragma unroll
            for (int q = 0; q < 2 * PROJ_RT; q++) red[q][threadIdx.x] = red[q][threadIdx.x] + red[q][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < nr) {
        int q = threadIdx.x;
        p1[((int64_t)blockIdx.x * k + i) * B + r0 + q] = red[q][0];
        p2[((int64_t)blockIdx.x * k + i) * B + r0 + q] = red[PROJ_RT + q][0];
    }
}

__global__ void proj_sum_kernel(const Cx<double>* p1, const Cx<double>* p2, int nchunk, int k, int B, Cx<double>* c1,
                                Cx<double>* c2) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= k * B) return;
    Cx<double> s1 = cmake(0.0, 0.0), s2 = cmake(0.0, 0.0);
    for (int ch = 0; ch < nchunk; ch++) {
        s1 = s1 + p1[(int64_t)ch * k * B + idx];
        s2 = s2 + p2[(int64_t)ch * k * B + idx];
    }
    c1[idx] = s1;
    c2[idx] = s2;
}

// c1, c2 (device, [k][B] complex) for a full internal field Z of precision zprec.
int project_field(dht_ctx* c, const void* Z, int zprec, int nrhs, Cx<double>* c1, Cx<double>* c2) {
    if (!c->W || c->k <= 0) return set_error(DHT_ERR_STATE, "no deflation basis");
    const int64_t Kn = 24 * c->g.Vh;   // complex entries per column
    const int k = c->k;
    int64_t chunk = 8192;
    int nchunk = (int)((Kn + chunk - 1) / chunk);
    while (nchunk > 256) {
        chunk *= 2;
        nchunk = (int)((Kn + chunk - 1) / chunk);
    }
    void *p1, *p2;
    size_t pb = (size_t)nchunk * k * nrhs * sizeof(Cx<double>);
    DHT_TRY(ws_get(c, WS_PROJ, pb, &p1));
    DHT_TRY(ws_get(c, WS_PROJ2, pb, &p2));
    for (int r0 = 0; r0 < nrhs; r0 += PROJ_RT) {
        int nr = std::min(PROJ_RT, nrhs - r0);
        dim3 grid(nchunk, k), block(PROJ_THREADS);
#define DHT_PG(PW, TW, PZ, TZ)                                                                                      \
    if (c->wprec == PW && zprec == PZ) {                                                                            \
        hipLaunchKernelGGL((proj_generic_kernel<TW, TZ>), grid, block, 0, c->stream,                                \
                           (const typename Store<TW>::elem*)c->W, (const typename Store<TZ>::elem*)Z, Kn,           \
                           (int64_t)c->g.Vh, nrhs, r0, nr, chunk, (Cx<double>*)p1, (Cx<double>*)p2, k);              \
        goto done;                                                                                                  \
    }
        DHT_PG(DHT_FP64, double, DHT_FP64, double)
        DHT_PG(DHT_FP32, float, DHT_FP64, double)
        DHT_PG(DHT_BF16, bf16x2, DHT_FP64, double)
#undef DHT_PG
        return set_error(DHT_ERR_INVALID_ARG, "unsupported projection precision pair");
    done:
        DHT_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(proj_sum_kernel, dim3((k * nrhs + 127) / 128), dim3(128), 0, c->stream, (const Cx<double>*)p1,
                       (const Cx<double>*)p2, nchunk, k, nrhs, c1, c2);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// ---------------------------------------------------------------------------
// basis management
// ---------------------------------------------------------------------------
static size_t col_bytes(dht_ctx* c) { return full_elems(c, 1) * elem_bytes(c->wprec); }

int deflation_begin(dht_ctx* c, int k, int prec) {
    if (k <= 0) return set_error(DHT_ERR_INVALID_ARG, "k must be positive");
    if (prec < DHT_FP64 || prec > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    if (c->W) {
        DHT_HIP(hipStreamSynchronize(c->stream));
        DHT_HIP(hipFree(c->W));
        c->W = nullptr;
    }
    c->k = k;
    c->wprec = prec;
    c->defl_ready = false;
    c->TD[0] = c->TD[1] = 0;
    size_t bytes = (size_t)k * full_elems(c, 1) * elem_bytes(prec);
    if (hipMalloc(&c->W, bytes) != hipSuccess) {
        c->W = nullptr;
        c->k = 0;
        (void)hipGetLastError();
        return set_error(DHT_ERR_OOM, "cannot allocate the deflation basis");
    }
    DHT_TRY(zero(c, c->W, bytes));
    return DHT_OK;
}

int deflation_set(dht_ctx* c, int first, int count, const double* W_dev) {
    if (!c->W) return set_error(DHT_ERR_STATE, "call dht_deflation_begin first");
    if (first < 0 || count < 0 || first + count > c->k) return set_error(DHT_ERR_INVALID_ARG, "column range");
    const int64_t N = 12 * c->g.V;
    for (int j = 0; j < count; j++)
        DHT_TRY(pack_spinor(c, W_dev + 2 * N * j, (char*)c->W + (size_t)(first + j) * col_bytes(c), c->wprec, 1));
    c->defl_ready = false;
    return DHT_OK;
}

// In-place inverse of an n x n complex matrix (row-major) by Gauss-Jordan
// elimination with partial pivoting.  Returns false if singular.
static bool invert(std::vector<std::complex<double>>& A, int n) {
    std::vector<int> piv(n);
    for (int i = 0; i < n; i++) piv[i] = i;
    std::vector<std::complex<double>> I(n * (size_t)n, 0.0);
    for (int i = 0; i < n; i++) I[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; col++) {
        int best = col;
        double bv = std::abs(A[(size_t)col * n + col]);
        for (int r = col + 1; r < n; r++) {
            double v = std::abs(A[(size_t)r * n + col]);
            if (v > bv) { bv = v; best = r; }
        }
        if (bv == 0.0 || !std::isfinite(bv)) return false;
        if (best != col) {
            for (int j = 0; j < n; j++) {
                std::swap(A[(size_t)col * n + j], A[(size_t)best * n + j]);
                std::swap(I[(size_t)col * n + j], I[(size_t)best * n + j]);
            }
        }
        std::complex<double> d = 1.0 / A[(size_t)col * n + col];
        for (int j = 0; j < n; j++) {
            A[(size_t)col * n + j] *= d;
            I[(size_t)col * n + j] *= d;
        }
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            std::complex<double> f = A[(size_t)r * n + col];
            if (f == 0.0) continue;
            for (int j = 0; j < n; j++) {
                A[(size_t)r * n + j] -= f * A[(size_t)col * n + j];
                I[(size_t)r * n + j] -= f * I[(size_t)col * n + j];
            }
        }
    }
    A.swap(I);
    return true;
}

int deflation_finalize(dht_ctx* c) {
    if (!c->W) return set_error(DHT_ERR_STATE, "no deflation basis");
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    const int k = c->k;
    const int nb = std::min(k, 32);
    const size_t fb = full_elems(c, nb) * 16;
    void *wb, *qwb, *cc;
    DHT_TRY(ws_get(c, WS_QW, fb, &wb));
    DHT_TRY(ws_get(c, WS_XF, fb, &qwb));
    DHT_TRY(ws_get(c, WS_COEF, sizeof(Cx<double>) * 4 * k * nb, &cc));
    Cx<double>* h1 = (Cx<double>*)cc;            // W^H (Q Wb)
    Cx<double>* h2 = h1 + (size_t)k * nb;         // W^H g5 (Q Wb)   (unused)
    Cx<double>* g1 = h2 + (size_t)k * nb;         // W^H Wb
    Cx<double>* g5m = g1 + (size_t)k * nb;        // W^H g5 Wb
    std::vector<std::complex<double>> H((size_t)k * k), G5((size_t)k * k);
    std::vector<Cx<double>> hb((size_t)4 * k * nb);
    const size_t cb = col_bytes(c);
    for (int j0 = 0; j0 < k; j0 += nb) {
        int n = std::min(nb, k - j0);
        // gather columns j0.. into an FP64 field with n RHS (RHS innermost)
        DHT_TRY(gather_columns(c, (const char*)c->W + (size_t)j0 * cb, c->wprec, n, wb));
        DHT_TRY(apply_full(c, DHT_OP_Q, DHT_FP64, wb, qwb, n));
        DHT_TRY(project_field(c, qwb, DHT_FP64, n, h1, h2));
        DHT_TRY(project_field(c, wb, DHT_FP64, n, g1, g5m));
        DHT_HIP(hipMemcpyAsync(hb.data(), cc, sizeof(Cx<double>) * 4 * k * nb, hipMemcpyDeviceToHost, c->stream));
        DHT_HIP(hipStreamSynchronize(c->stream));
        // blocks are [k][n] with stride n inside this batch
        for (int i = 0; i < k; i++)
            for (int jj = 0; jj < n; jj++) {
                Cx<double> hv = hb[(size_t)i * n + jj];
                Cx<double> gv = hb[(size_t)3 * k * nb + (size_t)i * n + jj];
                H[(size_t)i * k + j0 + jj] = std::complex<double>(hv.re, hv.im);
                G5[(size_t)i * k + j0 + jj] = std::complex<double>(gv.re, gv.im);
            }
    }
    // H is Hermitian in exact arithmetic: use its Hermitian part
    for (int i = 0; i < k; i++)
        for (int j = i; j < k; j++) {
            std::complex<double> a = 0.5 * (H[(size_t)i * k + j] + std::conj(H[(size_t)j * k + i]));
            H[(size_t)i * k + j] = a;
            H[(size_t)j * k + i] = std::conj(a);
        }
    if (!invert(H, k)) return set_error(DHT_ERR_BREAKDOWN, "W^H Q W is singular");
    std::complex<double> td = 0.0;
    for (int a = 0; a < k; a++)
        for (int b = 0; b < k; b++) td += H[(size_t)a * k + b] * G5[(size_t)b * k + a];
    c->M.assign((size_t)2 * k * k, 0.0);
    for (size_t i = 0; i < (size_t)k * k; i++) {
        c->M[2 * i] = H[i].real();
        c->M[2 * i + 1] = H[i].imag();
    }
    c->TD[0] = td.real();
    c->TD[1] = td.imag();
    c->defl_ready = true;
    return DHT_OK;
}

// d_j = c1_j^H M c2_j on the host (c1, c2 host arrays [k][B] complex)
void deflation_corrections(const dht_ctx* c, const Cx<double>* c1, const Cx<double>* c2, int B, double* dre,
                           double* dim) {
    const int k = c->k;
    const std::complex<double>* M = (const std::complex<double>*)c->M.data();
    std::vector<std::complex<double>> v(k);
    for (int r = 0; r < B; r++) {
        for (int a = 0; a < k; a++) {
            std::complex<double> s = 0.0;
            for (int b = 0; b < k; b++) s += M[(size_t)a * k + b] * std::complex<double>(c2[(size_t)b * B + r].re, c2[(size_t)b * B + r].im);
            v[a] = s;
        }
        std::complex<double> d = 0.0;
        for (int a = 0; a < k; a++) d += std::conj(std::complex<double>(c1[(size_t)a * B + r].re, c1[(size_t)a * B + r].im)) * v[a];
        dre[r] = d.real();
        dim[r] = d.imag();
    }
}

// ---------------------------------------------------------------------------
// column gather: n consecutive B=1 columns (precision wp) -> FP64 field [2][12][Vh][n]
// ---------------------------------------------------------------------------
template <typename SW>
__global__ void gather_kernel(const typename Store<SW>::elem* W, int64_t Kn, int n, Cx<double>* out) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= Kn * n) return;
    int64_t K = gid / n;
    int j = (int)(gid - K * n);
    auto v = Store<SW>::ld(W + (int64_t)j * Kn + K);
    out[gid] = cmake<double>(v.re, v.im);
}

int gather_columns(dht_ctx* c, const void* W, int wprec, int n, void* out) {
    const int64_t Kn = 24 * c->g.Vh;
    int64_t tot = Kn * n;
    dim3 grid((unsigned)((tot + 255) / 256)), block(256);
    switch (wprec) {
        case DHT_FP64: hipLaunchKernelGGL(gather_kernel<double>, grid, block, 0, c->stream, (const Cx<double>*)W, Kn, n, (Cx<double>*)out); break;
        case DHT_FP32: hipLaunchKernelGGL(gather_kernel<float>, grid, block, 0, c->stream, (const Cx<float>*)W, Kn, n, (Cx<double>*)out); break;
        case DHT_BF16: hipLaunchKernelGGL(gather_kernel<bf16x2>, grid, block, 0, c->stream, (const bf16x2*)W, Kn, n, (Cx<double>*)out); break;
        default: return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

}  // namespace dht
