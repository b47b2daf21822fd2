// Deflation basis: eigenvectors of Q = g5 D with the smallest |lambda|
// (Section 5.1: the singular triplets of D follow from the eigenpairs of the
// Hermitian Q, sigma = |lambda|, u = g5 v sign(lambda)).
//
// Chebyshev-filtered subspace iteration in FP64.  Q^2 = D^H D has the wanted
// vectors at the bottom of its spectrum, so a Chebyshev polynomial in Q^2 that
// is bounded on [a, b] (b >= ||Q||^2, a = the largest Ritz value of Q^2 in the
// current block) amplifies them; after each filter the block is
// orthonormalised (Cholesky QR, twice); a Rayleigh-Ritz step with Q^2 orders
// the block and one with Q on its converging leading part separates
// eigenvalues of opposite sign.  Convergence is tested on the true
// residuals ||Q w - lambda w|| of the k Ritz pairs of smallest |lambda|.
//
// Block vectors are internal FP64 full fields of nb right-hand sides, i.e.
// N x nb row-major complex matrices; Gram matrices, rotations and residual
// norms are tall-skinny kernels below, the small nb x nb eigenproblems and
// factorisations run on the host in FP64.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "solver.h"

namespace dht {

static constexpr int EG_T = 32;        // tile of the Gram / rotation kernels
static constexpr int EG_THREADS = 256;
static constexpr int EG_SPLITS = 64;   // row splits of a Gram product

// partial[s][i][j] = sum over rows of split s of conj(X[r][i]) Y[r][j]
__global__ __launch_bounds__(EG_THREADS) void eig_gram_kernel(const Cx<double>* X, const Cx<double>* Y, int64_t nrows,
                                                             int nb, Cx<double>* partial) {
    __shared__ Cx<double> xs[EG_T][EG_T + 1], ys[EG_T][EG_T + 1];
    const int i0 = blockIdx.x * EG_T, j0 = blockIdx.y * EG_T, s = blockIdx.z;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t rps = (nrows + gridDim.z - 1) / gridDim.z;
    const int64_t r0 = s * rps, r1 = std::min<int64_t>(nrows, r0 + rps);
    Cx<double> acc[2][2];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) acc[a][b] = cmake(0.0, 0.0);
    for (int64_t rb = r0; rb < r1; rb += EG_T) {
        for (int e = threadIdx.x; e < EG_T * EG_T; e += EG_THREADS) {
            const int rr = e / EG_T, cc = e % EG_T;
            const int64_t r = rb + rr;
            const bool ok = r < r1;
            xs[rr][cc] = ok ? X[r * nb + i0 + cc] : cmake(0.0, 0.0);
            ys[rr][cc] = ok ? Y[r * nb + j0 + cc] : cmake(0.0, 0.0);
        }
        __syncthreads();
        for (int rr = 0; rr < EG_T; rr++) {
            const Cx<double> x0 = xs[rr][2 * ty], x1 = xs[rr][2 * ty + 1];
            const Cx<double> y0 = ys[rr][2 * tx], y1 = ys[rr][2 * tx + 1];
            acc[0][0] = acc[0][0] + conjmul(x0, y0);
            acc[0][1] = acc[0][1] + conjmul(x0, y1);
            acc[1][0] = acc[1][0] + conjmul(x1, y0);
            acc[1][1] = acc[1][1] + conjmul(x1, y1);
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            partial[((int64_t)s * nb + i0 + 2 * ty + a) * nb + j0 + 2 * tx + b] = acc[a][b];
}

__global__ void eig_gram_sum_kernel(const Cx<double>* partial, int nb, int nsplit, Cx<double>* G) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nb * nb) return;
    Cx<double> s = cmake(0.0, 0.0);
    for (int k = 0; k < nsplit; k++) s = s + partial[(int64_t)k * nb * nb + e];
    G[e] = s;
}

// Z[r][j] = sum_i X[r][i] C[i][j]   (X: nrows x nb, C: nb x nb row-major, Z != X)
__global__ __launch_bounds__(EG_THREADS) void eig_rotate_kernel(const Cx<double>* X, const Cx<double>* C, int64_t nrows,
                                                               int nb, Cx<double>* Z) {
    __shared__ Cx<double> xs[EG_T][EG_T + 1], cs[EG_T][EG_T + 1];
    const int64_t r0 = (int64_t)blockIdx.x * EG_T;
    const int j0 = blockIdx.y * EG_T;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    Cx<double> acc[2][2];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) acc[a][b] = cmake(0.0, 0.0);
    for (int ib = 0; ib < nb; ib += EG_T) {
        for (int e = threadIdx.x; e < EG_T * EG_T; e += EG_THREADS) {
            const int rr = e / EG_T, cc = e % EG_T;
            const int64_t r = r0 + rr;
            xs[rr][cc] = r < nrows ? X[r * nb + ib + cc] : cmake(0.0, 0.0);
            cs[rr][cc] = C[(int64_t)(ib + rr) * nb + j0 + cc];
        }
        __syncthreads();
        for (int ii = 0; ii < EG_T; ii++) {
            const Cx<double> x0 = xs[2 * ty][ii], x1 = xs[2 * ty + 1][ii];
            const Cx<double> c0 = cs[ii][2 * tx], c1 = cs[ii][2 * tx + 1];
            acc[0][0] = acc[0][0] + x0 * c0;
            acc[0][1] = acc[0][1] + x0 * c1;
            acc[1][0] = acc[1][0] + x1 * c0;
            acc[1][1] = acc[1][1] + x1 * c1;
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; a++) {
        const int64_t r = r0 + 2 * ty + a;
        if (r < nrows)
            for (int b = 0; b < 2; b++) Z[r * nb + j0 + 2 * tx + b] = acc[a][b];
    }
}

// Z = a X + b Y + c W elementwise (Y, W may be null)
__global__ void eig_lincomb_kernel(Cx<double>* Z, double a, const Cx<double>* X, double b, const Cx<double>* Y, double c,
                                   const Cx<double>* W, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        Cx<double> v = a * X[e];
        if (Y) v = v + b * Y[e];
        if (W) v = v + c * W[e];
        Z[e] = v;
    }
}

// partial[blk][j] = sum over the block's rows of |W[r][j] - lambda_j V[r][j]|^2
__global__ __launch_bounds__(EG_THREADS) void eig_resid_kernel(const Cx<double>* W, const Cx<double>* V,
                                                              const double* lam, int64_t nrows, int nb,
                                                              double* partial) {
    __shared__ double red[EG_THREADS];
    const int slots = EG_THREADS / nb;   // rows handled side by side (nb divides 256)
    const int j = threadIdx.x % nb, slot = threadIdx.x / nb;
    const double l = lam[j];
    double s = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * slots + slot; r < nrows; r += (int64_t)gridDim.x * slots) {
        const Cx<double> d = W[r * nb + j] - l * V[r * nb + j];
        s += d.re * d.re + d.im * d.im;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (slot == 0) {
        for (int q = 1; q < slots; q++) s += red[q * nb + j];
        partial[(int64_t)blockIdx.x * nb + j] = s;
    }
}

// ---------------------------------------------------------------------------
// host FP64 dense helpers (nb x nb, row-major complex)
// ---------------------------------------------------------------------------
typedef std::vector<Cx<double>> CMat;

static inline Cx<double> cconj(Cx<double> a) { return cmake(a.re, -a.im); }

// Cholesky G = L L^H (lower); returns false if G is not positive definite
static bool cholesky(const CMat& G, int n, CMat& L) {
    L.assign((size_t)n * n, cmake(0.0, 0.0));
    for (int j = 0; j < n; j++) {
        double d = G[(size_t)j * n + j].re;
        for (int k = 0; k < j; k++) d -= L[(size_t)j * n + k].re * L[(size_t)j * n + k].re +
                                         L[(size_t)j * n + k].im * L[(size_t)j * n + k].im;
        if (!(d > 0.0)) return false;
        const double ljj = std::sqrt(d);
        L[(size_t)j * n + j] = cmake(ljj, 0.0);
        for (int i = j + 1; i < n; i++) {
            Cx<double> s = G[(size_t)i * n + j];
            for (int k = 0; k < j; k++) s = s - L[(size_t)i * n + k] * cconj(L[(size_t)j * n + k]);
            L[(size_t)i * n + j] = (1.0 / ljj) * s;
        }
    }
    return true;
}

// C = L^{-H} (upper triangular), so that X C has orthonormal columns when X^H X = L L^H
static void inv_lower_h(const CMat& L, int n, CMat& C) {
    CMat Li((size_t)n * n, cmake(0.0, 0.0));   // L^{-1}, lower
    for (int j = 0; j < n; j++) {
        Li[(size_t)j * n + j] = cmake(1.0 / L[(size_t)j * n + j].re, 0.0);
        for (int i = j + 1; i < n; i++) {
            Cx<double> s = cmake(0.0, 0.0);
            for (int k = j; k < i; k++) s = s + L[(size_t)i * n + k] * Li[(size_t)k * n + j];
            Li[(size_t)i * n + j] = (-1.0 / L[(size_t)i * n + i].re) * s;
        }
    }
    C.assign((size_t)n * n, cmake(0.0, 0.0));
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) C[(size_t)i * n + j] = cconj(Li[(size_t)j * n + i]);
}

// Cyclic Jacobi for a Hermitian matrix: A = V diag(w) V^H, w ascending
static void jacobi_eigh(CMat A, int n, std::vector<double>& w, CMat& V) {
    V.assign((size_t)n * n, cmake(0.0, 0.0));
    for (int i = 0; i < n; i++) V[(size_t)i * n + i] = cmake(1.0, 0.0);
    auto at = [&](int i, int j) -> Cx<double>& { return A[(size_t)i * n + j]; };
    double fro = 0.0;
    for (auto& e : A) fro += e.re * e.re + e.im * e.im;
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0.0;
        for (int i = 0; i < n; i++)
            for (int j = i + 1; j < n; j++) off += at(i, j).re * at(i, j).re + at(i, j).im * at(i, j).im;
        if (off <= 1e-32 * fro || off == 0.0) break;
        for (int p = 0; p < n - 1; p++)
            for (int q = p + 1; q < n; q++) {
                const Cx<double> apq = at(p, q);
                const double mag = std::sqrt(apq.re * apq.re + apq.im * apq.im);
                if (mag == 0.0) continue;
                // phase: with P = diag(1, e^{-i phi}) the (p, q) entry becomes |apq|
                const Cx<double> ph = cmake(apq.re / mag, -apq.im / mag);   // e^{-i phi}
                const double app = at(p, p).re, aqq = at(q, q).re;
                const double zeta = (aqq - app) / (2.0 * mag);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // U acting on columns p, q: U = P R, R = [[c, s], [-s, c]]
                const Cx<double> upp = cmake(c, 0.0), upq = cmake(s, 0.0);
                const Cx<double> uqp = (-s) * ph, uqq = c * ph;
                for (int k = 0; k < n; k++) {   // A <- A U
                    const Cx<double> akp = at(k, p), akq = at(k, q);
                    at(k, p) = akp * upp + akq * uqp;
                    at(k, q) = akp * upq + akq * uqq;
                }
                for (int k = 0; k < n; k++) {   // A <- U^H A
                    const Cx<double> apk = at(p, k), aqk = at(q, k);
                    at(p, k) = cconj(upp) * apk + cconj(uqp) * aqk;
                    at(q, k) = cconj(upq) * apk + cconj(uqq) * aqk;
                }
                at(p, q) = cmake(0.0, 0.0);
                at(q, p) = cmake(0.0, 0.0);
                for (int k = 0; k < n; k++) {   // V <- V U
                    const Cx<double> vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = vkp * upp + vkq * uqp;
                    V[(size_t)k * n + q] = vkp * upq + vkq * uqq;
                }
            }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; i++) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return at(a, a).re < at(b, b).re; });
    CMat Vs((size_t)n * n);
    w.resize(n);
    for (int jj = 0; jj < n; jj++) {
        w[jj] = at(idx[jj], idx[jj]).re;
        for (int i = 0; i < n; i++) Vs[(size_t)i * n + jj] = V[(size_t)i * n + idx[jj]];
    }
    V.swap(Vs);
}

// ---------------------------------------------------------------------------
// device block operations
// ---------------------------------------------------------------------------
struct EigWork {
    int64_t rows;   // N
    int nb;
    Cx<double>* part;    // Gram partials [EG_SPLITS][nb][nb]
    Cx<double>* small;   // nb x nb matrix on the device
    double* rpart;       // residual partials
    double* lam;         // nb values on the device
    int rblocks;
};

static int gram(dht_ctx* c, const EigWork& w, const Cx<double>* X, const Cx<double>* Y, CMat& G) {
    dim3 grid(w.nb / EG_T, w.nb / EG_T, EG_SPLITS);
    hipLaunchKernelGGL(eig_gram_kernel, grid, dim3(EG_THREADS), 0, c->stream, X, Y, w.rows, w.nb, w.part);
    DHT_HIP(hipGetLastError());
    const int nn = w.nb * w.nb;
    hipLaunchKernelGGL(eig_gram_sum_kernel, dim3((nn + 255) / 256), dim3(256), 0, c->stream, w.part, w.nb, EG_SPLITS,
                       w.small);
    DHT_HIP(hipGetLastError());
    G.resize(nn);
    DHT_HIP(hipMemcpyAsync(G.data(), w.small, sizeof(Cx<double>) * nn, hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    return DHT_OK;
}

static int rotate(dht_ctx* c, const EigWork& w, const Cx<double>* X, const CMat& C, Cx<double>* Z) {
    DHT_HIP(hipMemcpyAsync(w.small, C.data(), sizeof(Cx<double>) * C.size(), hipMemcpyHostToDevice, c->stream));
    dim3 grid((unsigned)((w.rows + EG_T - 1) / EG_T), w.nb / EG_T);
    hipLaunchKernelGGL(eig_rotate_kernel, grid, dim3(EG_THREADS), 0, c->stream, X, w.small, w.rows, w.nb, Z);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

static int lincomb(dht_ctx* c, const EigWork& w, Cx<double>* Z, double a, const Cx<double>* X, double b,
                   const Cx<double>* Y, double cc, const Cx<double>* W) {
    const int64_t n = w.rows * w.nb;
    const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(eig_lincomb_kernel, dim3(nb), dim3(256), 0, c->stream, Z, a, X, b, Y, cc, W, n);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

static int resid_norms(dht_ctx* c, const EigWork& w, const Cx<double>* W, const Cx<double>* V,
                       const std::vector<double>& lam, std::vector<double>& out) {
    DHT_HIP(hipMemcpyAsync(w.lam, lam.data(), sizeof(double) * w.nb, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(eig_resid_kernel, dim3(w.rblocks), dim3(EG_THREADS), 0, c->stream, W, V, w.lam, w.rows, w.nb,
                       w.rpart);
    DHT_HIP(hipGetLastError());
    std::vector<double> h((size_t)w.rblocks * w.nb);
    DHT_HIP(hipMemcpyAsync(h.data(), w.rpart, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    out.assign(w.nb, 0.0);
    for (int b = 0; b < w.rblocks; b++)
        for (int j = 0; j < w.nb; j++) out[j] += h[(size_t)b * w.nb + j];
    for (auto& v : out) v = std::sqrt(v);
    return DHT_OK;
}

// V <- V C with C = L^{-H} from X^H X = L L^H, twice (Cholesky QR 2); T is scratch
static int orthonormalise(dht_ctx* c, const EigWork& w, Cx<double>*& V, Cx<double>*& T) {
    for (int pass = 0; pass < 2; pass++) {
        CMat G, L, C;
        DHT_TRY(gram(c, w, V, V, G));
        for (int i = 0; i < w.nb; i++)   // exact Hermitian symmetry
            for (int j = i + 1; j < w.nb; j++) {
                Cx<double> a = G[(size_t)i * w.nb + j], b = cconj(G[(size_t)j * w.nb + i]);
                G[(size_t)i * w.nb + j] = 0.5 * (a + b);
                G[(size_t)j * w.nb + i] = cconj(G[(size_t)i * w.nb + j]);
            }
        if (!cholesky(G, w.nb, L)) return set_error(DHT_ERR_BREAKDOWN, "eigensolver block lost rank (Cholesky QR)");
        inv_lower_h(L, w.nb, C);
        DHT_TRY(rotate(c, w, V, C, T));
        std::swap(V, T);
    }
    return DHT_OK;
}

static int apply_q(dht_ctx* c, const EigWork& w, const Cx<double>* in, Cx<double>* out) {
    return apply_full(c, DHT_OP_Q, DHT_FP64, in, out, w.nb);
}

static void hermitise(CMat& H, int n) {
    for (int i = 0; i < n; i++)
        for (int j = i; j < n; j++) {
            Cx<double> a = H[(size_t)i * n + j], b = cconj(H[(size_t)j * n + i]);
            H[(size_t)i * n + j] = 0.5 * (a + b);
            H[(size_t)j * n + i] = cconj(H[(size_t)i * n + j]);
        }
}

// Rayleigh-Ritz on the orthonormal block V (T scratch).  Ordering and the
// filter bound come from Q^2, whose Rayleigh matrix is (Q V)^H (Q V): at the
// bottom of a positive spectrum Ritz values approach from above and none is
// spurious.  Signs are then separated by a Rayleigh-Ritz with Q restricted to
// the leading m >= k Ritz vectors of Q^2 (m extended past near-equal values so
// that a +-lambda pair is never split); a step with Q on the whole block would
// produce spurious near-zero Ritz values from unconverged +-lambda mixtures.
// Out: V (leading m columns Q-Ritz vectors ordered by |lambda|), W = Q V,
// lam[0..m) and their residual norms, theta = Q^2 Ritz values (ascending).
static int rayleigh_ritz(dht_ctx* c, const EigWork& w, int k, Cx<double>*& V, Cx<double>*& W, Cx<double>*& T,
                         std::vector<double>& lam, std::vector<double>& res, std::vector<double>& theta, int* m_out) {
    const int nb = w.nb;
    DHT_TRY(apply_q(c, w, V, W));
    CMat H, Y;
    DHT_TRY(gram(c, w, W, W, H));
    hermitise(H, nb);
    jacobi_eigh(H, nb, theta, Y);
    DHT_TRY(rotate(c, w, V, Y, T));
    std::swap(V, T);
    DHT_TRY(rotate(c, w, W, Y, T));
    std::swap(W, T);
    int m = k;
    while (m < nb && theta[m] - theta[m - 1] <= 1e-8 * std::max(theta[m], 1e-300)) m++;
    DHT_TRY(gram(c, w, V, W, H));
    CMat Hm((size_t)m * m);
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++) Hm[(size_t)i * m + j] = H[(size_t)i * nb + j];
    hermitise(Hm, m);
    std::vector<double> ev;
    CMat Ym;
    jacobi_eigh(Hm, m, ev, Ym);
    std::vector<int> idx(m);
    for (int i = 0; i < m; i++) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return std::fabs(ev[a]) < std::fabs(ev[b]); });
    CMat C((size_t)nb * nb, cmake(0.0, 0.0));
    for (int i = 0; i < nb; i++) C[(size_t)i * nb + i] = cmake(1.0, 0.0);
    lam.assign(nb, 0.0);
    for (int jj = 0; jj < m; jj++) {
        lam[jj] = ev[idx[jj]];
        for (int i = 0; i < m; i++) C[(size_t)i * nb + jj] = Ym[(size_t)i * m + idx[jj]];
    }
    DHT_TRY(rotate(c, w, V, C, T));
    std::swap(V, T);
    DHT_TRY(rotate(c, w, W, C, T));
    std::swap(W, T);
    *m_out = m;
    return resid_norms(c, w, W, V, lam, res);
}

int eigensolve(dht_ctx* c, const dht_eig_params* prm, double* lambda_host, double* resid_host, dht_eig_stats* st) {
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    if (!c->W || c->k <= 0) return set_error(DHT_ERR_STATE, "call dht_deflation_begin first");
    const int k = c->k;
    int guard = prm->guard > 0 ? prm->guard : std::max(16, k / 4);
    int nb = EG_T;
    while (nb < k + guard) nb *= 2;
    if (nb > DHT_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "k + guard must not exceed 256 block vectors");
    if (prm->degree < 1 || prm->max_iter < 1 || !(prm->tol > 0)) return set_error(DHT_ERR_INVALID_ARG, "bad eigensolver parameters");

    EigWork w;
    w.rows = c->g.V * 12;
    w.nb = nb;
    w.rblocks = 512;
    const size_t fb = sizeof(Cx<double>) * (size_t)w.rows * nb;
    void *p0, *p1, *p2, *p3, *pp, *ps, *pr, *pl;
    DHT_TRY(ws_get(c, WS_EIG_V, fb, &p0));
    DHT_TRY(ws_get(c, WS_EIG_W, fb, &p1));
    DHT_TRY(ws_get(c, WS_EIG_T, fb, &p2));
    DHT_TRY(ws_get(c, WS_EIG_U, fb, &p3));
    DHT_TRY(ws_get(c, WS_EIG_PART, sizeof(Cx<double>) * (size_t)EG_SPLITS * nb * nb, &pp));
    DHT_TRY(ws_get(c, WS_EIG_SMALL, sizeof(Cx<double>) * (size_t)nb * nb, &ps));
    DHT_TRY(ws_get(c, WS_EIG_RPART, sizeof(double) * (size_t)w.rblocks * nb, &pr));
    DHT_TRY(ws_get(c, WS_EIG_LAM, sizeof(double) * nb, &pl));
    w.part = (Cx<double>*)pp;
    w.small = (Cx<double>*)ps;
    w.rpart = (double*)pr;
    w.lam = (double*)pl;
    Cx<double>* V = (Cx<double>*)p0;
    Cx<double>* W = (Cx<double>*)p1;
    Cx<double>* T = (Cx<double>*)p2;
    Cx<double>* U = (Cx<double>*)p3;

    // start block: Z4 noise (run 0 of the given seed)
    dht_probe_spec sp = {prm->seed, 0u, 0};
    DHT_TRY(probes_gen(c, &sp, 0, nb, nb, V, DHT_FP64, nullptr, nullptr));
    const double qn = std::fabs(4.0 + c->mass) + 4.0;   // ||Q|| = ||D|| <= |4 + m| + 4
    const double b = qn * qn * 1.0001;
    std::vector<double> lam, res, theta;
    int m = k;
    DHT_TRY(orthonormalise(c, w, V, T));
    DHT_TRY(rayleigh_ritz(c, w, k, V, W, T, lam, res, theta, &m));
    int it = 0, conv = 0;
    int64_t matvecs = 1;
    for (; it < prm->max_iter; it++) {
        conv = 0;
        while (conv < k && res[conv] <= prm->tol * qn) conv++;
        if (conv == k) break;
        // damp [a, b] with a = the largest Q^2 Ritz value of the block
        double a = theta[nb - 1];
        if (!(a < b)) a = 0.5 * b;
        const double e = 0.5 * (b - a), cen = 0.5 * (b + a);
        // Chebyshev recurrence in Q^2: Y0 = V, Y1 = (Q^2 - cen) V / e,
        // Y_{j+1} = 2 (Q^2 - cen) Y_j / e - Y_{j-1}; buffers V (Y_{j-1}), U (Y_j), W, T
        DHT_TRY(apply_q(c, w, V, T));
        DHT_TRY(apply_q(c, w, T, W));
        DHT_TRY(lincomb(c, w, U, 1.0 / e, W, -cen / e, V, 0.0, nullptr));
        matvecs += 2;
        for (int j = 1; j < prm->degree; j++) {
            DHT_TRY(apply_q(c, w, U, T));
            DHT_TRY(apply_q(c, w, T, W));
            DHT_TRY(lincomb(c, w, V, 2.0 / e, W, -2.0 * cen / e, U, -1.0, V));
            std::swap(V, U);
            matvecs += 2;
        }
        std::swap(V, U);   // V = Y_degree
        DHT_TRY(orthonormalise(c, w, V, T));
        DHT_TRY(rayleigh_ritz(c, w, k, V, W, T, lam, res, theta, &m));
        matvecs += 1;
    }
    // the k Ritz vectors of smallest |lambda| into the stored basis
    const size_t cb = sizeof(double) * 2 * (size_t)w.rows;
    void* canon;
    DHT_TRY(ws_get(c, WS_EIG_CANON, cb * k, &canon));
    DHT_TRY(unpack_spinor(c, V, DHT_FP64, (double*)canon, k, nb));
    DHT_TRY(deflation_set(c, 0, k, (const double*)canon));
    DHT_HIP(hipStreamSynchronize(c->stream));
    for (int j = 0; j < k; j++) {
        if (lambda_host) lambda_host[j] = lam[j];
        if (resid_host) resid_host[j] = res[j] / qn;
    }
    if (st) {
        st->iters = it;
        st->converged = conv;
        st->block = nb;
        st->matvecs = matvecs;
    }
    return conv == k ? DHT_OK : set_error(DHT_ERR_NOT_CONVERGED, "eigensolver: not all k pairs reached the tolerance");
}

// ---------------------------------------------------------------------------
// Preconditioned block eigensolver with locking (Section 5.1: the paper's route
// to the deflation space is a preconditioned Davidson-type method with a
// window of block vectors and locking of converged ones).  Here: LOBPCG on
// Q^2 = D^H D, whose smallest eigenvalues are sigma^2 of the wanted singular
// triplets, with the window X of m vectors, the preconditioned residuals W
// and the previous directions P; a Rayleigh-Ritz step on [X, W, P] (the
// generalised form, with the Gram matrix of the three blocks factored by
// Cholesky, so that small losses of orthogonality between the blocks do no
// harm) gives the next window.  Converged leading Ritz vectors are locked
// (copied out, their slots refilled with fresh Z4 noise), and every new block
// is kept orthogonal to the locked ones.  The preconditioner approximates
// (Q^2)^-1 = D^-1 g5 D^-1 g5 by two loose mixed-precision solves with D.
// ---------------------------------------------------------------------------

// dst[:, d0 + j] = src[:, s0 + j] for j < ncols (both nrows x nb)
__global__ void eig_copy_cols_kernel(const Cx<double>* src, Cx<double>* dst, int64_t nrows, int nb, int s0, int d0,
                                     int ncols) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrows * ncols) return;
    const int64_t r = e / ncols;
    const int j = (int)(e - r * ncols);
    dst[r * nb + d0 + j] = src[r * nb + s0 + j];
}

struct Lobpcg {
    dht_ctx* c;
    EigWork w;
    int m;
    Cx<double> *X, *AX, *W, *AW, *P, *AP, *NX, *NAX, *NP, *NAP, *T1, *T2, *T3;
    std::vector<Cx<double>*> locked;   // chunks of m columns (unused columns zero)
    int nl = 0;                        // locked vectors
    int64_t qapps = 0, solves = 0;
    const dht_solver_params* sp = nullptr;   // preconditioner solves (null: none)
};

static int copy_cols(Lobpcg& L, const Cx<double>* src, Cx<double>* dst, int s0, int d0, int n) {
    const int64_t tot = L.w.rows * n;
    hipLaunchKernelGGL(eig_copy_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, L.c->stream, src, dst,
                       L.w.rows, L.w.nb, s0, d0, n);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

static int apply_q2(Lobpcg& L, const Cx<double>* in, Cx<double>* out) {
    DHT_TRY(apply_q(L.c, L.w, in, L.T3));
    DHT_TRY(apply_q(L.c, L.w, L.T3, out));
    L.qapps += 2;
    return DHT_OK;
}

// V -= B (B^H V) over every locked chunk, twice
static int project_locked(Lobpcg& L, Cx<double>* V) {
    for (int pass = 0; pass < 2; pass++)
        for (int ch = 0; ch * L.m < L.nl; ch++) {
            CMat G;
            DHT_TRY(gram(L.c, L.w, L.locked[ch], V, G));
            DHT_TRY(rotate(L.c, L.w, L.locked[ch], G, L.T1));
            DHT_TRY(lincomb(L.c, L.w, V, 1.0, V, -1.0, L.T1, 0.0, nullptr));
        }
    return DHT_OK;
}

// V -= B (B^H V) and, with AB/AV, AV -= AB (B^H V) (B orthonormal)
static int project_block(Lobpcg& L, const Cx<double>* B, const Cx<double>* AB, Cx<double>* V, Cx<double>* AV) {
    CMat G;
    DHT_TRY(gram(L.c, L.w, B, V, G));
    DHT_TRY(rotate(L.c, L.w, B, G, L.T1));
    DHT_TRY(lincomb(L.c, L.w, V, 1.0, V, -1.0, L.T1, 0.0, nullptr));
    if (AV) {
        DHT_TRY(rotate(L.c, L.w, AB, G, L.T1));
        DHT_TRY(lincomb(L.c, L.w, AV, 1.0, AV, -1.0, L.T1, 0.0, nullptr));
    }
    return DHT_OK;
}

// V <- V C, AV <- AV C with C = L^-H from V^H V = L L^H (Cholesky QR, twice);
// returns false in *ok when the block has lost rank
static int ortho_pair(Lobpcg& L, Cx<double>* V, Cx<double>* AV, bool* ok) {
    *ok = true;
    const size_t bytes = sizeof(Cx<double>) * (size_t)L.w.rows * L.w.nb;
    for (int pass = 0; pass < 2; pass++) {
        CMat G, Lc, C;
        DHT_TRY(gram(L.c, L.w, V, V, G));
        hermitise(G, L.m);
        if (!cholesky(G, L.m, Lc)) {
            *ok = false;
            return DHT_OK;
        }
        inv_lower_h(Lc, L.m, C);
        DHT_TRY(rotate(L.c, L.w, V, C, L.T1));
        DHT_HIP(hipMemcpyAsync(V, L.T1, bytes, hipMemcpyDeviceToDevice, L.c->stream));
        if (AV) {
            DHT_TRY(rotate(L.c, L.w, AV, C, L.T1));
            DHT_HIP(hipMemcpyAsync(AV, L.T1, bytes, hipMemcpyDeviceToDevice, L.c->stream));
        }
    }
    return DHT_OK;
}

// out = D^-1 g5 D^-1 g5 in (two loose solves), or out = in without a preconditioner
static int precondition(Lobpcg& L, const Cx<double>* in, Cx<double>* out) {
    const size_t bytes = sizeof(Cx<double>) * (size_t)L.w.rows * L.w.nb;
    if (!L.sp) {
        DHT_HIP(hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, L.c->stream));
        return DHT_OK;
    }
    std::vector<dht_solve_stats> st(L.m);
    for (int rep = 0; rep < 2; rep++) {
        DHT_TRY(g5_field(L.c, DHT_FP64, rep == 0 ? in : out, L.T2, L.m));
        const int rc = solve_fields(L.c, L.sp, L.T2, out, L.m, st.data(), nullptr, nullptr, DHT_FP64);
        if (rc != DHT_OK && rc != DHT_ERR_NOT_CONVERGED) return rc;   // a loose solve may miss: it only preconditions
        L.solves += L.m;
    }
    return DHT_OK;
}

// Rayleigh-Ritz on the blocks S[0..nbk) with images AS: the m smallest Ritz
// pairs; new X = S C_X, and (nbk > 1) new P = the W and P part of the same
// combination.  theta receives the m Ritz values (ascending).
static int rayleigh_ritz_blocks(Lobpcg& L, int nbk, std::vector<double>& theta, bool* ok) {
    Cx<double>* S[3] = {L.X, L.W, L.P};
    Cx<double>* AS[3] = {L.AX, L.AW, L.AP};
    const int m = L.m, n = nbk * m;
    CMat G((size_t)n * n), M((size_t)n * n);
    for (int i = 0; i < nbk; i++)
        for (int j = i; j < nbk; j++) {
            CMat g, h;
            DHT_TRY(gram(L.c, L.w, S[i], AS[j], g));
            DHT_TRY(gram(L.c, L.w, S[i], S[j], h));
            for (int a = 0; a < m; a++)
                for (int b = 0; b < m; b++) {
                    G[(size_t)(i * m + a) * n + j * m + b] = g[(size_t)a * m + b];
                    M[(size_t)(i * m + a) * n + j * m + b] = h[(size_t)a * m + b];
                    G[(size_t)(j * m + b) * n + i * m + a] = cconj(g[(size_t)a * m + b]);
                    M[(size_t)(j * m + b) * n + i * m + a] = cconj(h[(size_t)a * m + b]);
                }
        }
    hermitise(G, n);
    hermitise(M, n);
    CMat Lc, Li;   // M = Lc Lc^H, Li = Lc^-H
    *ok = cholesky(M, n, Lc);
    if (!*ok) return DHT_OK;
    inv_lower_h(Lc, n, Li);
    // Gt = Li^H G Li
    CMat T((size_t)n * n, cmake(0.0, 0.0)), Gt((size_t)n * n, cmake(0.0, 0.0));
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) {
            Cx<double> acc = cmake(0.0, 0.0);
            for (int e = 0; e < n; e++) acc = acc + G[(size_t)a * n + e] * Li[(size_t)e * n + b];
            T[(size_t)a * n + b] = acc;
        }
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) {
            Cx<double> acc = cmake(0.0, 0.0);
            for (int e = 0; e < n; e++) acc = acc + cconj(Li[(size_t)e * n + a]) * T[(size_t)e * n + b];
            Gt[(size_t)a * n + b] = acc;
        }
    hermitise(Gt, n);
    std::vector<double> ev;
    CMat Y;
    jacobi_eigh(Gt, n, ev, Y);   // ascending
    theta.assign(ev.begin(), ev.begin() + m);
    // C = Li Y[:, :m], split into m x m blocks C_i
    std::vector<CMat> C(nbk, CMat((size_t)m * m));
    for (int i = 0; i < nbk; i++)
        for (int a = 0; a < m; a++)
            for (int b = 0; b < m; b++) {
                Cx<double> acc = cmake(0.0, 0.0);
                for (int e = 0; e < n; e++) acc = acc + Li[(size_t)(i * m + a) * n + e] * Y[(size_t)e * n + b];
                C[i][(size_t)a * m + b] = acc;
            }
    // new X, AX (and P, AP from the W and P parts)
    for (int img = 0; img < 2; img++) {
        Cx<double>** src = img ? AS : S;
        Cx<double>* nx = img ? L.NAX : L.NX;
        Cx<double>* np_ = img ? L.NAP : L.NP;
        DHT_TRY(rotate(L.c, L.w, src[0], C[0], L.T1));
        if (nbk == 1) {
            DHT_HIP(hipMemcpyAsync(nx, L.T1, sizeof(Cx<double>) * (size_t)L.w.rows * L.w.nb, hipMemcpyDeviceToDevice,
                                   L.c->stream));
            continue;
        }
        DHT_TRY(rotate(L.c, L.w, src[1], C[1], L.T2));
        if (nbk == 3) {
            DHT_TRY(rotate(L.c, L.w, src[2], C[2], L.T3));
            DHT_TRY(lincomb(L.c, L.w, nx, 1.0, L.T1, 1.0, L.T2, 1.0, L.T3));
            DHT_TRY(lincomb(L.c, L.w, np_, 1.0, L.T2, 1.0, L.T3, 0.0, nullptr));
        } else {
            DHT_TRY(lincomb(L.c, L.w, nx, 1.0, L.T1, 1.0, L.T2, 0.0, nullptr));
            DHT_TRY(lincomb(L.c, L.w, np_, 1.0, L.T2, 0.0, nullptr, 0.0, nullptr));
        }
    }
    std::swap(L.X, L.NX);
    std::swap(L.AX, L.NAX);
    if (nbk > 1) {
        std::swap(L.P, L.NP);
        std::swap(L.AP, L.NAP);
    }
    return DHT_OK;
}

int lobpcg(dht_ctx* c, const dht_lobpcg_params* prm, double* sigma_host, double* resid_host, dht_lobpcg_stats* st) {
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    if (!c->W || c->k <= 0) return set_error(DHT_ERR_STATE, "call dht_deflation_begin first");
    if (!prm || !(prm->tol > 0) || prm->max_iter < 1 || (prm->block != 32 && prm->block != 64))
        return set_error(DHT_ERR_INVALID_ARG, "bad LOBPCG parameters (block 32 or 64)");
    if (prm->precond && !(prm->precond_tol > 0 && prm->precond_tol < 1))
        return set_error(DHT_ERR_INVALID_ARG, "preconditioner tolerance must lie in (0, 1)");
    const int k = c->k, m = prm->block;
    Lobpcg L;
    L.c = c;
    L.m = m;
    L.w.rows = c->g.V * 12;
    L.w.nb = m;
    L.w.rblocks = 512;
    const size_t fb = sizeof(Cx<double>) * (size_t)L.w.rows * m;
    const int nchunks = (k + m - 1) / m;
    void *work, *lock, *pp, *ps, *pr, *pl;
    DHT_TRY(ws_get(c, WS_EIG_U, fb * 13, &work));
    DHT_TRY(ws_get(c, WS_EIG_T, fb * nchunks, &lock));
    DHT_TRY(ws_get(c, WS_EIG_PART, sizeof(Cx<double>) * (size_t)EG_SPLITS * m * m, &pp));
    DHT_TRY(ws_get(c, WS_EIG_SMALL, sizeof(Cx<double>) * (size_t)m * m, &ps));
    DHT_TRY(ws_get(c, WS_EIG_RPART, sizeof(double) * (size_t)L.w.rblocks * m, &pr));
    DHT_TRY(ws_get(c, WS_EIG_LAM, sizeof(double) * m, &pl));
    L.w.part = (Cx<double>*)pp;
    L.w.small = (Cx<double>*)ps;
    L.w.rpart = (double*)pr;
    L.w.lam = (double*)pl;
    Cx<double>* bufs[13];
    for (int i = 0; i < 13; i++) bufs[i] = (Cx<double>*)((char*)work + fb * i);
    L.X = bufs[0]; L.AX = bufs[1]; L.W = bufs[2]; L.AW = bufs[3]; L.P = bufs[4]; L.AP = bufs[5];
    L.NX = bufs[6]; L.NAX = bufs[7]; L.NP = bufs[8]; L.NAP = bufs[9]; L.T1 = bufs[10]; L.T2 = bufs[11]; L.T3 = bufs[12];
    for (int ch = 0; ch < nchunks; ch++) L.locked.push_back((Cx<double>*)((char*)lock + fb * ch));
    DHT_TRY(zero(c, lock, fb * nchunks));
    dht_solver_params sp;
    if (prm->precond) {
        memset(&sp, 0, sizeof(sp));
        sp.method = DHT_SOLVER_DC_BICGSTAB;
        sp.inner = DHT_BF16;
        sp.tol = prm->precond_tol;
        sp.maxiter = 1000;
        L.sp = &sp;
    }
    const double qn = std::fabs(4.0 + c->mass) + 4.0;   // ||Q|| <= |4 + m| + 4
    const double tol = prm->tol * qn * qn;              // on ||Q^2 x - theta x||
    std::vector<double> sig(k, 0.0), rres(k, 0.0);
    // start block: Z4 noise
    uint32_t run = 0;
    dht_probe_spec spec = {(uint32_t)prm->seed, run, 0};
    DHT_TRY(probes_gen(c, &spec, 0, m, m, L.X, DHT_FP64, nullptr, nullptr));
    bool ok;
    DHT_TRY(ortho_pair(L, L.X, nullptr, &ok));
    if (!ok) return set_error(DHT_ERR_BREAKDOWN, "LOBPCG: start block lost rank");
    DHT_TRY(apply_q2(L, L.X, L.AX));
    std::vector<double> theta, res;
    DHT_TRY(rayleigh_ritz_blocks(L, 1, theta, &ok));
    if (!ok) return set_error(DHT_ERR_BREAKDOWN, "LOBPCG: start block lost rank");
    bool havep = false;
    int it = 0;
    for (; it < prm->max_iter && L.nl < k; it++) {
        DHT_TRY(resid_norms(c, L.w, L.AX, L.X, theta, res));
        // lock the leading converged Ritz vectors
        int nc = 0;
        while (nc < m && L.nl + nc < k && res[nc] <= tol) nc++;
        if (nc > 0) {
            for (int j = 0; j < nc; j++) {
                const int slot = L.nl + j;
                DHT_TRY(copy_cols(L, L.X, L.locked[slot / m], j, slot % m, 1));
                sig[slot] = std::sqrt(std::max(theta[j], 0.0));
                rres[slot] = res[j] / (qn * qn);
            }
            L.nl += nc;
            if (L.nl >= k) break;
            // refill the locked slots with fresh noise, keep the rest of the window
            spec.run = ++run;
            DHT_TRY(probes_gen(c, &spec, 0, m, m, L.T2, DHT_FP64, nullptr, nullptr));
            DHT_TRY(copy_cols(L, L.T2, L.X, 0, 0, nc));
            DHT_TRY(project_locked(L, L.X));
            DHT_TRY(ortho_pair(L, L.X, nullptr, &ok));
            if (!ok) return set_error(DHT_ERR_BREAKDOWN, "LOBPCG: window lost rank after locking");
            DHT_TRY(apply_q2(L, L.X, L.AX));
            DHT_TRY(rayleigh_ritz_blocks(L, 1, theta, &ok));
            if (!ok) return set_error(DHT_ERR_BREAKDOWN, "LOBPCG: window lost rank after locking");
            havep = false;
            continue;
        }
        // W = T (AX - X theta), orthogonal to the locked vectors, X and P
        CMat D((size_t)m * m, cmake(0.0, 0.0));
        for (int j = 0; j < m; j++) D[(size_t)j * m + j] = cmake(theta[j], 0.0);
        DHT_TRY(rotate(c, L.w, L.X, D, L.T1));
        DHT_TRY(lincomb(c, L.w, L.T2, 1.0, L.AX, -1.0, L.T1, 0.0, nullptr));   // R
        DHT_HIP(hipMemcpyAsync(L.NX, L.T2, fb, hipMemcpyDeviceToDevice, c->stream));
        DHT_TRY(precondition(L, L.NX, L.W));
        DHT_TRY(project_locked(L, L.W));
        DHT_TRY(project_block(L, L.X, nullptr, L.W, nullptr));
        if (havep) DHT_TRY(project_block(L, L.P, nullptr, L.W, nullptr));
        DHT_TRY(ortho_pair(L, L.W, nullptr, &ok));
        if (!ok) {   // W fell into span(X, P): restart without P
            havep = false;
            DHT_TRY(precondition(L, L.NX, L.W));
            DHT_TRY(project_locked(L, L.W));
            DHT_TRY(project_block(L, L.X, nullptr, L.W, nullptr));
            DHT_TRY(ortho_pair(L, L.W, nullptr, &ok));
            if (!ok) return set_error(DHT_ERR_BREAKDOWN, "LOBPCG: residual block lost rank");
        }
        DHT_TRY(apply_q2(L, L.W, L.AW));
        if (havep) {   // P orthonormal and orthogonal to X and W, its image alongside
            DHT_TRY(project_block(L, L.X, L.AX, L.P, L.AP));
            DHT_TRY(project_block(L, L.W, L.AW, L.P, L.AP));
            DHT_TRY(ortho_pair(L, L.P, L.AP, &ok));
            if (!ok) havep = false;
        }
        DHT_TRY(rayleigh_ritz_blocks(L, havep ? 3 : 2, theta, &ok));
        if (!ok) {   // the three blocks were dependent: drop P and retry on [X, W]
            havep = false;
            DHT_TRY(rayleigh_ritz_blocks(L, 2, theta, &ok));
            if (!ok) return set_error(DHT_ERR_BREAKDOWN, "LOBPCG: Rayleigh-Ritz basis lost rank");
        }
        havep = true;
    }
    // the locked vectors into the stored basis
    if (L.nl < k) {   // not all converged: the best current Ritz vectors fill the rest
        DHT_TRY(resid_norms(c, L.w, L.AX, L.X, theta, res));
        for (int j = 0; L.nl < k && j < m; j++) {
            const int slot = L.nl++;
            DHT_TRY(copy_cols(L, L.X, L.locked[slot / m], j, slot % m, 1));
            sig[slot] = std::sqrt(std::max(theta[j], 0.0));
            rres[slot] = res[j] / (qn * qn);
        }
    }
    const int filled = std::min(L.nl, k);
    void* canon;
    DHT_TRY(ws_get(c, WS_EIG_CANON, sizeof(double) * 2 * (size_t)L.w.rows * m, &canon));
    for (int ch = 0; ch * m < filled; ch++) {
        const int cnt = std::min(m, filled - ch * m);
        DHT_TRY(unpack_spinor(c, L.locked[ch], DHT_FP64, (double*)canon, cnt, m));
        DHT_TRY(deflation_set(c, ch * m, cnt, (const double*)canon));
    }
    DHT_HIP(hipStreamSynchronize(c->stream));
    DHT_TRY(prof_harvest(c));
    int conv = 0;
    for (int j = 0; j < k; j++) {
        if (sigma_host) sigma_host[j] = sig[j];
        if (resid_host) resid_host[j] = rres[j];
        if (rres[j] * qn * qn <= tol) conv++;
    }
    if (st) {
        st->iters = it;
        st->converged = conv;
        st->q_applications = L.qapps;
        st->precond_solves = L.solves;
    }
    return conv == k ? DHT_OK : set_error(DHT_ERR_NOT_CONVERGED, "LOBPCG: not all k vectors reached the tolerance");
}

}  // namespace dht

