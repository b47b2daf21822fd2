// The distance profile W_d of Section 6.2: for sampled rows i of B (D^-1, its
// deflated remainder D^-1 - P, or either one masked to the entries that the
// first 2^m hierarchical-probing vectors leave in the variance), the sum of
// |B_ij|^2 over the entries j whose site lies at torus Manhattan distance d
// from the site of i, divided by m_d, the number of such entries.
//
// Rows come from columns: D^H = g5 D g5 and P^H = g5 P g5 (M is Hermitian),
// so |B_ij| = |B_ji| and column i -- the solution of D x = e_i, minus
// W M (W^H g5 e_i) when deflated -- has the profile of row i.  The probing
// mask is symmetric too: entry (i, j) survives when the colours of the two
// sites agree on the low m bits (the first 2^m Hadamard vectors sum to 2^m
// times that indicator).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <vector>

#include "solver.h"

namespace dht {

static constexpr int WD_ROWS = 16;      // rows per batch of point sources
static constexpr int WD_THREADS = 256;
static constexpr int WD_MAX_BLOCKS = 1024;

struct UnitArgs {
    int64_t K[WD_ROWS];   // internal index of each source entry
    int n, bp;
};

__global__ void unit_sources_kernel(Cx<double>* E, UnitArgs a) {
    const int r = threadIdx.x;
    if (r < a.n) E[a.K[r] * a.bp + r] = cmake(1.0, 0.0);
}

struct WdArgs {
    Geom g;
    int bp, n, nd;
    int src[WD_ROWS][4];       // source site of each column
    uint64_t srccol[WD_ROWS];  // its colour bits under the mask
    uint64_t mask;             // 0: no probing mask
};

// partial[blk][r][d]: this block's sums of |X(site, comp, r)|^2 by distance d
__global__ __launch_bounds__(WD_THREADS) void wd_kernel(const Cx<double>* X, WdArgs a, double* partial) {
    extern __shared__ double bins[];   // [n][nd]
    for (int i = threadIdx.x; i < a.n * a.nd; i += WD_THREADS) bins[i] = 0.0;
    __syncthreads();
    const int64_t Vh = a.g.Vh;
    const int64_t total = 2 * Vh * a.bp;
    for (int64_t gid = (int64_t)blockIdx.x * WD_THREADS + threadIdx.x; gid < total;
         gid += (int64_t)gridDim.x * WD_THREADS) {
        const int64_t ps = gid / a.bp;
        const int r = (int)(gid - ps * a.bp);
        if (r >= a.n) continue;
        const int p = (int)(ps / Vh);
        const int64_t s = ps - (int64_t)p * Vh;
        int c[4];
        cb_coords(a.g, s, p, c);
        if (a.mask && ((hp_colour_bits(c, a.mask) ^ a.srccol[r]) & a.mask)) continue;
        int d = 0;
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            const int x = abs(c[mu] - a.src[r][mu]);
            d += min(x, a.g.L[mu] - x);
        }
        double sum = 0.0;
#pragma unroll
        for (int comp = 0; comp < 12; comp++) {
            const Cx<double> v = X[(((int64_t)p * 12 + comp) * Vh + s) * a.bp + r];
            sum += v.re * v.re + v.im * v.im;
        }
        atomicAdd(&bins[r * a.nd + d], sum);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.n * a.nd; i += WD_THREADS) partial[(int64_t)blockIdx.x * a.n * a.nd + i] = bins[i];
}

__global__ void wd_sum_kernel(const double* partial, int nblk, int n, double* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int b = 0; b < nblk; b++) s += partial[(int64_t)b * n + i];
    out[i] = s;
}

static void site_of(const Geom& g, int64_t n, int c[4]) {
    c[0] = (int)(n % g.L[0]);
    n /= g.L[0];
    c[1] = (int)(n % g.L[1]);
    n /= g.L[1];
    c[2] = (int)(n % g.L[2]);
    c[3] = (int)(n / g.L[2]);
}

}  // namespace dht

using namespace dht;

extern "C" {

int dht_distance_profile(dht_ctx* c, const int64_t* rows, int nrows, int deflate, int hp_vectors,
                         const dht_solver_params* prm, double* W_host, int64_t* m_host) {
    if (!c || !rows || !prm || !W_host || nrows <= 0) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    DHT_HIP(hipSetDevice(c->device));
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    const Geom& g = c->g;
    const int64_t N = 12 * g.V;
    for (int i = 0; i < nrows; i++)
        if (rows[i] < 0 || rows[i] >= N) return set_error(DHT_ERR_INVALID_ARG, "row index outside 0..N-1");
    if (hp_vectors < 0 || hp_vectors > 65536 || (hp_vectors & (hp_vectors - 1)))
        return set_error(DHT_ERR_INVALID_ARG, "hp_vectors must be 0 or a power of two <= 65536");
    if (deflate && (!c->defl_ready || c->k <= 0)) return set_error(DHT_ERR_STATE, "no finalized deflation basis");
    const uint64_t mask = hp_vectors > 1 ? (uint64_t)hp_vectors - 1 : 0;
    const int nd = g.L[0] / 2 + g.L[1] / 2 + g.L[2] / 2 + g.L[3] / 2 + 1;
    if (nd > 512) return set_error(DHT_ERR_INVALID_ARG, "lattice too large for the distance bins");
    // m_d relative to site 0 (the same for every site of the torus)
    std::vector<int64_t> m(nd, 0);
    for (int64_t n = 0; n < g.V; n++) {
        int cc[4];
        site_of(g, n, cc);
        int d = 0;
        for (int mu = 0; mu < 4; mu++) d += std::min(cc[mu], g.L[mu] - cc[mu]);
        m[d] += 12;
    }
    if (m_host) std::copy(m.begin(), m.end(), m_host);
    const int k = deflate ? c->k : 0;
    bool missed = false;
    std::string msg;
    for (int r0 = 0; r0 < nrows; r0 += WD_ROWS) {
        const int n = std::min(WD_ROWS, nrows - r0);
        const int bp = pad_rhs(n);
        const size_t fb = full_elems(c, bp) * 16;
        void *E, *X, *part, *outb;
        DHT_TRY(ws_get(c, WS_Z, fb, &E));
        DHT_TRY(ws_get(c, WS_PACK_OUT, fb, &X));
        UnitArgs ua;
        WdArgs wa;
        memset(&ua, 0, sizeof(ua));
        memset(&wa, 0, sizeof(wa));
        ua.n = n;
        ua.bp = bp;
        wa.g = g;
        wa.bp = bp;
        wa.n = n;
        wa.nd = nd;
        wa.mask = mask;
        for (int r = 0; r < n; r++) {
            const int64_t row = rows[r0 + r];
            const int64_t site = row / 12;
            const int comp = (int)(row % 12);
            int cc[4];
            site_of(g, site, cc);
            const int p = (cc[0] + cc[1] + cc[2] + cc[3]) & 1;
            ua.K[r] = ((int64_t)p * 12 + comp) * g.Vh + (site >> 1);
            for (int mu = 0; mu < 4; mu++) wa.src[r][mu] = cc[mu];
            wa.srccol[r] = mask ? (hp_colour_bits(cc, mask) & mask) : 0;
        }
        DHT_TRY(zero(c, E, fb));
        hipLaunchKernelGGL(unit_sources_kernel, dim3(1), dim3(WD_ROWS), 0, c->stream, (Cx<double>*)E, ua);
        DHT_HIP(hipGetLastError());
        std::vector<dht_solve_stats> st(bp);
        std::vector<double> zn2(bp, 0.0);
        for (int r = 0; r < n; r++) zn2[r] = 1.0;
        int rc = solve_fields(c, prm, E, X, bp, st.data(), zn2.data(), nullptr, DHT_FP64);
        if (rc == DHT_ERR_NOT_CONVERGED) {
            missed = true;
            msg = dht_last_error();
        } else if (rc != DHT_OK) {
            return rc;
        }
        if (k > 0) {   // column of D^-1 - P: x - W M (W^H g5 e_i)
            void* cc;
            DHT_TRY(ws_get(c, WS_COEF, sizeof(Cx<double>) * 3 * (size_t)k * bp, &cc));
            Cx<double>* c1 = (Cx<double>*)cc;
            Cx<double>* c2 = c1 + (size_t)k * bp;
            Cx<double>* vd = c2 + (size_t)k * bp;
            DHT_TRY(project_field(c, E, DHT_FP64, bp, c1, c2));
            std::vector<std::complex<double>> h2((size_t)k * bp), v((size_t)k * bp, 0.0);
            DHT_HIP(hipMemcpyAsync(h2.data(), c2, sizeof(Cx<double>) * h2.size(), hipMemcpyDeviceToHost, c->stream));
            DHT_HIP(hipStreamSynchronize(c->stream));
            const std::complex<double>* M = (const std::complex<double>*)c->M.data();
            for (int a = 0; a < k; a++)
                for (int r = 0; r < bp; r++) {
                    std::complex<double> acc = 0.0;
                    if (c->M_diag) acc = M[(size_t)a * k + a] * h2[(size_t)a * bp + r];
                    else
                        for (int b = 0; b < k; b++) acc += M[(size_t)a * k + b] * h2[(size_t)b * bp + r];
                    v[(size_t)a * bp + r] = acc;
                }
            DHT_HIP(hipMemcpyAsync(vd, v.data(), sizeof(Cx<double>) * v.size(), hipMemcpyHostToDevice, c->stream));
            DHT_HIP(hipStreamSynchronize(c->stream));   // v is pageable and goes out of scope
            DHT_TRY(basis_subtract(c, vd, bp, X));
        }
        const int nblk = (int)std::min<int64_t>(WD_MAX_BLOCKS, (2 * g.Vh * bp + WD_THREADS - 1) / WD_THREADS);
        const int nb = n * nd;
        DHT_TRY(ws_get(c, WS_WD_PART, sizeof(double) * (size_t)nblk * nb, &part));
        DHT_TRY(ws_get(c, WS_WD_OUT, sizeof(double) * (size_t)nb, &outb));
        hipLaunchKernelGGL(wd_kernel, dim3(nblk), dim3(WD_THREADS), sizeof(double) * nb, c->stream,
                           (const Cx<double>*)X, wa, (double*)part);
        DHT_HIP(hipGetLastError());
        hipLaunchKernelGGL(wd_sum_kernel, dim3((nb + 127) / 128), dim3(128), 0, c->stream, (const double*)part, nblk,
                           nb, (double*)outb);
        DHT_HIP(hipGetLastError());
        std::vector<double> h(nb);
        DHT_HIP(hipMemcpyAsync(h.data(), outb, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
        DHT_HIP(hipStreamSynchronize(c->stream));
        DHT_TRY(prof_harvest(c));
        for (int r = 0; r < n; r++)
            for (int d = 0; d < nd; d++) W_host[(size_t)(r0 + r) * nd + d] = h[(size_t)r * nd + d] / (double)m[d];
    }
    if (missed) return set_error(DHT_ERR_NOT_CONVERGED, msg);
    return DHT_OK;
}

}  // extern "C"
