// Variance analysis of the trace estimator (Sections 6.1-6.3): run-to-run
// variances of the hierarchical-probing estimate with Jackknife error bars,
// the speedup over plain Monte Carlo, and the playback of stored projection
// coefficients with fewer deflation vectors.  Host code only: these entry
// points take host arrays and need no device.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <vector>

#include "internal.h"

namespace dht {

typedef std::complex<double> cd;

// unbiased sample variance E|x - xbar|^2 of complex values, skipping index `skip`
static double cvar(const std::vector<cd>& x, int skip) {
    const int n = (int)x.size() - (skip >= 0 ? 1 : 0);
    if (n < 2) return NAN;
    cd m = 0.0;
    for (int i = 0; i < (int)x.size(); i++)
        if (i != skip) m += x[i];
    m /= (double)n;
    double v = 0.0;
    for (int i = 0; i < (int)x.size(); i++)
        if (i != skip) v += std::norm(x[i] - m);
    return v / (n - 1);
}

// Jackknife error of a statistic from its R leave-one-out values
static double jack_err(const std::vector<double>& loo) {
    const int R = (int)loo.size();
    double m = 0.0;
    for (double v : loo) m += v;
    m /= R;
    double s = 0.0;
    for (double v : loo) s += (v - m) * (v - m);
    return sqrt((R - 1.0) / R * s);
}

// In-place inverse of an n x n complex matrix (Gauss-Jordan, partial pivoting)
static bool cinvert(std::vector<cd>& A, int n) {
    std::vector<cd> I((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) I[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; col++) {
        int best = col;
        for (int r = col + 1; r < n; r++)
            if (std::abs(A[(size_t)r * n + col]) > std::abs(A[(size_t)best * n + col])) best = r;
        if (!(std::abs(A[(size_t)best * n + col]) > 0.0)) return false;
        for (int j = 0; j < n && best != col; j++) {
            std::swap(A[(size_t)col * n + j], A[(size_t)best * n + j]);
            std::swap(I[(size_t)col * n + j], I[(size_t)best * n + j]);
        }
        const cd d = 1.0 / A[(size_t)col * n + col];
        for (int j = 0; j < n; j++) {
            A[(size_t)col * n + j] *= d;
            I[(size_t)col * n + j] *= d;
        }
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            const cd f = A[(size_t)r * n + col];
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

}  // namespace dht

using namespace dht;

extern "C" {

int dht_hp_variance(const double* q, int R, int S, const int* s_list, int ns, double v_stoc, dht_hp_var* out) {
    if (!q || !s_list || !out || R < 3 || S <= 0 || ns <= 0) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    for (int i = 0; i < ns; i++) {
        const int s = s_list[i];
        if (s <= 0 || s > S) return set_error(DHT_ERR_INVALID_ARG, "s outside 1..S");
        std::vector<cd> t(R);
        for (int r = 0; r < R; r++) {   // the run's estimate after s probes
            cd acc = 0.0;
            for (int j = 0; j < s; j++) acc += cd(q[2 * ((size_t)r * S + j)], q[2 * ((size_t)r * S + j) + 1]);
            t[r] = acc / (double)s;
        }
        dht_hp_var& o = out[i];
        memset(&o, 0, sizeof(o));
        o.s = s;
        cd m = 0.0;
        for (const cd& v : t) m += v;
        m /= (double)R;
        o.mean_re = m.real();
        o.mean_im = m.imag();
        o.var = cvar(t, -1);
        o.mean_err = sqrt(o.var / R);
        std::vector<double> lv(R), lr(R);
        for (int r = 0; r < R; r++) {
            lv[r] = cvar(t, r);
            lr[r] = v_stoc > 0 ? v_stoc / (lv[r] * s) : 0.0;
        }
        o.var_err = jack_err(lv);
        o.rs = v_stoc > 0 ? v_stoc / (o.var * s) : 0.0;
        o.rs_err = v_stoc > 0 ? jack_err(lr) : 0.0;
    }
    return DHT_OK;
}

int dht_playback(const double* H, const double* G5, int k, int diagonal, const double* coef, const double* q, int n,
                 const int* k_list, int nk, double* qd_out, double* TD_out) {
    if (!H || !G5 || !coef || !q || !k_list || !qd_out || !TD_out || k <= 0 || n <= 0 || nk <= 0)
        return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    const cd* Hc = (const cd*)H;
    const cd* Gc = (const cd*)G5;
    const cd* c1 = (const cd*)coef;                 // [k][n]
    const cd* c2 = c1 + (size_t)k * n;              // [k][n]
    const cd* qc = (const cd*)q;
    cd* qd = (cd*)qd_out;
    cd* td = (cd*)TD_out;
    for (int a = 0; a < nk; a++) {
        const int kk = k_list[a];
        if (kk < 0 || kk > k) return set_error(DHT_ERR_INVALID_ARG, "playback size outside 0..k");
        // the Galerkin inverse on the leading kk vectors: M' = (H[:kk, :kk])^-1
        std::vector<cd> M((size_t)kk * kk, 0.0);
        for (int i = 0; i < kk; i++)
            for (int j = 0; j < kk; j++)
                if (!diagonal || i == j) M[(size_t)i * kk + j] = Hc[(size_t)i * k + j];
        if (kk > 0 && !cinvert(M, kk)) return set_error(DHT_ERR_BREAKDOWN, "leading block of W^H Q W is singular");
        cd t = 0.0;   // T_D' = Tr(M' G5[:kk, :kk])
        for (int i = 0; i < kk; i++)
            for (int j = 0; j < kk; j++) t += M[(size_t)i * kk + j] * Gc[(size_t)j * k + i];
        td[a] = t;
        for (int r = 0; r < n; r++) {   // q - c1^H M' c2 over the leading kk coefficients
            cd d = 0.0;
            for (int i = 0; i < kk; i++) {
                cd v = 0.0;
                for (int j = 0; j < kk; j++) v += M[(size_t)i * kk + j] * c2[(size_t)j * n + r];
                d += std::conj(c1[(size_t)i * n + r]) * v;
            }
            qd[(size_t)a * n + r] = qc[r] - d;
        }
    }
    return DHT_OK;
}

int dht_theorem2(int64_t N, int k, int hermitian, double sum_all, double sumsq_all, const double* top,
                 dht_thm2* out) {
    if (!out || N < 1 || k < 0 || k > N || (k > 0 && !top)) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (!isfinite(sumsq_all) || sumsq_all < 0 || (hermitian && !isfinite(sum_all)))
        return set_error(DHT_ERR_INVALID_ARG, "sums must be finite (the plain sum is needed for Hermitian matrices)");
    double st = 0.0, st2 = 0.0;
    for (int i = 0; i < k; i++) {
        if (!isfinite(top[i])) return set_error(DHT_ERR_INVALID_ARG, "non-finite deflated value");
        st += top[i];
        st2 += top[i] * top[i];
    }
    const double rest2 = sumsq_all - st2;   // sum of the squares of the N - k remaining values
    if (rest2 < -1e-12 * sumsq_all) return set_error(DHT_ERR_INVALID_ARG, "deflated values exceed the total sum of squares");
    const double Nd = (double)N, nr = (double)(N - k);
    memset(out, 0, sizeof(*out));
    out->mu_k = N > k ? (sum_all - st) / nr : 0.0;
    out->V_k = N > k ? std::max(0.0, rest2) / nr - out->mu_k * out->mu_k : 0.0;
    const double mu0 = sum_all / Nd, V0 = sumsq_all / Nd - mu0 * mu0;
    if (!hermitian) {
        out->var_k = (1.0 - 1.0 / Nd) * std::max(0.0, rest2);   // (N - k)(1 - 1/N)(V_k + mu_k^2)
        out->var_0 = (1.0 - 1.0 / Nd) * sumsq_all;              // (N - 1)(V_0 + mu_0^2)
    } else {
        out->var_k = nr * (out->V_k * Nd / (Nd + 1.0) + out->mu_k * out->mu_k * k / (Nd + 1.0));
        out->var_0 = Nd * Nd * V0 / (Nd + 1.0);
    }
    out->ratio = out->var_0 > 0 ? out->var_k / out->var_0 : NAN;
    out->reduces = out->var_k < out->var_0 ? 1 : 0;
    return DHT_OK;
}

int dht_deflation_get_galerkin(dht_ctx* c, double* H, double* G5, int* diagonal) {
    if (!c || !H || !G5 || !diagonal) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    if (!c->defl_ready || c->Hq.empty()) return set_error(DHT_ERR_STATE, "deflation not finalized");
    memcpy(H, c->Hq.data(), sizeof(double) * c->Hq.size());
    memcpy(G5, c->G5q.data(), sizeof(double) * c->G5q.size());
    *diagonal = c->M_diag ? 1 : 0;
    return DHT_OK;
}

}  // extern "C"
