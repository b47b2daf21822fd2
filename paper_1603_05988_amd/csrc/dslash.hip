// Even/odd Wilson hopping term on gfx950.
//
//   Hop(psi)(x) = sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^H psi(x-mu) ]
//
// (-1 on hops across the t boundary when antiperiodic), so that the Wilson
// matrix is D = (4+m) - Hop/2 and D^H uses the opposite projector signs.  The
// paper fixes only that D is a nearest-neighbour operator on a 4D lattice
// with 4 spin x 3 colour components per site (Section 1); the operator form
// is the plain r = 1 Wilson matrix.
//
// Chiral basis: g_mu = [[0, A_mu], [A_mu^H, 0]] with A_x = -i s1, A_y = -i s2,
// A_z = -i s3, A_t = 1.  (1 - s g_mu) psi = [h; -s A^H h] with
// h = psi_up - s A psi_lo, so each hop multiplies only a half spinor (2 spins x
// 3 colours) by the link and rebuilds the lower half by a signed permutation.
//
// Mapping: one lane per (checkerboard site, RHS), RHS fastest, so the B lanes
// of a site share the link loads and every spinor component load of a
// wavefront is contiguous.  Accumulation in FP64 for FP64 storage, FP32
// otherwise.  Workgroups are remapped so that each of the 8 XCDs walks a
// contiguous range of sites (neighbour reuse stays in one L2).
#include <type_traits>

#include "internal.h"

namespace dht {

struct HopArgs {
    void* out;
    const void* in;
    const void* x;       // xpay source (same parity as out) or null
    const void* U;
    Geom g;
    int out_parity;
    int B;
    int bshift;          // log2(B) if B is a power of two, else -1
    double ca, cb;       // out = ca * x + cb * Hop(in)
};

// h = psi_up - SGN * A_mu psi_lo  (SGN = +1 for (1 - g), -1 for (1 + g))
template <int MU, int SGN, typename T>
__device__ inline void project(const Cx<T>* p, Cx<T>* h) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        Cx<T> u0 = p[a], u1 = p[3 + a], l0 = p[6 + a], l1 = p[9 + a];
        Cx<T> A0, A1;   // A psi_lo
        if (MU == 0) { A0 = timesMinusI(l1); A1 = timesMinusI(l0); }
        if (MU == 1) { A0 = neg(l1); A1 = l0; }
        if (MU == 2) { A0 = timesMinusI(l0); A1 = timesI(l1); }
        if (MU == 3) { A0 = l0; A1 = l1; }
        if (SGN > 0) { h[a] = u0 - A0; h[3 + a] = u1 - A1; }
        else         { h[a] = u0 + A0; h[3 + a] = u1 + A1; }
    }
}

// acc += ph * [w; -SGN A^H w]
template <int MU, int SGN, typename T>
__device__ inline void reconstruct(Cx<T>* acc, const Cx<T>* w, T ph) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        Cx<T> w0 = ph * w[a], w1 = ph * w[3 + a];
        Cx<T> B0, B1;   // A^H w
        if (MU == 0) { B0 = timesI(w1); B1 = timesI(w0); }
        if (MU == 1) { B0 = w1; B1 = neg(w0); }
        if (MU == 2) { B0 = timesI(w0); B1 = timesMinusI(w1); }
        if (MU == 3) { B0 = w0; B1 = w1; }
        acc[a] = acc[a] + w0;
        acc[3 + a] = acc[3 + a] + w1;
        if (SGN > 0) { acc[6 + a] = acc[6 + a] - B0; acc[9 + a] = acc[9 + a] - B1; }
        else         { acc[6 + a] = acc[6 + a] + B0; acc[9 + a] = acc[9 + a] + B1; }
    }
}

template <typename S>
__device__ inline void load_spinor(const typename Store<S>::elem* base, int64_t cstride, Cx<typename Store<S>::acc>* p) {
#pragma unroll
    for (int c = 0; c < 12; c++) p[c] = Store<S>::ld(base + c * cstride);
}

template <typename S>
__device__ inline void load_link(const typename Store<S>::elem* base, int64_t estride, Cx<typename Store<S>::acc>* u) {
#pragma unroll
    for (int e = 0; e < 9; e++) u[e] = Store<S>::ld(base + e * estride);
}

// w = U h (per spin) or U^H h
template <bool ADJ, typename T>
__device__ inline void mul_link(const Cx<T>* u, const Cx<T>* h, Cx<T>* w) {
#pragma unroll
    for (int sp = 0; sp < 2; sp++) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            Cx<T> s = cmake<T>(0, 0);
#pragma unroll
            for (int b = 0; b < 3; b++) {
                if (!ADJ) s = s + u[3 * a + b] * h[3 * sp + b];
                else      s = s + conjmul(u[3 * b + a], h[3 * sp + b]);
            }
            w[3 * sp + a] = s;
        }
    }
}

template <typename S, int MU, bool DAG>
__device__ inline void hop_dir(const HopArgs& a, const int c[4], int64_t s, int r, Cx<typename Store<S>::acc>* acc) {
    typedef typename Store<S>::acc T;
    typedef typename Store<S>::elem E;
    const Geom& g = a.g;
    const int p = a.out_parity;
    const int64_t Vh = g.Vh;
    const E* in = (const E*)a.in;
    const E* U = (const E*)a.U;
    const int64_t cstride = Vh * a.B;
    constexpr int SF = DAG ? -1 : 1;   // sign of the forward projector (1 - SF g)
    // forward neighbour x + mu (parity 1 - p), link U_mu(x) at parity p
    {
        int n[4] = {c[0], c[1], c[2], c[3]};
        n[MU] = (c[MU] + 1 == g.L[MU]) ? 0 : c[MU] + 1;
        int64_t sf = lex_index(g, n) >> 1;
        T ph = (MU == 3 && g.antiperiodic && c[3] == g.L[3] - 1) ? T(-1) : T(1);
        Cx<T> psi[12], h[6], u[9], w[6];
        load_spinor<S>(in + sf * a.B + r, cstride, psi);
        project<MU, SF>(psi, h);
        load_link<S>(U + ((int64_t)(MU * 9) * 2 + p) * Vh + s, 2 * Vh, u);
        mul_link<false>(u, h, w);
        reconstruct<MU, SF>(acc, w, ph);
    }
    // backward neighbour x - mu (parity 1 - p), link U_mu(x - mu)^H at parity 1 - p
    {
        int n[4] = {c[0], c[1], c[2], c[3]};
        n[MU] = (c[MU] == 0) ? g.L[MU] - 1 : c[MU] - 1;
        int64_t sb = lex_index(g, n) >> 1;
        T ph = (MU == 3 && g.antiperiodic && c[3] == 0) ? T(-1) : T(1);
        Cx<T> psi[12], h[6], u[9], w[6];
        load_spinor<S>(in + sb * a.B + r, cstride, psi);
        project<MU, -SF>(psi, h);
        load_link<S>(U + ((int64_t)(MU * 9) * 2 + (1 - p)) * Vh + sb, 2 * Vh, u);
        mul_link<true>(u, h, w);
        reconstruct<MU, -SF>(acc, w, ph);
    }
}

// Workgroup index remap: hardware dispatches workgroup i to XCD i mod 8;
// give XCD j the contiguous logical range [j * per, (j+1) * per).
__device__ inline int64_t xcd_remap(int64_t bid, int64_t nblocks) {
    const int64_t nx = 8;
    int64_t per = (nblocks + nx - 1) / nx;
    int64_t xcd = bid % nx, k = bid / nx;
    int64_t full = nblocks % nx == 0 ? nx : nblocks % nx;   // XCDs that receive `per` blocks
    int64_t start = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1);
    return start + k;
}

template <typename S, bool DAG, bool G5OUT, bool XPAY>
__global__ __launch_bounds__(256) void hop_kernel(HopArgs a) {
    typedef typename Store<S>::acc T;
    typedef typename Store<S>::elem E;
    int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    int64_t gid = blk * blockDim.x + threadIdx.x;
    int64_t s;
    int r;
    if (a.bshift >= 0) { s = gid >> a.bshift; r = (int)(gid & (a.B - 1)); }
    else { s = gid / a.B; r = (int)(gid - s * a.B); }
    if (s >= a.g.Vh) return;
    int c[4];
    cb_coords(a.g, s, a.out_parity, c);
    Cx<T> acc[12];
#pragma unroll
    for (int i = 0; i < 12; i++) acc[i] = cmake<T>(0, 0);
    hop_dir<S, 0, DAG>(a, c, s, r, acc);
    hop_dir<S, 1, DAG>(a, c, s, r, acc);
    hop_dir<S, 2, DAG>(a, c, s, r, acc);
    hop_dir<S, 3, DAG>(a, c, s, r, acc);
    const int64_t cstride = a.g.Vh * a.B;
    const int64_t off = s * a.B + r;
    E* out = (E*)a.out;
    const T cb = (T)a.cb, ca = (T)a.ca;
#pragma unroll
    for (int i = 0; i < 12; i++) {
        Cx<T> v = cb * acc[i];
        if (XPAY) v = v + ca * Store<S>::ld((const E*)a.x + i * cstride + off);
        if (G5OUT && i >= 6) v = neg(v);
        Store<S>::st(out + i * cstride + off, v);
    }
}

template <typename S>
static int launch_hop(dht_ctx* c, int out_parity, const void* in, void* out, const void* x, double ca, double cb,
                      int nrhs, bool dagger, bool g5out) {
    HopArgs a;
    a.out = out;
    a.in = in;
    a.x = x;
    a.U = c->U[std::is_same<S, double>::value ? 0 : (std::is_same<S, float>::value ? 1 : 2)];
    a.g = c->g;
    a.out_parity = out_parity;
    a.B = nrhs;
    a.bshift = -1;
    for (int b = 0; b < 8; b++)
        if ((1 << b) == nrhs) a.bshift = b;
    a.ca = ca;
    a.cb = cb;
    int64_t nthreads = c->g.Vh * (int64_t)nrhs;
    dim3 grid((unsigned)((nthreads + 255) / 256)), block(256);
    bool xp = x != nullptr;
#define DHT_HOP_CASE(D_, G_, X_)                                                            \
    if (dagger == D_ && g5out == G_ && xp == X_) {                                          \
        hipLaunchKernelGGL((hop_kernel<S, D_, G_, X_>), grid, block, 0, c->stream, a);     \
        goto launched;                                                                      \
    }
    DHT_HOP_CASE(false, false, false)
    DHT_HOP_CASE(false, false, true)
    DHT_HOP_CASE(false, true, false)
    DHT_HOP_CASE(false, true, true)
    DHT_HOP_CASE(true, false, false)
    DHT_HOP_CASE(true, false, true)
    DHT_HOP_CASE(true, true, false)
    DHT_HOP_CASE(true, true, true)
#undef DHT_HOP_CASE
launched:
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

int hop(dht_ctx* c, int prec, int out_parity, const void* in, void* out, const void* x, double a, double b,
        int nrhs, bool dagger, bool g5out) {
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    if (prec < DHT_FP64 || prec > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    int tok;
    DHT_TRY(prof_begin(c, &tok));
    int rc = DHT_OK;
    switch (prec) {
        case DHT_FP64: rc = launch_hop<double>(c, out_parity, in, out, x, a, b, nrhs, dagger, g5out); break;
        case DHT_FP32: rc = launch_hop<float>(c, out_parity, in, out, x, a, b, nrhs, dagger, g5out); break;
        case DHT_BF16: rc = launch_hop<bf16x2>(c, out_parity, in, out, x, a, b, nrhs, dagger, g5out); break;
    }
    if (rc != DHT_OK) return rc;
    // algorithmic bytes: read the input half field (and the xpay source), write
    // the output, read each of the 8 Vh link matrices of this parity once
    const double eb = (double)elem_bytes(prec);
    const double bytes = (2.0 + (x ? 1.0 : 0.0)) * 12.0 * c->g.Vh * nrhs * eb + 72.0 * c->g.Vh * eb;
    return prof_end(c, tok, PROF_HOP64 + prec, bytes);
}

// g5 on a full field: copy, negating spin components 2 and 3 (c >= 6)
template <typename S>
__global__ void g5_kernel(const typename Store<S>::elem* in, typename Store<S>::elem* out, int64_t per_comp,
                          size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int comp = (int)((i / per_comp) % 12);
    auto v = Store<S>::ld(in + i);
    Store<S>::st(out + i, comp >= 6 ? neg(v) : v);
}

int g5_field(dht_ctx* c, int prec, const void* in, void* out, int nrhs) {
    size_t n = full_elems(c, nrhs);
    int64_t per = c->g.Vh * nrhs;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (prec) {
#define C_(P, T) case P: hipLaunchKernelGGL((g5_kernel<T>), grid, block, 0, c->stream, \
        (const typename Store<T>::elem*)in, (typename Store<T>::elem*)out, per, n); break;
        C_(DHT_FP64, double) C_(DHT_FP32, float) C_(DHT_BF16, bf16x2)
#undef C_
        default: return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// Full-lattice operators on full internal fields: D, D^H, g5, Q = g5 D.
int apply_full(dht_ctx* c, int op, int prec, const void* in, void* out, int nrhs) {
    if (op == DHT_OP_G5) return g5_field(c, prec, in, out, nrhs);
    if (op != DHT_OP_D && op != DHT_OP_DDAG && op != DHT_OP_Q) return set_error(DHT_ERR_INVALID_ARG, "bad operator");
    const size_t hb = half_elems(c, nrhs) * elem_bytes(prec);
    const char* ic = (const char*)in;
    char* oc = (char*)out;
    const double a = 4.0 + c->mass;
    for (int p = 0; p < 2; p++) {
        DHT_TRY(hop(c, prec, p, ic + (1 - p) * hb, oc + p * hb, ic + p * hb, a, -0.5, nrhs, op == DHT_OP_DDAG,
                    op == DHT_OP_Q));
    }
    return DHT_OK;
}

}  // namespace dht
