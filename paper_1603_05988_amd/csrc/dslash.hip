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
// of a site share the link loads and every 16-byte vector load of a
// wavefront is contiguous.  Site arithmetic is 32-bit; neighbours are found by
// offsets from the site's own index.  Accumulation in FP64 for FP64 storage,
// FP32 otherwise.  Workgroups are remapped so that each of the 8 XCDs walks
// a contiguous range of sites (neighbour reuse stays in one L2).  An optional
// epilogue reduces per-RHS dot products of the result (BiCGStab's (rhat, v),
// (t, s), (t, t)) into workgroup partial sums, saving a pass over the field.
#include <type_traits>

#include "internal.h"

namespace dht {

struct HopArgs {
    void* out;
    const void* in;
    const void* x;       // xpay source (same parity as out) or null
    const void* U;
    const void* da;      // dot operand a (HOPDOT_A_OUT)
    Cx<double>* partial;
    int Lx, Ly, Lz, Lt, Lxh;
    int Vh;
    int antiperiodic;
    int out_parity;
    int bshift;          // log2(B)
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

// 12 components of (site s, rhs r): 12 / VW vectors at stride Vh * B
template <typename S>
__device__ inline void load_spinor(const void* base, int64_t v0, int64_t vstride, Cx<typename Store<S>::acc>* p) {
    constexpr int VW = Store<S>::VW;
#pragma unroll
    for (int j = 0; j < 12 / VW; j++) Store<S>::ldv(base, v0 + j * vstride, p + j * VW);
}

template <typename S>
__device__ inline void load_link(const void* base, int64_t v0, Cx<typename Store<S>::acc>* u) {
    constexpr int VW = Store<S>::VW;
    constexpr int NV = (9 + VW - 1) / VW;
    Cx<typename Store<S>::acc> tmp[NV * VW];
#pragma unroll
    for (int j = 0; j < NV; j++) Store<S>::ldv(base, v0 + j, tmp + j * VW);
#pragma unroll
    for (int e = 0; e < 9; e++) u[e] = tmp[e];
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

// Ordering fence for the accumulation: the accumulators pass through an
// empty asm (so the arithmetic producing them cannot sink below it) that also
// clobbers memory (so later loads cannot rise above it).  Emits no code.
template <typename T>
__device__ inline void fence_acc(Cx<T>* acc) {
#pragma unroll
    for (int i = 0; i < 12; i++) asm volatile("" : "+v"(acc[i].re), "+v"(acc[i].im) : : "memory");
}

// one direction: forward neighbour sf (link at this site), backward sb (link at sb, other parity)
template <typename S, int MU, bool DAG>
__device__ inline void hop_dir(const HopArgs& a, int s, int sf, int sb, int r, bool phf, bool phb,
                               Cx<typename Store<S>::acc>* acc) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    constexpr int NV = (9 + VW - 1) / VW;
    const int p = a.out_parity;
    const int64_t vstride = (int64_t)a.Vh << a.bshift;
    constexpr int SF = DAG ? -1 : 1;   // sign of the forward projector (1 - SF g)
    {
        Cx<T> psi[12], h[6], u[9], w[6];
        load_spinor<S>(a.in, ((int64_t)sf << a.bshift) + r, vstride, psi);
        project<MU, SF>(psi, h);
        load_link<S>(a.U, ((int64_t)(MU * 2 + p) * a.Vh + s) * NV, u);
        mul_link<false>(u, h, w);
        reconstruct<MU, SF>(acc, w, phf ? T(-1) : T(1));
    }
    // keep each half-direction's loads next to their use: unfenced, the
    // optimiser issues all sixteen neighbour/link loads first and exhausts registers
    fence_acc(acc);
    {
        Cx<T> psi[12], h[6], u[9], w[6];
        load_spinor<S>(a.in, ((int64_t)sb << a.bshift) + r, vstride, psi);
        project<MU, -SF>(psi, h);
        load_link<S>(a.U, ((int64_t)(MU * 2 + (1 - p)) * a.Vh + sb) * NV, u);
        mul_link<true>(u, h, w);
        reconstruct<MU, -SF>(acc, w, phb ? T(-1) : T(1));
    }
    fence_acc(acc);
}

// Workgroup index remap: hardware dispatches workgroup i to XCD i mod 8;
// give XCD j the contiguous logical range [j * per, (j+1) * per).
__device__ inline int xcd_remap(int bid, int nblocks) {
    const int nx = 8;
    int per = (nblocks + nx - 1) / nx;
    int xcd = bid % nx, k = bid / nx;
    int full = nblocks % nx == 0 ? nx : nblocks % nx;   // XCDs that receive `per` blocks
    int start = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1);
    return start + k;
}

static constexpr int HOP_THREADS = 256;

template <typename S, bool DAG, bool G5OUT, bool XPAY, int DOT>
__global__ __launch_bounds__(HOP_THREADS) void hop_kernel(HopArgs a) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    constexpr int NP = DOT == HOPDOT_A_OUT ? 1 : (DOT == HOPDOT_OUT_X ? 2 : 0);
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int gid = blk * HOP_THREADS + threadIdx.x;
    const int B = 1 << a.bshift;
    const int s = gid >> a.bshift;
    const int r = gid & (B - 1);
    const bool live = s < a.Vh;
    Cx<double> d0 = cmake(0.0, 0.0), d1 = cmake(0.0, 0.0);
    if (live) {
        // coordinates of checkerboard site s
        const int xh = s % a.Lxh;
        int rest = s / a.Lxh;
        const int y = rest % a.Ly;
        rest /= a.Ly;
        const int z = rest % a.Lz;
        const int t = rest / a.Lz;
        const int x = 2 * xh + ((a.out_parity + y + z + t) & 1);
        const int row = s - xh;   // index of (x = 0, y, z, t) / 2
        const int sy = a.Lxh, sz = a.Lxh * a.Ly, st = sz * a.Lz;
        const int xf = x + 1 == a.Lx ? 0 : x + 1, xb = x == 0 ? a.Lx - 1 : x - 1;
        Cx<T> acc[12];
#pragma unroll
        for (int i = 0; i < 12; i++) acc[i] = cmake<T>(0, 0);
        hop_dir<S, 0, DAG>(a, s, row + (xf >> 1), row + (xb >> 1), r, false, false, acc);
        hop_dir<S, 1, DAG>(a, s, y == a.Ly - 1 ? s - (a.Ly - 1) * sy : s + sy, y == 0 ? s + (a.Ly - 1) * sy : s - sy,
                           r, false, false, acc);
        hop_dir<S, 2, DAG>(a, s, z == a.Lz - 1 ? s - (a.Lz - 1) * sz : s + sz, z == 0 ? s + (a.Lz - 1) * sz : s - sz,
                           r, false, false, acc);
        hop_dir<S, 3, DAG>(a, s, t == a.Lt - 1 ? s - (a.Lt - 1) * st : s + st, t == 0 ? s + (a.Lt - 1) * st : s - st,
                           r, a.antiperiodic && t == a.Lt - 1, a.antiperiodic && t == 0, acc);
        const int64_t vstride = (int64_t)a.Vh << a.bshift;
        const int64_t v0 = ((int64_t)s << a.bshift) + r;
        const T cb = (T)a.cb, ca = (T)a.ca;
        Cx<T> xv[12];
        if (XPAY) load_spinor<S>(a.x, v0, vstride, xv);
#pragma unroll
        for (int i = 0; i < 12; i++) {
            Cx<T> v = cb * acc[i];
            if (XPAY) v = v + ca * xv[i];
            if (G5OUT && i >= 6) v = neg(v);
            acc[i] = v;
        }
#pragma unroll
        for (int j = 0; j < 12 / VW; j++) Store<S>::stv(a.out, v0 + j * vstride, acc + j * VW);
        if (DOT != HOPDOT_NONE) {
            // the stored (rounded) values, so the sums match a separate pass
            Cx<T> ov[12];
#pragma unroll
            for (int i = 0; i < 12; i++) ov[i] = Store<S>::round(acc[i]);
            if (DOT == HOPDOT_A_OUT) {
                Cx<T> av[12];
                load_spinor<S>(a.da, v0, vstride, av);
#pragma unroll
                for (int i = 0; i < 12; i++)
                    d0 = d0 + conjmul(cmake<double>(av[i].re, av[i].im), cmake<double>(ov[i].re, ov[i].im));
            } else {
#pragma unroll
                for (int i = 0; i < 12; i++) {
                    Cx<double> o = cmake<double>(ov[i].re, ov[i].im);
                    d0 = d0 + conjmul(o, cmake<double>(xv[i].re, xv[i].im));
                    d1.re += o.re * o.re + o.im * o.im;
                }
            }
        }
    }
    if (NP > 0) {
        __shared__ Cx<double> red[NP > 0 ? NP : 1][HOP_THREADS];
        red[0][threadIdx.x] = d0;
        if (NP > 1) red[NP - 1][threadIdx.x] = d1;
        __syncthreads();
        for (int w = HOP_THREADS / 2; w >= B; w >>= 1) {
            if ((int)threadIdx.x < w) {
#pragma unroll
                for (int q = 0; q < NP; q++) red[q][threadIdx.x] = red[q][threadIdx.x] + red[q][threadIdx.x + w];
            }
            __syncthreads();
        }
        if ((int)threadIdx.x < B) {
#pragma unroll
            for (int q = 0; q < NP; q++) a.partial[((int64_t)blk * NP + q) * B + threadIdx.x] = red[q][threadIdx.x];
        }
    }
}

int hop_blocks(const dht_ctx* c, int nrhs) {
    int64_t n = c->g.Vh * (int64_t)nrhs;
    return (int)((n + HOP_THREADS - 1) / HOP_THREADS);
}

template <typename S>
static int launch_hop(dht_ctx* c, int out_parity, const void* in, void* out, const void* x, double ca, double cb,
                      int nrhs, bool dagger, bool g5out, HopDot* dot) {
    HopArgs a;
    a.out = out;
    a.in = in;
    a.x = x;
    a.U = c->U[std::is_same<S, double>::value ? 0 : (std::is_same<S, float>::value ? 1 : 2)];
    a.Lx = c->g.L[0];
    a.Ly = c->g.L[1];
    a.Lz = c->g.L[2];
    a.Lt = c->g.L[3];
    a.Lxh = c->g.Lxh;
    a.Vh = (int)c->g.Vh;
    a.antiperiodic = c->g.antiperiodic;
    a.out_parity = out_parity;
    a.bshift = -1;
    for (int b = 0; b < 9; b++)
        if ((1 << b) == nrhs) a.bshift = b;
    if (a.bshift < 0) return set_error(DHT_ERR_INVALID_ARG, "internal batch must be a power of two <= 256");
    a.ca = ca;
    a.cb = cb;
    int kind = dot ? dot->kind : HOPDOT_NONE;
    a.da = dot ? dot->a : nullptr;
    a.partial = dot ? dot->partial : nullptr;
    if (kind == HOPDOT_OUT_X && !x) return set_error(DHT_ERR_INVALID_ARG, "fused (out, x) needs an xpay source");
    const int nb = hop_blocks(c, nrhs);
    if (dot) dot->nblocks = nb;
    dim3 grid(nb), block(HOP_THREADS);
    bool xp = x != nullptr;
#define DHT_HOP_CASE(D_, G_, X_, K_)                                                               \
    if (dagger == D_ && g5out == G_ && xp == X_ && kind == K_) {                                   \
        hipLaunchKernelGGL((hop_kernel<S, D_, G_, X_, K_>), grid, block, 0, c->stream, a);        \
        goto launched;                                                                             \
    }
    DHT_HOP_CASE(false, false, false, HOPDOT_NONE)
    DHT_HOP_CASE(false, false, true, HOPDOT_NONE)
    DHT_HOP_CASE(false, true, false, HOPDOT_NONE)
    DHT_HOP_CASE(false, true, true, HOPDOT_NONE)
    DHT_HOP_CASE(true, false, false, HOPDOT_NONE)
    DHT_HOP_CASE(true, false, true, HOPDOT_NONE)
    DHT_HOP_CASE(true, true, false, HOPDOT_NONE)
    DHT_HOP_CASE(true, true, true, HOPDOT_NONE)
    DHT_HOP_CASE(false, false, true, HOPDOT_A_OUT)
    DHT_HOP_CASE(false, false, true, HOPDOT_OUT_X)
#undef DHT_HOP_CASE
    return set_error(DHT_ERR_INVALID_ARG, "unsupported hop variant");
launched:
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

int hop(dht_ctx* c, int prec, int out_parity, const void* in, void* out, const void* x, double a, double b,
        int nrhs, bool dagger, bool g5out, HopDot* dot) {
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    if (prec < DHT_FP64 || prec > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    int tok;
    DHT_TRY(prof_begin(c, &tok));
    int rc = DHT_OK;
    switch (prec) {
        case DHT_FP64: rc = launch_hop<double>(c, out_parity, in, out, x, a, b, nrhs, dagger, g5out, dot); break;
        case DHT_FP32: rc = launch_hop<float>(c, out_parity, in, out, x, a, b, nrhs, dagger, g5out, dot); break;
        case DHT_BF16: rc = launch_hop<bf16x2>(c, out_parity, in, out, x, a, b, nrhs, dagger, g5out, dot); break;
    }
    if (rc != DHT_OK) return rc;
    // algorithmic bytes: read the input half field (and the xpay / dot operand),
    // write the output, read each of the 8 Vh link matrices of this parity once
    const double eb = (double)elem_bytes(prec);
    double nfield = 2.0 + (x ? 1.0 : 0.0) + ((dot && dot->kind == HOPDOT_A_OUT) ? 1.0 : 0.0);
    const double bytes = nfield * 12.0 * c->g.Vh * nrhs * eb + 72.0 * c->g.Vh * eb;
    return prof_end(c, tok, PROF_HOP64 + prec, bytes);
}

// g5 on a full field: negate spin components 2 and 3 (c >= 6)
template <typename S>
__global__ void g5_kernel(const void* in, void* out, int64_t per_group, size_t nvec) {
    constexpr int VW = Store<S>::VW;
    size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvec) return;
    int cv = (int)((v / per_group) % (12 / VW));
    Cx<typename Store<S>::acc> e[VW];
    Store<S>::ldv(in, v, e);
#pragma unroll
    for (int j = 0; j < VW; j++)
        if (cv * VW + j >= 6) e[j] = neg(e[j]);
    Store<S>::stv(out, v, e);
}

int g5_field(dht_ctx* c, int prec, const void* in, void* out, int nrhs) {
    const int VW = vec_width(prec);
    size_t nvec = full_elems(c, nrhs) / VW;
    int64_t per = c->g.Vh * nrhs;
    dim3 grid((unsigned)((nvec + 255) / 256)), block(256);
    switch (prec) {
        case DHT_FP64: hipLaunchKernelGGL(g5_kernel<double>, grid, block, 0, c->stream, in, out, per, nvec); break;
        case DHT_FP32: hipLaunchKernelGGL(g5_kernel<float>, grid, block, 0, c->stream, in, out, per, nvec); break;
        case DHT_BF16: hipLaunchKernelGGL(g5_kernel<bf16x2>, grid, block, 0, c->stream, in, out, per, nvec); break;
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
