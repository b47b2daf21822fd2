// Reductions and vector updates for the batched Krylov solvers.
//
// Every dot product is accumulated in FP64: each lane converts its products
// to double, lanes of one RHS are combined by a fixed-order tree in LDS, and
// the per-workgroup partial sums are added in workgroup order by a one-block
// finalise kernel.  The result is therefore deterministic for a fixed grid.
//
// Per-RHS solver scalars live on the device (struct RhsState) and are read by
// the update kernels, so a BiCGStab iteration needs no host round trip.
#include <algorithm>
#include <type_traits>

#include "solver.h"

namespace dht {

static constexpr int RED_THREADS = 256;
static constexpr int RED_MAX_BLOCKS = 1024;

static int pow2_at_least(int b) {
    int p = 1;
    while (p < b) p <<= 1;
    return p;
}

// --------------------------------------------------------------------------
// generic multi-dot: out[pair][r] = sum conj(a_pair) b_pair over one field
// --------------------------------------------------------------------------
template <typename S, int NP>
__global__ __launch_bounds__(RED_THREADS) void dot_partials_kernel(DotArgs d) {
    typedef typename Store<S>::elem E;
    __shared__ Cx<double> red[NP][RED_THREADS];
    const int tid = threadIdx.x;
    const int Bp = d.Bp;
    const int r = tid & (Bp - 1);
    const int sites_per_block = RED_THREADS / Bp;
    Cx<double> acc[NP];
#pragma unroll
    for (int i = 0; i < NP; i++) acc[i] = cmake(0.0, 0.0);
    if (r < d.B) {
        for (int64_t s = (int64_t)blockIdx.x * sites_per_block + tid / Bp; s < d.nsite;
             s += (int64_t)gridDim.x * sites_per_block) {
            for (int c = 0; c < 12; c++) {
                int64_t o = ((int64_t)c * d.nsite + s) * d.B + r;
#pragma unroll
                for (int i = 0; i < NP; i++) {
                    auto x = Store<S>::ld((const E*)d.a[i] + o);
                    auto y = Store<S>::ld((const E*)d.b[i] + o);
                    acc[i] = acc[i] + conjmul(cmake<double>(x.re, x.im), cmake<double>(y.re, y.im));
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NP; i++) red[i][tid] = acc[i];
    __syncthreads();
    for (int st = RED_THREADS / 2; st >= Bp; st >>= 1) {
        if (tid < st) {
#pragma unroll
            for (int i = 0; i < NP; i++) red[i][tid] = red[i][tid] + red[i][tid + st];
        }
        __syncthreads();
    }
    if (tid < d.B) {
#pragma unroll
        for (int i = 0; i < NP; i++) d.partial[((int64_t)blockIdx.x * NP + i) * d.B + tid] = red[i][tid];
    }
}

int dot_blocks(int64_t nsite, int Bp) {
    int64_t spb = RED_THREADS / Bp;
    int64_t nb = (nsite + spb - 1) / spb;
    return (int)(nb < RED_MAX_BLOCKS ? nb : RED_MAX_BLOCKS);
}

template <typename S>
static int launch_dots_t(dht_ctx* c, DotArgs& d, int np, hipStream_t st) {
    dim3 grid(d.nblocks), block(RED_THREADS);
    switch (np) {
        case 1: hipLaunchKernelGGL((dot_partials_kernel<S, 1>), grid, block, 0, st, d); break;
        case 2: hipLaunchKernelGGL((dot_partials_kernel<S, 2>), grid, block, 0, st, d); break;
        case 3: hipLaunchKernelGGL((dot_partials_kernel<S, 3>), grid, block, 0, st, d); break;
        default: return set_error(DHT_ERR_INVALID_ARG, "npair must be 1..3");
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

int launch_dot_partials(dht_ctx* c, int prec, int np, const void* const* a, const void* const* b, int64_t nsite,
                        int nrhs, Cx<double>* partial, int* nblocks_out) {
    DotArgs d;
    for (int i = 0; i < 3; i++) {
        d.a[i] = i < np ? a[i] : nullptr;
        d.b[i] = i < np ? b[i] : nullptr;
    }
    d.nsite = nsite;
    d.B = nrhs;
    d.Bp = pow2_at_least(nrhs);
    if (d.Bp > RED_THREADS) return set_error(DHT_ERR_INVALID_ARG, "too many right-hand sides for a reduction");
    d.partial = partial;
    d.nblocks = dot_blocks(nsite, d.Bp);
    *nblocks_out = d.nblocks;
    switch (prec) {
        case DHT_FP64: return launch_dots_t<double>(c, d, np, c->stream);
        case DHT_FP32: return launch_dots_t<float>(c, d, np, c->stream);
        case DHT_BF16: return launch_dots_t<bf16x2>(c, d, np, c->stream);
    }
    return set_error(DHT_ERR_INVALID_ARG, "bad precision");
}

// sum partials over blocks: out[pair][r]
__global__ void sum_partials_kernel(const Cx<double>* partial, int nblocks, int np, int B, Cx<double>* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np * B) return;
    int pair = i / B, r = i - pair * B;
    Cx<double> s = cmake(0.0, 0.0);
    for (int b = 0; b < nblocks; b++) s = s + partial[((int64_t)b * np + pair) * B + r];
    out[i] = s;
}

int dots(dht_ctx* c, int prec, int np, const void* const* a, const void* const* b, int64_t nsite, int nrhs,
         Cx<double>* out_dev) {
    void* part;
    DHT_TRY(ws_get(c, WS_PARTIAL, (size_t)RED_MAX_BLOCKS * 3 * nrhs * sizeof(Cx<double>), &part));
    int nb;
    DHT_TRY(launch_dot_partials(c, prec, np, a, b, nsite, nrhs, (Cx<double>*)part, &nb));
    hipLaunchKernelGGL(sum_partials_kernel, dim3((np * nrhs + 63) / 64), dim3(64), 0, c->stream,
                       (const Cx<double>*)part, nb, np, nrhs, out_dev);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// --------------------------------------------------------------------------
// BiCGStab scalar updates (one thread per RHS)
// --------------------------------------------------------------------------
__device__ inline Cx<double> cdiv(Cx<double> a, Cx<double> b) {
    double d = b.re * b.re + b.im * b.im;
    return cmake((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
__device__ inline double cabs2(Cx<double> a) { return a.re * a.re + a.im * a.im; }
__device__ inline bool cfinite(Cx<double> a) { return isfinite(a.re) && isfinite(a.im); }

__global__ void finalize_kernel(const Cx<double>* partial, int nblocks, int np, int B, RhsState* st, int op,
                                double bd_eps) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B) return;
    Cx<double> v[3];
    for (int pair = 0; pair < np; pair++) {
        Cx<double> s = cmake(0.0, 0.0);
        for (int b = 0; b < nblocks; b++) s = s + partial[((int64_t)b * np + pair) * B + r];
        v[pair] = s;
    }
    RhsState& x = st[r];
    if (op == FIN_INIT) {   // v0 = (r, r) with rhat = r = b
        x.rnorm2 = v[0].re;
        x.rhat2 = v[0].re;
        x.rho = cmake(1.0, 0.0);
        x.alpha = cmake(1.0, 0.0);
        x.omega = cmake(1.0, 0.0);
        x.beta = cmake(0.0, 0.0);
        x.iters = 0;
        if (!isfinite(v[0].re)) { x.active = 0; x.status = RS_NAN; }
        else if (x.rnorm2 <= x.target2) { x.active = 0; x.status = RS_CONVERGED; }
        else { x.active = 1; x.status = RS_RUNNING; }
        return;
    }
    if (!x.active) return;
    if (op == FIN_ALPHA) {   // v0 = (rhat, v)
        if (!cfinite(v[0])) { x.active = 0; x.status = RS_NAN; return; }
        if (cabs2(v[0]) == 0.0) { x.active = 0; x.status = RS_BREAKDOWN; return; }
        x.alpha = cdiv(x.rho, v[0]);
    } else if (op == FIN_OMEGA) {   // v0 = (t, s), v1 = (t, t)
        if (!cfinite(v[0]) || !isfinite(v[1].re)) { x.active = 0; x.status = RS_NAN; return; }
        x.omega = v[1].re > 0.0 ? cmake(v[0].re / v[1].re, v[0].im / v[1].re) : cmake(0.0, 0.0);
    } else if (op == FIN_RHO) {     // v0 = (rhat, r), v1 = (r, r)
        x.iters++;
        x.rnorm2 = v[1].re;
        if (!cfinite(v[0]) || !isfinite(v[1].re)) { x.active = 0; x.status = RS_NAN; return; }
        if (x.rnorm2 <= x.target2) { x.active = 0; x.status = RS_CONVERGED; return; }
        if (cabs2(x.omega) == 0.0 || cabs2(v[0]) <= bd_eps * bd_eps * x.rhat2 * x.rnorm2) {
            x.active = 0; x.status = RS_BREAKDOWN; return;
        }
        x.beta = cdiv(v[0], x.rho) * cdiv(x.alpha, x.omega);
        x.rho = v[0];
    }
}

int finalize(dht_ctx* c, const Cx<double>* partial, int nblocks, int np, int nrhs, RhsState* st, int op, double bd_eps) {
    hipLaunchKernelGGL(finalize_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, partial, nblocks, np, nrhs, st,
                       op, bd_eps);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// --------------------------------------------------------------------------
// vector updates (elementwise over [12][nsite][B]; r = index mod B)
// --------------------------------------------------------------------------
template <typename S>
__global__ void p_update_kernel(typename Store<S>::elem* p, const typename Store<S>::elem* r_,
                                const typename Store<S>::elem* v, const RhsState* st, size_t n, int B) {
    typedef typename Store<S>::acc T;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int r = (int)(i % B);
    const RhsState& x = st[r];
    if (!x.active) return;
    Cx<T> beta = cmake<T>((T)x.beta.re, (T)x.beta.im), om = cmake<T>((T)x.omega.re, (T)x.omega.im);
    Cx<T> pv = Store<S>::ld(p + i), rv = Store<S>::ld(r_ + i), vv = Store<S>::ld(v + i);
    Store<S>::st(p + i, rv + beta * (pv - om * vv));
}

template <typename S>
__global__ void s_update_kernel(typename Store<S>::elem* s, const typename Store<S>::elem* r_,
                                const typename Store<S>::elem* v, const RhsState* st, size_t n, int B) {
    typedef typename Store<S>::acc T;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int r = (int)(i % B);
    const RhsState& x = st[r];
    if (!x.active) return;
    Cx<T> al = cmake<T>((T)x.alpha.re, (T)x.alpha.im);
    Store<S>::st(s + i, Store<S>::ld(r_ + i) - al * Store<S>::ld(v + i));
}

template <typename S>
__global__ void xr_update_kernel(typename Store<S>::elem* x_, typename Store<S>::elem* r_,
                                 const typename Store<S>::elem* p, const typename Store<S>::elem* s,
                                 const typename Store<S>::elem* t, const RhsState* st, size_t n, int B) {
    typedef typename Store<S>::acc T;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int r = (int)(i % B);
    const RhsState& x = st[r];
    if (!x.active) return;
    Cx<T> al = cmake<T>((T)x.alpha.re, (T)x.alpha.im), om = cmake<T>((T)x.omega.re, (T)x.omega.im);
    Cx<T> sv = Store<S>::ld(s + i);
    Store<S>::st(x_ + i, Store<S>::ld(x_ + i) + al * Store<S>::ld(p + i) + om * sv);
    Store<S>::st(r_ + i, sv - om * Store<S>::ld(t + i));
}

static dim3 egrid(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

int p_update(dht_ctx* c, int prec, void* p, const void* r, const void* v, const RhsState* st, size_t n, int B) {
    switch (prec) {
#define C_(P, T) case P: hipLaunchKernelGGL((p_update_kernel<T>), egrid(n), dim3(256), 0, c->stream, \
        (typename Store<T>::elem*)p, (const typename Store<T>::elem*)r, (const typename Store<T>::elem*)v, st, n, B); break;
        C_(DHT_FP64, double) C_(DHT_FP32, float) C_(DHT_BF16, bf16x2)
#undef C_
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}
int s_update(dht_ctx* c, int prec, void* s, const void* r, const void* v, const RhsState* st, size_t n, int B) {
    switch (prec) {
#define C_(P, T) case P: hipLaunchKernelGGL((s_update_kernel<T>), egrid(n), dim3(256), 0, c->stream, \
        (typename Store<T>::elem*)s, (const typename Store<T>::elem*)r, (const typename Store<T>::elem*)v, st, n, B); break;
        C_(DHT_FP64, double) C_(DHT_FP32, float) C_(DHT_BF16, bf16x2)
#undef C_
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}
int xr_update(dht_ctx* c, int prec, void* x, void* r, const void* p, const void* s, const void* t, const RhsState* st,
              size_t n, int B) {
    switch (prec) {
#define C_(P, T) case P: hipLaunchKernelGGL((xr_update_kernel<T>), egrid(n), dim3(256), 0, c->stream, \
        (typename Store<T>::elem*)x, (typename Store<T>::elem*)r, (const typename Store<T>::elem*)p, \
        (const typename Store<T>::elem*)s, (const typename Store<T>::elem*)t, st, n, B); break;
        C_(DHT_FP64, double) C_(DHT_FP32, float) C_(DHT_BF16, bf16x2)
#undef C_
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// --------------------------------------------------------------------------
// defect-correction helpers
// --------------------------------------------------------------------------
// out_lo = scale[r] * in_hi  (scale = 1 / ||r||, 0 for finished RHS)
template <typename SO>
__global__ void scale_down_kernel(const Cx<double>* in, typename Store<SO>::elem* out, const double* scale, size_t n,
                                  int B) {
    typedef typename Store<SO>::acc T;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sc = scale[i % B];
    Cx<double> v = in[i];
    Store<SO>::st(out + i, cmake<T>((T)(sc * v.re), (T)(sc * v.im)));
}
// x_hi += scale[r] * e_lo
template <typename SI>
__global__ void accum_up_kernel(Cx<double>* x, const typename Store<SI>::elem* e, const double* scale, size_t n, int B) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sc = scale[i % B];
    if (sc == 0.0) return;
    auto v = Store<SI>::ld(e + i);
    x[i] = cmake(x[i].re + sc * (double)v.re, x[i].im + sc * (double)v.im);
}

int scale_down(dht_ctx* c, const void* in, void* out, int pout, const double* scale, size_t n, int B) {
    switch (pout) {
#define C_(P, T) case P: hipLaunchKernelGGL((scale_down_kernel<T>), egrid(n), dim3(256), 0, c->stream, \
        (const Cx<double>*)in, (typename Store<T>::elem*)out, scale, n, B); break;
        C_(DHT_FP64, double) C_(DHT_FP32, float) C_(DHT_BF16, bf16x2)
#undef C_
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}
int accum_up(dht_ctx* c, void* x, const void* e, int pin, const double* scale, size_t n, int B) {
    switch (pin) {
#define C_(P, T) case P: hipLaunchKernelGGL((accum_up_kernel<T>), egrid(n), dim3(256), 0, c->stream, \
        (Cx<double>*)x, (const typename Store<T>::elem*)e, scale, n, B); break;
        C_(DHT_FP64, double) C_(DHT_FP32, float) C_(DHT_BF16, bf16x2)
#undef C_
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// y = a - b (FP64 elementwise) -- residual r = b - A x
__global__ void sub_kernel(const Cx<double>* a, const Cx<double>* b, Cx<double>* y, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = a[i] - b[i];
}
int sub(dht_ctx* c, const void* a, const void* b, void* y, size_t n) {
    hipLaunchKernelGGL(sub_kernel, egrid(n), dim3(256), 0, c->stream, (const Cx<double>*)a, (const Cx<double>*)b,
                       (Cx<double>*)y, n);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// fill with zero (a kernel rather than a memset so that the stream can be captured)
// grid-stride: the deflation basis can exceed 2^32 words (a launch is capped at 2^32 threads)
__global__ void zero_kernel(uint4* p, size_t n16, uint32_t* tail, size_t ntail) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t j = i; j < n16; j += stride) p[j] = make_uint4(0u, 0u, 0u, 0u);
    for (size_t j = i; j < ntail; j += stride) tail[j] = 0u;
}
int zero(dht_ctx* c, void* p, size_t bytes) {
    size_t n = bytes / 4;
    if (n == 0) return DHT_OK;
    size_t n16 = ((uintptr_t)p & 15) ? 0 : n / 4;   // 16-byte stores only on aligned buffers
    size_t blocks = std::min<size_t>((n16 + 255) / 256, 65536);
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, c->stream, (uint4*)p, n16,
                       (uint32_t*)p + 4 * n16, n - 4 * n16);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

}  // namespace dht
