// Reductions and vector updates for the batched Krylov solvers.
//
// Fields are arrays of 16-byte vectors (VW complex numbers of one site and
// RHS); with the batch B a power of two the RHS of vector v is v & (B - 1),
// so these kernels do not depend on the site layout.
//
// Every dot product is accumulated in FP64: each lane converts its products
// to double, the lanes of one RHS are combined by a fixed-order tree in LDS,
// and the per-workgroup partial sums are added in workgroup order by the
// finalise kernel (one workgroup per RHS).  Results are deterministic for a
// fixed grid.  Per-RHS solver scalars live on the device (struct RhsState)
// and are read by the update kernels, so a BiCGStab iteration needs no host
// round trip.
#include <algorithm>
#include <type_traits>

#include "solver.h"

namespace dht {

static constexpr int RED_THREADS = 256;
static constexpr int RED_MAX_BLOCKS = 16384;

static int red_blocks(size_t nvec) {
    size_t nb = (nvec + RED_THREADS - 1) / RED_THREADS;
    return (int)std::max<size_t>(1, std::min<size_t>(nb, RED_MAX_BLOCKS));
}

// Position v = cv * SB + sr of a grid-stride loop over vectors whose
// component groups lie SB apart, advanced without a 64-bit division per step
struct StridePos {
    int64_t cv, sr, qs, rs, SB;
    __device__ StridePos(size_t v0, size_t stride, int64_t SB_) : SB(SB_) {
        cv = (int64_t)v0 / SB;
        sr = (int64_t)v0 - cv * SB;
        qs = (int64_t)stride / SB;
        rs = (int64_t)stride - qs * SB;
    }
    __device__ void next() {
        cv += qs;
        sr += rs;
        if (sr >= SB) {
            sr -= SB;
            cv++;
        }
    }
};

// fixed-order tree over the RED_THREADS lanes down to B entries (lane r keeps RHS r)
template <int NP>
__device__ inline void block_reduce_rhs(Cx<double> (*red)[RED_THREADS], int B) {
    __syncthreads();
    for (int w = RED_THREADS / 2; w >= B; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < NP; q++) red[q][threadIdx.x] = red[q][threadIdx.x] + red[q][threadIdx.x + w];
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// generic multi-dot: partial[block][pair][r] = sum conj(a_pair) b_pair
// --------------------------------------------------------------------------
template <typename S, int NP>
__global__ __launch_bounds__(RED_THREADS) void dot_partials_kernel(DotArgs d) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    __shared__ Cx<double> red[NP][RED_THREADS];
    Cx<double> acc[NP];
#pragma unroll
    for (int i = 0; i < NP; i++) acc[i] = cmake(0.0, 0.0);
    const size_t stride = (size_t)gridDim.x * RED_THREADS;
    for (size_t v = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; v < d.nvec; v += stride) {
#pragma unroll
        for (int i = 0; i < NP; i++) {
            Cx<T> x[VW], y[VW];
            Store<S>::ldv(d.a[i], v, x);
            Store<S>::ldv(d.b[i], v, y);
#pragma unroll
            for (int j = 0; j < VW; j++)
                acc[i] = acc[i] + conjmul(cmake<double>(x[j].re, x[j].im), cmake<double>(y[j].re, y[j].im));
        }
    }
#pragma unroll
    for (int i = 0; i < NP; i++) red[i][threadIdx.x] = acc[i];
    block_reduce_rhs<NP>(red, d.B);
    if ((int)threadIdx.x < d.B) {
#pragma unroll
        for (int i = 0; i < NP; i++) d.partial[((int64_t)blockIdx.x * NP + i) * d.B + threadIdx.x] = red[i][threadIdx.x];
    }
}

int launch_dot_partials(dht_ctx* c, int prec, int np, const void* const* a, const void* const* b, size_t nvec,
                        int nrhs, Cx<double>* partial, int* nblocks_out) {
    if (nrhs > RED_THREADS || (nrhs & (nrhs - 1))) return set_error(DHT_ERR_INVALID_ARG, "batch must be a power of two <= 256");
    DotArgs d;
    for (int i = 0; i < 3; i++) {
        d.a[i] = i < np ? a[i] : nullptr;
        d.b[i] = i < np ? b[i] : nullptr;
    }
    d.nvec = nvec;
    d.B = nrhs;
    d.partial = partial;
    d.nblocks = red_blocks(nvec);
    *nblocks_out = d.nblocks;
    dim3 grid(d.nblocks), block(RED_THREADS);
#define DHT_DOT(P, T)                                                                              \
    if (prec == P) {                                                                               \
        if (np == 1) hipLaunchKernelGGL((dot_partials_kernel<T, 1>), grid, block, 0, c->stream, d); \
        else if (np == 2) hipLaunchKernelGGL((dot_partials_kernel<T, 2>), grid, block, 0, c->stream, d); \
        else hipLaunchKernelGGL((dot_partials_kernel<T, 3>), grid, block, 0, c->stream, d);       \
        DHT_HIP(hipGetLastError());                                                                \
        return DHT_OK;                                                                             \
    }
    if (np < 1 || np > 3) return set_error(DHT_ERR_INVALID_ARG, "npair must be 1..3");
    DHT_DOT(DHT_FP64, double)
    DHT_DOT(DHT_FP32, float)
    DHT_DOT(DHT_BF16, bf16x2)
#undef DHT_DOT
    return set_error(DHT_ERR_INVALID_ARG, "bad precision");
}

// --------------------------------------------------------------------------
// finalise: one workgroup per RHS sums the partials in a fixed order, then
// (op != FIN_SUM) applies the BiCGStab scalar update for that RHS
// --------------------------------------------------------------------------
__device__ inline Cx<double> cdiv(Cx<double> a, Cx<double> b) {
    double d = b.re * b.re + b.im * b.im;
    return cmake((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
__device__ inline double cabs2(Cx<double> a) { return a.re * a.re + a.im * a.im; }
__device__ inline bool cfinite(Cx<double> a) { return isfinite(a.re) && isfinite(a.im); }

__device__ void state_update(RhsState& x, const Cx<double>* v, int op, double bd_eps) {
    if (op == FIN_INIT) {   // v0 = (r, r) with rhat = r = b
        x.rnorm2 = v[0].re;
        x.rhat2 = v[0].re;
        x.rho = cmake(v[0].re, 0.0);   // (rhat, r) with rhat = r
        x.alpha = cmake(1.0, 0.0);
        x.omega = cmake(1.0, 0.0);
        x.beta = cmake(0.0, 0.0);
        x.iters = 0;
        if (x.target2 < 0.0) { x.active = 0; x.status = RS_CONVERGED; }   // not part of this solve
        else if (!isfinite(v[0].re)) { x.active = 0; x.status = RS_NAN; }
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

__global__ __launch_bounds__(RED_THREADS) void finalize_kernel(const Cx<double>* partial, int nblocks, int np, int B,
                                                               RhsState* st, int op, double bd_eps, Cx<double>* sums) {
    __shared__ Cx<double> red[RED_THREADS];
    __shared__ Cx<double> v[3];
    const int r = blockIdx.x;
    for (int pair = 0; pair < np; pair++) {
        Cx<double> s = cmake(0.0, 0.0);
        for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) s = s + partial[((int64_t)b * np + pair) * B + r];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) v[pair] = red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (sums)
            for (int pair = 0; pair < np; pair++) sums[pair * B + r] = v[pair];
        if (op != FIN_SUM) state_update(st[r], v, op, bd_eps);
    }
}

// First stage for long partial lists (one row per hop workgroup): workgroup f
// sums a contiguous slice of rows [b][np * B]; the rows are read coalesced.
static constexpr int FOLD_ROWS = 256;
__global__ __launch_bounds__(RED_THREADS) void fold_partials_kernel(const Cx<double>* partial, int nblocks, int w,
                                                                    Cx<double>* out) {
    __shared__ Cx<double> red[RED_THREADS];
    const int per = (nblocks + gridDim.x - 1) / gridDim.x;
    const int b0 = blockIdx.x * per, b1 = min(nblocks, b0 + per);
    const int rows = RED_THREADS / w;   // rows summed side by side (w <= RED_THREADS)
    const int col = threadIdx.x % w, slot = threadIdx.x / w;
    Cx<double> s = cmake(0.0, 0.0);
    if (slot < rows)
        for (int b = b0 + slot; b < b1; b += rows) s = s + partial[(int64_t)b * w + col];
    red[threadIdx.x] = s;
    __syncthreads();
    if (slot == 0) {
        for (int q = 1; q < rows; q++) s = s + red[q * w + col];
        out[(int64_t)blockIdx.x * w + col] = s;
    }
}

int finalize(dht_ctx* c, const Cx<double>* partial, int nblocks, int np, int nrhs, RhsState* st, int op, double bd_eps,
             Cx<double>* sums) {
    const int w = np * nrhs;
    if (nblocks > 4 * FOLD_ROWS && w <= RED_THREADS) {
        void* fold;
        DHT_TRY(ws_get(c, WS_FOLD, sizeof(Cx<double>) * FOLD_ROWS * RED_THREADS, &fold));
        hipLaunchKernelGGL(fold_partials_kernel, dim3(FOLD_ROWS), dim3(RED_THREADS), 0, c->stream, partial, nblocks, w,
                           (Cx<double>*)fold);
        DHT_HIP(hipGetLastError());
        partial = (const Cx<double>*)fold;
        nblocks = FOLD_ROWS;
    }
    hipLaunchKernelGGL(finalize_kernel, dim3(nrhs), dim3(RED_THREADS), 0, c->stream, partial, nblocks, np, nrhs, st,
                       op, bd_eps, sums);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

int dots(dht_ctx* c, int prec, int np, const void* const* a, const void* const* b, size_t nvec, int nrhs,
         Cx<double>* out_dev) {
    void* part;
    DHT_TRY(ws_get(c, WS_PARTIAL, partial_bytes(c, nrhs), &part));
    int nb;
    DHT_TRY(launch_dot_partials(c, prec, np, a, b, nvec, nrhs, (Cx<double>*)part, &nb));
    return finalize(c, (const Cx<double>*)part, nb, np, nrhs, nullptr, FIN_SUM, 0.0, out_dev);
}

size_t partial_bytes(const dht_ctx* c, int nrhs) {
    // enough for a fused hop epilogue (one partial per hop workgroup, at most
    // hop_blocks + nrhs of them with RHS groups) with 3 pairs
    size_t nb = std::max<size_t>(RED_MAX_BLOCKS, (size_t)hop_blocks(c, nrhs) + nrhs);
    return nb * 3 * nrhs * sizeof(Cx<double>);
}

// reduction workspace of a fused epilogue or a generic dot: partials and the
// fold of a long partial list
void ws_plan_dots(const dht_ctx* c, int nrhs, size_t* plan) {
    plan_max(plan, WS_PARTIAL, partial_bytes(c, nrhs));
    plan_max(plan, WS_FOLD, sizeof(Cx<double>) * FOLD_ROWS * RED_THREADS);
}

// --------------------------------------------------------------------------
// vector updates (one lane per 16-byte vector; r = v & (B - 1))
// --------------------------------------------------------------------------
template <typename T> __device__ inline Cx<T> cscal(Cx<double> a) { return cmake<T>((T)a.re, (T)a.im); }

template <typename S>
__global__ void p_update_kernel(void* p, const void* p_in, const void* r_, const void* v, const RhsState* st,
                                size_t nvec, int B) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nvec) return;
    const RhsState& x = st[i & (B - 1)];
    if (!x.active) return;
    Cx<T> beta = cscal<T>(x.beta), om = cscal<T>(x.omega);
    Cx<T> pv[VW], rv[VW], vv[VW];
    Store<S>::ldv(p_in, i, pv);
    Store<S>::ldv(r_, i, rv);
    Store<S>::ldv(v, i, vv);
#pragma unroll
    for (int j = 0; j < VW; j++) pv[j] = rv[j] + beta * (pv[j] - om * vv[j]);
    Store<S>::stv(p, i, pv);
}

template <typename S>
__global__ void s_update_kernel(void* s, const void* r_, const void* v, const RhsState* st, size_t nvec, int B) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nvec) return;
    const RhsState& x = st[i & (B - 1)];
    if (!x.active) return;
    Cx<T> al = cscal<T>(x.alpha);
    Cx<T> rv[VW], vv[VW];
    Store<S>::ldv(r_, i, rv);
    Store<S>::ldv(v, i, vv);
#pragma unroll
    for (int j = 0; j < VW; j++) rv[j] = rv[j] - al * vv[j];
    Store<S>::stv(s, i, rv);
}

// x += alpha p + omega s;  r = s - omega t;  partials of (rhat, r) and (r, r).
// X32: x is kept in FP32 storage (vector index cv * SB + sr of S holds
// components VW cv .. VW cv + VW - 1, which FP32 keeps in VW / 2 vectors)
template <typename S, bool X32>
__device__ inline void ld_x(const void* x_, size_t i, int64_t SB, Cx<typename Store<S>::acc>* xv) {
    constexpr int VW = Store<S>::VW;
    if constexpr (X32) {
        const int64_t cv = (int64_t)i / SB, sr = (int64_t)i - cv * SB;
#pragma unroll
        for (int h = 0; h < VW / 2; h++) Store<float>::ldv(x_, (cv * (VW / 2) + h) * SB + sr, xv + 2 * h);
    } else {
        Store<S>::ldv(x_, i, xv);
    }
}
template <typename S, bool X32>
__device__ inline void st_x(void* x_, size_t i, int64_t SB, const Cx<typename Store<S>::acc>* xv) {
    constexpr int VW = Store<S>::VW;
    if constexpr (X32) {
        const int64_t cv = (int64_t)i / SB, sr = (int64_t)i - cv * SB;
#pragma unroll
        for (int h = 0; h < VW / 2; h++) Store<float>::stv(x_, (cv * (VW / 2) + h) * SB + sr, xv + 2 * h);
    } else {
        Store<S>::stv(x_, i, xv);
    }
}

template <typename S, bool X32>
__global__ __launch_bounds__(RED_THREADS) void xr_update_kernel(void* x_, void* r_, const void* p, const void* s,
                                                                const void* t, const void* rh, const RhsState* st,
                                                                size_t nvec, int B, Cx<double>* partial, int x_zero,
                                                                int64_t SB) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    __shared__ Cx<double> red[2][RED_THREADS];
    Cx<double> d0 = cmake(0.0, 0.0), d1 = cmake(0.0, 0.0);
    const size_t stride = (size_t)gridDim.x * RED_THREADS;
    const RhsState& x = st[threadIdx.x & (B - 1)];   // the stride keeps each lane on one RHS
    if (x.active) {
        Cx<T> al = cscal<T>(x.alpha), om = cscal<T>(x.omega);
        for (size_t i = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; i < nvec; i += stride) {
            Cx<T> xv[VW], pv[VW], sv[VW], tv[VW], hv[VW];
            if (x_zero) {   // first iteration from x = 0: x is written, not read
#pragma unroll
                for (int j = 0; j < VW; j++) xv[j] = cmake<T>(0, 0);
            } else {
                ld_x<S, X32>(x_, i, SB, xv);
            }
            Store<S>::ldv(p, i, pv);
            Store<S>::ldv(s, i, sv);
            Store<S>::ldv(t, i, tv);
            Store<S>::ldv(rh, i, hv);
#pragma unroll
            for (int j = 0; j < VW; j++) {
                xv[j] = xv[j] + al * pv[j] + om * sv[j];
                sv[j] = Store<S>::round(sv[j] - om * tv[j]);   // the new r, as stored
                Cx<double> rd = cmake<double>(sv[j].re, sv[j].im);
                d0 = d0 + conjmul(cmake<double>(hv[j].re, hv[j].im), rd);
                d1.re += rd.re * rd.re + rd.im * rd.im;
            }
            st_x<S, X32>(x_, i, SB, xv);
            Store<S>::stv(r_, i, sv);
        }
    } else if (x_zero) {   // an RHS that stopped before its first x update keeps x = 0
        const Cx<T> zv[VW] = {};
        for (size_t i = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; i < nvec; i += stride) st_x<S, X32>(x_, i, SB, zv);
    }
    red[0][threadIdx.x] = d0;
    red[1][threadIdx.x] = d1;
    block_reduce_rhs<2>(red, B);
    if ((int)threadIdx.x < B) {
        partial[((int64_t)blockIdx.x * 2 + 0) * B + threadIdx.x] = red[0][threadIdx.x];
        partial[((int64_t)blockIdx.x * 2 + 1) * B + threadIdx.x] = red[1][threadIdx.x];
    }
}

static dim3 egrid(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

#define DHT_PREC_SWITCH(prec, LAUNCH)                 \
    switch (prec) {                                   \
        case DHT_FP64: { typedef double T_; LAUNCH; } break; \
        case DHT_FP32: { typedef float T_; LAUNCH; } break;  \
        case DHT_BF16: { typedef bf16x2 T_; LAUNCH; } break; \
        default: return set_error(DHT_ERR_INVALID_ARG, "bad precision"); \
    }

int p_update(dht_ctx* c, int prec, void* p, const void* r, const void* v, const RhsState* st, size_t nvec, int B,
             const void* p_in) {
    DHT_PREC_SWITCH(prec, hipLaunchKernelGGL(p_update_kernel<T_>, egrid(nvec), dim3(256), 0, c->stream, p,
                                             p_in ? p_in : p, r, v, st, nvec, B))
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}
int s_update(dht_ctx* c, int prec, void* s, const void* r, const void* v, const RhsState* st, size_t nvec, int B) {
    DHT_PREC_SWITCH(prec, hipLaunchKernelGGL(s_update_kernel<T_>, egrid(nvec), dim3(256), 0, c->stream, s, r, v, st, nvec, B))
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}
int xr_update_dots(dht_ctx* c, int prec, void* x, void* r, const void* p, const void* s, const void* t, const void* rh,
                   const RhsState* st, size_t nvec, int B, Cx<double>* partial, int* nblocks, bool x_zero, bool x32) {
    int nb = red_blocks(nvec);
    *nblocks = nb;
    const int64_t SB = c->g.Vh * (int64_t)B;
    if (x32 && prec == DHT_BF16) {
        hipLaunchKernelGGL((xr_update_kernel<bf16x2, true>), dim3(nb), dim3(RED_THREADS), 0, c->stream, x, r, p, s, t,
                           rh, st, nvec, B, partial, (int)x_zero, SB);
    } else {
        if (x32 && prec != DHT_FP32) return set_error(DHT_ERR_INVALID_ARG, "FP32 x needs BF16 or FP32 vectors");
        DHT_PREC_SWITCH(prec, hipLaunchKernelGGL((xr_update_kernel<T_, false>), dim3(nb), dim3(RED_THREADS), 0, c->stream,
                                                 x, r, p, s, t, rh, st, nvec, B, partial, (int)x_zero, SB))
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// r = s - omega t with the partials of (rhat, r) and (r, r), x left alone: the
// iteration's (alpha, omega) go to hist[B] (zero for an RHS that is not
// active) and x is rebuilt later from the stored p and s (accum_hist)
template <typename S>
__global__ __launch_bounds__(RED_THREADS) void r_update_kernel(void* r_, const void* s, const void* t, const void* rh,
                                                               const RhsState* st, size_t nvec, int B,
                                                               Cx<double>* partial, Cx<double>* hist) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    __shared__ Cx<double> red[2][RED_THREADS];
    Cx<double> d0 = cmake(0.0, 0.0), d1 = cmake(0.0, 0.0);
    const size_t stride = (size_t)gridDim.x * RED_THREADS;
    const RhsState& x = st[threadIdx.x & (B - 1)];   // the stride keeps each lane on one RHS
    if (blockIdx.x == 0 && (int)threadIdx.x < B) {
        hist[threadIdx.x] = x.active ? x.alpha : cmake(0.0, 0.0);
        hist[B + threadIdx.x] = x.active ? x.omega : cmake(0.0, 0.0);
    }
    if (x.active) {
        Cx<T> om = cscal<T>(x.omega);
        // four vectors per step, all loaded before any is used (more loads in
        // flight than two: -7 % at 32^3x64); the sums keep the order of a
        // one-vector loop
        constexpr int U = 4;
        for (size_t i = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; i < nvec; i += U * stride) {
            Cx<T> sv[U][VW], tv[U][VW], hv[U][VW];
#pragma unroll
            for (int u = 0; u < U; u++)
                if (i + u * stride < nvec) {
                    Store<S>::ldv(s, i + u * stride, sv[u]);
                    Store<S>::ldv(t, i + u * stride, tv[u]);
                    Store<S>::ldv(rh, i + u * stride, hv[u]);
                }
#pragma unroll
            for (int u = 0; u < U; u++)
                if (i + u * stride < nvec) {
#pragma unroll
                    for (int j = 0; j < VW; j++) {
                        sv[u][j] = Store<S>::round(sv[u][j] - om * tv[u][j]);   // the new r, as stored
                        Cx<double> rd = cmake<double>(sv[u][j].re, sv[u][j].im);
                        d0 = d0 + conjmul(cmake<double>(hv[u][j].re, hv[u][j].im), rd);
                        d1.re += rd.re * rd.re + rd.im * rd.im;
                    }
                    Store<S>::stv(r_, i + u * stride, sv[u]);
                }
        }
    }
    red[0][threadIdx.x] = d0;
    red[1][threadIdx.x] = d1;
    block_reduce_rhs<2>(red, B);
    if ((int)threadIdx.x < B) {
        partial[((int64_t)blockIdx.x * 2 + 0) * B + threadIdx.x] = red[0][threadIdx.x];
        partial[((int64_t)blockIdx.x * 2 + 1) * B + threadIdx.x] = red[1][threadIdx.x];
    }
}

// X (FP64 half field) = [X +] scale_r * sum_j (alpha_j p_j + omega_j s_j) over
// the n stored iterations (p_j, s_j: slot j of the rings, storage S; hist:
// [n][2][B]); a zero coefficient skips its vector (its slot may hold another
// RHS's stale values).  With E32 (FP32 half field) the sum is also kept there,
// E = [E +] sum rounded to FP32, and X moves by scale_r times exactly what E
// moved by, so that X - scale_r E stays what it was (exact to FP64 rounding).
template <typename S>
__global__ void accum_hist_kernel(Cx<double>* X, const void* P, const void* Sv, const Cx<double>* hist, int n,
                                  size_t nvec, int64_t SB, int B, const double* scale, int assign, const void* P0,
                                  void* E32, int e_assign) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nvec) return;
    const int rr = (int)(i & (B - 1));
    const int64_t cv = (int64_t)i / SB, sr = (int64_t)i - cv * SB;
    const double sc = scale[rr];
    Cx<double> acc[VW];
#pragma unroll
    for (int q = 0; q < VW; q++) acc[q] = cmake(0.0, 0.0);
    if (sc != 0.0) {
        for (int j = 0; j < n; j++) {
            const Cx<double> al = hist[(int64_t)j * 2 * B + rr], om = hist[((int64_t)j * 2 + 1) * B + rr];
            Cx<T> v[VW];
            if (al.re != 0.0 || al.im != 0.0) {
                Store<S>::ldv((j == 0 && P0) ? P0 : (const void*)((const char*)P + (size_t)j * nvec * 16), i, v);
#pragma unroll
                for (int q = 0; q < VW; q++) acc[q] = acc[q] + al * cmake<double>(v[q].re, v[q].im);
            }
            if (om.re != 0.0 || om.im != 0.0) {
                Store<S>::ldv((const char*)Sv + (size_t)j * nvec * 16, i, v);
#pragma unroll
                for (int q = 0; q < VW; q++) acc[q] = acc[q] + om * cmake<double>(v[q].re, v[q].im);
            }
        }
    }
    if constexpr (VW >= 2) {
        if (E32 && (sc != 0.0 || e_assign)) {
#pragma unroll
            for (int h = 0; h < VW / 2; h++) {
                const int64_t ev = (cv * (VW / 2) + h) * SB + sr;
                Cx<float> eo[2] = {cmake(0.f, 0.f), cmake(0.f, 0.f)};
                if (!e_assign) Store<float>::ldv(E32, ev, eo);
                Cx<float> en[2];
#pragma unroll
                for (int q2 = 0; q2 < 2; q2++) {
                    Cx<double>& a = acc[2 * h + q2];
                    en[q2] = cmake((float)((double)eo[q2].re + a.re), (float)((double)eo[q2].im + a.im));
                    a = cmake((double)en[q2].re - (double)eo[q2].re, (double)en[q2].im - (double)eo[q2].im);
                }
                Store<float>::stv(E32, ev, en);
            }
        }
    }
    if (sc == 0.0 && !assign) return;
#pragma unroll
    for (int q = 0; q < VW; q++) {
        Cx<double>& xd = X[(cv * VW + q) * SB + sr];
        const Cx<double> x0 = assign ? cmake(0.0, 0.0) : xd;
        xd = cmake(x0.re + sc * acc[q].re, x0.im + sc * acc[q].im);
    }
}

// r = r_in - scale_r * w (FP64 half fields r, r_in; FP32 w), with the
// per-RHS partials of (r, r) for the new r; with rh16 also s16_r * r in BF16
// (the next inner solve's right-hand side).  One item is one BF16 vector:
// components 4m .. 4m+3 of one (site, RHS), i.e. FP32 vectors 2m and 2m+1.
__global__ __launch_bounds__(RED_THREADS) void residual_step_kernel(Cx<double>* r, const Cx<double>* r_in,
                                                                    const void* w, const double* scale,
                                                                    size_t nitem, int64_t SB, int B,
                                                                    Cx<double>* partial, void* rh16,
                                                                    const double* s16) {
    __shared__ Cx<double> red[1][RED_THREADS];
    Cx<double> d0 = cmake(0.0, 0.0);
    const double sc = scale[threadIdx.x & (B - 1)];   // the stride keeps each lane on one RHS
    const double s16r = rh16 ? s16[threadIdx.x & (B - 1)] : 0.0;
    const size_t stride = (size_t)gridDim.x * RED_THREADS;
    const size_t v0 = (size_t)blockIdx.x * RED_THREADS + threadIdx.x;
    StridePos pos(v0, stride, SB);   // pos.cv = m
    // four items per step, all loaded before any is used (sums in the order
    // of a one-item loop)
    constexpr int U = 4;
    for (size_t v = v0; v < nitem; v += U * stride) {
        Cx<float> wv[U][4];
        Cx<double> ri[U][4];
        int64_t e0[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (v + u * stride < nitem) {
                const int64_t w0 = pos.cv * 2 * SB + pos.sr;
                Store<float>::ldv(w, w0, wv[u]);
                Store<float>::ldv(w, w0 + SB, wv[u] + 2);
                e0[u] = pos.cv * 4 * SB + pos.sr;
#pragma unroll
                for (int q = 0; q < 4; q++) ri[u][q] = r_in[e0[u] + q * SB];
            }
            pos.next();
        }
#pragma unroll
        for (int u = 0; u < U; u++)
            if (v + u * stride < nitem) {
                Cx<float> o16[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const Cx<double> nr =
                        cmake(ri[u][q].re - sc * (double)wv[u][q].re, ri[u][q].im - sc * (double)wv[u][q].im);
                    r[e0[u] + q * SB] = nr;
                    d0.re += nr.re * nr.re + nr.im * nr.im;
                    o16[q] = cmake<float>((float)(s16r * nr.re), (float)(s16r * nr.im));
                }
                if (rh16) Store<bf16x2>::stv(rh16, v + u * stride, o16);
            }
    }
    red[0][threadIdx.x] = d0;
    block_reduce_rhs<1>(red, B);
    if ((int)threadIdx.x < B) partial[(int64_t)blockIdx.x * B + threadIdx.x] = red[0][threadIdx.x];
}

int residual_step(dht_ctx* c, void* r, const void* r_in, const void* w32, const double* scale, int nrhs,
                  Cx<double>* partial, int* nblocks, void* rh16, const double* s16) {
    if (rh16 && !s16) return set_error(DHT_ERR_INVALID_ARG, "BF16 residual copy needs its scales");
    const int64_t SB = c->g.Vh * (int64_t)nrhs;
    const size_t nitem = half_vecs(c, nrhs, DHT_BF16);
    const int nb = red_blocks(nitem);
    *nblocks = nb;
    hipLaunchKernelGGL(residual_step_kernel, dim3(nb), dim3(RED_THREADS), 0, c->stream, (Cx<double>*)r,
                       (const Cx<double>*)r_in, w32, scale, nitem, SB, nrhs, partial, rh16, s16);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

int r_update_dots(dht_ctx* c, int prec, void* r, const void* s, const void* t, const void* rh, const RhsState* st,
                  size_t nvec, int B, Cx<double>* partial, int* nblocks, Cx<double>* hist) {
    int nb = red_blocks(nvec);
    *nblocks = nb;
    DHT_PREC_SWITCH(prec, hipLaunchKernelGGL(r_update_kernel<T_>, dim3(nb), dim3(RED_THREADS), 0, c->stream, r, s, t, rh,
                                             st, nvec, B, partial, hist))
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

int accum_hist(dht_ctx* c, int prec, void* X, const void* P, const void* Sv, const Cx<double>* hist, int n, int nrhs,
               const double* scale, bool assign, const void* P0, void* E32, bool e_assign) {
    if (E32 && prec == DHT_FP64) return set_error(DHT_ERR_INVALID_ARG, "an FP32 copy of the sum needs 16- or 32-bit vectors");
    const int64_t SB = c->g.Vh * (int64_t)nrhs;
    const size_t nvec = half_vecs(c, nrhs, prec);
    DHT_PREC_SWITCH(prec, hipLaunchKernelGGL(accum_hist_kernel<T_>, egrid(nvec), dim3(256), 0, c->stream, (Cx<double>*)X,
                                             P, Sv, hist, n, nvec, SB, nrhs, scale, (int)assign, P0, E32, (int)e_assign))
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// --------------------------------------------------------------------------
// defect-correction helpers (FP64 half field <-> low-precision half field)
// --------------------------------------------------------------------------
// low vector v = (cv, site-rhs sr) holds components cv*VW .. cv*VW+VW-1;
// the FP64 vector of component c is c * SB + sr.
template <typename SO>
__global__ void scale_down_kernel(const Cx<double>* in, void* out, const double* scale, size_t nlo, int64_t SB, int B) {
    typedef typename Store<SO>::acc T;
    constexpr int VW = Store<SO>::VW;
    size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nlo) return;
    int64_t cv = v / SB, sr = v - cv * SB;
    double sc = scale[sr & (B - 1)];
    Cx<T> e[VW];
#pragma unroll
    for (int j = 0; j < VW; j++) {
        Cx<double> d = in[(cv * VW + j) * SB + sr];
        e[j] = cmake<T>((T)(sc * d.re), (T)(sc * d.im));
    }
    Store<SO>::stv(out, v, e);
}
// Start of an inner solve from x = 0: r = rhat = p = round(scale_r * in) in the
// inner precision (in: FP64 half field; r or p = null: not written), with
// the per-RHS partials of (r, r).
template <typename SO>
__global__ __launch_bounds__(RED_THREADS) void solve_init_kernel(const Cx<double>* in, const double* scale, void* r,
                                                                 void* rh, void* p, size_t nlo, int64_t SB, int B,
                                                                 Cx<double>* partial) {
    typedef typename Store<SO>::acc T;
    constexpr int VW = Store<SO>::VW;
    __shared__ Cx<double> red[1][RED_THREADS];
    Cx<double> d0 = cmake(0.0, 0.0);
    const double sc = scale[threadIdx.x & (B - 1)];   // the stride keeps each lane on one RHS
    const size_t stride = (size_t)gridDim.x * RED_THREADS;
    const size_t v0 = (size_t)blockIdx.x * RED_THREADS + threadIdx.x;
    StridePos pos(v0, stride, SB);
    // two vectors per step, both loaded before either is used (sums in the
    // order of a one-vector loop)
    for (size_t v = v0; v < nlo; v += 2 * stride) {
        const bool two = v + stride < nlo;
        Cx<double> d[2][VW];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            if (u == 0 || two) {
#pragma unroll
                for (int j = 0; j < VW; j++) d[u][j] = in[(pos.cv * VW + j) * SB + pos.sr];
            }
            pos.next();
        }
#pragma unroll
        for (int u = 0; u < 2; u++)
            if (u == 0 || two) {
                Cx<T> e[VW];
#pragma unroll
                for (int j = 0; j < VW; j++) {
                    e[j] = Store<SO>::round(cmake<T>((T)(sc * d[u][j].re), (T)(sc * d[u][j].im)));
                    d0.re += (double)e[j].re * e[j].re + (double)e[j].im * e[j].im;
                }
                const size_t vu = v + u * stride;
                if (r) Store<SO>::stv(r, vu, e);
                Store<SO>::stv(rh, vu, e);
                if (p) Store<SO>::stv(p, vu, e);
            }
    }
    red[0][threadIdx.x] = d0;
    block_reduce_rhs<1>(red, B);
    if ((int)threadIdx.x < B) partial[(int64_t)blockIdx.x * B + threadIdx.x] = red[0][threadIdx.x];
}

int solve_init(dht_ctx* c, const void* in, int pout, const double* scale, void* r, void* rh, void* p, int nrhs,
               Cx<double>* partial, int* nblocks) {
    const int64_t SB = c->g.Vh * (int64_t)nrhs;
    size_t nlo = half_elems(c, nrhs) / vec_width(pout);
    const int nb = red_blocks(nlo);
    *nblocks = nb;
    DHT_PREC_SWITCH(pout, hipLaunchKernelGGL(solve_init_kernel<T_>, dim3(nb), dim3(RED_THREADS), 0, c->stream,
                                             (const Cx<double>*)in, scale, r, rh, p, nlo, SB, nrhs, partial))
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// x += scale_r * e (assign: x = scale_r * e, x not read)
template <typename SI>
__global__ void accum_up_kernel(Cx<double>* x, const void* e_, const double* scale, size_t nlo, int64_t SB, int B,
                                int assign) {
    typedef typename Store<SI>::acc T;
    constexpr int VW = Store<SI>::VW;
    size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nlo) return;
    int64_t cv = v / SB, sr = v - cv * SB;
    double sc = scale[sr & (B - 1)];
    if (sc == 0.0) {
        if (assign)
#pragma unroll
            for (int j = 0; j < VW; j++) x[(cv * VW + j) * SB + sr] = cmake(0.0, 0.0);
        return;
    }
    Cx<T> e[VW];
    Store<SI>::ldv(e_, v, e);
#pragma unroll
    for (int j = 0; j < VW; j++) {
        Cx<double>& xd = x[(cv * VW + j) * SB + sr];
        const Cx<double> x0 = assign ? cmake(0.0, 0.0) : xd;
        xd = cmake(x0.re + sc * (double)e[j].re, x0.im + sc * (double)e[j].im);
    }
}

int scale_down(dht_ctx* c, const void* in, void* out, int pout, const double* scale, int nrhs) {
    const int64_t SB = c->g.Vh * (int64_t)nrhs;
    size_t nlo = half_elems(c, nrhs) / vec_width(pout);
    DHT_PREC_SWITCH(pout, hipLaunchKernelGGL(scale_down_kernel<T_>, egrid(nlo), dim3(256), 0, c->stream,
                                             (const Cx<double>*)in, out, scale, nlo, SB, nrhs))
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}
int accum_up(dht_ctx* c, void* x, const void* e, int pin, const double* scale, int nrhs, bool assign) {
    const int64_t SB = c->g.Vh * (int64_t)nrhs;
    size_t nlo = half_elems(c, nrhs) / vec_width(pin);
    DHT_PREC_SWITCH(pin, hipLaunchKernelGGL(accum_up_kernel<T_>, egrid(nlo), dim3(256), 0, c->stream,
                                            (Cx<double>*)x, e, scale, nlo, SB, nrhs, (int)assign))
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

// fill with zero (a kernel rather than a memset so that the stream can be
// captured); grid-stride because the deflation basis can exceed 2^32 words
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
    size_t blocks = std::min<size_t>((std::max(n16, n - 4 * n16) + 255) / 256, 65536);
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, c->stream, (uint4*)p, n16,
                       (uint32_t*)p + 4 * n16, n - 4 * n16);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

}  // namespace dht
