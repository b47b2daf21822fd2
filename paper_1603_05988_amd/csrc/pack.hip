// Layout conversion between the canonical interface layout and the internal
// even/odd, RHS-innermost, 16-byte-vector layout, with precision conversion
// (round to nearest even for FP64 -> FP32 -> BF16).
#include <type_traits>

#include "internal.h"

namespace dht {

template <typename S>
__device__ inline Cx<typename Store<S>::acc> from_double(Cx<double> v) {
    typedef typename Store<S>::acc T;
    return cmake<T>((T)v.re, (T)v.im);   // double -> float is RNE; BF16 rounds again on store
}

// links: canonical [4][V][9] complex128 -> [4][2][Vh][nvec] 16-byte vectors per precision
template <typename S>
__device__ inline void store_link(void* U, int mu, int p, int64_t s, int64_t Vh, const Cx<double>* m) {
    constexpr int VW = Store<S>::VW;
    constexpr int NV = (9 + VW - 1) / VW;
    Cx<typename Store<S>::acc> e[NV * VW];
#pragma unroll
    for (int i = 0; i < NV * VW; i++) e[i] = i < 9 ? from_double<S>(m[i]) : from_double<S>(cmake(0.0, 0.0));
#pragma unroll
    for (int j = 0; j < NV; j++) Store<S>::stv_rne(U, ((int64_t)(mu * 2 + p) * Vh + s) * NV + j, e + j * VW);
}

__global__ void pack_gauge_kernel(const Cx<double>* __restrict__ Uc, void* U64, void* U32, void* U16, Geom g) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 4 * g.V) return;
    int mu = (int)(gid / g.V);
    int64_t n = gid - (int64_t)mu * g.V;
    int64_t r = n;
    int x = (int)(r % g.L[0]); r /= g.L[0];
    int y = (int)(r % g.L[1]); r /= g.L[1];
    int z = (int)(r % g.L[2]);
    int t = (int)(r / g.L[2]);
    int p = (x + y + z + t) & 1;
    int64_t s = n >> 1;
    Cx<double> m[9];
    for (int e = 0; e < 9; e++) m[e] = Uc[gid * 9 + e];
    store_link<double>(U64, mu, p, s, g.Vh, m);
    store_link<float>(U32, mu, p, s, g.Vh, m);
    store_link<bf16x2>(U16, mu, p, s, g.Vh, m);
}

int pack_gauge(dht_ctx* c, const double* U_dev) {
    int64_t n = 4 * c->g.V;
    hipLaunchKernelGGL(pack_gauge_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       (const Cx<double>*)U_dev, c->U[0], c->U[1], c->U[2], c->g);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// spinors: canonical [n][V][12] complex128 <-> internal [2][12/VW][Vh][bp][VW]
template <typename S, bool PACK>
__global__ void spinor_pack_kernel(Cx<double>* canon, void* field, Geom g, int n, int bp) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (p, s, r), r fastest
    if (gid >= g.V * (int64_t)bp) return;
    int64_t ps = gid / bp;
    int r = (int)(gid - ps * bp);
    if (!PACK && r >= n) return;
    int p = (int)(ps / g.Vh);
    int64_t s = ps - (int64_t)p * g.Vh;
    int cc[4];
    cb_coords(g, s, p, cc);
    int64_t nsite = lex_index(g, cc);
    const int64_t SB = g.Vh * bp;
    const int64_t vbase = (int64_t)p * (12 / VW) * SB + s * bp + r;
    Cx<T> e[12];
    if (PACK) {
        for (int comp = 0; comp < 12; comp++)
            e[comp] = r < n ? from_double<S>(canon[((int64_t)r * g.V + nsite) * 12 + comp]) : cmake<T>(0, 0);
#pragma unroll
        for (int j = 0; j < 12 / VW; j++) Store<S>::stv_rne(field, vbase + j * SB, e + j * VW);
    } else {
#pragma unroll
        for (int j = 0; j < 12 / VW; j++) Store<S>::ldv(field, vbase + j * SB, e + j * VW);
        for (int comp = 0; comp < 12; comp++)
            canon[((int64_t)r * g.V + nsite) * 12 + comp] = cmake<double>((double)e[comp].re, (double)e[comp].im);
    }
}

template <bool PACK>
static int spinor_dispatch(dht_ctx* c, double* canon, void* field, int prec, int n, int bp) {
    if (n > bp) return set_error(DHT_ERR_INVALID_ARG, "batch exceeds its padded size");
    int64_t tot = c->g.V * (int64_t)bp;
    dim3 grid((unsigned)((tot + 255) / 256)), block(256);
    switch (prec) {
        case DHT_FP64:
            hipLaunchKernelGGL((spinor_pack_kernel<double, PACK>), grid, block, 0, c->stream, (Cx<double>*)canon, field,
                               c->g, n, bp);
            break;
        case DHT_FP32:
            hipLaunchKernelGGL((spinor_pack_kernel<float, PACK>), grid, block, 0, c->stream, (Cx<double>*)canon, field,
                               c->g, n, bp);
            break;
        case DHT_BF16:
            hipLaunchKernelGGL((spinor_pack_kernel<bf16x2, PACK>), grid, block, 0, c->stream, (Cx<double>*)canon, field,
                               c->g, n, bp);
            break;
        default:
            return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

int pack_spinor(dht_ctx* c, const double* canon, void* field, int prec, int n, int bp) {
    return spinor_dispatch<true>(c, const_cast<double*>(canon), field, prec, n, bp);
}
int unpack_spinor(dht_ctx* c, const void* field, int prec, double* canon, int n, int bp) {
    return spinor_dispatch<false>(c, canon, const_cast<void*>(field), prec, n, bp);
}

}  // namespace dht
