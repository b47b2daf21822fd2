// Layout conversion between the canonical interface layout and the internal
// even/odd RHS-innermost layout, and precision conversion (round to nearest
// even for FP64 -> FP32 -> BF16).
#include <type_traits>

#include "internal.h"

namespace dht {

template <typename S>
__device__ inline void store_from_double(typename Store<S>::elem* p, Cx<double> v) {
    typedef typename Store<S>::acc T;
    Store<S>::st(p, cmake<T>((T)v.re, (T)v.im));
}
template <>
__device__ inline void store_from_double<bf16x2>(bf16x2* p, Cx<double> v) {
    // double -> float (RNE) -> bf16 (RNE); documented double rounding
    Store<bf16x2>::st(p, cmake<float>((float)v.re, (float)v.im));
}

template <typename S>
__device__ inline Cx<double> load_to_double(const typename Store<S>::elem* p) {
    auto v = Store<S>::ld(p);
    return cmake<double>((double)v.re, (double)v.im);
}

// links: canonical [4][V][9] complex128 -> [4][9][2][Vh] in FP64, FP32, BF16
__global__ void pack_gauge_kernel(const Cx<double>* __restrict__ Uc, Cx<double>* U64, Cx<float>* U32,
                                  bf16x2* U16, Geom g) {
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
    for (int e = 0; e < 9; e++) {
        Cx<double> v = Uc[gid * 9 + e];
        int64_t o = ((int64_t)(mu * 9 + e) * 2 + p) * g.Vh + s;
        U64[o] = v;
        store_from_double<float>(U32 + o, v);
        store_from_double<bf16x2>(U16 + o, v);
    }
}

int pack_gauge(dht_ctx* c, const double* U_dev) {
    int64_t n = 4 * c->g.V;
    hipLaunchKernelGGL(pack_gauge_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       (const Cx<double>*)U_dev, (Cx<double>*)c->U[0], (Cx<float>*)c->U[1], (bf16x2*)c->U[2], c->g);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// spinors: canonical [B][V][12] complex128 <-> internal [2][12][Vh][B]
template <typename S, bool PACK>
__global__ void spinor_pack_kernel(Cx<double>* canon, typename Store<S>::elem* field, Geom g, int B) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (p, s, r), r fastest
    int64_t tot = g.V * (int64_t)B;
    if (gid >= tot) return;
    int64_t ps = gid / B;
    int r = (int)(gid - ps * B);
    int p = (int)(ps / g.Vh);
    int64_t s = ps - (int64_t)p * g.Vh;
    int cc[4];
    cb_coords(g, s, p, cc);
    int64_t n = lex_index(g, cc);
    Cx<double>* cp = canon + ((int64_t)r * g.V + n) * 12;
    typename Store<S>::elem* fp = field + (int64_t)p * 12 * g.Vh * B + s * B + r;
    int64_t cs = g.Vh * B;
    for (int comp = 0; comp < 12; comp++) {
        if (PACK) store_from_double<S>(fp + comp * cs, cp[comp]);
        else cp[comp] = load_to_double<S>(fp + comp * cs);
    }
}

template <bool PACK>
static int spinor_dispatch(dht_ctx* c, double* canon, void* field, int prec, int nrhs) {
    int64_t n = c->g.V * (int64_t)nrhs;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (prec) {
        case DHT_FP64:
            hipLaunchKernelGGL((spinor_pack_kernel<double, PACK>), grid, block, 0, c->stream, (Cx<double>*)canon,
                               (Cx<double>*)field, c->g, nrhs);
            break;
        case DHT_FP32:
            hipLaunchKernelGGL((spinor_pack_kernel<float, PACK>), grid, block, 0, c->stream, (Cx<double>*)canon,
                               (Cx<float>*)field, c->g, nrhs);
            break;
        case DHT_BF16:
            hipLaunchKernelGGL((spinor_pack_kernel<bf16x2, PACK>), grid, block, 0, c->stream, (Cx<double>*)canon,
                               (bf16x2*)field, c->g, nrhs);
            break;
        default:
            return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

int pack_spinor(dht_ctx* c, const double* canon, void* field, int prec, int nrhs) {
    return spinor_dispatch<true>(c, const_cast<double*>(canon), field, prec, nrhs);
}
int unpack_spinor(dht_ctx* c, const void* field, int prec, double* canon, int nrhs) {
    return spinor_dispatch<false>(c, canon, const_cast<void*>(field), prec, nrhs);
}

// elementwise precision conversion
template <typename SI, typename SO>
__global__ void convert_kernel(const typename Store<SI>::elem* in, typename Store<SO>::elem* out, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Cx<double> v = load_to_double<SI>(in + i);
    store_from_double<SO>(out + i, v);
}

int convert_field(dht_ctx* c, const void* in, int pin, void* out, int pout, size_t n) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define DHT_CONV(PI, TI, PO, TO)                                                                          \
    if (pin == PI && pout == PO) {                                                                        \
        hipLaunchKernelGGL((convert_kernel<TI, TO>), grid, block, 0, c->stream,                           \
                           (const typename Store<TI>::elem*)in, (typename Store<TO>::elem*)out, n);        \
        DHT_HIP(hipGetLastError());                                                                       \
        return DHT_OK;                                                                                    \
    }
    DHT_CONV(DHT_FP64, double, DHT_FP64, double)
    DHT_CONV(DHT_FP64, double, DHT_FP32, float)
    DHT_CONV(DHT_FP64, double, DHT_BF16, bf16x2)
    DHT_CONV(DHT_FP32, float, DHT_FP64, double)
    DHT_CONV(DHT_FP32, float, DHT_FP32, float)
    DHT_CONV(DHT_FP32, float, DHT_BF16, bf16x2)
    DHT_CONV(DHT_BF16, bf16x2, DHT_FP64, double)
    DHT_CONV(DHT_BF16, bf16x2, DHT_FP32, float)
    DHT_CONV(DHT_BF16, bf16x2, DHT_BF16, bf16x2)
#undef DHT_CONV
    return set_error(DHT_ERR_INVALID_ARG, "bad precision pair");
}

}  // namespace dht
