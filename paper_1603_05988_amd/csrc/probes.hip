// Probe vectors on the device (Algorithm 1: the Z4 base vector, the
// hierarchical-probing Hadamard vectors and their elementwise product).
//
// z_j(n) = i^k(n) * h_j(site(n)):  k(n) in {0,1,2,3} is the Z4 noise index
// (Section 1: entries uniform in {1, i, -1, -i}) from the counter-based
// SplitMix64 generator (Steele, Lea and Flood 2014); h_j is the
// hierarchical-probing Hadamard sign (Section 5.2), 1 for plain noise.
//
// SplitMix64: out(s, i) = mix(s + (i + 1) * 0x9E3779B97F4A7C15) with the
// finaliser mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
// z *= 0x94D049BB133111EB; z ^= z >> 31.  Keys: K_run = out(seed, run); the
// hierarchical-probing base vector uses K_run, plain probe j uses
// out(K_run, j).  Component n of a probe takes the 2 bits at 2 (n mod 32) of
// out(key, n / 32).
//
// Colour of a site for level l: bit 4l = parity of sum_mu floor(x_mu / 2^l),
// bits 4l+1..4l+3 = floor(x_mu / 2^l) mod 2 for mu = x, y, z; the Hadamard
// sign of probe j is (-1)^popcount(colour & j).  The first 2^m probes span the
// indicator vectors of the partition by the low m colour bits, which nest as
// m grows (the hierarchical property).
#include "internal.h"

namespace dht {

__host__ __device__ inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm64_out(uint64_t state, uint64_t i) {
    return sm64_mix(state + (i + 1) * 0x9E3779B97F4A7C15ull);
}

struct ProbeArgs {
    Geom g;
    int n;      // real probes
    int B;      // padded slots (power of two)
    int hp;
    uint64_t krun;
    int64_t first;
    void* field;
    int prec;
    uint8_t* kout;
    int8_t* sout;
    uint8_t* zcode;
};

template <typename S>
__global__ void probe_kernel(ProbeArgs a) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (p, s, r), r fastest
    if (gid >= a.g.V * (int64_t)a.B) return;
    int64_t ps = gid / a.B;
    int r = (int)(gid - ps * a.B);
    int p = (int)(ps / a.g.Vh);
    int64_t s = ps - (int64_t)p * a.g.Vh;
    const bool real = r < a.n;
    int c[4];
    cb_coords(a.g, s, p, c);
    int64_t n = lex_index(a.g, c);
    uint64_t j = (uint64_t)(a.first + r);
    uint64_t key = a.hp ? a.krun : sm64_out(a.krun, j);
    float sign = 1.0f;
    if (a.hp) sign = (__popcll(hp_colour_bits(c, j) & j) & 1) ? -1.0f : 1.0f;
    if (a.sout && real) a.sout[(int64_t)r * a.g.V + n] = (int8_t)sign;
    const int64_t N = 12 * a.g.V;
    uint64_t widx = ~0ull, word = 0;
    Cx<T> e[12];
    for (int comp = 0; comp < 12; comp++) {
        uint64_t nc = (uint64_t)(12 * n + comp);
        if ((nc >> 5) != widx) {
            widx = nc >> 5;
            word = sm64_out(key, widx);
        }
        int k = (int)((word >> (2 * (nc & 31))) & 3ull);
        if (a.kout && real) a.kout[(int64_t)r * N + (int64_t)nc] = (uint8_t)k;
        if (a.zcode)   // z = i^k * sign = i^(k + 2 [sign < 0]); padding slots hold code 0 but are never read
            a.zcode[((int64_t)p * 12 * a.g.Vh + (int64_t)comp * a.g.Vh + s) * a.B + r] =
                (uint8_t)((k + (sign < 0.0f ? 2 : 0)) & 3);
        T re = (k == 0) ? T(1) : (k == 2 ? T(-1) : T(0));
        T im = (k == 1) ? T(1) : (k == 3 ? T(-1) : T(0));
        e[comp] = real ? cmake<T>((T)sign * re, (T)sign * im) : cmake<T>(0, 0);
    }
    if (a.field) {
        const int64_t SB = a.g.Vh * a.B;
        const int64_t vbase = (int64_t)p * (12 / VW) * SB + s * a.B + r;
#pragma unroll
        for (int q = 0; q < 12 / VW; q++) Store<S>::stv(a.field, vbase + q * SB, e + q * VW);
    }
}

int probes_gen(dht_ctx* c, const dht_probe_spec* spec, int64_t first, int n, int bp, void* field, int prec,
               uint8_t* kout, int8_t* sout, uint8_t* zcode) {
    if (first < 0) return set_error(DHT_ERR_INVALID_ARG, "negative probe index");
    if (n > bp) return set_error(DHT_ERR_INVALID_ARG, "batch exceeds its padded size");
    const int nrhs = bp;
    ProbeArgs a;
    a.g = c->g;
    a.n = n;
    a.B = nrhs;
    a.hp = spec->hp ? 1 : 0;
    a.krun = sm64_out(spec->seed, spec->run);
    a.first = first;
    a.field = field;
    a.prec = prec;
    a.kout = kout;
    a.sout = sout;
    a.zcode = zcode;
    int64_t nthreads = c->g.V * (int64_t)nrhs;
    dim3 grid((unsigned)((nthreads + 255) / 256)), block(256);
    switch (prec) {
        case DHT_FP64: hipLaunchKernelGGL(probe_kernel<double>, grid, block, 0, c->stream, a); break;
        case DHT_FP32: hipLaunchKernelGGL(probe_kernel<float>, grid, block, 0, c->stream, a); break;
        case DHT_BF16: hipLaunchKernelGGL(probe_kernel<bf16x2>, grid, block, 0, c->stream, a); break;
        default: return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

}  // namespace dht
