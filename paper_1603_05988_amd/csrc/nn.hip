// Learned right preconditioner: a 3-layer 4D convolutional network on BF16
// matrix cores (gfx950), with its training (forward, backward, Adam).
//
// The paper leaves the linear solver open (Algorithm 1, "Solve Ay = z"); the
// network M(r) ~ D^-1 r serves as the right preconditioner of FGMRES.
// Architecture: 3^4-tap convolutions over the periodic lattice, channels
// 24 -> 48 -> 48 -> 24 (real and imaginary parts of the 12 spin-colour
// components: channel 2c + part), ReLU after layers 1 and 2, no bias.
//
// Activations: [batch][V][C] with lexicographic sites -- for 24 channels this
// is exactly the canonical spinor layout read as reals.  Hidden activations
// and gradients are BF16; the network output is FP32.  Weights: FP32 master
// copy [81][Cout][Cin] (tap t = (dx+1) + 3 (dy+1) + 9 (dz+1) + 27 (dt+1),
// out[x] = sum_t W[t] in[x + d_t]) plus BF16 copies for the matrix cores:
// Wf [81][Cout16][Cin] (Cout padded to 16) for the forward pass and
// Wb [81][Cin16][Cout] with Wb[80 - t][i][o] = W[t][o][i] for the backward
// (data) pass, which is the forward convolution with reflected, transposed taps.
//
// Convolution as implicit GEMM on v_mfma_f32_16x16x32_bf16: rows = sites,
// columns = output channels, K = 81 taps x Cin (8 channels of one tap per
// lane per step, a 16-byte load of the neighbour's channels-last vector).
// Each wave owns 64 sites x all output channels; accumulation in FP32.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "solver.h"

namespace dht {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

static const int NN_CH[4] = {24, 48, 48, 24};

__device__ inline uint16_t f2bf(float f) { return (uint16_t)(f32x2_to_bf16x2_bits(f, 0.f) & 0xffffu); }
__device__ inline float bf2f(uint16_t h) { return bf16_bits_to_f32(h); }

struct ConvArgs {
    const uint16_t* in;     // [B][V][CIN] BF16
    const uint16_t* W;      // [81][COUT16][CIN] BF16
    void* out0;             // [B][V][COUT]: FP32 if out0_fp32 else BF16
    uint16_t* out1;         // [B][V][COUT] BF16 relu(out) or null
    const uint16_t* mask;   // [B][V][COUT] BF16: zero the output where mask <= 0 (or null)
    int L0, L1, L2, L3;
    int V;
    int64_t nsites;         // B * V
    int out0_fp32;
};

static constexpr int CONV_WAVES = 4;

template <int CIN, int COUT>
__global__ __launch_bounds__(64 * CONV_WAVES) void conv_fwd_kernel(ConvArgs a) {
    constexpr int COUTP = (COUT + 15) / 16 * 16;
    constexpr int CT = COUTP / 16;
    constexpr int KG = CIN / 8;          // 8-channel groups per tap
    constexpr int KTOT = 81 * KG;
    constexpr int NSTEP = (KTOT + 3) / 4;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t base = ((int64_t)blockIdx.x * CONV_WAVES + wave) * 64;
    // the four row sites of this lane in the A operand (row = lane % 16)
    int cx[4][4];
    int64_t brow[4];
    bool vrow[4];
#pragma unroll
    for (int rt = 0; rt < 4; rt++) {
        int64_t gs = base + rt * 16 + (lane & 15);
        vrow[rt] = gs < a.nsites;
        if (!vrow[rt]) gs = 0;
        int64_t b = gs / a.V;
        int x = (int)(gs - b * a.V);
        brow[rt] = b * a.V;
        cx[rt][0] = x % a.L0;
        x /= a.L0;
        cx[rt][1] = x % a.L1;
        x /= a.L1;
        cx[rt][2] = x % a.L2;
        cx[rt][3] = x / a.L2;
    }
    f32x4_t acc[4][CT];
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++) acc[rt][ct] = (f32x4_t){0.f, 0.f, 0.f, 0.f};

    for (int step = 0; step < NSTEP; step++) {
        const int g = step * 4 + (lane >> 4);
        const bool vk = g < KTOT;
        const int tap = vk ? g / KG : 0;
        const int i0 = (g - tap * KG) * 8;
        const int d0 = tap % 3 - 1, d1 = (tap / 3) % 3 - 1, d2 = (tap / 9) % 3 - 1, d3 = tap / 27 - 1;
        bf16x8_t bf[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ct++) {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (vk) v = *(const uint4*)(a.W + ((int64_t)(tap * COUTP + ct * 16 + (lane & 15)) * CIN + i0));
            bf[ct] = __builtin_bit_cast(bf16x8_t, v);
        }
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            int n0 = cx[rt][0] + d0, n1 = cx[rt][1] + d1, n2 = cx[rt][2] + d2, n3 = cx[rt][3] + d3;
            n0 = n0 < 0 ? n0 + a.L0 : (n0 >= a.L0 ? n0 - a.L0 : n0);
            n1 = n1 < 0 ? n1 + a.L1 : (n1 >= a.L1 ? n1 - a.L1 : n1);
            n2 = n2 < 0 ? n2 + a.L2 : (n2 >= a.L2 ? n2 - a.L2 : n2);
            n3 = n3 < 0 ? n3 + a.L3 : (n3 >= a.L3 ? n3 - a.L3 : n3);
            const int64_t nb = brow[rt] + n0 + (int64_t)a.L0 * (n1 + a.L1 * (n2 + (int64_t)a.L2 * n3));
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (vk && vrow[rt]) v = *(const uint4*)(a.in + nb * CIN + i0);
            bf16x8_t af = __builtin_bit_cast(bf16x8_t, v);
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[ct], acc[rt][ct], 0, 0, 0);
        }
    }
    // C layout: column = lane % 16, rows 4 (lane / 16) + q
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++) {
            const int o = ct * 16 + (lane & 15);
            if (o >= COUT) continue;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int64_t s = base + rt * 16 + 4 * (lane >> 4) + q;
                if (s >= a.nsites) continue;
                float v = acc[rt][ct][q];
                const int64_t idx = s * COUT + o;
                if (a.mask && !(bf2f(a.mask[idx]) > 0.f)) v = 0.f;
                if (a.out0_fp32) ((float*)a.out0)[idx] = v;
                else ((uint16_t*)a.out0)[idx] = f2bf(v);
                if (a.out1) a.out1[idx] = f2bf(v > 0.f ? v : 0.f);
            }
        }
}

// Weight gradient for one layer: gW[t][o][i] = sum over sites s of g[s][o] in[s + d_t][i]
// (neighbours inside the same sample).  Rows o, columns i, K = sites; each
// workgroup sums its share of sites for one tap into FP32 partials.
struct WgradArgs {
    const uint16_t* g;    // [B][V][COUT] BF16
    const uint16_t* in;   // [B][V][CIN] BF16
    float* partial;       // [chunks][81][COUT][CIN]
    int L0, L1, L2, L3;
    int V;
    int64_t nsites;
    int64_t sites_per_chunk;   // multiple of 32 * CONV_WAVES
};

template <int CIN, int COUT>
__global__ __launch_bounds__(64 * CONV_WAVES) void conv_wgrad_kernel(WgradArgs a) {
    constexpr int OT = (COUT + 15) / 16;
    constexpr int IT = (CIN + 15) / 16;
    __shared__ float red[CONV_WAVES][OT * IT * 4][64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tap = blockIdx.y;
    const int d0 = tap % 3 - 1, d1 = (tap / 3) % 3 - 1, d2 = (tap / 9) % 3 - 1, d3 = tap / 27 - 1;
    const int64_t s_begin = (int64_t)blockIdx.x * a.sites_per_chunk;
    const int64_t s_end = s_begin + a.sites_per_chunk < a.nsites ? s_begin + a.sites_per_chunk : a.nsites;
    f32x4_t acc[OT][IT];
#pragma unroll
    for (int ot = 0; ot < OT; ot++)
#pragma unroll
        for (int it = 0; it < IT; it++) acc[ot][it] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
    const int kq = 8 * (lane >> 4);   // this lane's 8 consecutive K (sites) within a step of 32
    for (int64_t s0 = s_begin + wave * 32; s0 < s_end; s0 += 32 * CONV_WAVES) {
        // A: rows o, K = sites; B: K = sites, columns i (neighbour input)
        bf16x8_t af[OT], bfr[IT];
        uint16_t av[OT][8], bv[IT][8];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int64_t s = s0 + kq + e;
            const bool vs = s < s_end;
            int64_t nb = 0;
            if (vs) {
                int64_t b = s / a.V;
                int x = (int)(s - b * a.V);
                int c0 = x % a.L0;
                x /= a.L0;
                int c1 = x % a.L1;
                x /= a.L1;
                int c2 = x % a.L2;
                int c3 = x / a.L2;
                c0 += d0; c1 += d1; c2 += d2; c3 += d3;
                c0 = c0 < 0 ? c0 + a.L0 : (c0 >= a.L0 ? c0 - a.L0 : c0);
                c1 = c1 < 0 ? c1 + a.L1 : (c1 >= a.L1 ? c1 - a.L1 : c1);
                c2 = c2 < 0 ? c2 + a.L2 : (c2 >= a.L2 ? c2 - a.L2 : c2);
                c3 = c3 < 0 ? c3 + a.L3 : (c3 >= a.L3 ? c3 - a.L3 : c3);
                nb = b * a.V + c0 + (int64_t)a.L0 * (c1 + a.L1 * (c2 + (int64_t)a.L2 * c3));
            }
#pragma unroll
            for (int ot = 0; ot < OT; ot++) {
                const int o = ot * 16 + (lane & 15);
                av[ot][e] = (vs && o < COUT) ? a.g[s * COUT + o] : (uint16_t)0;
            }
#pragma unroll
            for (int it = 0; it < IT; it++) {
                const int i = it * 16 + (lane & 15);
                bv[it][e] = (vs && i < CIN) ? a.in[nb * CIN + i] : (uint16_t)0;
            }
        }
#pragma unroll
        for (int ot = 0; ot < OT; ot++) {
            uint4 v;
            v.x = av[ot][0] | ((uint32_t)av[ot][1] << 16);
            v.y = av[ot][2] | ((uint32_t)av[ot][3] << 16);
            v.z = av[ot][4] | ((uint32_t)av[ot][5] << 16);
            v.w = av[ot][6] | ((uint32_t)av[ot][7] << 16);
            af[ot] = __builtin_bit_cast(bf16x8_t, v);
        }
#pragma unroll
        for (int it = 0; it < IT; it++) {
            uint4 v;
            v.x = bv[it][0] | ((uint32_t)bv[it][1] << 16);
            v.y = bv[it][2] | ((uint32_t)bv[it][3] << 16);
            v.z = bv[it][4] | ((uint32_t)bv[it][5] << 16);
            v.w = bv[it][6] | ((uint32_t)bv[it][7] << 16);
            bfr[it] = __builtin_bit_cast(bf16x8_t, v);
        }
#pragma unroll
        for (int ot = 0; ot < OT; ot++)
#pragma unroll
            for (int it = 0; it < IT; it++)
                acc[ot][it] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ot], bfr[it], acc[ot][it], 0, 0, 0);
    }
    // sum the waves in a fixed order, then write this chunk's partial for the tap
#pragma unroll
    for (int ot = 0; ot < OT; ot++)
#pragma unroll
        for (int it = 0; it < IT; it++)
#pragma unroll
            for (int q = 0; q < 4; q++) red[wave][(ot * IT + it) * 4 + q][lane] = acc[ot][it][q];
    __syncthreads();
    if (wave == 0) {
        float* out = a.partial + ((int64_t)blockIdx.x * 81 + tap) * COUT * CIN;
#pragma unroll
        for (int ot = 0; ot < OT; ot++)
#pragma unroll
            for (int it = 0; it < IT; it++)
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    float v = 0.f;
                    for (int w = 0; w < CONV_WAVES; w++) v += red[w][(ot * IT + it) * 4 + q][lane];
                    const int o = ot * 16 + 4 * (lane >> 4) + q;   // C row
                    const int i = it * 16 + (lane & 15);          // C column
                    if (o < COUT && i < CIN) out[o * CIN + i] = v;
                }
    }
}

__global__ void wgrad_sum_kernel(const float* partial, int nchunk, int64_t n, float* gw) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; c++) s += partial[(int64_t)c * n + i];
    gw[i] = (float)s;
}

// ---------------------------------------------------------------------------
// loss (relative squared error per sample), its gradient, Adam, conversions
// ---------------------------------------------------------------------------
// y: network output, rs: skip term s r (or null), e: target
__global__ void loss_partial_kernel(const float* y, const float* rs, const float* e, int64_t per_sample, double* s1,
                                    double* s2) {
    __shared__ double r1[256], r2[256];
    const int b = blockIdx.x;
    double a1 = 0.0, a2 = 0.0;
    for (int64_t i = threadIdx.x; i < per_sample; i += 256) {
        double yy = y[b * per_sample + i], ee = e[b * per_sample + i];
        if (rs) yy += rs[b * per_sample + i];
        a1 += (yy - ee) * (yy - ee);
        a2 += ee * ee;
    }
    r1[threadIdx.x] = a1;
    r2[threadIdx.x] = a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        s1[b] = r1[0];
        s2[b] = r2[0];
    }
}

__global__ void loss_grad_kernel(const float* y, const float* rs, const float* e, const double* s2, int64_t per_sample,
                                 int64_t n, double scale, uint16_t* gy) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t b = i / per_sample;
    double den = s2[b] > 0 ? s2[b] : 1.0;
    double yy = (double)y[i] + (rs ? (double)rs[i] : 0.0);
    gy[i] = f2bf((float)(2.0 * (yy - e[i]) / den * scale));
}

__global__ void adam_kernel(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float c1, float c2, float eps) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// FP32 master [81][COUT][CIN] -> BF16 forward [81][COUT16][CIN] and backward [81][CIN16][COUT]
__global__ void weight_copies_kernel(const float* w, int cin, int cout, uint16_t* wf, uint16_t* wb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)81 * cout * cin;
    if (i >= n) return;
    int t = (int)(i / ((int64_t)cout * cin));
    int rem = (int)(i - (int64_t)t * cout * cin);
    int o = rem / cin, ci = rem - o * cin;
    uint16_t h = f2bf(w[i]);
    int cout16 = (cout + 15) / 16 * 16, cin16 = (cin + 15) / 16 * 16;
    wf[((int64_t)t * cout16 + o) * cin + ci] = h;
    wb[((int64_t)(80 - t) * cin16 + ci) * cout + o] = h;
}

// canonical complex128 spinors [n][V][12] <-> NN channels [n][V][24]
__global__ void canon_to_bf16_kernel(const double* in, uint16_t* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf((float)in[i]);
}
__global__ void canon_to_f32_kernel(const double* in, float* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}
__global__ void canon_scaled_to_f32_kernel(const double* in, float s, float* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = s * (float)in[i];
}
__global__ void f32_skip_to_canon_kernel(const float* in, const double* r, float s, double* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i] + (double)(s * (float)r[i]);
}
__global__ void f32_to_canon_kernel(const float* in, double* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}
__global__ void scaled_to_bf16_kernel(const float* in, uint16_t* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(in[i]);
}

static dim3 g256(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int64_t layer_size(int l) { return (int64_t)81 * NN_CH[l] * NN_CH[l + 1]; }
static int64_t pad16(int c) { return (c + 15) / 16 * 16; }

int nn_alloc(dht_ctx* c) {
    if (c->nn.ready) return DHT_OK;
    int64_t tot = 0;
    for (int l = 0; l < 3; l++) tot += layer_size(l);
    size_t fb = sizeof(float) * tot;
    size_t hb = 0;
    for (int l = 0; l < 3; l++) hb += sizeof(uint16_t) * 81 * (pad16(NN_CH[l + 1]) * NN_CH[l] + pad16(NN_CH[l]) * NN_CH[l + 1]);
    void* p;
    if (hipMalloc(&p, 4 * fb + hb) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(DHT_ERR_OOM, "cannot allocate network weights");
    }
    c->nn.mem = p;
    char* q = (char*)p;
    int64_t off = 0;
    for (int l = 0; l < 3; l++) {
        c->nn.w[l] = (float*)q + off;
        c->nn.g[l] = (float*)(q + fb) + off;
        c->nn.m[l] = (float*)(q + 2 * fb) + off;
        c->nn.v[l] = (float*)(q + 3 * fb) + off;
        off += layer_size(l);
    }
    uint16_t* h = (uint16_t*)(q + 4 * fb);
    for (int l = 0; l < 3; l++) {
        c->nn.wf[l] = h;
        h += 81 * pad16(NN_CH[l + 1]) * NN_CH[l];
        c->nn.wb[l] = h;
        h += 81 * pad16(NN_CH[l]) * NN_CH[l + 1];
    }
    DHT_TRY(zero(c, p, 4 * fb + hb));
    c->nn.ready = true;
    return DHT_OK;
}

int nn_refresh_copies(dht_ctx* c) {
    for (int l = 0; l < 3; l++) {
        hipLaunchKernelGGL(weight_copies_kernel, g256(layer_size(l)), dim3(256), 0, c->stream, c->nn.w[l], NN_CH[l],
                           NN_CH[l + 1], c->nn.wf[l], c->nn.wb[l]);
        DHT_HIP(hipGetLastError());
    }
    return DHT_OK;
}

int nn_set_weights(dht_ctx* c, const float* host) {
    DHT_TRY(nn_alloc(c));
    int64_t off = 0;
    for (int l = 0; l < 3; l++) {
        DHT_HIP(hipMemcpyAsync(c->nn.w[l], host + off, sizeof(float) * layer_size(l), hipMemcpyHostToDevice, c->stream));
        off += layer_size(l);
    }
    // a new set of weights restarts the optimiser
    for (int l = 0; l < 3; l++) {
        DHT_TRY(zero(c, c->nn.m[l], sizeof(float) * layer_size(l)));
        DHT_TRY(zero(c, c->nn.v[l], sizeof(float) * layer_size(l)));
    }
    c->nn.step = 0;
    DHT_TRY(nn_refresh_copies(c));
    DHT_HIP(hipStreamSynchronize(c->stream));
    return DHT_OK;
}

int nn_get_weights(dht_ctx* c, float* host, bool grads) {
    if (!c->nn.ready) return set_error(DHT_ERR_STATE, "network not initialised");
    int64_t off = 0;
    for (int l = 0; l < 3; l++) {
        DHT_HIP(hipMemcpyAsync(host + off, grads ? c->nn.g[l] : c->nn.w[l], sizeof(float) * layer_size(l),
                               hipMemcpyDeviceToHost, c->stream));
        off += layer_size(l);
    }
    DHT_HIP(hipStreamSynchronize(c->stream));
    return DHT_OK;
}

int64_t nn_num_weights() {
    int64_t t = 0;
    for (int l = 0; l < 3; l++) t += layer_size(l);
    return t;
}

template <int CIN, int COUT>
static void launch_conv(dht_ctx* c, const uint16_t* in, const uint16_t* W, void* out0, bool out0_fp32, uint16_t* out1,
                        const uint16_t* mask, int nb) {
    ConvArgs a;
    a.in = in;
    a.W = W;
    a.out0 = out0;
    a.out1 = out1;
    a.mask = mask;
    a.L0 = c->g.L[0];
    a.L1 = c->g.L[1];
    a.L2 = c->g.L[2];
    a.L3 = c->g.L[3];
    a.V = (int)c->g.V;
    a.nsites = (int64_t)nb * c->g.V;
    a.out0_fp32 = out0_fp32 ? 1 : 0;
    int64_t blocks = (a.nsites + 64 * CONV_WAVES - 1) / (64 * CONV_WAVES);
    hipLaunchKernelGGL((conv_fwd_kernel<CIN, COUT>), dim3((unsigned)blocks), dim3(64 * CONV_WAVES), 0, c->stream, a);
}

static int conv(dht_ctx* c, int cin, int cout, const uint16_t* in, const uint16_t* W, void* out0, bool out0_fp32,
                uint16_t* out1, const uint16_t* mask, int nb) {
    int tok;
    DHT_TRY(prof_begin(c, &tok));
    if (cin == 24 && cout == 48) launch_conv<24, 48>(c, in, W, out0, out0_fp32, out1, mask, nb);
    else if (cin == 48 && cout == 48) launch_conv<48, 48>(c, in, W, out0, out0_fp32, out1, mask, nb);
    else if (cin == 48 && cout == 24) launch_conv<48, 24>(c, in, W, out0, out0_fp32, out1, mask, nb);
    else return set_error(DHT_ERR_INVALID_ARG, "unsupported convolution shape");
    DHT_HIP(hipGetLastError());
    // the profile of this class counts flops (2 per multiply-add) in place of bytes
    return prof_end(c, tok, PROF_CONV, 2.0 * 81.0 * cin * cout * (double)nb * (double)c->g.V);
}

template <int CIN, int COUT>
static int launch_wgrad(dht_ctx* c, const uint16_t* g, const uint16_t* in, float* gw, int nb) {
    WgradArgs a;
    a.g = g;
    a.in = in;
    a.L0 = c->g.L[0];
    a.L1 = c->g.L[1];
    a.L2 = c->g.L[2];
    a.L3 = c->g.L[3];
    a.V = (int)c->g.V;
    a.nsites = (int64_t)nb * c->g.V;
    const int64_t quantum = 32 * CONV_WAVES;
    int64_t chunks = std::max<int64_t>(1, std::min<int64_t>(64, (a.nsites + 4 * quantum - 1) / (4 * quantum)));
    int64_t spc = (a.nsites + chunks - 1) / chunks;
    spc = (spc + quantum - 1) / quantum * quantum;
    chunks = (a.nsites + spc - 1) / spc;
    a.sites_per_chunk = spc;
    const int64_t n = (int64_t)81 * COUT * CIN;
    void* part;
    DHT_TRY(ws_get(c, WS_NN_PART, sizeof(float) * n * chunks, &part));
    a.partial = (float*)part;
    hipLaunchKernelGGL((conv_wgrad_kernel<CIN, COUT>), dim3((unsigned)chunks, 81), dim3(64 * CONV_WAVES), 0, c->stream,
                       a);
    DHT_HIP(hipGetLastError());
    hipLaunchKernelGGL(wgrad_sum_kernel, g256(n), dim3(256), 0, c->stream, (const float*)part, (int)chunks, n, gw);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

static int wgrad(dht_ctx* c, int l, const uint16_t* g, const uint16_t* in, int nb) {
    if (l == 0) return launch_wgrad<24, 48>(c, g, in, c->nn.g[0], nb);
    if (l == 1) return launch_wgrad<48, 48>(c, g, in, c->nn.g[1], nb);
    return launch_wgrad<48, 24>(c, g, in, c->nn.g[2], nb);
}

// activation workspace for nb samples
struct NNBufs {
    uint16_t *x, *h1, *a1, *h2, *a2, *gy, *g2, *g1;
    float *y, *e, *rs;   // output, target, skip term s r (FP32, from the unrounded input)
};

static int nn_bufs(dht_ctx* c, int nb, NNBufs* b) {
    const int64_t V = c->g.V;
    const size_t s24 = (size_t)nb * V * 24, s48 = (size_t)nb * V * 48;
    void* p;
    size_t bytes = sizeof(uint16_t) * (s24 * 2 + s48 * 6) + sizeof(float) * s24 * 3 + 1536;
    DHT_TRY(ws_get(c, WS_NN_ACT, bytes, &p));
    char* q = (char*)p;
    auto take = [&](size_t nbytes) {
        char* r = q;
        q += (nbytes + 255) / 256 * 256;
        return r;
    };
    b->x = (uint16_t*)take(2 * s24);
    b->gy = (uint16_t*)take(2 * s24);
    b->h1 = (uint16_t*)take(2 * s48);
    b->a1 = (uint16_t*)take(2 * s48);
    b->h2 = (uint16_t*)take(2 * s48);
    b->a2 = (uint16_t*)take(2 * s48);
    b->g2 = (uint16_t*)take(2 * s48);
    b->g1 = (uint16_t*)take(2 * s48);
    b->y = (float*)take(4 * s24);
    b->e = (float*)take(4 * s24);
    b->rs = (float*)take(4 * s24);
    (void)bytes;
    return DHT_OK;
}

// inference only (the preconditioner inside FGMRES): input, the two hidden
// activations and the output; the pre-activation values, which only the
// backward pass reads, share one scratch block
size_t nn_infer_bytes(const dht_ctx* c, int nb) {
    const size_t s24 = (size_t)nb * c->g.V * 24, s48 = (size_t)nb * c->g.V * 48;
    return sizeof(uint16_t) * (s24 + s48 * 3) + sizeof(float) * s24 + 1024;
}

static int nn_bufs_infer(dht_ctx* c, int nb, NNBufs* b) {
    const int64_t V = c->g.V;
    const size_t s24 = (size_t)nb * V * 24, s48 = (size_t)nb * V * 48;
    void* p;
    DHT_TRY(ws_get(c, WS_NN_ACT, nn_infer_bytes(c, nb), &p));
    char* q = (char*)p;
    auto take = [&](size_t nbytes) {
        char* r = q;
        q += (nbytes + 255) / 256 * 256;
        return r;
    };
    memset(b, 0, sizeof(*b));
    b->x = (uint16_t*)take(2 * s24);
    b->h1 = (uint16_t*)take(2 * s48);
    b->h2 = b->h1;
    b->a1 = (uint16_t*)take(2 * s48);
    b->a2 = (uint16_t*)take(2 * s48);
    b->y = (float*)take(4 * s24);
    return DHT_OK;
}

// forward of nb samples already in b.x (BF16); output in b.y (FP32)
static int nn_forward_bufs(dht_ctx* c, NNBufs& b, int nb) {
    DHT_TRY(conv(c, 24, 48, b.x, c->nn.wf[0], b.h1, false, b.a1, nullptr, nb));
    DHT_TRY(conv(c, 48, 48, b.a1, c->nn.wf[1], b.h2, false, b.a2, nullptr, nb));
    DHT_TRY(conv(c, 48, 24, b.a2, c->nn.wf[2], b.y, true, nullptr, nullptr, nb));
    return DHT_OK;
}

// loss over nb samples (b.y vs b.e), gradients into c->nn.g; returns the loss on the host
static int nn_loss_backward(dht_ctx* c, NNBufs& b, int nb, double* loss) {
    const int64_t per = c->g.V * 24;
    void* s;
    DHT_TRY(ws_get(c, WS_NN_SCAL, sizeof(double) * 2 * nb, &s));
    double* s1 = (double*)s;
    double* s2 = s1 + nb;
    const float* rs = c->nn.skip != 0.f ? b.rs : nullptr;
    hipLaunchKernelGGL(loss_partial_kernel, dim3(nb), dim3(256), 0, c->stream, b.y, rs, b.e, per, s1, s2);
    DHT_HIP(hipGetLastError());
    hipLaunchKernelGGL(loss_grad_kernel, g256(per * nb), dim3(256), 0, c->stream, b.y, rs, b.e, s2, per, per * nb,
                       1.0 / nb, b.gy);
    DHT_HIP(hipGetLastError());
    // layer 3: weight gradient from a2; data gradient through layer 3, masked by h2 > 0
    DHT_TRY(wgrad(c, 2, b.gy, b.a2, nb));
    DHT_TRY(conv(c, 24, 48, b.gy, c->nn.wb[2], b.g2, false, nullptr, b.h2, nb));
    DHT_TRY(wgrad(c, 1, b.g2, b.a1, nb));
    DHT_TRY(conv(c, 48, 48, b.g2, c->nn.wb[1], b.g1, false, nullptr, b.h1, nb));
    DHT_TRY(wgrad(c, 0, b.g1, b.x, nb));
    if (loss) {
        std::vector<double> h(2 * nb);
        DHT_HIP(hipMemcpyAsync(h.data(), s1, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, c->stream));
        DHT_HIP(hipStreamSynchronize(c->stream));
        double L = 0.0;
        for (int i = 0; i < nb; i++) L += h[nb + i] > 0 ? h[i] / h[nb + i] : 0.0;
        *loss = L / nb;
    }
    return DHT_OK;
}

static int nn_adam(dht_ctx* c, float lr) {
    c->nn.step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)c->nn.step), c2 = 1.f - powf(b2, (float)c->nn.step);
    for (int l = 0; l < 3; l++) {
        hipLaunchKernelGGL(adam_kernel, g256(layer_size(l)), dim3(256), 0, c->stream, c->nn.w[l], c->nn.g[l],
                           c->nn.m[l], c->nn.v[l], layer_size(l), lr, b1, b2, c1, c2, 1e-8f);
        DHT_HIP(hipGetLastError());
    }
    return nn_refresh_copies(c);
}

// canonical complex128 [nb][V][12] -> b.x (BF16) and optionally b.e (FP32)
static int nn_load(dht_ctx* c, NNBufs& b, const double* R, const double* E, int nb) {
    const int64_t n = (int64_t)nb * c->g.V * 24;
    hipLaunchKernelGGL(canon_to_bf16_kernel, g256(n), dim3(256), 0, c->stream, R, b.x, n);
    DHT_HIP(hipGetLastError());
    if (E) {
        hipLaunchKernelGGL(canon_to_f32_kernel, g256(n), dim3(256), 0, c->stream, E, b.e, n);
        DHT_HIP(hipGetLastError());
        if (c->nn.skip != 0.f) {
            hipLaunchKernelGGL(canon_scaled_to_f32_kernel, g256(n), dim3(256), 0, c->stream, R, c->nn.skip, b.rs, n);
            DHT_HIP(hipGetLastError());
        }
    }
    return DHT_OK;
}

int nn_forward_canon(dht_ctx* c, const double* R, double* E, int n) {
    if (!c->nn.ready) return set_error(DHT_ERR_STATE, "network not initialised");
    for (int r0 = 0; r0 < n; r0 += NN_MAX_BATCH) {
        const int nb = std::min(NN_MAX_BATCH, n - r0);
        NNBufs b;
        DHT_TRY(nn_bufs(c, nb, &b));
        const int64_t off = (int64_t)r0 * c->g.V * 24;
        DHT_TRY(nn_load(c, b, R + off, nullptr, nb));
        DHT_TRY(nn_forward_bufs(c, b, nb));
        const int64_t m = (int64_t)nb * c->g.V * 24;
        hipLaunchKernelGGL(f32_skip_to_canon_kernel, g256(m), dim3(256), 0, c->stream, b.y, R + off, c->nn.skip,
                           E + off, m);
        DHT_HIP(hipGetLastError());
    }
    DHT_HIP(hipStreamSynchronize(c->stream));
    return DHT_OK;
}

int nn_grad_canon(dht_ctx* c, const double* R, const double* E, int n, double* loss) {
    if (!c->nn.ready) return set_error(DHT_ERR_STATE, "network not initialised");
    if (n > NN_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "gradient batch too large");
    NNBufs b;
    DHT_TRY(nn_bufs(c, n, &b));
    DHT_TRY(nn_load(c, b, R, E, n));
    DHT_TRY(nn_forward_bufs(c, b, n));
    DHT_TRY(nn_loss_backward(c, b, n, loss));
    DHT_HIP(hipStreamSynchronize(c->stream));
    return DHT_OK;
}

int nn_train_canon(dht_ctx* c, const double* R, const double* E, int npairs, int epochs, int batch, float lr,
                   double* final_loss) {
    if (!c->nn.ready) return set_error(DHT_ERR_STATE, "network not initialised");
    if (batch <= 0 || batch > NN_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "bad minibatch size");
    double last = 0.0;
    const int64_t per = c->g.V * 24;
    for (int ep = 0; ep < epochs; ep++) {
        double sum = 0.0;
        int cnt = 0;
        for (int p0 = 0; p0 < npairs; p0 += batch) {
            const int nb = std::min(batch, npairs - p0);
            NNBufs b;
            DHT_TRY(nn_bufs(c, nb, &b));
            DHT_TRY(nn_load(c, b, R + p0 * per, E + p0 * per, nb));
            DHT_TRY(nn_forward_bufs(c, b, nb));
            double L;
            DHT_TRY(nn_loss_backward(c, b, nb, &L));
            DHT_TRY(nn_adam(c, lr));
            sum += L * nb;
            cnt += nb;
        }
        last = cnt ? sum / cnt : 0.0;
    }
    DHT_HIP(hipStreamSynchronize(c->stream));
    if (final_loss) *final_loss = last;
    return DHT_OK;
}

// Apply the network to a full internal FP32 field (nrhs slots) in place of
// the preconditioner: out = M(in).  in/out: [2][6][Vh][B][2] complex FP32.
template <bool TO_NN>
__global__ void field_nn_kernel(float* field, uint16_t* xin, const float* yout, const float* fin, float skip, Geom g,
                                int B, int n) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (p, s, r)
    if (gid >= g.V * (int64_t)B) return;
    int64_t ps = gid / B;
    int r = (int)(gid - ps * B);
    int p = (int)(ps / g.Vh);
    int64_t s = ps - (int64_t)p * g.Vh;
    int cc[4];
    cb_coords(g, s, p, cc);
    int64_t site = lex_index(g, cc);
    const int64_t SB = g.Vh * B;
    const int64_t vbase = (int64_t)p * 6 * SB + s * B + r;
    for (int j = 0; j < 6; j++) {
        float4* v = (float4*)field + vbase + j * SB;
        if (TO_NN) {
            float4 d = *v;
            uint16_t* o = xin + ((int64_t)r * g.V + site) * 24 + 4 * j;
            if (r < n) {
                o[0] = f2bf(d.x);
                o[1] = f2bf(d.y);
                o[2] = f2bf(d.z);
                o[3] = f2bf(d.w);
            }
        } else {
            float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < n) {
                const float* y = yout + ((int64_t)r * g.V + site) * 24 + 4 * j;
                const float4 x = ((const float4*)fin)[vbase + j * SB];
                d = make_float4(y[0] + skip * x.x, y[1] + skip * x.y, y[2] + skip * x.z, y[3] + skip * x.w);
            }
            *v = d;
        }
    }
}

int nn_apply_field(dht_ctx* c, const void* in, void* out, int nrhs) {
    if (!c->nn.ready) return set_error(DHT_ERR_STATE, "network not initialised");
    if (nrhs > NN_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "preconditioner batch too large");
    NNBufs b;
    DHT_TRY(nn_bufs_infer(c, nrhs, &b));
    int64_t tot = c->g.V * (int64_t)nrhs;
    hipLaunchKernelGGL(field_nn_kernel<true>, g256(tot), dim3(256), 0, c->stream, (float*)in, b.x, (const float*)nullptr,
                       (const float*)nullptr, 0.f, c->g, nrhs, nrhs);
    DHT_HIP(hipGetLastError());
    DHT_TRY(nn_forward_bufs(c, b, nrhs));
    hipLaunchKernelGGL(field_nn_kernel<false>, g256(tot), dim3(256), 0, c->stream, (float*)out, (uint16_t*)nullptr,
                       (const float*)b.y, (const float*)in, c->nn.skip, c->g, nrhs, nrhs);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

}  // namespace dht
