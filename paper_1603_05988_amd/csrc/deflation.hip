// Deflation of the trace estimator (Section 5.2; Algorithm 1: the deflation space, T_D, and the
// deflation correction of each probe's quadratic form).
//
// With k eigenvectors W of the Hermitian Q = g5 D (stored rounded to FP64,
// FP32 or BF16), the deflated part of D^-1 = Q^-1 g5 is P = W M W^H g5 with
// M = (W^H Q W)^-1, the Galerkin inverse of Q on span(W) (equal to Lambda^-1
// for exact orthonormal eigenvectors, i.e. V Sigma^-1 U^H of Section 5.2).
// H = W^H Q W and the trace T_D = Tr(P) = Tr(M W^H g5 W) are accumulated in
// FP64 from the stored vectors, so the estimator stays unbiased whatever the
// storage precision: only its variance depends on how good W is.  A diagonal
// variant (M = diag(1 / w_i^H Q w_i), T_D = sum M_ii w_i^H g5 w_i) needs only
// k dot products and is exact for orthonormal eigenvectors.
//
// Per probe: c1 = W^H z and c2 = W^H g5 z (g5 = +1 on spins 0, 1 and -1 on
// spins 2, 3 in the chiral basis, so both come from one pass over W), and
// z^H P z = c1^H M c2.
//
// Storage of W.  FP64 / FP32: k full internal fields with one RHS each,
// column after column ([k][2][12][Vh]).  BF16: the MFMA A-fragment order of
// v_mfma_f32_32x32x16_bf16 -- rows (columns of W) grouped in tiles of 32,
// the real K axis (2 x complex entries) in steps of 16; one step of one tile
// is 64 lanes x 16 bytes, lane = row % 32 + 32 * ((K' % 16) / 8), so every
// step of the projection is a single coalesced 1 KB wavefront load.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>

#include "solver.h"

namespace dht {

// ---------------------------------------------------------------------------
// W addressing
// ---------------------------------------------------------------------------
struct WLayout {
    int64_t Kn;       // complex entries per column (24 Vh)
    int64_t nsteps;   // Kn / 8: MFMA K-steps (16 reals) per tile
    int kp;           // rows padded to a multiple of 32
    int tiled;        // BF16 fragment order
};

// element index (in complex units of the storage type) of W(i, K)
__host__ __device__ inline int64_t w_index(const WLayout& L, int64_t i, int64_t K) {
    if (!L.tiled) return i * L.Kn + K;
    int64_t t = i >> 5, lr = i & 31;
    return (((t * L.nsteps + (K >> 3)) * 64 + lr + 32 * ((K & 7) >> 2)) << 2) + (K & 3);
}

static WLayout wlayout(const dht_ctx* c) {
    WLayout L;
    L.Kn = 24 * c->g.Vh;
    L.nsteps = L.Kn / 8;
    L.kp = ((c->k + 31) / 32) * 32;
    L.tiled = c->wprec == DHT_BF16;
    return L;
}

static size_t w_bytes(const dht_ctx* c, int k, int prec) {
    int64_t Kn = 24 * c->g.Vh;
    int64_t rows = prec == DHT_BF16 ? ((k + 31) / 32) * 32 : k;
    return (size_t)rows * Kn * elem_bytes(prec);
}

// ---------------------------------------------------------------------------
// generic projection (any storage precision, FP64 probes), FP64 accumulation
// ---------------------------------------------------------------------------
static constexpr int PROJ_THREADS = 256;
static constexpr int PROJ_RT = 4;    // right-hand sides per pass

template <typename SW, typename SZ>
__global__ __launch_bounds__(PROJ_THREADS) void proj_generic_kernel(const typename Store<SW>::elem* W, WLayout wl,
                                                                    const typename Store<SZ>::elem* Z,
                                                                    int64_t per_comp, int B, int r0, int nr,
                                                                    int64_t chunk, Cx<double>* p1, Cx<double>* p2,
                                                                    int k) {
    __shared__ Cx<double> red[2 * PROJ_RT][PROJ_THREADS];
    const int i = blockIdx.y;
    const int64_t Kn = wl.Kn;
    const int64_t cbeg = (int64_t)blockIdx.x * chunk;
    const int64_t cend = cbeg + chunk < Kn ? cbeg + chunk : Kn;
    Cx<double> a1[PROJ_RT], a2[PROJ_RT];
#pragma unroll
    for (int q = 0; q < PROJ_RT; q++) a1[q] = a2[q] = cmake(0.0, 0.0);
    for (int64_t K = cbeg + threadIdx.x; K < cend; K += PROJ_THREADS) {
        auto wv = Store<SW>::ld(W + w_index(wl, i, K));
        Cx<double> wd = cmake<double>(wv.re, wv.im);
        int comp = (int)((K / per_comp) % 12);
        double sg = comp < 6 ? 1.0 : -1.0;
        const typename Store<SZ>::elem* zp = Z + K * B + r0;
#pragma unroll
        for (int q = 0; q < PROJ_RT; q++) {
            if (q < nr) {
                auto zv = Store<SZ>::ld(zp + q);
                Cx<double> pr = conjmul(wd, cmake<double>(zv.re, zv.im));
                a1[q] = a1[q] + pr;
                a2[q] = a2[q] + sg * pr;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PROJ_RT; q++) {
        red[q][threadIdx.x] = a1[q];
        red[PROJ_RT + q][threadIdx.x] = a2[q];
    }
    __syncthreads();
    for (int st = PROJ_THREADS / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
#pragma unroll
            for (int q = 0; q < 2 * PROJ_RT; q++) red[q][threadIdx.x] = red[q][threadIdx.x] + red[q][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < nr) {
        int q = threadIdx.x;
        p1[((int64_t)blockIdx.x * k + i) * B + r0 + q] = red[q][0];
        p2[((int64_t)blockIdx.x * k + i) * B + r0 + q] = red[PROJ_RT + q][0];
    }
}

__global__ void proj_sum_kernel(const Cx<double>* p1, const Cx<double>* p2, int nchunk, int k, int B, Cx<double>* c1,
                                Cx<double>* c2) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= k * B) return;
    Cx<double> s1 = cmake(0.0, 0.0), s2 = cmake(0.0, 0.0);
    for (int ch = 0; ch < nchunk; ch++) {
        s1 = s1 + p1[(int64_t)ch * k * B + idx];
        s2 = s2 + p2[(int64_t)ch * k * B + idx];
    }
    c1[idx] = s1;
    c2[idx] = s2;
}

// split of the basis entries over workgroups of the generic projection: at
// most 256 chunks of at least 8192 entries
static int field_chunks(const dht_ctx* c, int64_t* chunk_out) {
    const int64_t Kn = 24 * c->g.Vh;
    int64_t chunk = 8192;
    int nchunk = (int)((Kn + chunk - 1) / chunk);
    while (nchunk > 256) {
        chunk *= 2;
        nchunk = (int)((Kn + chunk - 1) / chunk);
    }
    if (chunk_out) *chunk_out = chunk;
    return nchunk;
}

void ws_plan_project_field(const dht_ctx* c, int nrhs, size_t* plan) {
    const size_t pb = (size_t)field_chunks(c, nullptr) * c->k * nrhs * sizeof(Cx<double>);
    plan_max(plan, WS_PROJ, pb);
    plan_max(plan, WS_PROJ2, pb);
}

int project_field(dht_ctx* c, const void* Z, int zprec, int nrhs, Cx<double>* c1, Cx<double>* c2) {
    if (!c->W || c->k <= 0) return set_error(DHT_ERR_STATE, "no deflation basis");
    const WLayout wl = wlayout(c);
    const int k = c->k;
    int64_t chunk;
    const int nchunk = field_chunks(c, &chunk);
    void *p1, *p2;
    size_t pb = (size_t)nchunk * k * nrhs * sizeof(Cx<double>);
    DHT_TRY(ws_get(c, WS_PROJ, pb, &p1));
    DHT_TRY(ws_get(c, WS_PROJ2, pb, &p2));
    int tok;
    DHT_TRY(prof_begin(c, &tok));
    for (int r0 = 0; r0 < nrhs; r0 += PROJ_RT) {
        int nr = std::min(PROJ_RT, nrhs - r0);
        dim3 grid(nchunk, k), block(PROJ_THREADS);
#define DHT_PG(PW, TW, PZ, TZ)                                                                                     \
    if (c->wprec == PW && zprec == PZ) {                                                                           \
        hipLaunchKernelGGL((proj_generic_kernel<TW, TZ>), grid, block, 0, c->stream,                               \
                           (const typename Store<TW>::elem*)c->W, wl, (const typename Store<TZ>::elem*)Z,          \
                           (int64_t)c->g.Vh, nrhs, r0, nr, chunk, (Cx<double>*)p1, (Cx<double>*)p2, k);             \
        goto done;                                                                                                 \
    }
        DHT_PG(DHT_FP64, double, DHT_FP64, double)
        DHT_PG(DHT_FP32, float, DHT_FP64, double)
        DHT_PG(DHT_BF16, bf16x2, DHT_FP64, double)
#undef DHT_PG
        return set_error(DHT_ERR_INVALID_ARG, "unsupported projection precision pair");
    done:
        DHT_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(proj_sum_kernel, dim3((k * nrhs + 127) / 128), dim3(128), 0, c->stream, (const Cx<double>*)p1,
                       (const Cx<double>*)p2, nchunk, k, nrhs, c1, c2);
    DHT_HIP(hipGetLastError());
    return prof_end(c, tok, PROF_PROJ_GENERIC,
                    (double)k * wl.Kn * elem_bytes(c->wprec) + (double)wl.Kn * nrhs * elem_bytes(zprec));
}

// ---------------------------------------------------------------------------
// MFMA projection: BF16 W (fragment order) x probes given as 2-bit codes
// (z = i^code, exact in BF16), FP32 MFMA accumulation flushed to FP64
// registers after every chunk of kc complex entries, FP64 cross-workgroup sum.
//
// As a real GEMM: conj(w) z = (wr zr + wi zi) + i (wr zi - wi zr), so with
// W viewed as a real [k][2 Kn] BF16 matrix (its storage), the B operand has
// two columns per RHS: (zr, zi) interleaved for the real part and (zi, -zr)
// for the imaginary part.  The K axis is split into the four groups
// (parity, upper/lower spins) of 6 Vh entries; a workgroup works inside one
// group, so the g5 sign is a per-workgroup constant.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

static constexpr int MP_WAVES = 8;
static constexpr int MP_THREADS = 64 * MP_WAVES;

struct MfmaProjArgs {
    const uint4* W;          // fragment-ordered BF16 W
    const uint8_t* zc;       // probe codes [Kn][B]
    int64_t nsteps;          // K-steps per tile (Kn / 8)
    int64_t group_len;       // 6 Vh complex entries
    int64_t chunks_per_group;
    int wg_per_group;
    int kc;                  // complex entries per chunk (multiple of 8, divides group_len)
    int B;
    int ntiles;              // row tiles of 32 (kp / 32)
    double* partial;         // [gridDim.x][kp][NT*32]
    int kp;
};

__device__ inline uint32_t bf16_unit(int v) { return v > 0 ? 0x3F80u : (v < 0 ? 0xBF80u : 0u); }

// Each workgroup takes a contiguous run of chunks of one group.  The probe
// codes of MP_FILL chunks (a contiguous run of bytes) are fetched with 8-byte
// loads one fill ahead, so their latency hides behind the previous fill's
// MFMAs; each fill stages them in LDS and expands them there into B
// fragments.  Inside a chunk every wave issues all of its A-fragment loads
// (RT tiles x the chunk's K-steps) before the MFMAs, so that RT * kc / 8
// 16-byte loads per lane are in flight; the FP32 accumulators are flushed
// to FP64 after every chunk.
static constexpr int MP_FILL = 4;
static constexpr int MP_KC_MAX = 64;   // largest chunk (complex entries)

// Spin-pair form (SP): the groups are (parity, spin s) of 3 Vh entries, and
// the B operand holds the probe codes of all four spins t at the same
// (parity, colour, site) entries, one run of codes per t, so that one pass
// gives W_s^H z_t for the 16 pairs (s, t); the column of probe r and spin t
// is slot t B + r.
template <int RT, int NT, bool SP>
__global__ __launch_bounds__(MP_THREADS) void proj_mfma_kernel(MfmaProjArgs a) {
    extern __shared__ uint4 bfr[];   // [MP_FILL][kc/8][NT][64] B fragments, then the raw codes
    // raw codes of one fill: RUNS * MP_FILL * kc * B bytes <= MP_FILL * 64 * NT * 16
    // (2 RUNS B <= 32 NT columns)
    constexpr int RUNS = SP ? 4 : 1;
    constexpr int RAW_PER_THREAD = (MP_FILL * MP_KC_MAX * NT * 16 / 8 + MP_THREADS - 1) / MP_THREADS;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int g = blockIdx.x / a.wg_per_group;           // group: parity * 2 + (lower spins)
    const int wslot = blockIdx.x - g * a.wg_per_group;
    const int tile0 = (blockIdx.y * MP_WAVES + wave) * RT;
    const int nks = a.kc >> 3;
    const int64_t per = (a.chunks_per_group + a.wg_per_group - 1) / a.wg_per_group;
    const int64_t c_begin = wslot * per;
    const int64_t c_end = c_begin + per < a.chunks_per_group ? c_begin + per : a.chunks_per_group;
    uint8_t* raw = (uint8_t*)(bfr + (size_t)MP_FILL * nks * NT * 64);

    f32x16_t acc[RT][NT];
    double facc[RT][NT][16];
#pragma unroll
    for (int rt = 0; rt < RT; rt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
#pragma unroll
            for (int q = 0; q < 16; q++) {
                acc[rt][nt][q] = 0.f;
                facc[rt][nt][q] = 0.0;
            }
        }

    // 8-byte words of the codes of the fill starting at chunk cf
    uint2 rv[RAW_PER_THREAD];
    auto fetch = [&](int64_t cf) {
        const int nfill = (int)(c_end - cf < MP_FILL ? c_end - cf : MP_FILL);
        const int run_words = (nfill * a.kc * a.B) >> 3;
#pragma unroll
        for (int j = 0; j < RAW_PER_THREAD; j++) {
            const int w = tid + j * MP_THREADS;
            if (w < RUNS * run_words) {
                const int t = SP ? w / run_words : 0;
                const int64_t grp = SP ? (int64_t)(g & ~3) + t : g;   // (parity, spin t) for SP
                const uint2* src = (const uint2*)(a.zc + (grp * a.group_len + cf * a.kc) * a.B);
                rv[j] = src[w - t * run_words];
            }
        }
    };
    if (c_begin < c_end) fetch(c_begin);

    for (int64_t cf = c_begin; cf < c_end; cf += MP_FILL) {
        const int nfill = (int)(c_end - cf < MP_FILL ? c_end - cf : MP_FILL);
        const int64_t K0 = (int64_t)g * a.group_len + cf * a.kc;
        __syncthreads();   // the previous fill's fragments and codes are no longer read
        const int run_bytes = nfill * a.kc * a.B;
        {
            const int nwords = (RUNS * run_bytes) >> 3;
#pragma unroll
            for (int j = 0; j < RAW_PER_THREAD; j++) {
                const int w = tid + j * MP_THREADS;
                if (w < nwords) ((uint2*)raw)[w] = rv[j];
            }
        }
        __syncthreads();
        if (cf + MP_FILL < c_end) fetch(cf + MP_FILL);   // in flight during this fill
        // expand: item (K-step, half, probe) -> the fragments of columns 2r
        // (real part: zr, zi) and 2r + 1 (imaginary part: zi, -zr) for the
        // complex entries K = 8 ks + 4 half + e, e = 0..3
        constexpr int RCOLS = NT * 16;
        for (int f = tid; f < nfill * nks * 2 * RCOLS; f += MP_THREADS) {
            const int r = f % RCOLS;
            const int rest = f / RCOLS;
            const int hh = rest & 1, ks = rest >> 1;
            uint32_t w0[4], w1[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                uint32_t z0 = 0, z1 = 0;
                if (r < RUNS * a.B) {
                    const int t = SP ? r / a.B : 0;
                    const int code = raw[t * run_bytes + (8 * ks + 4 * hh + e) * a.B + (r - t * a.B)] & 3;
                    const int zr = code == 0 ? 1 : (code == 2 ? -1 : 0);
                    const int zi = code == 1 ? 1 : (code == 3 ? -1 : 0);
                    z0 = bf16_unit(zr) | (bf16_unit(zi) << 16);
                    z1 = bf16_unit(zi) | (bf16_unit(-zr) << 16);
                }
                w0[e] = z0;
                w1[e] = z1;
            }
            const int col = 2 * r;
            const int nt = col >> 5, l = (col & 31) + 32 * hh;
            bfr[(ks * NT + nt) * 64 + l] = make_uint4(w0[0], w0[1], w0[2], w0[3]);
            bfr[(ks * NT + nt) * 64 + l + 1] = make_uint4(w1[0], w1[1], w1[2], w1[3]);
        }
        __syncthreads();
        for (int cc = 0; cc < nfill; cc++) {
            const int64_t step0 = (K0 >> 3) + (int64_t)cc * nks;
            for (int kb = 0; kb < nks; kb += 8) {   // the chunk in blocks of 8 K-steps
                uint4 av[RT][8];
#pragma unroll
                for (int rt = 0; rt < RT; rt++) {
                    const int t = tile0 + rt < a.ntiles ? tile0 + rt : a.ntiles - 1;
#pragma unroll
                    for (int u = 0; u < 8; u++)
                        if (kb + u < nks) av[rt][u] = a.W[((int64_t)t * a.nsteps + step0 + kb + u) * 64 + lane];
                }
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    if (kb + u >= nks) break;
                    bf16x8_t bf[NT];
#pragma unroll
                    for (int nt = 0; nt < NT; nt++)
                        bf[nt] = __builtin_bit_cast(bf16x8_t, bfr[((cc * nks + kb + u) * NT + nt) * 64 + lane]);
#pragma unroll
                    for (int rt = 0; rt < RT; rt++) {
                        bf16x8_t af = __builtin_bit_cast(bf16x8_t, av[rt][u]);
#pragma unroll
                        for (int nt = 0; nt < NT; nt++)
                            acc[rt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bf[nt], acc[rt][nt], 0, 0, 0);
                    }
                }
            }
            // flush the chunk sums into FP64
#pragma unroll
            for (int rt = 0; rt < RT; rt++)
#pragma unroll
                for (int nt = 0; nt < NT; nt++)
#pragma unroll
                    for (int q = 0; q < 16; q++) {
                        facc[rt][nt][q] += (double)acc[rt][nt][q];
                        acc[rt][nt][q] = 0.f;
                    }
        }
    }
    // this workgroup's partial sums; C layout: row = 8 (q/4) + 4 (lane/32) + q%4, col = lane % 32
    const int ncol = NT * 32;
    double* out = a.partial + (int64_t)blockIdx.x * a.kp * ncol;
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
        const int t = tile0 + rt;
        if (t >= a.ntiles) continue;
#pragma unroll
        for (int nt = 0; nt < NT; nt++)
#pragma unroll
            for (int q = 0; q < 16; q++) {
                int row = t * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                int col = nt * 32 + (lane & 31);
                out[(int64_t)row * ncol + col] = facc[rt][nt][q];
            }
    }
}

// c1[i][r] = sum over workgroups; c2 adds the lower-spin groups with a minus sign
__global__ void proj_mfma_sum_kernel(const double* partial, int nwg, int wg_per_group, int kp, int ncol, int k, int B,
                                     Cx<double>* c1, Cx<double>* c2) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= k * B) return;
    int i = idx / B, r = idx - i * B;
    double a1r = 0, a1i = 0, a2r = 0, a2i = 0;
    for (int w = 0; w < nwg; w++) {
        int g = w / wg_per_group;
        double s = (g & 1) ? -1.0 : 1.0;
        const double* p = partial + ((int64_t)w * kp + i) * ncol + 2 * r;
        a1r += p[0];
        a1i += p[1];
        a2r += s * p[0];
        a2i += s * p[1];
    }
    c1[idx] = cmake(a1r, a1i);
    c2[idx] = cmake(a2r, a2i);
}

// launch shape of the MFMA projection for nrhs probes: the K chunk, the
// column tiles of 32 (NT) and row tiles per wave (RT), the row groups of
// workgroups and the workgroups per K group; the partials it writes
struct MfmaShape {
    int kc, chunks_per_group, NT, RT, rowgroups, wpg, nwg;
    size_t partial_bytes;
};
// (sp: the spin-pair form, 8 groups of 3 Vh entries, four code slots per probe)
static MfmaShape mfma_shape(const dht_ctx* c, int nrhs, bool sp = false) {
    const WLayout wl = wlayout(c);
    MfmaShape sh;
    const int ngroups = sp ? 8 : 4;
    const int64_t group_len = (sp ? 3 : 6) * c->g.Vh;
    sh.kc = 8;
    for (int kc = 64; kc >= 8; kc >>= 1)
        if (group_len % kc == 0) { sh.kc = kc; break; }
    sh.chunks_per_group = (int)(group_len / sh.kc);
    sh.NT = (2 * (sp ? 4 * nrhs : nrhs) + 31) / 32;
    if (sh.NT == 3) sh.NT = 4;
    sh.RT = sh.NT == 1 ? 2 : 1;
    const int rows_per_wg = MP_WAVES * sh.RT * 32;
    sh.rowgroups = (wl.kp + rows_per_wg - 1) / rows_per_wg;
    const int target = c->proj_wgs > 0 ? c->proj_wgs : 512;   // split of the basis entries (tuned)
    sh.wpg = (int)std::min<int64_t>(sh.chunks_per_group, std::max(1, target / (ngroups * sh.rowgroups)));
    sh.nwg = ngroups * sh.wpg;
    sh.partial_bytes = (size_t)sh.nwg * wl.kp * sh.NT * 32 * sizeof(double);
    return sh;
}

void ws_plan_project_codes(const dht_ctx* c, int nrhs, size_t* plan) {
    if (c->k > 0 && c->wprec == DHT_BF16) plan_max(plan, WS_PROJ, mfma_shape(c, nrhs).partial_bytes);
}

int project_codes(dht_ctx* c, const uint8_t* zc, int nrhs, Cx<double>* c1, Cx<double>* c2) {
    if (!c->W || c->k <= 0) return set_error(DHT_ERR_STATE, "no deflation basis");
    if (c->wprec != DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "MFMA projection needs a BF16 basis");
    if (nrhs <= 0 || nrhs > 64) return set_error(DHT_ERR_INVALID_ARG, "1..64 right-hand sides per projection");
    const WLayout wl = wlayout(c);
    const MfmaShape sh = mfma_shape(c, nrhs);
    MfmaProjArgs a;
    a.W = (const uint4*)c->W;
    a.zc = zc;
    a.nsteps = wl.nsteps;
    a.group_len = 6 * c->g.Vh;
    a.kc = sh.kc;
    a.chunks_per_group = sh.chunks_per_group;
    a.B = nrhs;
    a.kp = wl.kp;
    a.ntiles = wl.kp / 32;
    const int NT = sh.NT, rowgroups = sh.rowgroups, wpg = sh.wpg, nwg = sh.nwg;
    a.wg_per_group = wpg;
    void* part;
    DHT_TRY(ws_get(c, WS_PROJ, sh.partial_bytes, &part));
    a.partial = (double*)part;
    DHT_TRY(zero(c, part, (size_t)nwg * wl.kp * NT * 32 * sizeof(double)));
    dim3 grid(nwg, rowgroups), block(MP_THREADS);
    if (a.group_len % 8 != 0 || a.kc > MP_KC_MAX) return set_error(DHT_ERR_INVALID_ARG, "lattice volume not a multiple of 8");
    // B fragments of one fill, then its raw codes
    size_t lds = (size_t)MP_FILL * (a.kc / 8) * NT * 64 * sizeof(uint4) + (size_t)MP_FILL * a.kc * nrhs;
    int tok;
    DHT_TRY(prof_begin(c, &tok));
    if (NT == 1) hipLaunchKernelGGL((proj_mfma_kernel<2, 1, false>), grid, block, lds, c->stream, a);
    else if (NT == 2) hipLaunchKernelGGL((proj_mfma_kernel<1, 2, false>), grid, block, lds, c->stream, a);
    else hipLaunchKernelGGL((proj_mfma_kernel<1, 4, false>), grid, block, lds, c->stream, a);
    DHT_HIP(hipGetLastError());
    // algorithmic bytes: the stored basis once, the probe codes once per row group, the partials
    DHT_TRY(prof_end(c, tok, PROF_PROJ_MFMA,
                     (double)wl.kp * wl.Kn * 4.0 + (double)rowgroups * wl.Kn * nrhs +
                         (double)nwg * wl.kp * NT * 32 * 8.0));
    hipLaunchKernelGGL(proj_mfma_sum_kernel, dim3((c->k * nrhs + 127) / 128), dim3(128), 0, c->stream,
                       (const double*)part, nwg, wpg, wl.kp, NT * 32, c->k, nrhs, c1, c2);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// ---------------------------------------------------------------------------
// spin-pair projections (traces with a spin matrix Gamma, end of Section 5.2)
//
// P_st[i][r] = sum over parity, colour and site of conj(W_i(s, c, x)) z_r(t, c, x)
// for the 16 spin pairs (s, t), stored [4 s + t][k][B].  For any 4 x 4 spin
// matrix Gamma, W^H Gamma^H z = sum_st conj(Gamma_ts) P_st, and W^H g5 z =
// sum_s g5_s P_ss: one pass serves every Gamma.
// ---------------------------------------------------------------------------
__global__ void proj_mfma_sp_sum_kernel(const double* partial, int wpg, int kp, int ncol, int k, int B,
                                        Cx<double>* P) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)16 * k * B) return;
    const int st = (int)(idx / ((int64_t)k * B));
    const int rem = (int)(idx - (int64_t)st * k * B);
    const int i = rem / B, r = rem - i * B;
    const int s = st >> 2, t = st & 3;
    double re = 0, im = 0;
    for (int par = 0; par < 2; par++)
        for (int w = 0; w < wpg; w++) {
            const int wg = (par * 4 + s) * wpg + w;
            const double* p = partial + ((int64_t)wg * kp + i) * ncol + 2 * (t * B + r);
            re += p[0];
            im += p[1];
        }
    P[idx] = cmake(re, im);
}

int project_codes_sp(dht_ctx* c, const uint8_t* zc, int nrhs, Cx<double>* P) {
    if (!c->W || c->k <= 0) return set_error(DHT_ERR_STATE, "no deflation basis");
    if (c->wprec != DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "MFMA projection needs a BF16 basis");
    if (nrhs <= 0 || nrhs > 16) return set_error(DHT_ERR_INVALID_ARG, "1..16 right-hand sides per spin-pair projection");
    const WLayout wl = wlayout(c);
    const MfmaShape sh = mfma_shape(c, nrhs, true);
    MfmaProjArgs a;
    a.W = (const uint4*)c->W;
    a.zc = zc;
    a.nsteps = wl.nsteps;
    a.group_len = 3 * c->g.Vh;
    a.kc = sh.kc;
    a.chunks_per_group = sh.chunks_per_group;
    a.B = nrhs;
    a.kp = wl.kp;
    a.ntiles = wl.kp / 32;
    a.wg_per_group = sh.wpg;
    if (a.group_len % 8 != 0 || a.kc > MP_KC_MAX)
        return set_error(DHT_ERR_INVALID_ARG, "lattice half volume not a multiple of 8");
    void* part;
    DHT_TRY(ws_get(c, WS_PROJ, sh.partial_bytes, &part));
    a.partial = (double*)part;
    DHT_TRY(zero(c, part, sh.partial_bytes));
    dim3 grid(sh.nwg, sh.rowgroups), block(MP_THREADS);
    const size_t lds = (size_t)MP_FILL * (a.kc / 8) * sh.NT * 64 * sizeof(uint4) + (size_t)MP_FILL * a.kc * 4 * nrhs;
    int tok;
    DHT_TRY(prof_begin(c, &tok));
    if (sh.NT == 1) hipLaunchKernelGGL((proj_mfma_kernel<2, 1, true>), grid, block, lds, c->stream, a);
    else if (sh.NT == 2) hipLaunchKernelGGL((proj_mfma_kernel<1, 2, true>), grid, block, lds, c->stream, a);
    else hipLaunchKernelGGL((proj_mfma_kernel<1, 4, true>), grid, block, lds, c->stream, a);
    DHT_HIP(hipGetLastError());
    // algorithmic bytes: the basis once, four code runs per row group, the partials
    DHT_TRY(prof_end(c, tok, PROF_PROJ_SP,
                     (double)wl.kp * wl.Kn * 4.0 + (double)sh.rowgroups * wl.Kn * nrhs +
                         (double)sh.partial_bytes));
    hipLaunchKernelGGL(proj_mfma_sp_sum_kernel, dim3((unsigned)((16 * (int64_t)c->k * nrhs + 127) / 128)), dim3(128),
                       0, c->stream, (const double*)part, sh.wpg, wl.kp, sh.NT * 32, c->k, nrhs, P);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// generic form: any storage precision of W, FP64 probe fields ([2][12][Vh][B]),
// FP64 accumulation; each workgroup takes one basis row and one run of
// (parity, colour, site) entries for SPG_RT right-hand sides
static constexpr int SPG_THREADS = 256;
static constexpr int SPG_RT = 2;

template <typename SW>
__global__ __launch_bounds__(SPG_THREADS) void proj_sp_generic_kernel(const typename Store<SW>::elem* W, WLayout wl,
                                                                      const Cx<double>* Z, int64_t Vh, int B, int r0,
                                                                      int nr, int64_t chunk, Cx<double>* part, int k) {
    __shared__ Cx<double> red[SPG_THREADS / 64][SPG_RT * 16];
    const int i = blockIdx.y;
    const int64_t nE = 6 * Vh;
    const int64_t ebeg = (int64_t)blockIdx.x * chunk;
    const int64_t eend = ebeg + chunk < nE ? ebeg + chunk : nE;
    Cx<double> acc[SPG_RT][16];
#pragma unroll
    for (int q = 0; q < SPG_RT; q++)
#pragma unroll
        for (int st = 0; st < 16; st++) acc[q][st] = cmake(0.0, 0.0);
    for (int64_t E = ebeg + threadIdx.x; E < eend; E += SPG_THREADS) {
        // entry E = (parity, colour, site): spin s sits at K = 12 Vh parity + 3 Vh s + (E - 3 Vh parity)
        const int64_t par = E / (3 * Vh);
        const int64_t K0 = E + 9 * Vh * par;
        Cx<double> w[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            auto v = Store<SW>::ld(W + w_index(wl, i, K0 + s * 3 * Vh));
            w[s] = cmake<double>(v.re, v.im);
        }
#pragma unroll
        for (int q = 0; q < SPG_RT; q++) {
            if (q >= nr) break;
            Cx<double> z[4];
#pragma unroll
            for (int t = 0; t < 4; t++) z[t] = Z[(K0 + t * 3 * Vh) * B + r0 + q];
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int t = 0; t < 4; t++) acc[q][s * 4 + t] = acc[q][s * 4 + t] + conjmul(w[s], z[t]);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < SPG_RT; q++)
#pragma unroll
        for (int st = 0; st < 16; st++) {
            double re = acc[q][st].re, im = acc[q][st].im;
            for (int off = 32; off > 0; off >>= 1) {
                re += __shfl_xor(re, off);
                im += __shfl_xor(im, off);
            }
            if (lane == 0) red[wave][q * 16 + st] = cmake(re, im);
        }
    __syncthreads();
    if (threadIdx.x < SPG_RT * 16) {
        const int q = threadIdx.x / 16, st = threadIdx.x % 16;
        if (q < nr) {
            Cx<double> sum = cmake(0.0, 0.0);
            for (int wv = 0; wv < SPG_THREADS / 64; wv++) sum = sum + red[wv][threadIdx.x];
            part[(((int64_t)blockIdx.x * 16 + st) * k + i) * B + r0 + q] = sum;
        }
    }
}

__global__ void proj_sp_sum_kernel(const Cx<double>* part, int nchunk, int64_t n, Cx<double>* P) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    Cx<double> s = cmake(0.0, 0.0);
    for (int ch = 0; ch < nchunk; ch++) s = s + part[(int64_t)ch * n + idx];
    P[idx] = s;
}

// split of the (parity, colour, site) entries: at most 64 runs of at least 4096
static int sp_chunks(const dht_ctx* c, int64_t* chunk_out) {
    const int64_t nE = 6 * c->g.Vh;
    int64_t chunk = 4096;
    int n = (int)((nE + chunk - 1) / chunk);
    while (n > 64) {
        chunk *= 2;
        n = (int)((nE + chunk - 1) / chunk);
    }
    if (chunk_out) *chunk_out = chunk;
    return n;
}

int project_field_sp(dht_ctx* c, const void* Z, int nrhs, Cx<double>* P) {
    if (!c->W || c->k <= 0) return set_error(DHT_ERR_STATE, "no deflation basis");
    const WLayout wl = wlayout(c);
    const int k = c->k;
    int64_t chunk;
    const int nchunk = sp_chunks(c, &chunk);
    const int64_t n = (int64_t)16 * k * nrhs;
    void* part;
    DHT_TRY(ws_get(c, WS_GAM_PART, (size_t)nchunk * n * sizeof(Cx<double>), &part));
    int tok;
    DHT_TRY(prof_begin(c, &tok));
    for (int r0 = 0; r0 < nrhs; r0 += SPG_RT) {
        const int nr = std::min(SPG_RT, nrhs - r0);
        dim3 grid(nchunk, k), block(SPG_THREADS);
        switch (c->wprec) {
            case DHT_FP64:
                hipLaunchKernelGGL(proj_sp_generic_kernel<double>, grid, block, 0, c->stream, (const Cx<double>*)c->W,
                                   wl, (const Cx<double>*)Z, c->g.Vh, nrhs, r0, nr, chunk, (Cx<double>*)part, k);
                break;
            case DHT_FP32:
                hipLaunchKernelGGL(proj_sp_generic_kernel<float>, grid, block, 0, c->stream, (const Cx<float>*)c->W,
                                   wl, (const Cx<double>*)Z, c->g.Vh, nrhs, r0, nr, chunk, (Cx<double>*)part, k);
                break;
            case DHT_BF16:
                hipLaunchKernelGGL(proj_sp_generic_kernel<bf16x2>, grid, block, 0, c->stream, (const bf16x2*)c->W,
                                   wl, (const Cx<double>*)Z, c->g.Vh, nrhs, r0, nr, chunk, (Cx<double>*)part, k);
                break;
            default: return set_error(DHT_ERR_INVALID_ARG, "bad basis precision");
        }
        DHT_HIP(hipGetLastError());
    }
    DHT_TRY(prof_end(c, tok, PROF_PROJ_GENERIC,
                     (double)k * wl.Kn * elem_bytes(c->wprec) + (double)wl.Kn * nrhs * 16.0));
    hipLaunchKernelGGL(proj_sp_sum_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, c->stream,
                       (const Cx<double>*)part, nchunk, n, P);
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// X[K][r] -= sum_a W_a(K) v[a][r] (X: FP64 full field [2][12][Vh][bp]; v: device [k][bp])
template <typename SW>
__global__ void basis_subtract_kernel(const typename Store<SW>::elem* W, WLayout wl, const Cx<double>* v, int k,
                                      int bp, Cx<double>* X) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= wl.Kn * bp) return;
    const int64_t K = gid / bp;
    const int r = (int)(gid - K * bp);
    Cx<double> acc = cmake(0.0, 0.0);
    for (int a = 0; a < k; a++) {
        auto w = Store<SW>::ld(W + w_index(wl, a, K));
        acc = acc + cmake<double>(w.re, w.im) * v[(int64_t)a * bp + r];
    }
    X[gid] = X[gid] - acc;
}

int basis_subtract(dht_ctx* c, const Cx<double>* v, int bp, void* X) {
    if (!c->W || c->k <= 0) return set_error(DHT_ERR_STATE, "no deflation basis");
    const WLayout wl = wlayout(c);
    const int64_t tot = wl.Kn * bp;
    dim3 grid((unsigned)((tot + 255) / 256)), block(256);
    switch (c->wprec) {
        case DHT_FP64: hipLaunchKernelGGL(basis_subtract_kernel<double>, grid, block, 0, c->stream, (const Cx<double>*)c->W, wl, v, c->k, bp, (Cx<double>*)X); break;
        case DHT_FP32: hipLaunchKernelGGL(basis_subtract_kernel<float>, grid, block, 0, c->stream, (const Cx<float>*)c->W, wl, v, c->k, bp, (Cx<double>*)X); break;
        case DHT_BF16: hipLaunchKernelGGL(basis_subtract_kernel<bf16x2>, grid, block, 0, c->stream, (const bf16x2*)c->W, wl, v, c->k, bp, (Cx<double>*)X); break;
        default: return set_error(DHT_ERR_INVALID_ARG, "bad basis precision");
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// ---------------------------------------------------------------------------
// basis management
// ---------------------------------------------------------------------------
int deflation_begin(dht_ctx* c, int k, int prec) {
    if (k <= 0) return set_error(DHT_ERR_INVALID_ARG, "k must be positive");
    if (prec < DHT_FP64 || prec > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    if (c->W) {
        DHT_HIP(hipStreamSynchronize(c->stream));
        DHT_HIP(hipFree(c->W));
        c->W = nullptr;
    }
    c->k = 0;
    c->defl_ready = false; c->defl_gen++;
    c->TD[0] = c->TD[1] = 0;
    size_t bytes = w_bytes(c, k, prec);
    if (hipMalloc(&c->W, bytes) != hipSuccess) {
        c->W = nullptr;
        (void)hipGetLastError();
        return set_error(DHT_ERR_OOM, "cannot allocate the deflation basis");
    }
    c->k = k;
    c->wprec = prec;
    DHT_TRY(zero(c, c->W, bytes));
    return DHT_OK;
}

// canonical FP64 columns [count][V][12] -> stored basis rows first..first+count-1
template <typename SW>
__global__ void pack_w_kernel(const Cx<double>* canon, typename Store<SW>::elem* W, WLayout wl, Geom g, int first,
                              int count) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (j, K), K fastest
    if (gid >= (int64_t)count * wl.Kn) return;
    int j = (int)(gid / wl.Kn);
    int64_t K = gid - (int64_t)j * wl.Kn;
    int p = (int)(K / (12 * g.Vh));
    int64_t rem = K - (int64_t)p * 12 * g.Vh;
    int comp = (int)(rem / g.Vh);
    int64_t s = rem - (int64_t)comp * g.Vh;
    int cc[4];
    cb_coords(g, s, p, cc);
    int64_t n = lex_index(g, cc);
    Cx<double> v = canon[((int64_t)j * g.V + n) * 12 + comp];
    typedef typename Store<SW>::acc T;
    Store<SW>::st_rne(W + w_index(wl, first + j, K), cmake<T>((T)v.re, (T)v.im));
}

int deflation_set(dht_ctx* c, int first, int count, const double* W_dev) {
    if (!c->W) return set_error(DHT_ERR_STATE, "call dht_deflation_begin first");
    if (first < 0 || count < 0 || first + count > c->k) return set_error(DHT_ERR_INVALID_ARG, "column range");
    if (count == 0) return DHT_OK;
    const WLayout wl = wlayout(c);
    int64_t n = (int64_t)count * wl.Kn;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (c->wprec) {
        case DHT_FP64: hipLaunchKernelGGL(pack_w_kernel<double>, grid, block, 0, c->stream, (const Cx<double>*)W_dev, (Cx<double>*)c->W, wl, c->g, first, count); break;
        case DHT_FP32: hipLaunchKernelGGL(pack_w_kernel<float>, grid, block, 0, c->stream, (const Cx<double>*)W_dev, (Cx<float>*)c->W, wl, c->g, first, count); break;
        case DHT_BF16: hipLaunchKernelGGL(pack_w_kernel<bf16x2>, grid, block, 0, c->stream, (const Cx<double>*)W_dev, (bf16x2*)c->W, wl, c->g, first, count); break;
    }
    DHT_HIP(hipGetLastError());
    c->defl_ready = false; c->defl_gen++;
    return DHT_OK;
}

// n consecutive basis rows j0.. -> FP64 field [2][12][Vh][bp] (RHS innermost,
// slots n..bp-1 zero)
template <typename SW>
__global__ void gather_kernel(const typename Store<SW>::elem* W, WLayout wl, int j0, int n, int bp, Cx<double>* out) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= wl.Kn * bp) return;
    int64_t K = gid / bp;
    int j = (int)(gid - K * bp);
    if (j >= n) {
        out[gid] = cmake(0.0, 0.0);
        return;
    }
    auto v = Store<SW>::ld(W + w_index(wl, j0 + j, K));
    out[gid] = cmake<double>(v.re, v.im);
}

int gather_columns(dht_ctx* c, int j0, int n, int bp, void* out) {
    const WLayout wl = wlayout(c);
    int64_t tot = wl.Kn * bp;
    dim3 grid((unsigned)((tot + 255) / 256)), block(256);
    switch (c->wprec) {
        case DHT_FP64: hipLaunchKernelGGL(gather_kernel<double>, grid, block, 0, c->stream, (const Cx<double>*)c->W, wl, j0, n, bp, (Cx<double>*)out); break;
        case DHT_FP32: hipLaunchKernelGGL(gather_kernel<float>, grid, block, 0, c->stream, (const Cx<float>*)c->W, wl, j0, n, bp, (Cx<double>*)out); break;
        case DHT_BF16: hipLaunchKernelGGL(gather_kernel<bf16x2>, grid, block, 0, c->stream, (const bf16x2*)c->W, wl, j0, n, bp, (Cx<double>*)out); break;
        default: return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    }
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

// In-place inverse of an n x n complex matrix (row-major) by Gauss-Jordan
// elimination with partial pivoting.  Returns false if singular.
static bool invert(std::vector<std::complex<double>>& A, int n) {
    std::vector<std::complex<double>> I(n * (size_t)n, 0.0);
    for (int i = 0; i < n; i++) I[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; col++) {
        int best = col;
        double bv = std::abs(A[(size_t)col * n + col]);
        for (int r = col + 1; r < n; r++) {
            double v = std::abs(A[(size_t)r * n + col]);
            if (v > bv) { bv = v; best = r; }
        }
        if (bv == 0.0 || !std::isfinite(bv)) return false;
        if (best != col) {
            for (int j = 0; j < n; j++) {
                std::swap(A[(size_t)col * n + j], A[(size_t)best * n + j]);
                std::swap(I[(size_t)col * n + j], I[(size_t)best * n + j]);
            }
        }
        std::complex<double> d = 1.0 / A[(size_t)col * n + col];
        for (int j = 0; j < n; j++) {
            A[(size_t)col * n + j] *= d;
            I[(size_t)col * n + j] *= d;
        }
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            std::complex<double> f = A[(size_t)r * n + col];
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

static int store_M(dht_ctx* c, const std::vector<std::complex<double>>& M, std::complex<double> td, bool diagonal) {
    const int k = c->k;
    c->M.assign((size_t)2 * k * k, 0.0);
    for (size_t i = 0; i < (size_t)k * k; i++) {
        c->M[2 * i] = M[i].real();
        c->M[2 * i + 1] = M[i].imag();
    }
    c->M_diag = diagonal;
    c->TD[0] = td.real();
    c->TD[1] = td.imag();
    c->defl_ready = true; c->defl_gen++;
    return DHT_OK;
}

int deflation_finalize(dht_ctx* c, bool diagonal) {
    if (!c->W) return set_error(DHT_ERR_STATE, "no deflation basis");
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    const int k = c->k;
    const int nb = std::min(k, 32);
    const int nbp = pad_rhs(nb);   // array stride: every block is padded to a power of two
    const size_t fb = full_elems(c, nbp) * 16;
    void *wb, *qwb, *cc;
    DHT_TRY(ws_get(c, WS_QW, fb, &wb));
    DHT_TRY(ws_get(c, WS_XF, fb, &qwb));
    // four [k][nbp] blocks (H columns, their g5 twins, W^H W, W^H g5 W): the
    // stride is the padded block width, which exceeds nb when nb is not a
    // power of two
    const size_t coef_elems = (size_t)4 * k * nbp;
    DHT_TRY(ws_get(c, WS_COEF, sizeof(Cx<double>) * coef_elems, &cc));
    std::vector<std::complex<double>> H, G5;
    std::vector<double> hdiag(k), gdiag(k);
    if (!diagonal) {
        H.assign((size_t)k * k, 0.0);
        G5.assign((size_t)k * k, 0.0);
    }
    std::vector<Cx<double>> hb(coef_elems);
    Cx<double>* h1 = (Cx<double>*)cc;
    const size_t fvec = full_elems(c, 1);   // FP64 vectors per column
    for (int j0 = 0; j0 < k; j0 += nb) {
        const int n = std::min(nb, k - j0);
        const int bp = pad_rhs(n);
        DHT_TRY(gather_columns(c, j0, n, bp, wb));
        DHT_TRY(apply_full(c, DHT_OP_Q, DHT_FP64, wb, qwb, bp));
        if (diagonal) {
            const void* a1[1] = {wb};
            const void* b1[1] = {qwb};
            DHT_TRY(dots(c, DHT_FP64, 1, a1, b1, fvec * bp, bp, h1));        // w^H Q w
            DHT_TRY(g5_field(c, DHT_FP64, wb, qwb, bp));                       // qwb <- g5 w
            DHT_TRY(dots(c, DHT_FP64, 1, a1, b1, fvec * bp, bp, h1 + bp));   // w^H g5 w
            DHT_HIP(hipMemcpyAsync(hb.data(), cc, sizeof(Cx<double>) * 2 * bp, hipMemcpyDeviceToHost, c->stream));
            DHT_HIP(hipStreamSynchronize(c->stream));
            for (int jj = 0; jj < n; jj++) {
                hdiag[j0 + jj] = hb[jj].re;
                gdiag[j0 + jj] = hb[bp + jj].re;
            }
            continue;
        }
        Cx<double>* h2 = h1 + (size_t)k * nbp;
        Cx<double>* g1 = h2 + (size_t)k * nbp;
        Cx<double>* g5m = g1 + (size_t)k * nbp;
        DHT_TRY(project_field(c, qwb, DHT_FP64, bp, h1, h2));
        DHT_TRY(project_field(c, wb, DHT_FP64, bp, g1, g5m));
        DHT_HIP(hipMemcpyAsync(hb.data(), cc, sizeof(Cx<double>) * coef_elems, hipMemcpyDeviceToHost, c->stream));
        DHT_HIP(hipStreamSynchronize(c->stream));
        for (int i = 0; i < k; i++)
            for (int jj = 0; jj < n; jj++) {
                Cx<double> hv = hb[(size_t)i * bp + jj];
                Cx<double> gv = hb[(size_t)3 * k * nbp + (size_t)i * bp + jj];
                H[(size_t)i * k + j0 + jj] = std::complex<double>(hv.re, hv.im);
                G5[(size_t)i * k + j0 + jj] = std::complex<double>(gv.re, gv.im);
            }
    }
    // the Galerkin matrices stay with the context: playback over fewer vectors
    // inverts their leading blocks (Section 6.3)
    c->Hq.assign((size_t)2 * k * k, 0.0);
    c->G5q.assign((size_t)2 * k * k, 0.0);
    for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++) {
            const size_t o = 2 * ((size_t)i * k + j);
            std::complex<double> h = diagonal ? (i == j ? hdiag[i] : 0.0) : H[(size_t)i * k + j];
            std::complex<double> g = diagonal ? (i == j ? gdiag[i] : 0.0) : G5[(size_t)i * k + j];
            if (!diagonal && j >= i) h = 0.5 * (H[(size_t)i * k + j] + std::conj(H[(size_t)j * k + i]));
            if (!diagonal && j < i) h = 0.5 * (std::conj(H[(size_t)j * k + i]) + H[(size_t)i * k + j]);
            c->Hq[o] = h.real();
            c->Hq[o + 1] = h.imag();
            c->G5q[o] = g.real();
            c->G5q[o + 1] = g.imag();
        }
    if (diagonal) {
        std::vector<std::complex<double>> M((size_t)k * k, 0.0);
        std::complex<double> td = 0.0;
        for (int i = 0; i < k; i++) {
            if (hdiag[i] == 0.0 || !std::isfinite(hdiag[i])) return set_error(DHT_ERR_BREAKDOWN, "w^H Q w = 0");
            M[(size_t)i * k + i] = 1.0 / hdiag[i];
            td += gdiag[i] / hdiag[i];
        }
        return store_M(c, M, td, true);
    }
    // H is Hermitian in exact arithmetic: use its Hermitian part
    for (int i = 0; i < k; i++)
        for (int j = i; j < k; j++) {
            std::complex<double> a = 0.5 * (H[(size_t)i * k + j] + std::conj(H[(size_t)j * k + i]));
            H[(size_t)i * k + j] = a;
            H[(size_t)j * k + i] = std::conj(a);
        }
    if (!invert(H, k)) return set_error(DHT_ERR_BREAKDOWN, "W^H Q W is singular");
    std::complex<double> td = 0.0;
    for (int a = 0; a < k; a++)
        for (int b = 0; b < k; b++) td += H[(size_t)a * k + b] * G5[(size_t)b * k + a];
    return store_M(c, H, td, false);
}

// d_j = c1_j^H M c2_j on the host for columns r < nuse (c1, c2 host arrays [k][B] complex)
void deflation_corrections(const dht_ctx* c, const Cx<double>* c1, const Cx<double>* c2, int B, int nuse, double* dre,
                           double* dim) {
    const int k = c->k;
    const std::complex<double>* M = (const std::complex<double>*)c->M.data();
    std::vector<std::complex<double>> v(k);
    for (int r = 0; r < nuse; r++) {
        for (int a = 0; a < k; a++) {
            std::complex<double> s = 0.0;
            if (c->M_diag) {
                s = M[(size_t)a * k + a] * std::complex<double>(c2[(size_t)a * B + r].re, c2[(size_t)a * B + r].im);
            } else {
                for (int b = 0; b < k; b++)
                    s += M[(size_t)a * k + b] * std::complex<double>(c2[(size_t)b * B + r].re, c2[(size_t)b * B + r].im);
            }
            v[a] = s;
        }
        std::complex<double> d = 0.0;
        for (int a = 0; a < k; a++)
            d += std::conj(std::complex<double>(c1[(size_t)a * B + r].re, c1[(size_t)a * B + r].im)) * v[a];
        dre[r] = d.real();
        dim[r] = d.imag();
    }
}

}  // namespace dht
