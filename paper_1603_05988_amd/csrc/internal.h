// Internal declarations of the dhtrace library (gfx950).
//
// Internal field layout ("even/odd, RHS-innermost, 16-byte vectors"): a
// field of B right-hand sides on one parity is complex<T>[12/VW][Vh][B][VW],
// where VW = 16 / sizeof(complex<T>) spin-colour components (c = 3 spin +
// colour) share one 16-byte vector: 1 in FP64, 2 in FP32, 4 in BF16.  A lane
// owns one (site s, RHS r) pair and reads each group of VW components with a
// single 16-byte load; the lanes of a wavefront read one contiguous run.  B is
// always a power of two (callers' batches are padded with zero right-hand
// sides), so the RHS of vector v is v & (B - 1).  A full-lattice field is two
// parity fields back to back (parity 0 = even first).  Checkerboard index of
// site (x, y, z, t): s = lexicographic(x, y, z, t) / 2 (Lx even), parity =
// (x+y+z+t) & 1.
//
// Links: for each (direction mu, parity, site) one 3x3 complex matrix
// (row-major) in ceil(9 / VW) consecutive 16-byte vectors, stored in FP64,
// FP32 and BF16: [4][2][Vh][nvec].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dhtrace.h"

namespace dht {

// ---------------------------------------------------------------------------
// scalars
// ---------------------------------------------------------------------------
struct bf16x2 {   // one complex number in BF16: low half = re, high half = im
    uint32_t bits;
};

template <typename T> struct Cx { T re, im; };

template <typename T> __host__ __device__ inline Cx<T> cmake(T r, T i) { Cx<T> c; c.re = r; c.im = i; return c; }
template <typename T> __host__ __device__ inline Cx<T> operator+(Cx<T> a, Cx<T> b) { return cmake(a.re + b.re, a.im + b.im); }
template <typename T> __host__ __device__ inline Cx<T> operator-(Cx<T> a, Cx<T> b) { return cmake(a.re - b.re, a.im - b.im); }
template <typename T> __host__ __device__ inline Cx<T> operator*(Cx<T> a, Cx<T> b) {
    return cmake(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> __host__ __device__ inline Cx<T> operator*(T s, Cx<T> a) { return cmake(s * a.re, s * a.im); }
template <typename T> __host__ __device__ inline Cx<T> conjmul(Cx<T> a, Cx<T> b) {  // conj(a) * b
    return cmake(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename T> __host__ __device__ inline Cx<T> timesI(Cx<T> a) { return cmake(-a.im, a.re); }
template <typename T> __host__ __device__ inline Cx<T> timesMinusI(Cx<T> a) { return cmake(a.im, -a.re); }
template <typename T> __host__ __device__ inline Cx<T> neg(Cx<T> a) { return cmake(-a.re, -a.im); }

// FP32 -> BF16 with round-to-nearest-even; NaN stays NaN (quiet bit set).
__host__ __device__ inline uint32_t f32_to_bf16_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
// Hardware conversion of two values in one instruction (v_cvt_pk_bf16_f32 on
// gfx950): round to nearest, but exact ties do not go to even, so it is used
// only for values the kernels compute, not where RNE is part of the contract.
typedef __bf16 bf16x2_vec_t __attribute__((ext_vector_type(2)));
__device__ inline uint32_t f32x2_to_bf16x2_bits(float lo, float hi) {
    bf16x2_vec_t b = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, b);
}
__host__ __device__ inline float bf16_bits_to_f32(uint32_t h) {
    uint32_t u = h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// Storage traits: how a complex<T> element is loaded/stored, what it
// accumulates in, and how VW of them pack into one 16-byte vector.
// 16-byte vector types for streaming (non-temporal) accesses: data touched once
// is marked so that it does not displace reused lines in L2.
typedef double f64x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

template <typename S> struct Store;
template <> struct Store<double> {
    typedef double acc;
    typedef Cx<double> elem;
    static constexpr int VW = 1;
    __device__ static inline Cx<double> round(Cx<double> v) { return v; }
    __device__ static inline Cx<double> ld(const elem* p) { return *p; }
    __device__ static inline void st(elem* p, Cx<double> v) { *p = v; }
    __device__ static inline void ldv(const void* base, int64_t v, Cx<double>* o) {
        double2 d = ((const double2*)base)[v];
        o[0] = cmake(d.x, d.y);
    }
    __device__ static inline void stv(void* base, int64_t v, const Cx<double>* i) {
        ((double2*)base)[v] = make_double2(i[0].re, i[0].im);
    }
    __device__ static inline void stv_rne(void* base, int64_t v, const Cx<double>* i) { stv(base, v, i); }
    __device__ static inline void st_rne(elem* p, Cx<double> v) { *p = v; }
    __device__ static inline void ldv_nt(const void* base, int64_t v, Cx<double>* o) {
        f64x2_t d = __builtin_nontemporal_load((const f64x2_t*)base + v);
        o[0] = cmake(d.x, d.y);
    }
    __device__ static inline void stv_nt(void* base, int64_t v, const Cx<double>* i) {
        f64x2_t d = {i[0].re, i[0].im};
        __builtin_nontemporal_store(d, (f64x2_t*)base + v);
    }
};
template <> struct Store<float> {
    typedef float acc;
    typedef Cx<float> elem;
    static constexpr int VW = 2;
    __device__ static inline Cx<float> round(Cx<float> v) { return v; }
    __device__ static inline Cx<float> ld(const elem* p) { return *p; }
    __device__ static inline void st(elem* p, Cx<float> v) { *p = v; }
    __device__ static inline void ldv(const void* base, int64_t v, Cx<float>* o) {
        float4 d = ((const float4*)base)[v];
        o[0] = cmake(d.x, d.y);
        o[1] = cmake(d.z, d.w);
    }
    __device__ static inline void stv(void* base, int64_t v, const Cx<float>* i) {
        ((float4*)base)[v] = make_float4(i[0].re, i[0].im, i[1].re, i[1].im);
    }
    __device__ static inline void stv_rne(void* base, int64_t v, const Cx<float>* i) { stv(base, v, i); }
    __device__ static inline void st_rne(elem* p, Cx<float> v) { *p = v; }
    __device__ static inline void ldv_nt(const void* base, int64_t v, Cx<float>* o) {
        f32x4_t d = __builtin_nontemporal_load((const f32x4_t*)base + v);
        o[0] = cmake(d.x, d.y);
        o[1] = cmake(d.z, d.w);
    }
    __device__ static inline void stv_nt(void* base, int64_t v, const Cx<float>* i) {
        f32x4_t d = {i[0].re, i[0].im, i[1].re, i[1].im};
        __builtin_nontemporal_store(d, (f32x4_t*)base + v);
    }
};
template <> struct Store<bf16x2> {
    typedef float acc;
    typedef bf16x2 elem;
    static constexpr int VW = 4;
    __device__ static inline Cx<float> unpack(uint32_t b) {
        return cmake(bf16_bits_to_f32(b & 0xffffu), bf16_bits_to_f32(b >> 16));
    }
    // values the kernels compute: the hardware conversion (round to nearest;
    // its tie rule is not ties-to-even)
    __device__ static inline uint32_t pack(Cx<float> v) {
        return f32x2_to_bf16x2_bits(v.re, v.im);
    }
    // stored inputs (links, basis, packed spinors): IEEE round-to-nearest-even
    __device__ static inline uint32_t pack_rne(Cx<float> v) {
        return f32_to_bf16_bits(v.re) | (f32_to_bf16_bits(v.im) << 16);
    }
    __device__ static inline void st_rne(elem* p, Cx<float> v) { p->bits = pack_rne(v); }
    __device__ static inline void stv_rne(void* base, int64_t v, const Cx<float>* i) {
        ((uint4*)base)[v] = make_uint4(pack_rne(i[0]), pack_rne(i[1]), pack_rne(i[2]), pack_rne(i[3]));
    }
    __device__ static inline Cx<float> round(Cx<float> v) { return unpack(pack(v)); }
    __device__ static inline Cx<float> ld(const elem* p) { return unpack(p->bits); }
    __device__ static inline void st(elem* p, Cx<float> v) { p->bits = pack(v); }
    __device__ static inline void ldv(const void* base, int64_t v, Cx<float>* o) {
        uint4 d = ((const uint4*)base)[v];
        o[0] = unpack(d.x);
        o[1] = unpack(d.y);
        o[2] = unpack(d.z);
        o[3] = unpack(d.w);
    }
    __device__ static inline void stv(void* base, int64_t v, const Cx<float>* i) {
        ((uint4*)base)[v] = make_uint4(pack(i[0]), pack(i[1]), pack(i[2]), pack(i[3]));
    }
    __device__ static inline void ldv_nt(const void* base, int64_t v, Cx<float>* o) {
        u32x4_t d = __builtin_nontemporal_load((const u32x4_t*)base + v);
        o[0] = unpack(d.x);
        o[1] = unpack(d.y);
        o[2] = unpack(d.z);
        o[3] = unpack(d.w);
    }
    __device__ static inline void stv_nt(void* base, int64_t v, const Cx<float>* i) {
        u32x4_t d = {pack(i[0]), pack(i[1]), pack(i[2]), pack(i[3])};
        __builtin_nontemporal_store(d, (u32x4_t*)base + v);
    }
};

inline size_t elem_bytes(int prec) { return prec == DHT_FP64 ? 16 : (prec == DHT_FP32 ? 8 : 4); }
inline int vec_width(int prec) { return prec == DHT_FP64 ? 1 : (prec == DHT_FP32 ? 2 : 4); }
// 16-byte vectors holding one link matrix (9 complex, padded)
inline int link_vecs(int prec) { return (9 + vec_width(prec) - 1) / vec_width(prec); }

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct Geom {
    int L[4];
    int Lxh;          // Lx / 2
    int64_t V, Vh;
    int antiperiodic;
};

// Coordinates of checkerboard site s of parity p.
__device__ __host__ inline void cb_coords(const Geom& g, int64_t s, int p, int c[4]) {
    int64_t r = s / g.Lxh;
    int xh = (int)(s - r * g.Lxh);
    c[1] = (int)(r % g.L[1]);
    r /= g.L[1];
    c[2] = (int)(r % g.L[2]);
    c[3] = (int)(r / g.L[2]);
    c[0] = 2 * xh + ((p + c[1] + c[2] + c[3]) & 1);
}
__device__ __host__ inline int64_t lex_index(const Geom& g, const int c[4]) {
    return (int64_t)c[0] + (int64_t)g.L[0] * ((int64_t)c[1] + (int64_t)g.L[1] * ((int64_t)c[2] + (int64_t)g.L[2] * c[3]));
}

// hierarchical-probing colour bits of a site for the levels that probe index j
// reaches (bit 4l = parity of sum_mu floor(x_mu / 2^l), bits 4l+1..4l+3 =
// floor(x_mu / 2^l) mod 2 for mu = x, y, z); the sign of probe j is
// (-1)^popcount(colour & j) (Section 5.2)
__device__ __host__ inline uint64_t hp_colour_bits(const int c[4], uint64_t j) {
    uint64_t col = 0;
    for (int l = 0; l < 16 && (j >> (4 * l)) != 0; l++) {
        int q0 = c[0] >> l, q1 = c[1] >> l, q2 = c[2] >> l, q3 = c[3] >> l;
        uint64_t bits = (uint64_t)((q0 + q1 + q2 + q3) & 1) | ((uint64_t)(q0 & 1) << 1) |
                        ((uint64_t)(q1 & 1) << 2) | ((uint64_t)(q2 & 1) << 3);
        col |= bits << (4 * l);
    }
    return col;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

// kernel classes for the instrumentation (dht_profile_get)
enum { PROF_HOP64 = 0, PROF_HOP32, PROF_HOP16, PROF_PROJ_MFMA, PROF_PROJ_GENERIC, PROF_CONV, PROF_PROJ_SP, PROF_NCLASS };
struct ProfPending {
    int cls;
    int ev0, ev1;       // indices into the event pool
    double bytes;       // algorithmic bytes of the launch
};
struct ProfStat {
    int64_t count = 0;
    double ms = 0.0;
    double bytes = 0.0;
};

// learned preconditioner weights (device)
// hopping-kernel launch shape (dht_hop_config); form < 0: unset
inline bool hop_form_tmarch(int form) {
    return form == DHT_HOP_TMARCH || form == DHT_HOP_TMARCH_ROWL || form == DHT_HOP_TSKEW || form == DHT_HOP_TSKEW_ROWL;
}
struct HopConfig {
    int form = -1;
    int nt = 1;
    int tc = 0;
    int rg = 0;   // RHS per sweep of the lattice (0: all)
    int zb = 0;   // t-marching: log2 of the z block of the row order
};

struct NNState {
    bool ready = false;
    void* mem = nullptr;
    float* w[3] = {nullptr, nullptr, nullptr};     // FP32 master [81][Cout][Cin]
    float* g[3] = {nullptr, nullptr, nullptr};     // gradients
    float* m[3] = {nullptr, nullptr, nullptr};     // Adam first moments
    float* v[3] = {nullptr, nullptr, nullptr};     // Adam second moments
    uint16_t* wf[3] = {nullptr, nullptr, nullptr}; // BF16 forward copy
    uint16_t* wb[3] = {nullptr, nullptr, nullptr}; // BF16 reflected/transposed copy
    int64_t step = 0;
    float skip = 0.f;                              // M(r) = net(r) + skip r
};

// solver branch counters (dht_solver_counters)
enum { SC_PREDICT = 0, SC_PREDICT_FAILED, SC_INPLACE, SC_REENTRY, SC_NCOUNT };

struct Welford {   // running mean / second moments of complex samples (Chan et al. update)
    int64_t n = 0;
    double mre = 0, mim = 0;   // means
    double m2re = 0, m2im = 0; // sums of squared deviations
    void add(double re, double im) {
        n++;
        double dre = re - mre, dim = im - mim;
        mre += dre / n;
        mim += dim / n;
        m2re += dre * (re - mre);
        m2im += dim * (im - mim);
    }
};

}  // namespace dht

struct dht_ctx {
    dht::Geom g;
    double mass;
    int device;
    hipStream_t stream;
    bool have_gauge = false;
    void* U[3] = {nullptr, nullptr, nullptr};   // links per precision
    // deflation
    int k = 0, wprec = DHT_FP64;
    bool defl_ready = false;
    void* W = nullptr;                 // [k][2][12][Vh] complex<wprec>
    std::vector<double> M;             // k x k complex128 row-major (host)
    bool M_diag = false;               // M is diagonal (Rayleigh-quotient finalize)
    std::vector<double> Hq, G5q;       // W^H Q W and W^H g5 W (k x k complex128; diagonals only when M_diag)
    double TD[2] = {0, 0};
    // per-kernel-class timing with HIP events (off unless enabled)
    bool prof = false;
    std::vector<hipEvent_t> prof_events;           // pool
    std::vector<int> prof_free;                    // pool events not in use
    std::vector<dht::ProfPending> prof_pending;    // launches not yet harvested
    dht::ProfStat prof_stat[dht::PROF_NCLASS];
    // estimator
    dht::Welford est_q, est_qd;
    // traces Tr(Gamma D^-1) (dht_gamma_set): ng spin matrices, complex128
    // [ng][4][4]; the spin-pair traces T_st of the deflated part (complex128
    // [16]) for basis generation gam_gen; running estimates per matrix
    std::vector<double> gam;
    int ng = 0;
    double gamT[32] = {0};
    bool gamT_valid = false;
    uint64_t gam_gen = 0;
    std::vector<dht::Welford> gest_q, gest_qd;
    // defect-correction branch counts since creation (dht_solver_counters)
    int64_t solver_count[dht::SC_NCOUNT] = {0, 0, 0, 0};
    // learned preconditioner
    dht::NNState nn;
    // hopping-kernel shape per (precision, log2 batch); hop_force overrides
    // every entry while the autotuner times a candidate
    dht::HopConfig hop_cfg[3][9][3];   // [precision][log2 batch][epilogue class]
    bool hop_force = false;
    dht::HopConfig hop_forced;
    // workspace slots (grow-only)
    std::vector<dht::Buf> ws;
    // caller-owned workspace (dht_set_workspace): the planned slots at fixed
    // offsets of one caller buffer; plan from dht_workspace_size
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::vector<size_t> plan, plan_off;      // in effect (set with the buffer)
    std::vector<size_t> plan_next;           // from the last dht_workspace_size
    size_t plan_next_total = 0;
    int planned_call = 0;   // > 0 inside a call the plan covers
    // timings of the last call (ms)
    double timings[5] = {0, 0, 0, 0, 0};
    hipEvent_t ev[6];
    bool events = false;
    // second stream (default priority) on which the deflation projection of
    // a batch runs concurrently with its solve; created on first use
    hipStream_t side = nullptr;
    hipEvent_t side_ev[4];
    // projection window (BF16 basis): the coefficients of probes
    // [pw_first, pw_first + pw_count) of pw_spec, computed in one pass over
    // the basis for basis generation pw_gen; defl_gen changes with the basis
    int proj_window = 0;
    int proj_wgs = 0;        // MFMA projection: target workgroup count of a pass (0: 512)
    bool pw_valid = false;
    int64_t pw_first = 0;
    int pw_count = 0, pw_pad = 0;
    dht_probe_spec pw_spec = {0u, 0u, 0};
    uint64_t pw_gen = 0, defl_gen = 0;
};

namespace dht {

// error reporting ------------------------------------------------------------
int set_error(int code, const std::string& msg);
#define DHT_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::dht::set_error(DHT_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define DHT_TRY(call)              \
    do {                           \
        int rc_ = (call);          \
        if (rc_ != DHT_OK) return rc_; \
    } while (0)

// workspace: slot ids --------------------------------------------------------
enum Slot {
    WS_PACK_IN = 0, WS_PACK_OUT, WS_TMP_HALF, WS_B, WS_RE, WS_TMPO,
    WS_K64,                 // 9 FP64 Krylov vectors: r, rhat, p, v, s, t, tmp, inner rhs, inner x
    WS_KLO = WS_K64 + 9,    // 9 low-precision Krylov vectors (same roles)
    WS_PARTIAL = WS_KLO + 9, WS_SCAL, WS_SCAL2, WS_FLAGS, WS_HOSTPIN,
    WS_Z, WS_XF, WS_QW, WS_PROJ, WS_COEF, WS_PROJ2, WS_ZCODE,
    WS_NN_PART, WS_NN_ACT, WS_NN_SCAL, WS_FG_V, WS_FG_Z, WS_FG_W, WS_FG_COEF, WS_FG_R, WS_FG_E, WS_XSTAR,
    WS_TUNE_REF, WS_TUNE_RED, WS_TUNE_A,
    WS_NORMS, WS_FOLD,
    WS_EIG_V, WS_EIG_W, WS_EIG_T, WS_EIG_U, WS_EIG_PART, WS_EIG_SMALL, WS_EIG_RPART, WS_EIG_LAM, WS_EIG_CANON, WS_DEFL_GET,
    WS_PW_CODE, WS_PW_COEF,
    WS_RING_P, WS_RING_S, WS_HIST, WS_HIST_SCALE, WS_E32, WS_W32, WS_T32, WS_S16,
    WS_GAM_PART, WS_GAM_FPART, WS_GAM_OUT, WS_GAM_CODE, WS_WD_PART, WS_WD_OUT,
    WS_NSLOTS
};
int ws_get(dht_ctx* c, int slot, size_t bytes, void** out);
// workspace plan: plan[slot] = max(plan[slot], bytes)
inline void plan_max(size_t* plan, int slot, size_t bytes) {
    if (bytes > plan[slot]) plan[slot] = bytes;
}

// instrumentation: bracket one launch of class `cls` (no-op unless profiling)
int prof_begin(dht_ctx* c, int* token);
int prof_end(dht_ctx* c, int token, int cls, double bytes);
int prof_harvest(dht_ctx* c);   // after a stream synchronisation
// the context's second stream (default priority) and its events, created on first use
int side_stream(dht_ctx* c);

// field helpers -------------------------------------------------------------
// (nrhs is the padded power-of-two batch in every internal call)
inline size_t half_elems(const dht_ctx* c, int nrhs) { return (size_t)12 * c->g.Vh * nrhs; }
inline size_t full_elems(const dht_ctx* c, int nrhs) { return 2 * half_elems(c, nrhs); }
inline int pad_rhs(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// kernels (launchers) -------------------------------------------------------
// pack.hip
int pack_gauge(dht_ctx* c, const double* U_dev);
// canonical [n][V][12] complex128 <-> full internal field with bp >= n RHS slots
// (pack writes zeros into slots n..bp-1; unpack reads slots < n only)
int pack_spinor(dht_ctx* c, const double* canon, void* field, int prec, int n, int bp);
int unpack_spinor(dht_ctx* c, const void* field, int prec, double* canon, int n, int bp);

// dslash.hip: out_p = a * x_p + b * Hop_{p <- 1-p}(in) (+ cz * z_p when z is
// given), optionally g5 on the result and/or dagger hop.  A per-RHS FP64
// reduction can be fused into the epilogue: HOPDOT_A_OUT gives (a, out) =
// sum conj(a) out; HOPDOT_OUT_X gives (out, x) and (out, out); HOPDOT_NORM
// gives (out, out); HOPDOT_NORM_ZX gives (out, out) and (z, x) (a residual
// z - D x with its norm and the quadratic form z^H x of the same operands).
// Partial sums go to partial[block][pair][nrhs]; nblocks receives the count.
enum { HOPDOT_NONE = 0, HOPDOT_A_OUT = 1, HOPDOT_OUT_X = 2, HOPDOT_NORM = 3, HOPDOT_NORM_ZX = 4 };
struct HopDot {
    int kind = HOPDOT_NONE;
    const void* a = nullptr;
    Cx<double>* partial = nullptr;
    int nblocks = 0;
};
// Operands of an FP64 hop that hold values exact in BF16 (probe fields) may
// be passed in the BF16 layout: mix is a set of HOP_IN16 (the stencil input),
// HOP_X16 (the x-pay source), HOP_Z16 (the second axpy source).  HOP_OUT16:
// the result scaled by s16[r] (device, per RHS) is also stored in BF16 at
// out16 (a residual that starts the next BF16 inner solve).  HOP_NOOUT: the
// result itself is not stored (only the fused sums are wanted; out unused).
enum { HOP_IN16 = 1, HOP_X16 = 2, HOP_Z16 = 4, HOP_OUT16 = 8, HOP_NOOUT = 16 };
int hop(dht_ctx* c, int prec, int out_parity, const void* in, void* out, const void* x, double a, double b,
        int nrhs, bool dagger, bool g5out, HopDot* dot = nullptr, const void* z = nullptr, double cz = 0.0,
        int mix = 0, void* out16 = nullptr, const double* s16 = nullptr);
int hop_blocks(const dht_ctx* c, int nrhs);   // workgroups of one hop launch
constexpr int HOP_LANES = 256;   // lanes per hop workgroup
// the shape a hop launch for (prec, nrhs) uses (t chunk resolved), and a check
// that a shape fits the lattice and batch
// epilogue classes: plain (out = b Hop(in)) and fused (x-pay, second operand or a fused dot)
enum { HOP_PLAIN = 0, HOP_FUSED = 1, HOP_FUSED_A = 2, HOP_NCLASS = 3 };
HopConfig hop_config(const dht_ctx* c, int prec, int nrhs, int cls);
HopConfig hop_default_config(const dht_ctx* c, int prec, int nrhs);
int hop_config_check(const dht_ctx* c, int nrhs, const HopConfig& h);
int apply_full(dht_ctx* c, int op, int prec, const void* in, void* out, int nrhs);   // full-lattice D, D^H, g5, Q
int g5_field(dht_ctx* c, int prec, const void* in, void* out, int nrhs);              // full-lattice g5

// probes.hip: probes j = first.. first+nrhs-1 into a full internal field of
// precision prec (may be null), plus optional index/sign outputs.
// Probes j = first .. first+n-1 into the first n of bp RHS slots of a full
// internal field (slots n..bp-1 are zero).  kout [n][N] and sout [n][V] are the
// raw noise indices and Hadamard signs; zcode (may be null) holds per (complex
// entry K of the full field in FP64 order, slot) the 2-bit code k' with
// z = i^k' ([24 Vh][bp] bytes), the input of the MFMA projection.
int probes_gen(dht_ctx* c, const dht_probe_spec* spec, int64_t first, int n, int bp, void* field, int prec,
               uint8_t* kout, int8_t* sout, uint8_t* zcode = nullptr);

}  // namespace dht
