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
    const void* z;       // second axpy source (same parity as out) or null
    const void* U;
    const void* da;      // dot operand a (HOPDOT_A_OUT)
    Cx<double>* partial;
    int Lx, Ly, Lz, Lt, Lxh;
    int Vh;
    int antiperiodic;
    int out_parity;
    int bshift;          // log2(B): the layout's RHS count
    int gshift;          // log2(G): RHS handled per sweep of the lattice (G divides B)
    int bpg;             // workgroups per RHS group; logical workgroup = group * bpg + index
    int tc, nchunk;      // t-marching: slices per chunk (even, divides Lt) and chunks
    int nt;              // non-temporal (streaming) output stores
    double ca, cb, cz;   // out = ca * x + cb * Hop(in) + cz * z
    void* out16;         // HOP_OUT16: s16[r] * out also stored in BF16 (an inner right-hand side)
    const double* s16;
    int zbs;             // t-marching: log2 of the z block of the row order
};

static constexpr int HOP_THREADS = HOP_LANES;

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


// the same with non-temporal loads (operands read once: kept out of the way
// of the stencil input's neighbour reuse in the caches)
template <typename S>
__device__ inline void load_spinor_nt(const void* base, int64_t v0, int64_t vstride, Cx<typename Store<S>::acc>* p) {
    constexpr int VW = Store<S>::VW;
#pragma unroll
    for (int j = 0; j < 12 / VW; j++) Store<S>::ldv_nt(base, v0 + j * vstride, p + j * VW);
}

// 12 components of an operand stored in S, or with B16 (an FP64 hop whose
// operand holds values exact in BF16: probe fields) read from BF16 storage
// and widened exactly; NT selects non-temporal loads
template <typename S, bool B16, bool NT>
__device__ inline void load_operand(const void* base, int64_t v0, int64_t vstride, Cx<typename Store<S>::acc>* p) {
    typedef typename Store<S>::acc T;
    if constexpr (B16 && !std::is_same<S, bf16x2>::value) {
        Cx<float> q[12];
        if (NT) load_spinor_nt<bf16x2>(base, v0, vstride, q);
        else load_spinor<bf16x2>(base, v0, vstride, q);
#pragma unroll
        for (int i = 0; i < 12; i++) p[i] = cmake<T>((T)q[i].re, (T)q[i].im);
    } else {
        if (NT) load_spinor_nt<S>(base, v0, vstride, p);
        else load_spinor<S>(base, v0, vstride, p);
    }
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

// ---------------------------------------------------------------------------
// BF16 storage: the link product on packed values.  A BF16 complex is one
// 32-bit word as stored (re in the low half, im in the high half).  For a link
// entry L and an operand x, Re(L x) and Im(L x) are each Lr a + Li b for a pair
// (a, b) made of +-xr, +-xi; v_dot2_f32_bf16 forms Lr a + Li b + acc in FP32
// straight from the packed link entry and the packed pair, so neither operand
// is unpacked and each pair of products costs one instruction (the products of
// two BF16 values are exact in FP32).  The pairs are signed selections of the
// stored (vr, vi) of v with x = i^K v: one half swap and per-half signs at
// most, fixed at compile time.
//   Re(U x) = Ur xr - Ui xi -> (xr, -xi)      Im(U x) = Ur xi + Ui xr -> (xi, xr)
//   Re(U* x) = Ur xr + Ui xi -> (xr, xi)      Im(U* x) = Ur xi - Ui xr -> (xi, -xr)
// (U* is the entry U_ba of U^H at (a, b), so ADJ reads U transposed.)
// ---------------------------------------------------------------------------
template <bool ADJ, bool IMPART, int K>
struct PairForm {
    // x = i^K v in terms of v: xr = sgn_r * v[sel_r], xi = sgn_i * v[sel_i] (sel 0 = re, 1 = im)
    static constexpr int sel_r = (K & 1) ? 1 : 0;
    static constexpr int sgn_r = (K == 0 || K == 3) ? 1 : -1;
    static constexpr int sel_i = (K & 1) ? 0 : 1;
    static constexpr int sgn_i = (K == 0 || K == 1) ? 1 : -1;
    static constexpr int lo_sel = IMPART ? sel_i : sel_r;
    static constexpr int lo_sgn = IMPART ? sgn_i : sgn_r;
    static constexpr int hi_sgn = IMPART ? (ADJ ? -sgn_r : sgn_r) : (ADJ ? sgn_i : -sgn_i);
    static constexpr bool swap = lo_sel == 1;
    static constexpr uint32_t mask = (lo_sgn < 0 ? 0x8000u : 0u) | (hi_sgn < 0 ? 0x80000000u : 0u);
};
// One chain: sum over b = 0..2 of Lr a + Li b for the pairs (a, b) of the
// upper-spin operand u_b (form UF, K = 0) and of the lower-spin operand w_b
// (form WF), Re or Im per IMPART, in FP32 from the packed BF16 words.  The
// signs of a pair are the instruction's per-half negation modifiers on the
// operand (neg_lo / neg_hi), so a sign flip costs no instruction (the
// compiler folds no negation into the BF16 dot2 itself).  The six products
// are one asm block: the chain starts from the inline constant 0 and keeps
// its partial sum in the block's own output register, passed from one dot2
// to the next as the accumulator (same opcode, accumulator operand: forwarded
// without wait states), and the block ends with s_nop 2, the three wait
// states a dot2 result needs before another vector instruction may read or
// overwrite its register.  The compiler sees neither the dot2s nor that
// rule, so it must not place its own instructions between them: with the
// products as separate statements, a compiler v_dot2c reading an asm dot2
// result one or two cycles later read a stale value.
#define DHT_MOD0 ""
#define DHT_MOD1 " neg_lo:[0,1,0]"
#define DHT_MOD2 " neg_hi:[0,1,0]"
#define DHT_MOD3 " neg_lo:[0,1,0] neg_hi:[0,1,0]"
#define DHT_CHAIN(MU_, MW_)                                                                          \
    asm("v_dot2_f32_bf16 %0, %1, %4, 0" MU_ "\n\t"                                                   \
        "v_dot2_f32_bf16 %0, %1, %7, %0" MW_ "\n\t"                                                  \
        "v_dot2_f32_bf16 %0, %2, %5, %0" MU_ "\n\t"                                                  \
        "v_dot2_f32_bf16 %0, %2, %8, %0" MW_ "\n\t"                                                  \
        "v_dot2_f32_bf16 %0, %3, %6, %0" MU_ "\n\t"                                                  \
        "v_dot2_f32_bf16 %0, %3, %9, %0" MW_ "\n\t"                                                  \
        "s_nop 2"                                                                                    \
        : "=&v"(d)                                                                                   \
        : "v"(l0), "v"(l1), "v"(l2), "v"(u0), "v"(u1), "v"(u2), "v"(w0), "v"(w1), "v"(w2))
#define DHT_CHAIN_W(MU_)                                                                             \
    if constexpr (MW == 0) DHT_CHAIN(MU_, DHT_MOD0);                                                 \
    else if constexpr (MW == 1) DHT_CHAIN(MU_, DHT_MOD1);                                            \
    else if constexpr (MW == 2) DHT_CHAIN(MU_, DHT_MOD2);                                            \
    else DHT_CHAIN(MU_, DHT_MOD3);
template <int MUM, int MW>
__device__ inline float dot2_chain(uint32_t l0, uint32_t l1, uint32_t l2, uint32_t u0, uint32_t u1, uint32_t u2,
                                   uint32_t w0, uint32_t w1, uint32_t w2) {
    float d;
    if constexpr (MUM == 0) {
        DHT_CHAIN_W(DHT_MOD0)
    } else if constexpr (MUM == 1) {
        DHT_CHAIN_W(DHT_MOD1)
    } else if constexpr (MUM == 2) {
        DHT_CHAIN_W(DHT_MOD2)
    } else {
        DHT_CHAIN_W(DHT_MOD3)
    }
    return d;
}
#undef DHT_CHAIN_W
#undef DHT_CHAIN
#undef DHT_MOD0
#undef DHT_MOD1
#undef DHT_MOD2
#undef DHT_MOD3
// the negation modifiers of a pair form: bit 0 neg_lo, bit 1 neg_hi
template <bool ADJ, bool IMPART, int K>
constexpr int pair_mods() {
    return ((PairForm<ADJ, IMPART, K>::mask & 0x8000u) ? 1 : 0) | ((PairForm<ADJ, IMPART, K>::mask & 0x80000000u) ? 2 : 0);
}
__device__ inline uint32_t half_swap(uint32_t v) { return (v >> 16) | (v << 16); }

// The projected half spinor of (1 - SGN g_mu) is h_sp = u_sp + i^K_sp l_(pi_sp)
// for the upper spins sp = 0, 1 (u) and a lower spin pi_sp (l), read off the
// chiral g_mu (the same combination as project<MU, SGN>).
template <int MU, int SGN, int SP> struct HalfSpin {
    static constexpr int kp = SGN > 0 ? 0 : 2;   // i^kp = SGN
    static constexpr int K = MU == 0 ? (1 + kp) & 3
                           : MU == 1 ? (SP == 0 ? kp : (2 + kp) & 3)
                           : MU == 2 ? (SP == 0 ? (1 + kp) & 3 : (3 + kp) & 3)
                                     : (2 + kp) & 3;
    static constexpr int lower = MU == 0 ? (SP == 0 ? 3 : 2) : MU == 1 ? (SP == 0 ? 3 : 2) : (SP == 0 ? 2 : 3);
};

// w = L h_SP for one half-spinor spin (3 colours), h_SP = u_SP + i^K l_lower
template <int MU, int SGN, bool ADJ, int SP>
__device__ inline void link_mult_spin(const uint32_t* p, const uint32_t* u, Cx<float>* w) {
    constexpr int K = HalfSpin<MU, SGN, SP>::K, LO = HalfSpin<MU, SGN, SP>::lower;
    uint32_t us[3], ls[3];
#pragma unroll
    for (int b = 0; b < 3; b++) {
        us[b] = half_swap(p[3 * SP + b]);
        ls[b] = half_swap(p[3 * LO + b]);
    }
    typedef PairForm<ADJ, false, 0> UR;
    typedef PairForm<ADJ, true, 0> UI;
    typedef PairForm<ADJ, false, K> WR;
    typedef PairForm<ADJ, true, K> WI;
#define DHT_U(F, b) (F::swap ? us[b] : p[3 * SP + (b)])
#define DHT_W(F, b) (F::swap ? ls[b] : p[3 * LO + (b)])
#define DHT_L(b) (ADJ ? u[3 * (b) + a] : u[3 * a + (b)])
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const float re = dot2_chain<pair_mods<ADJ, false, 0>(), pair_mods<ADJ, false, K>()>(
            DHT_L(0), DHT_L(1), DHT_L(2), DHT_U(UR, 0), DHT_U(UR, 1), DHT_U(UR, 2), DHT_W(WR, 0), DHT_W(WR, 1),
            DHT_W(WR, 2));
        const float im = dot2_chain<pair_mods<ADJ, true, 0>(), pair_mods<ADJ, true, K>()>(
            DHT_L(0), DHT_L(1), DHT_L(2), DHT_U(UI, 0), DHT_U(UI, 1), DHT_U(UI, 2), DHT_W(WI, 0), DHT_W(WI, 1),
            DHT_W(WI, 2));
        w[a] = cmake(re, im);
    }
#undef DHT_L
#undef DHT_W
#undef DHT_U
}

// w = L h of both half-spinor spins, L = U or U^H (ADJ), h of (1 - SGN g_mu),
// from the packed spinor p[12] (index 3 spin + colour) and packed link u[9]
template <int MU, int SGN, bool ADJ>
__device__ inline void link_mult_bf16(const uint32_t* p, const uint32_t* u, Cx<float>* w) {
    link_mult_spin<MU, SGN, ADJ, 0>(p, u, w);
    link_mult_spin<MU, SGN, ADJ, 1>(p, u, w + 3);
}

// 12 packed components of (site s, rhs r) and the 9 packed entries of a link
__device__ inline void load_packed_spinor(const void* base, int64_t v0, int64_t vstride, uint32_t* p) {
#pragma unroll
    for (int j = 0; j < 3; j++) {
        uint4 d = ((const uint4*)base)[v0 + j * vstride];
        p[4 * j] = d.x;
        p[4 * j + 1] = d.y;
        p[4 * j + 2] = d.z;
        p[4 * j + 3] = d.w;
    }
}
__device__ inline void load_packed_link(const void* base, int64_t v0, uint32_t* u) {
#pragma unroll
    for (int j = 0; j < 3; j++) {
        uint4 d = ((const uint4*)base)[v0 + j];
        u[4 * j] = d.x;
        if (4 * j + 1 < 9) u[4 * j + 1] = d.y;
        if (4 * j + 2 < 9) u[4 * j + 2] = d.z;
        if (4 * j + 3 < 9) u[4 * j + 3] = d.w;
    }
}

// Row-shared links (BF16, sweeps of >= 16 right-hand sides).  The 16 lanes of
// a DPP row hold the 16 right-hand sides of one site and need the same 8 link
// matrices.  Lane q of the row loads half (6 words) of the step's link slot
// q / 2 -- slots 2 mu and 2 mu + 1 are U_mu at the output site (forward) and
// U_mu at its backward link site (other parity) -- and each link's 9 words
// are broadcast from its two owner lanes (DPP row_newbcast) just before its
// product: 3 eight-byte loads per lane and step instead of the 16-byte link
// loads that every lane of the row would otherwise repeat.
struct RowLinks {
    uint32_t w[6];
};
__device__ inline void row_links_load(const void* U, int Vh, int p, int s, int sbx, int sby, int sbz, int sbt,
                                      RowLinks& rl) {
    const int q = threadIdx.x & 15, d = q >> 1, mu = d >> 1;
    const bool bwd = d & 1;
    int site = s;
    if (bwd) site = mu == 0 ? sbx : (mu == 1 ? sby : (mu == 2 ? sbz : sbt));
    const int64_t v = ((int64_t)(mu * 2 + (bwd ? 1 - p : p)) * Vh + site) * 3;   // 3 vectors per BF16 link
    const uint2* ptr = (const uint2*)((const uint4*)U + v) + 3 * (q & 1);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const uint2 d2 = ptr[k];
        rl.w[2 * k] = d2.x;
        rl.w[2 * k + 1] = d2.y;
    }
}
template <int D, int K>
__device__ inline uint32_t row_link_word(const RowLinks& rl) {   // word K of slot D, from its owner lane
    constexpr int lane = 2 * D + (K < 6 ? 0 : 1), slot = K < 6 ? K : K - 6;
    // every lane of the row reads an active lane of its row, so the old value
    // is never used (bound_ctrl set: no move to initialise it)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)rl.w[slot], 0x150 + lane, 0xf, 0xf, true);
}
template <int D>
__device__ inline void row_link_get(const RowLinks& rl, uint32_t* u) {
    u[0] = row_link_word<D, 0>(rl);
    u[1] = row_link_word<D, 1>(rl);
    u[2] = row_link_word<D, 2>(rl);
    u[3] = row_link_word<D, 3>(rl);
    u[4] = row_link_word<D, 4>(rl);
    u[5] = row_link_word<D, 5>(rl);
    u[6] = row_link_word<D, 6>(rl);
    u[7] = row_link_word<D, 7>(rl);
    u[8] = row_link_word<D, 8>(rl);
}

// Ordering fence for the accumulation: the accumulators pass through an
// empty asm (so the arithmetic producing them cannot sink below it) that also
// clobbers memory (so later loads cannot rise above it).  Emits no code.
template <int N, typename T>
__device__ inline void fence_n(Cx<T>* v) {
#pragma unroll
    for (int i = 0; i < N; i++) asm volatile("" : "+v"(v[i].re), "+v"(v[i].im) : : "memory");
}
template <typename T>
__device__ inline void fence_acc(Cx<T>* acc) { fence_n<12>(acc); }

// one direction: forward neighbour sf with its link at (lf, lfv), backward
// neighbour sb with its link at (lb, lbv) (16-byte vector indices; the links
// come from global memory or from the workgroup's LDS copy)
template <typename S, int MU, bool DAG, int MIX, bool ROWL = false>
__device__ inline void hop_dir(const HopArgs& a, int sf, int sb, int r, bool phf, bool phb, const void* lf,
                               int64_t lfv, const void* lb, int64_t lbv, Cx<typename Store<S>::acc>* acc,
                               const RowLinks* rl = nullptr) {
    typedef typename Store<S>::acc T;
    const int64_t vstride = (int64_t)a.Vh << a.bshift;
    constexpr int SF = DAG ? -1 : 1;   // sign of the forward projector (1 - SF g)
    if constexpr (std::is_same<S, bf16x2>::value) {
        {
            uint32_t psi[12], u[12];
            Cx<float> w[6];
            load_packed_spinor(a.in, ((int64_t)sf << a.bshift) + r, vstride, psi);
            if constexpr (ROWL) row_link_get<2 * MU>(*rl, u);
            else load_packed_link(lf, lfv, u);
            link_mult_bf16<MU, SF, false>(psi, u, w);
            reconstruct<MU, SF>(acc, w, phf ? -1.f : 1.f);
        }
        fence_acc(acc);
        {
            uint32_t psi[12], u[12];
            Cx<float> w[6];
            load_packed_spinor(a.in, ((int64_t)sb << a.bshift) + r, vstride, psi);
            if constexpr (ROWL) row_link_get<2 * MU + 1>(*rl, u);
            else load_packed_link(lb, lbv, u);
            link_mult_bf16<MU, -SF, true>(psi, u, w);
            reconstruct<MU, -SF>(acc, w, phb ? -1.f : 1.f);
        }
        fence_acc(acc);
        return;
    }
    {
        Cx<T> psi[12], h[6], u[9], w[6];
        load_operand<S, (MIX & HOP_IN16) != 0, false>(a.in, ((int64_t)sf << a.bshift) + r, vstride, psi);
        project<MU, SF>(psi, h);
        load_link<S>(lf, lfv, u);
        mul_link<false>(u, h, w);
        reconstruct<MU, SF>(acc, w, phf ? T(-1) : T(1));
    }
    // keep loads next to their use: unfenced, the optimiser issues all sixteen
    // neighbour/link loads first and exhausts registers
    fence_acc(acc);
    {
        Cx<T> psi[12], h[6], u[9], w[6];
        load_operand<S, (MIX & HOP_IN16) != 0, false>(a.in, ((int64_t)sb << a.bshift) + r, vstride, psi);
        project<MU, -SF>(psi, h);
        load_link<S>(lb, lbv, u);
        mul_link<true>(u, h, w);
        reconstruct<MU, -SF>(acc, w, phb ? T(-1) : T(1));
    }
    fence_acc(acc);
}

// checkerboard index of the backward neighbour x - mu of site s (parity p)
__device__ inline int bwd_site(const HopArgs& a, int s, int mu) {
    const int xh = s % a.Lxh;
    int rest = s / a.Lxh;
    const int y = rest % a.Ly;
    rest /= a.Ly;
    const int z = rest % a.Lz;
    const int t = rest / a.Lz;
    const int sy = a.Lxh, sz = a.Lxh * a.Ly, st = sz * a.Lz;
    if (mu == 0) {
        const int x = 2 * xh + ((a.out_parity + y + z + t) & 1);
        return s - xh + ((x == 0 ? a.Lx - 1 : x - 1) >> 1);
    }
    if (mu == 1) return y == 0 ? s + (a.Ly - 1) * sy : s - sy;
    if (mu == 2) return z == 0 ? s + (a.Lz - 1) * sz : s - sz;
    return t == 0 ? s + (a.Lt - 1) * st : s - st;
}

// Cooperative copy of the links a workgroup needs into LDS: slot
// ((d * ns + k) * NV + j), d = 2 mu (forward: U_mu at site k) or 2 mu + 1
// (backward: U_mu at the neighbour k - mu, other parity).  site(k) gives the
// checkerboard index of local site k, or -1 for an idle slot.  One coalesced
// pass replaces the per-lane link loads that the B lanes of a site would
// otherwise each issue.
template <typename S, typename SiteFn>
__device__ inline void stage_links(const HopArgs& a, uint4* lds, int ns, SiteFn site) {
    constexpr int NV = (9 + Store<S>::VW - 1) / Store<S>::VW;
    const int total = 8 * ns * NV;
    const int p = a.out_parity;
    for (int k = threadIdx.x; k < total; k += HOP_THREADS) {
        const int d = k / (ns * NV);
        const int rem = k - d * ns * NV;
        const int sl = rem / NV, j = rem - sl * NV;
        const int s = site(sl);
        if (s < 0) continue;
        const int mu = d >> 1;
        const int ls = (d & 1) ? bwd_site(a, s, mu) : s;
        const int par = (d & 1) ? 1 - p : p;
        lds[k] = ((const uint4*)a.U)[((int64_t)(mu * 2 + par) * a.Vh + ls) * NV + j];
    }
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

// t-marching default: halve the chunk while the grid holds fewer lanes than this
static constexpr int64_t HOP_MIN_LANES = 1 << 20;

// components NG c .. NG c + NG - 1 (NG a multiple of 4) of an operand of
// (site, rhs) at vector v0, stored in S or, with B16, held in BF16 (4
// components per vector) and widened exactly; NT: non-temporal loads
template <typename S, int NG, bool B16, bool NT>
__device__ inline void load_operand_group(const void* base, int64_t v0, int64_t vstride, int c,
                                          Cx<typename Store<S>::acc>* p) {
    typedef typename Store<S>::acc T;
    if constexpr (B16 && !std::is_same<S, bf16x2>::value) {
#pragma unroll
        for (int g = 0; g < NG / 4; g++) {
            Cx<float> q[4];
            const int64_t v = v0 + (c * (NG / 4) + g) * vstride;
            if (NT) Store<bf16x2>::ldv_nt(base, v, q);
            else Store<bf16x2>::ldv(base, v, q);
#pragma unroll
            for (int i = 0; i < 4; i++) p[4 * g + i] = cmake<T>((T)q[i].re, (T)q[i].im);
        }
    } else {
        constexpr int VW = Store<S>::VW, NV = NG / VW;
#pragma unroll
        for (int j = 0; j < NV; j++) {
            const int64_t v = v0 + (c * NV + j) * vstride;
            if (NT) Store<S>::ldv_nt(base, v, p + j * VW);
            else Store<S>::ldv(base, v, p + j * VW);
        }
    }
}

// out = cb * acc + ca * x (g5 applied on request), stored; the fused dot
// products use the stored (rounded) values, so they match a separate pass.
// BF16 hops take the 12 components in three groups of 4 (one vector each),
// holding only a group of each operand at a time, which keeps the BF16
// t-marching (a, out) form at 4 waves per SIMD; FP32 / FP64 hops, with one or
// two waves per SIMD, load all 12 at once to overlap the loads.  The sums keep
// the order of a one-component loop.
template <typename S, bool G5OUT, bool XPAY, int DOT, int MIX>
__device__ inline void hop_epilogue(const HopArgs& a, int s, int r, Cx<typename Store<S>::acc>* acc, Cx<double>& d0,
                                    Cx<double>& d1) {
    typedef typename Store<S>::acc T;
    constexpr int VW = Store<S>::VW;
    constexpr int NG = std::is_same<S, bf16x2>::value ? 4 : 12;   // components per group
    const int64_t vstride = (int64_t)a.Vh << a.bshift;
    const int64_t v0 = ((int64_t)s << a.bshift) + r;
    const T cb = (T)a.cb, ca = (T)a.ca;
    fence_acc(acc);   // the epilogue's operand loads stay below the stencil arithmetic
#pragma unroll
    for (int c = 0; c < 12 / NG; c++) {
        Cx<T>* o = acc + NG * c;
        Cx<T> xv[NG], zv[NG];
        if (XPAY) load_operand_group<S, NG, (MIX & HOP_X16) != 0, true>(a.x, v0, vstride, c, xv);
#pragma unroll
        for (int q = 0; q < NG; q++) {
            Cx<T> v = cb * o[q];
            if (XPAY) v = v + ca * xv[q];
            o[q] = v;
        }
        if (XPAY && a.z) {   // out += cz * z (residuals z - D x in one pass)
            const T cz = (T)a.cz;
            load_operand_group<S, NG, (MIX & HOP_Z16) != 0, true>(a.z, v0, vstride, c, zv);
#pragma unroll
            for (int q = 0; q < NG; q++) o[q] = o[q] + cz * zv[q];
        }
#pragma unroll
        for (int q = 0; q < NG; q++)
            if (G5OUT && NG * c + q >= 6) o[q] = neg(o[q]);
        if constexpr ((MIX & HOP_OUT16) != 0) {
            const double sc = a.s16[r];
#pragma unroll
            for (int g = 0; g < NG / 4; g++) {
                Cx<float> o16[4];
#pragma unroll
                for (int q = 0; q < 4; q++)
                    o16[q] = cmake<float>((float)(sc * o[4 * g + q].re), (float)(sc * o[4 * g + q].im));
                Store<bf16x2>::stv(a.out16, v0 + (c * (NG / 4) + g) * vstride, o16);
            }
        }
        if constexpr ((MIX & HOP_NOOUT) == 0) {   // else only the epilogue sums are wanted
#pragma unroll
            for (int j = 0; j < NG / VW; j++) {
                const int64_t v = v0 + (c * (NG / VW) + j) * vstride;
                if (a.nt) Store<S>::stv_nt(a.out, v, o + j * VW);
                else Store<S>::stv(a.out, v, o + j * VW);
            }
        }
        if (DOT != HOPDOT_NONE) {
            Cx<T> ov[NG];
#pragma unroll
            for (int q = 0; q < NG; q++) ov[q] = Store<S>::round(o[q]);
            if (DOT == HOPDOT_A_OUT) {
                Cx<T> av[NG];
                load_operand_group<S, NG, false, true>(a.da, v0, vstride, c, av);
#pragma unroll
                for (int q = 0; q < NG; q++)
                    d0 = d0 + conjmul(cmake<double>(av[q].re, av[q].im), cmake<double>(ov[q].re, ov[q].im));
            } else if (DOT == HOPDOT_NORM) {
#pragma unroll
                for (int q = 0; q < NG; q++) d0.re += (double)ov[q].re * ov[q].re + (double)ov[q].im * ov[q].im;
            } else if (DOT == HOPDOT_NORM_ZX) {
#pragma unroll
                for (int q = 0; q < NG; q++) {
                    d0.re += (double)ov[q].re * ov[q].re + (double)ov[q].im * ov[q].im;
                    d1 = d1 + conjmul(cmake<double>(zv[q].re, zv[q].im), cmake<double>(xv[q].re, xv[q].im));
                }
            } else {
#pragma unroll
                for (int q = 0; q < NG; q++) {
                    Cx<double> oo = cmake<double>(ov[q].re, ov[q].im);
                    d0 = d0 + conjmul(oo, cmake<double>(xv[q].re, xv[q].im));
                    d1.re += oo.re * oo.re + oo.im * oo.im;
                }
            }
        }
    }
}

// workgroup tree over the lanes of equal RHS, partial[blk][q][B]; a workgroup
// of RHS group g (G RHS from g * G) writes zeros for the other RHS
template <int NP>
__device__ inline void hop_block_reduce(const HopArgs& a, int blk, int g, Cx<double> d0, Cx<double> d1) {
    if (NP > 0) {
        const int B = 1 << a.bshift, G = 1 << a.gshift;
        __shared__ Cx<double> red[NP > 0 ? NP : 1][HOP_THREADS];
        red[0][threadIdx.x] = d0;
        if (NP > 1) red[NP - 1][threadIdx.x] = d1;
        __syncthreads();
        for (int w = HOP_THREADS / 2; w >= G; w >>= 1) {
            if ((int)threadIdx.x < w) {
#pragma unroll
                for (int q = 0; q < NP; q++) red[q][threadIdx.x] = red[q][threadIdx.x] + red[q][threadIdx.x + w];
            }
            __syncthreads();
        }
        if ((int)threadIdx.x < B) {
            const int lr = (int)threadIdx.x - g * G;
            const bool mine = lr >= 0 && lr < G;
#pragma unroll
            for (int q = 0; q < NP; q++)
                a.partial[((int64_t)blk * NP + q) * B + threadIdx.x] = mine ? red[q][lr] : cmake(0.0, 0.0);
        }
    }
}

// Site-parallel form: one lane per (site, RHS), RHS fastest.  With LDSL the
// workgroup's ns = 256 / B sites take their links from LDS.
template <typename S, bool DAG, bool G5OUT, bool XPAY, int DOT, bool LDSL, int MIX, bool ROWL = false>
__global__ __launch_bounds__(HOP_THREADS) void hop_kernel(HopArgs a) {
    typedef typename Store<S>::acc T;
    constexpr int NV = (9 + Store<S>::VW - 1) / Store<S>::VW;
    constexpr int NP = (DOT == HOPDOT_A_OUT || DOT == HOPDOT_NORM) ? 1 : ((DOT == HOPDOT_OUT_X || DOT == HOPDOT_NORM_ZX) ? 2 : 0);
    extern __shared__ uint4 hop_lds[];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g = blk / a.bpg;                 // RHS group
    const int bl = blk - g * a.bpg;            // workgroup within the group's sweep
    const int G = 1 << a.gshift;
    const int ns = HOP_THREADS >> a.gshift;
    const int sl = threadIdx.x >> a.gshift;
    const int s = bl * ns + sl;
    const int r = g * G + (threadIdx.x & (G - 1));
    const int p = a.out_parity;
    if (LDSL) {
        const int s0 = bl * ns;
        stage_links<S>(a, hop_lds, ns, [&](int k) { return s0 + k < a.Vh ? s0 + k : -1; });
        __syncthreads();
    }
    Cx<double> d0 = cmake(0.0, 0.0), d1 = cmake(0.0, 0.0);
    if (s < a.Vh) {
        const int xh = s % a.Lxh;
        int rest = s / a.Lxh;
        const int y = rest % a.Ly;
        rest /= a.Ly;
        const int z = rest % a.Lz;
        const int t = rest / a.Lz;
        const int x = 2 * xh + ((p + y + z + t) & 1);
        const int row = s - xh;   // index of (x = 0, y, z, t) / 2
        const int sy = a.Lxh, sz = a.Lxh * a.Ly, st = sz * a.Lz;
        const int xf = x + 1 == a.Lx ? 0 : x + 1, xb = x == 0 ? a.Lx - 1 : x - 1;
        const int sn[8] = {row + (xf >> 1), row + (xb >> 1),
                           y == a.Ly - 1 ? s - (a.Ly - 1) * sy : s + sy, y == 0 ? s + (a.Ly - 1) * sy : s - sy,
                           z == a.Lz - 1 ? s - (a.Lz - 1) * sz : s + sz, z == 0 ? s + (a.Lz - 1) * sz : s - sz,
                           t == a.Lt - 1 ? s - (a.Lt - 1) * st : s + st, t == 0 ? s + (a.Lt - 1) * st : s - st};
        Cx<T> acc[12];
#pragma unroll
        for (int i = 0; i < 12; i++) acc[i] = cmake<T>(0, 0);
        RowLinks rl;
        if constexpr (ROWL) row_links_load(a.U, a.Vh, p, s, sn[1], sn[3], sn[5], sn[7], rl);
#define DHT_DIR(MU, PHF, PHB)                                                                              \
    if (ROWL)                                                                                            \
        hop_dir<S, MU, DAG, MIX, ROWL>(a, sn[2 * MU], sn[2 * MU + 1], r, PHF, PHB, nullptr, 0, nullptr, 0, acc, &rl); \
    else if (LDSL)                                                                                       \
        hop_dir<S, MU, DAG, MIX>(a, sn[2 * MU], sn[2 * MU + 1], r, PHF, PHB, hop_lds,                         \
                            (int64_t)((2 * MU) * ns + sl) * NV, hop_lds, (int64_t)((2 * MU + 1) * ns + sl) * NV, acc); \
    else                                                                                                 \
        hop_dir<S, MU, DAG, MIX>(a, sn[2 * MU], sn[2 * MU + 1], r, PHF, PHB, a.U,                             \
                            ((int64_t)(MU * 2 + p) * a.Vh + s) * NV, a.U,                                \
                            ((int64_t)(MU * 2 + 1 - p) * a.Vh + sn[2 * MU + 1]) * NV, acc);
        DHT_DIR(0, false, false)
        DHT_DIR(1, false, false)
        DHT_DIR(2, false, false)
        DHT_DIR(3, a.antiperiodic && t == a.Lt - 1, a.antiperiodic && t == 0)
#undef DHT_DIR
        hop_epilogue<S, G5OUT, XPAY, DOT, MIX>(a, s, r, acc, d0, d1);
    }
    hop_block_reduce<NP>(a, blk, g, d0, d1);
}

// Column of a t-marching lane from its index j in the chunk: x-rows (16 lanes
// per row at 16 RHS) in blocks of 2^zbs consecutive z, y next, z blocks last,
// so that the workgroups resident on one XCD at a time (dispatched in index
// order) hold both the y and the z neighbours of most rows and the neighbour
// reads meet in its L2 (2^zbs = 1: y fastest, z neighbours Ly rows apart).
__device__ inline void tm_column(const HopArgs& a, int j, int& s3, int& xh, int& y, int& z) {
    xh = j % a.Lxh;
    const int rho = j / a.Lxh;
    const int zl = rho & ((1 << a.zbs) - 1);
    const int rest = rho >> a.zbs;
    y = rest % a.Ly;
    z = ((rest / a.Ly) << a.zbs) | zl;
    s3 = xh + a.Lxh * (y + a.Ly * z);
}

// ---------------------------------------------------------------------------
// t-marching form.  A lane owns one (x, y, z) column of the output parity and
// one RHS and walks t upward through a chunk of tc slices.  The t-forward
// neighbour psi(t+1) read at step t is also the t-backward neighbour of the
// output two slices later (same x), so its other projection times U_t^H is
// kept in registers for step t + 2: every input site is fetched once for the
// t direction, and the x, y, z neighbours of a step all lie in one slice that
// the step before has just brought into the caches.
// ---------------------------------------------------------------------------
// The pending backward t-hops live in LDS, [slot][6][lanes] per workgroup
// (one lane's entries are HOP_THREADS apart: conflict-free), which keeps the
// kernel's registers at the level of the site-parallel form.
template <typename T>
__device__ inline void wb_store(Cx<T>* wbs, const Cx<T>* w) {
#pragma unroll
    for (int i = 0; i < 6; i++) wbs[i * HOP_THREADS + threadIdx.x] = w[i];
}
template <typename T>
__device__ inline void wb_load(const Cx<T>* wbs, Cx<T>* w) {
#pragma unroll
    for (int i = 0; i < 6; i++) w[i] = wbs[i * HOP_THREADS + threadIdx.x];
}

template <typename S, int SGN, int MIX>
__device__ inline void t_back(const HopArgs& a, int sin, int r, int64_t vstride, typename Store<S>::acc ph,
                              Cx<typename Store<S>::acc>* wbs) {
    typedef typename Store<S>::acc T;
    constexpr int NV = (9 + Store<S>::VW - 1) / Store<S>::VW;
    Cx<T> wb[6];
    if constexpr (std::is_same<S, bf16x2>::value) {
        uint32_t psi[12], u[12];
        load_packed_spinor(a.in, ((int64_t)sin << a.bshift) + r, vstride, psi);
        load_packed_link(a.U, ((int64_t)(6 + 1 - a.out_parity) * a.Vh + sin) * NV, u);
        link_mult_bf16<3, SGN, true>(psi, u, wb);
    } else {
        Cx<T> psi[12], h[6], u[9];
        load_operand<S, (MIX & HOP_IN16) != 0, false>(a.in, ((int64_t)sin << a.bshift) + r, vstride, psi);
        project<3, SGN>(psi, h);
        load_link<S>(a.U, ((int64_t)(6 + 1 - a.out_parity) * a.Vh + sin) * NV, u);
        mul_link<true>(u, h, wb);
    }
#pragma unroll
    for (int i = 0; i < 6; i++) wb[i] = ph * wb[i];
    wb_store(wbs, wb);
}

template <typename S, bool DAG, bool G5OUT, bool XPAY, int DOT, int MIX, bool ROWL = false>
__device__ inline void tm_step(const HopArgs& a, int t, int t1, int s3, int xh, int y, int z, int r, int V3, int yf,
                               int yb, int zf, int zb, Cx<typename Store<S>::acc>* wbs, Cx<double>& d0,
                               Cx<double>& d1) {
    typedef typename Store<S>::acc T;
    constexpr int NV = (9 + Store<S>::VW - 1) / Store<S>::VW;
    constexpr int SF = DAG ? -1 : 1;
    const int p = a.out_parity;
    const int64_t vstride = (int64_t)a.Vh << a.bshift;
    int s = t * V3 + s3;
    // opaque to the optimiser: otherwise it keeps one strength-reduced 64-bit
    // pointer per direction and vector live across the t loop
    asm volatile("" : "+v"(s));
    const int x = 2 * xh + ((p + y + z + t) & 1);
    const int row = s - xh;
    const int xf = x + 1 == a.Lx ? 0 : x + 1, xb = x == 0 ? a.Lx - 1 : x - 1;
    Cx<T> acc[12];
#pragma unroll
    for (int i = 0; i < 12; i++) acc[i] = cmake<T>(0, 0);
    const int sx = row + (xb >> 1), sy = s + yb, sz = s + zb;
    const int sn = (t + 1 == a.Lt ? 0 : t + 1) * V3 + s3;
    RowLinks rl;
    if constexpr (ROWL) row_links_load(a.U, a.Vh, p, s, sx, sy, sz, sn, rl);
    hop_dir<S, 0, DAG, MIX, ROWL>(a, row + (xf >> 1), sx, r, false, false, a.U, ((int64_t)p * a.Vh + s) * NV, a.U,
                       ((int64_t)(1 - p) * a.Vh + sx) * NV, acc, &rl);
    hop_dir<S, 1, DAG, MIX, ROWL>(a, s + yf, sy, r, false, false, a.U, ((int64_t)(2 + p) * a.Vh + s) * NV, a.U,
                       ((int64_t)(3 - p) * a.Vh + sy) * NV, acc, &rl);
    hop_dir<S, 2, DAG, MIX, ROWL>(a, s + zf, sz, r, false, false, a.U, ((int64_t)(4 + p) * a.Vh + s) * NV, a.U,
                       ((int64_t)(5 - p) * a.Vh + sz) * NV, acc, &rl);
    {
        Cx<T> wb[6];
        wb_load(wbs, wb);
        reconstruct<3, -SF>(acc, wb, T(1));
    }
    if constexpr (std::is_same<S, bf16x2>::value) {
        uint32_t psi[12], u[12];
        Cx<float> w[6];
        load_packed_spinor(a.in, ((int64_t)sn << a.bshift) + r, vstride, psi);
        if constexpr (ROWL) row_link_get<6>(rl, u);
        else load_packed_link(a.U, ((int64_t)(6 + p) * a.Vh + s) * NV, u);
        link_mult_bf16<3, SF, false>(psi, u, w);
        reconstruct<3, SF>(acc, w, (a.antiperiodic && t == a.Lt - 1) ? -1.f : 1.f);
        if (t + 2 < t1) {   // backward t-hop of step t + 2, from the same input spinor
            fence_acc(acc);
            if constexpr (ROWL) row_link_get<7>(rl, u);
            else load_packed_link(a.U, ((int64_t)(6 + 1 - p) * a.Vh + sn) * NV, u);
            link_mult_bf16<3, -SF, true>(psi, u, w);
            wb_store(wbs, w);
        }
    } else {
        Cx<T> psi[12], h[6], u[9], w[6];
        load_operand<S, (MIX & HOP_IN16) != 0, false>(a.in, ((int64_t)sn << a.bshift) + r, vstride, psi);
        project<3, SF>(psi, h);
        load_link<S>(a.U, ((int64_t)(6 + p) * a.Vh + s) * NV, u);
        mul_link<false>(u, h, w);
        reconstruct<3, SF>(acc, w, (a.antiperiodic && t == a.Lt - 1) ? T(-1) : T(1));
        if (t + 2 < t1) {   // backward t-hop of step t + 2, from the same input spinor
            fence_acc(acc);
            project<3, -SF>(psi, h);
            load_link<S>(a.U, ((int64_t)(6 + 1 - p) * a.Vh + sn) * NV, u);
            mul_link<true>(u, h, w);
            wb_store(wbs, w);
        }
    }
    hop_epilogue<S, G5OUT, XPAY, DOT, MIX>(a, s, r, acc, d0, d1);
    fence_acc(acc);   // the next step's loads stay below this step's arithmetic
}

// BF16 with no fused sums or the single (a, out) sum: held to 128 registers,
// i.e. 4 waves per SIMD (the (a, out) row-link form needs 129 otherwise;
// neither then spills); the two-sum forms would spill and keep 2-3 waves
template <typename S, int DOT>
constexpr int tm_min_waves() {
    return (std::is_same<S, bf16x2>::value && (DOT == HOPDOT_NONE || DOT == HOPDOT_A_OUT)) ? 4 : 1;
}

template <typename S, bool DAG, bool G5OUT, bool XPAY, int DOT, int MIX, bool ROWL = false>
__global__ __launch_bounds__(HOP_THREADS) __attribute__((amdgpu_waves_per_eu(tm_min_waves<S, DOT>(), 8)))
void hop_tm_kernel(HopArgs a) {
    typedef typename Store<S>::acc T;
    extern __shared__ uint4 hop_lds[];   // [2][6][HOP_THREADS] Cx<T>
    constexpr int NP = (DOT == HOPDOT_A_OUT || DOT == HOPDOT_NORM) ? 1 : ((DOT == HOPDOT_OUT_X || DOT == HOPDOT_NORM_ZX) ? 2 : 0);
    constexpr int SF = DAG ? -1 : 1;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g = blk / a.bpg;                 // RHS group
    const int gid = (blk - g * a.bpg) * HOP_THREADS + threadIdx.x;
    const int G = 1 << a.gshift;
    const int col = gid >> a.gshift;   // chunk * V3 + column
    const int r = g * G + (gid & (G - 1));
    const int V3 = a.Vh / a.Lt;
    const int chunk = col / V3;
    Cx<double> d0 = cmake(0.0, 0.0), d1 = cmake(0.0, 0.0);
    if (chunk < a.nchunk) {
        int s3, xh, y, z;
        tm_column(a, col - chunk * V3, s3, xh, y, z);
        const int sy = a.Lxh, sz = a.Lxh * a.Ly;
        const int yf = y == a.Ly - 1 ? -(a.Ly - 1) * sy : sy, yb = y == 0 ? (a.Ly - 1) * sy : -sy;
        const int zf = z == a.Lz - 1 ? -(a.Lz - 1) * sz : sz, zb = z == 0 ? (a.Lz - 1) * sz : -sz;
        const int64_t vstride = (int64_t)a.Vh << a.bshift;
        const int t0 = chunk * a.tc, t1 = t0 + a.tc;
        // pending backward t-hops of the even / odd steps of the chunk
        Cx<T>* wb0 = (Cx<T>*)hop_lds;
        Cx<T>* wb1 = wb0 + 6 * HOP_THREADS;
        t_back<S, -SF, MIX>(a, (t0 == 0 ? a.Lt - 1 : t0 - 1) * V3 + s3, r, vstride,
                       (a.antiperiodic && t0 == 0) ? T(-1) : T(1), wb0);
        t_back<S, -SF, MIX>(a, t0 * V3 + s3, r, vstride, T(1), wb1);
#pragma nounroll
        for (int t = t0; t < t1; t += 2) {
            tm_step<S, DAG, G5OUT, XPAY, DOT, MIX, ROWL>(a, t, t1, s3, xh, y, z, r, V3, yf, yb, zf, zb, wb0, d0, d1);
            tm_step<S, DAG, G5OUT, XPAY, DOT, MIX, ROWL>(a, t + 1, t1, s3, xh, y, z, r, V3, yf, yb, zf, zb, wb1, d0,
                                                         d1);
        }
    }
    hop_block_reduce<NP>(a, blk, g, d0, d1);
}

// ---------------------------------------------------------------------------
// Skewed t-marching form.  As above, a lane owns one (x, y, z) column and one
// RHS and walks a chunk of t slices, but step t reads a single input slice,
// t + 1: the column's own spinor there completes output t (its forward t-hop)
// and gives the backward t-hop of output t + 2, and the x, y, z neighbours
// there start output t + 1, whose accumulator is carried into the next step.
// The plain t-march reads slice t + 1 at step t (the own column) and again at
// step t + 1 (as the spatial neighbours of the next output), one step of
// every resident workgroup's traffic apart; here both reads fall in one step,
// so the neighbour reuse between columns meets in the caches sooner.
// ---------------------------------------------------------------------------

// row-shared links of a skewed step: the spatial slots (forward at s, backward
// at sbx, sby, sbz) belong to output t + 1, the forward t slot to output t
// (site sft) and the backward t slot to the input site sbt of slice t + 1
__device__ inline void row_links_load_skew(const void* U, int Vh, int p, int s, int sft, int sbx, int sby, int sbz,
                                           int sbt, RowLinks& rl) {
    const int q = threadIdx.x & 15, d = q >> 1, mu = d >> 1;
    const bool bwd = d & 1;
    int site = mu == 3 ? sft : s;
    if (bwd) site = mu == 0 ? sbx : (mu == 1 ? sby : (mu == 2 ? sbz : sbt));
    const int64_t v = ((int64_t)(mu * 2 + (bwd ? 1 - p : p)) * Vh + site) * 3;   // 3 vectors per BF16 link
    const uint2* ptr = (const uint2*)((const uint4*)U + v) + 3 * (q & 1);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const uint2 d2 = ptr[k];
        rl.w[2 * k] = d2.x;
        rl.w[2 * k + 1] = d2.y;
    }
}

// One skewed step t (OPEN: the step before the chunk's first output, which
// only starts output t + 1 = t0).  acc carries output t in and output t + 1
// out; wprod receives the backward t-hop of output t + 2, wcons holds that of
// output t + 1.
template <typename S, bool DAG, bool G5OUT, bool XPAY, int DOT, int MIX, bool ROWL, bool OPEN>
__device__ inline void tsk_step(const HopArgs& a, int t, int t1, int s3, int xh, int y, int z, int r, int V3, int yf,
                                int yb, int zf, int zb, Cx<typename Store<S>::acc>* wprod,
                                const Cx<typename Store<S>::acc>* wcons, Cx<typename Store<S>::acc>* acc,
                                Cx<double>& d0, Cx<double>& d1) {
    typedef typename Store<S>::acc T;
    constexpr int NV = (9 + Store<S>::VW - 1) / Store<S>::VW;
    constexpr int SF = DAG ? -1 : 1;
    const int p = a.out_parity;
    const int64_t vstride = (int64_t)a.Vh << a.bshift;
    const int tn = t + 1 == a.Lt ? 0 : t + 1;   // the input slice of this step
    int sn = tn * V3 + s3;                      // own column there; also output t + 1's site
    int s0 = OPEN ? sn : t * V3 + s3;           // output t
    asm volatile("" : "+v"(sn), "+v"(s0));
    const int x = 2 * xh + ((p + y + z + tn) & 1);
    const int row = sn - xh;
    const int xf = x + 1 == a.Lx ? 0 : x + 1, xb = x == 0 ? a.Lx - 1 : x - 1;
    const int sx = row + (xb >> 1), sy = sn + yb, sz = sn + zb;
    RowLinks rl;
    if constexpr (ROWL) row_links_load_skew(a.U, a.Vh, p, sn, s0, sx, sy, sz, sn, rl);
    const bool more = t + 1 < t1, more2 = t + 2 < t1;
    if constexpr (std::is_same<S, bf16x2>::value) {
        uint32_t psi[12], u[12];
        Cx<float> w[6];
        load_packed_spinor(a.in, ((int64_t)sn << a.bshift) + r, vstride, psi);
        if constexpr (!OPEN) {   // forward t-hop completes output t
            if constexpr (ROWL) row_link_get<6>(rl, u);
            else load_packed_link(a.U, ((int64_t)(6 + p) * a.Vh + s0) * NV, u);
            link_mult_bf16<3, SF, false>(psi, u, w);
            reconstruct<3, SF>(acc, w, (a.antiperiodic && t == a.Lt - 1) ? -1.f : 1.f);
            fence_acc(acc);
        }
        if (more2) {   // backward t-hop of output t + 2, from the same input spinor
            if constexpr (ROWL) row_link_get<7>(rl, u);
            else load_packed_link(a.U, ((int64_t)(6 + 1 - p) * a.Vh + sn) * NV, u);
            link_mult_bf16<3, -SF, true>(psi, u, w);
            wb_store(wprod, w);
        }
    } else {
        Cx<T> psi[12], h[6], u[9], w[6];
        load_operand<S, (MIX & HOP_IN16) != 0, false>(a.in, ((int64_t)sn << a.bshift) + r, vstride, psi);
        if constexpr (!OPEN) {
            project<3, SF>(psi, h);
            load_link<S>(a.U, ((int64_t)(6 + p) * a.Vh + s0) * NV, u);
            mul_link<false>(u, h, w);
            reconstruct<3, SF>(acc, w, (a.antiperiodic && t == a.Lt - 1) ? T(-1) : T(1));
            fence_acc(acc);
        }
        if (more2) {
            project<3, -SF>(psi, h);
            load_link<S>(a.U, ((int64_t)(6 + 1 - p) * a.Vh + sn) * NV, u);
            mul_link<true>(u, h, w);
            wb_store(wprod, w);
        }
    }
    if constexpr (!OPEN) {
        hop_epilogue<S, G5OUT, XPAY, DOT, MIX>(a, s0, r, acc, d0, d1);
        fence_acc(acc);
    }
    if (more) {   // start output t + 1: its pending backward t-hop, then x, y, z from this slice
        Cx<T> wb[6];
        wb_load(wcons, wb);
#pragma unroll
        for (int i = 0; i < 12; i++) acc[i] = cmake<T>(0, 0);
        reconstruct<3, -SF>(acc, wb, T(1));
        fence_acc(acc);
        hop_dir<S, 0, DAG, MIX, ROWL>(a, row + (xf >> 1), sx, r, false, false, a.U, ((int64_t)p * a.Vh + sn) * NV, a.U,
                                      ((int64_t)(1 - p) * a.Vh + sx) * NV, acc, &rl);
        hop_dir<S, 1, DAG, MIX, ROWL>(a, sn + yf, sy, r, false, false, a.U, ((int64_t)(2 + p) * a.Vh + sn) * NV, a.U,
                                      ((int64_t)(3 - p) * a.Vh + sy) * NV, acc, &rl);
        hop_dir<S, 2, DAG, MIX, ROWL>(a, sn + zf, sz, r, false, false, a.U, ((int64_t)(4 + p) * a.Vh + sn) * NV, a.U,
                                      ((int64_t)(5 - p) * a.Vh + sz) * NV, acc, &rl);
    }
}

template <typename S, bool DAG, bool G5OUT, bool XPAY, int DOT, int MIX, bool ROWL = false>
__global__ __launch_bounds__(HOP_THREADS) void hop_tsk_kernel(HopArgs a) {
    typedef typename Store<S>::acc T;
    extern __shared__ uint4 hop_lds[];   // [2][6][HOP_THREADS] Cx<T>
    constexpr int NP = (DOT == HOPDOT_A_OUT || DOT == HOPDOT_NORM) ? 1 : ((DOT == HOPDOT_OUT_X || DOT == HOPDOT_NORM_ZX) ? 2 : 0);
    constexpr int SF = DAG ? -1 : 1;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g = blk / a.bpg;                 // RHS group
    const int gid = (blk - g * a.bpg) * HOP_THREADS + threadIdx.x;
    const int G = 1 << a.gshift;
    const int col = gid >> a.gshift;   // chunk * V3 + column
    const int r = g * G + (gid & (G - 1));
    const int V3 = a.Vh / a.Lt;
    const int chunk = col / V3;
    Cx<double> d0 = cmake(0.0, 0.0), d1 = cmake(0.0, 0.0);
    if (chunk < a.nchunk) {
        int s3, xh, y, z;
        tm_column(a, col - chunk * V3, s3, xh, y, z);
        const int sy = a.Lxh, sz = a.Lxh * a.Ly;
        const int yf = y == a.Ly - 1 ? -(a.Ly - 1) * sy : sy, yb = y == 0 ? (a.Ly - 1) * sy : -sy;
        const int zf = z == a.Lz - 1 ? -(a.Lz - 1) * sz : sz, zb = z == 0 ? (a.Lz - 1) * sz : -sz;
        const int64_t vstride = (int64_t)a.Vh << a.bshift;
        const int t0 = chunk * a.tc, t1 = t0 + a.tc;
        // step k of the chunk (k = t - t0, from -1) leaves the backward t-hop
        // of output t + 2 in slot k & 1 and takes that of output t + 1 from
        // slot (k + 1) & 1
        Cx<T>* wb0 = (Cx<T>*)hop_lds;
        Cx<T>* wb1 = wb0 + 6 * HOP_THREADS;
        t_back<S, -SF, MIX>(a, (t0 == 0 ? a.Lt - 1 : t0 - 1) * V3 + s3, r, vstride,
                            (a.antiperiodic && t0 == 0) ? T(-1) : T(1), wb0);
        Cx<T> acc[12];
        tsk_step<S, DAG, G5OUT, XPAY, DOT, MIX, ROWL, true>(a, t0 - 1, t1, s3, xh, y, z, r, V3, yf, yb, zf, zb, wb1,
                                                             wb0, acc, d0, d1);
#pragma nounroll
        for (int t = t0; t < t1; t += 2) {
            tsk_step<S, DAG, G5OUT, XPAY, DOT, MIX, ROWL, false>(a, t, t1, s3, xh, y, z, r, V3, yf, yb, zf, zb, wb0,
                                                                  wb1, acc, d0, d1);
            tsk_step<S, DAG, G5OUT, XPAY, DOT, MIX, ROWL, false>(a, t + 1, t1, s3, xh, y, z, r, V3, yf, yb, zf, zb,
                                                                  wb1, wb0, acc, d0, d1);
        }
    }
    hop_block_reduce<NP>(a, blk, g, d0, d1);
}

template <typename S> constexpr int prec_of() {
    return std::is_same<S, double>::value ? DHT_FP64 : (std::is_same<S, float>::value ? DHT_FP32 : DHT_BF16);
}

static int log2_batch(int nrhs) {
    for (int b = 0; b < 9; b++)
        if ((1 << b) == nrhs) return b;
    return -1;
}

static int auto_chunk(const dht_ctx* c, int nrhs) {
    const int Lt = c->g.L[3];
    const int64_t cols = c->g.Vh / Lt * (int64_t)nrhs;
    int tc = Lt;
    while (tc % 4 == 0 && cols * (Lt / tc) < HOP_MIN_LANES) tc /= 2;
    return tc;
}

int hop_config_check(const dht_ctx* c, int nrhs, const HopConfig& h) {
    if (log2_batch(nrhs) < 0) return set_error(DHT_ERR_INVALID_ARG, "batch must be a power of two <= 256");
    if (h.form < DHT_HOP_SITE || h.form > DHT_HOP_TSKEW_ROWL || (h.nt != 0 && h.nt != 1))
        return set_error(DHT_ERR_INVALID_ARG, "bad hop form");
    const int G = h.rg > 0 ? h.rg : nrhs;
    if (log2_batch(G) < 0 || G > nrhs) return set_error(DHT_ERR_INVALID_ARG, "RHS group must be a power of two <= nrhs");
    if (h.form == DHT_HOP_SITE_LDS && (HOP_THREADS / G) > 32)
        return set_error(DHT_ERR_INVALID_ARG, "LDS-link form needs at least 8 right-hand sides per sweep");
    if (hop_form_tmarch(h.form) && h.tc != 0 && (h.tc < 2 || (h.tc & 1) || c->g.L[3] % h.tc))
        return set_error(DHT_ERR_INVALID_ARG, "t chunk must be even and divide Lt");
    if (h.zb < 0 || h.zb > 8 || (h.zb > 0 && (!hop_form_tmarch(h.form) || c->g.L[2] % (1 << h.zb))))
        return set_error(DHT_ERR_INVALID_ARG, "z block must be a power of two dividing Lz (t-marching forms only)");
    return DHT_OK;
}

// Default shape: links from LDS for FP32 / FP64 batches of >= 8, otherwise one
// lane per site; streaming stores.  (Measured on the 32^3x64 lattice at 16
// RHS: the LDS copy pays in FP32 and FP64 and not in BF16, whose links take
// only three 16-byte loads.)
HopConfig hop_default_config(const dht_ctx* c, int prec, int nrhs) {
    HopConfig h;
    h.form = (prec != DHT_BF16 && HOP_THREADS / nrhs <= 32) ? DHT_HOP_SITE_LDS : DHT_HOP_SITE;
    h.nt = 1;
    h.tc = auto_chunk(c, nrhs);
    return h;
}

HopConfig hop_config(const dht_ctx* c, int prec, int nrhs, int cls) {
    HopConfig h;
    const int b = log2_batch(nrhs);
    if (c->hop_force) h = c->hop_forced;
    else if (b >= 0 && prec >= 0 && prec < 3 && c->hop_cfg[prec][b][cls].form >= 0) h = c->hop_cfg[prec][b][cls];
    else h = hop_default_config(c, prec, nrhs);
    if (h.tc == 0) h.tc = auto_chunk(c, nrhs);
    return h;
}

// workgroups of the site-parallel forms with one sweep over all RHS; the
// other shapes use at most this many plus one per RHS group
int hop_blocks(const dht_ctx* c, int nrhs) {
    int64_t n = c->g.Vh * (int64_t)nrhs;
    return (int)((n + HOP_THREADS - 1) / HOP_THREADS);
}

template <typename S>
static int launch_hop(dht_ctx* c, int out_parity, const void* in, void* out, const void* x, double ca, double cb,
                      int nrhs, bool dagger, bool g5out, HopDot* dot, const void* z, double cz, int mix, void* out16,
                      const double* s16) {
    HopArgs a;
    a.out = out;
    a.in = in;
    a.x = x;
    a.z = z;
    a.cz = cz;
    if (z && !x) return set_error(DHT_ERR_INVALID_ARG, "second axpy source needs an xpay source");
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
    a.out16 = out16;
    a.s16 = s16;
    if (((mix & HOP_OUT16) != 0) != (out16 != nullptr) || (out16 && !s16))
        return set_error(DHT_ERR_INVALID_ARG, "BF16 output copy needs its buffer and scales");
    if (kind == HOPDOT_OUT_X && !x) return set_error(DHT_ERR_INVALID_ARG, "fused (out, x) needs an xpay source");
    if (kind == HOPDOT_NORM_ZX && !z) return set_error(DHT_ERR_INVALID_ARG, "fused (z, x) needs both axpy sources");
    const int cls = (dot && kind == HOPDOT_A_OUT) ? HOP_FUSED_A : ((x || dot) ? HOP_FUSED : HOP_PLAIN);
    const HopConfig cfg = hop_config(c, prec_of<S>(), nrhs, cls);
    a.tc = cfg.tc;
    a.nchunk = a.Lt / cfg.tc;
    a.zbs = hop_form_tmarch(cfg.form) ? cfg.zb : 0;
    a.nt = cfg.nt;
    // the row-shared forms need BF16 rows of one site (>= 16 RHS per sweep);
    // otherwise they run as their plain form
    const int G0 = cfg.rg > 0 ? cfg.rg : nrhs;
    const bool rowl = std::is_same<S, bf16x2>::value && G0 >= 16 &&
                      (cfg.form == DHT_HOP_SITE_ROWL || cfg.form == DHT_HOP_TMARCH_ROWL ||
                       cfg.form == DHT_HOP_TSKEW_ROWL);
    const bool skew = cfg.form == DHT_HOP_TSKEW || cfg.form == DHT_HOP_TSKEW_ROWL;
    const int mode = hop_form_tmarch(cfg.form) ? DHT_HOP_TMARCH : (cfg.form == DHT_HOP_SITE_ROWL ? DHT_HOP_SITE : cfg.form);
    const int G = cfg.rg > 0 ? cfg.rg : nrhs;   // RHS per sweep
    a.gshift = log2_batch(G);
    if (a.gshift < 0 || G > nrhs) return set_error(DHT_ERR_INVALID_ARG, "bad RHS group");
    const int ns = HOP_THREADS >> a.gshift;   // sites per workgroup (site-parallel forms)
    a.bpg = mode == DHT_HOP_TMARCH
                ? (int)((c->g.Vh / a.Lt * (int64_t)a.nchunk * G + HOP_THREADS - 1) / HOP_THREADS)
                : (int)((c->g.Vh + ns - 1) / ns);
    const int nb = a.bpg * (nrhs / G);
    const size_t lds = mode == DHT_HOP_SITE_LDS ? (size_t)8 * ns * ((9 + Store<S>::VW - 1) / Store<S>::VW) * 16 : 0;
    const size_t tm_lds = (size_t)2 * 6 * HOP_THREADS * sizeof(Cx<typename Store<S>::acc>);
    if (dot) dot->nblocks = nb;
    dim3 grid(nb), block(HOP_THREADS);
    bool xp = x != nullptr;
#define DHT_HOP_CASE_M(D_, G_, X_, K_, M_)                                                                   \
    if (dagger == D_ && g5out == G_ && xp == X_ && kind == K_ && mix == (M_)) {                              \
        if constexpr (std::is_same<S, bf16x2>::value) {                                                      \
            if (rowl) {                                                                                      \
                if (skew)                                                                                    \
                    hipLaunchKernelGGL((hop_tsk_kernel<S, D_, G_, X_, K_, M_, true>), grid, block, tm_lds,   \
                                       c->stream, a);                                                        \
                else if (mode == DHT_HOP_TMARCH)                                                             \
                    hipLaunchKernelGGL((hop_tm_kernel<S, D_, G_, X_, K_, M_, true>), grid, block, tm_lds,    \
                                       c->stream, a);                                                        \
                else                                                                                         \
                    hipLaunchKernelGGL((hop_kernel<S, D_, G_, X_, K_, false, M_, true>), grid, block, 0,     \
                                       c->stream, a);                                                        \
                goto launched;                                                                               \
            }                                                                                                \
        }                                                                                                    \
        if (skew)                                                                                            \
            hipLaunchKernelGGL((hop_tsk_kernel<S, D_, G_, X_, K_, M_>), grid, block, tm_lds, c->stream, a);  \
        else if (mode == DHT_HOP_TMARCH)                                                                     \
            hipLaunchKernelGGL((hop_tm_kernel<S, D_, G_, X_, K_, M_>), grid, block, tm_lds, c->stream, a);   \
        else if (mode == DHT_HOP_SITE_LDS)                                                                   \
            hipLaunchKernelGGL((hop_kernel<S, D_, G_, X_, K_, true, M_>), grid, block, lds, c->stream, a);   \
        else                                                                                                 \
            hipLaunchKernelGGL((hop_kernel<S, D_, G_, X_, K_, false, M_>), grid, block, 0, c->stream, a);    \
        goto launched;                                                                                       \
    }
#define DHT_HOP_CASE(D_, G_, X_, K_) DHT_HOP_CASE_M(D_, G_, X_, K_, 0)
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
    DHT_HOP_CASE(false, false, true, HOPDOT_NORM)
    DHT_HOP_CASE(false, false, true, HOPDOT_NORM_ZX)
    if constexpr (std::is_same<S, double>::value) {
        // FP64 residuals whose probe operand is held in BF16 (exact values):
        // the Schur right-hand side from z, the odd sites, the final residual
        DHT_HOP_CASE_M(false, false, true, HOPDOT_NORM, HOP_IN16 | HOP_X16)
        DHT_HOP_CASE_M(false, false, true, HOPDOT_NORM, HOP_IN16 | HOP_X16 | HOP_OUT16)
        DHT_HOP_CASE_M(false, false, true, HOPDOT_NORM, HOP_OUT16)
        DHT_HOP_CASE_M(false, false, true, HOPDOT_NONE, HOP_X16)
        DHT_HOP_CASE_M(false, false, true, HOPDOT_OUT_X, HOP_X16)
        DHT_HOP_CASE_M(false, false, true, HOPDOT_NORM, HOP_Z16)
        DHT_HOP_CASE_M(false, false, true, HOPDOT_NORM_ZX, HOP_Z16)
        DHT_HOP_CASE_M(false, false, true, HOPDOT_NORM_ZX, HOP_Z16 | HOP_NOOUT)
        DHT_HOP_CASE_M(false, false, true, HOPDOT_NORM_ZX, HOP_NOOUT)
    }
#undef DHT_HOP_CASE
#undef DHT_HOP_CASE_M
    return set_error(DHT_ERR_INVALID_ARG, "unsupported hop variant");
launched:
    DHT_HIP(hipGetLastError());
    return DHT_OK;
}

int hop(dht_ctx* c, int prec, int out_parity, const void* in, void* out, const void* x, double a, double b,
        int nrhs, bool dagger, bool g5out, HopDot* dot, const void* z, double cz, int mix, void* out16,
        const double* s16) {
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    if (prec < DHT_FP64 || prec > DHT_BF16) return set_error(DHT_ERR_INVALID_ARG, "bad precision");
    if (mix != 0 && prec != DHT_FP64) return set_error(DHT_ERR_INVALID_ARG, "BF16 operands only in FP64 hops");
    int tok;
    DHT_TRY(prof_begin(c, &tok));
    int rc = DHT_OK;
    switch (prec) {
        case DHT_FP64: rc = launch_hop<double>(c, out_parity, in, out, x, a, b, nrhs, dagger, g5out, dot, z, cz, mix, out16, s16);
            break;
        case DHT_FP32: rc = launch_hop<float>(c, out_parity, in, out, x, a, b, nrhs, dagger, g5out, dot, z, cz, mix, out16, s16);
            break;
        case DHT_BF16: rc = launch_hop<bf16x2>(c, out_parity, in, out, x, a, b, nrhs, dagger, g5out, dot, z, cz, mix, out16, s16);
            break;
    }
    if (rc != DHT_OK) return rc;
    // algorithmic bytes: read the input half field (and the xpay / dot operand),
    // write the output, read each of the 8 Vh link matrices of this parity once
    const double eb = (double)elem_bytes(prec), e16 = (double)elem_bytes(DHT_BF16);
    const double nbytes = ((mix & HOP_NOOUT) ? 0.0 : eb) + ((mix & HOP_IN16) ? e16 : eb) +
                          (x ? ((mix & HOP_X16) ? e16 : eb) : 0.0) + (z ? ((mix & HOP_Z16) ? e16 : eb) : 0.0) +
                          ((dot && dot->kind == HOPDOT_A_OUT) ? eb : 0.0) + ((mix & HOP_OUT16) ? e16 : 0.0);
    const double bytes = nbytes * 12.0 * c->g.Vh * nrhs + 72.0 * c->g.Vh * eb;
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
