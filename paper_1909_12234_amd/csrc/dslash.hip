// Wilson-Dirac operator on gfx950.
//
//   (A psi)(x) = (4+m) psi(x)
//              - 1/2 sum_mu [ (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu) ]
//
// Each hop is done on a half spinor: the rank-2 projector (1 + s g_mu) (s = -1 forward,
// +1 backward; swapped for A^+) maps the 4 spin components to two colour vectors h0, h1,
// the 3x3 link multiplies only those two, and the lower two spin rows are rebuilt from
// them.  The projection and rebuild rules follow from the DeGrand-Rossi matrices:
//   mu=x: h0 = p0 + s i p3, h1 = p1 + s i p2;  rows 2,3 += -s i Uh1, -s i Uh0
//   mu=y: h0 = p0 - s p3,   h1 = p1 + s p2;    rows 2,3 +=  s Uh1,   -s Uh0
//   mu=z: h0 = p0 + s i p2, h1 = p1 - s i p3;  rows 2,3 += -s i Uh0,  s i Uh1
//   mu=t: h0 = p0 + s p2,   h1 = p1 + s p3;    rows 2,3 +=  s Uh0,    s Uh1
// giving 1320 flops per site and right-hand side for the hopping term.
//
// One thread owns one site and R right-hand sides: each link is loaded once and applied
// to R spinors.  Algorithmic traffic per site: 72 link reals + R*(24 in + 24 out) reals.
#include <iterator>

#include "blas.h"
#include "dslash_mfma.h"
#include "lqt_internal.h"

namespace lqt {

template <typename C>
struct cpx {
    C x, y;
};

template <typename C>
__device__ __forceinline__ cpx<C> ld_c(const double2* p) {
    double2 v = *p;
    return {(C)v.x, (C)v.y};
}
template <typename C, typename S>
__device__ __forceinline__ cpx<C> ld_c(const S* p) {
    float2 v = io<S>::ld(p);
    return {(C)v.x, (C)v.y};
}
template <typename C>
__device__ __forceinline__ void st_c(double2* p, cpx<C> v) {
    *p = make_double2((double)v.x, (double)v.y);
}
template <typename C, typename S>
__device__ __forceinline__ void st_c(S* p, cpx<C> v) {
    io<S>::st(p, make_float2((float)v.x, (float)v.y));
}

// element i of a field through a wave-uniform base and a 32-bit byte offset: the load
// forms the address itself (scalar base + vector offset), no 64-bit vector arithmetic.
// Valid while 12 V sizeof(S) < 4 GiB (checked when a context is created).
template <typename S>
__device__ __forceinline__ const S* at(const S* base, uint32_t i) {
    return (const S*)((const char*)base + i * (uint32_t)sizeof(S));
}
template <typename S>
__device__ __forceinline__ S* at(S* base, uint32_t i) {
    return (S*)((char*)base + i * (uint32_t)sizeof(S));
}

// a + s*i*b  (s = +1 or -1)
template <int SG, typename C>
__device__ __forceinline__ cpx<C> add_si(cpx<C> a, cpx<C> b) {
    return SG > 0 ? cpx<C>{a.x - b.y, a.y + b.x} : cpx<C>{a.x + b.y, a.y - b.x};
}
template <int SG, typename C>
__device__ __forceinline__ cpx<C> add_s(cpx<C> a, cpx<C> b) {
    return SG > 0 ? cpx<C>{a.x + b.x, a.y + b.y} : cpx<C>{a.x - b.x, a.y - b.y};
}

// h = (1 + SG g_MU) p restricted to its two independent rows
template <int MU, int SG, typename C>
__device__ __forceinline__ void project(const cpx<C> p[12], cpx<C> h0[3], cpx<C> h1[3]) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (MU == 0) {
            h0[a] = add_si<SG>(p[a], p[9 + a]);
            h1[a] = add_si<SG>(p[3 + a], p[6 + a]);
        } else if (MU == 1) {
            h0[a] = add_s<-SG>(p[a], p[9 + a]);
            h1[a] = add_s<SG>(p[3 + a], p[6 + a]);
        } else if (MU == 2) {
            h0[a] = add_si<SG>(p[a], p[6 + a]);
            h1[a] = add_si<-SG>(p[3 + a], p[9 + a]);
        } else {
            h0[a] = add_s<SG>(p[a], p[6 + a]);
            h1[a] = add_s<SG>(p[3 + a], p[9 + a]);
        }
    }
}

template <int MU, int SG, typename C>
__device__ __forceinline__ void rebuild_add(cpx<C> acc[12], const cpx<C> u0[3], const cpx<C> u1[3]) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        acc[a].x += u0[a].x;
        acc[a].y += u0[a].y;
        acc[3 + a].x += u1[a].x;
        acc[3 + a].y += u1[a].y;
        if (MU == 0) {
            acc[6 + a] = add_si<-SG>(acc[6 + a], u1[a]);
            acc[9 + a] = add_si<-SG>(acc[9 + a], u0[a]);
        } else if (MU == 1) {
            acc[6 + a] = add_s<SG>(acc[6 + a], u1[a]);
            acc[9 + a] = add_s<-SG>(acc[9 + a], u0[a]);
        } else if (MU == 2) {
            acc[6 + a] = add_si<-SG>(acc[6 + a], u0[a]);
            acc[9 + a] = add_si<SG>(acc[9 + a], u1[a]);
        } else {
            acc[6 + a] = add_s<SG>(acc[6 + a], u0[a]);
            acc[9 + a] = add_s<SG>(acc[9 + a], u1[a]);
        }
    }
}

__device__ __forceinline__ float fm(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fm(double a, double b, double c) { return fma(a, b, c); }

// o = l h with l = U (forward) or U^+ (backward), written as fused multiply-add chains
template <bool DAGGER_LINK, typename C>
__device__ __forceinline__ void su3_mul(const cpx<C> u[9], const cpx<C> h[3], cpx<C> o[3]) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        // l_b = U[a][b], or conj(U[b][a]) for the dagger
        const cpx<C> l0 = DAGGER_LINK ? cpx<C>{u[a].x, -u[a].y} : u[3 * a];
        C re = l0.x * h[0].x, im = l0.x * h[0].y;
        re = fm(-l0.y, h[0].y, re);
        im = fm(l0.y, h[0].x, im);
#pragma unroll
        for (int b = 1; b < 3; b++) {
            const cpx<C> l = DAGGER_LINK ? cpx<C>{u[3 * b + a].x, -u[3 * b + a].y} : u[3 * a + b];
            re = fm(l.x, h[b].x, re);
            re = fm(-l.y, h[b].y, re);
            im = fm(l.x, h[b].y, im);
            im = fm(l.y, h[b].x, im);
        }
        o[a] = {re, im};
    }
}

// Fields are read through a wave-uniform base pointer (one right-hand side) and a 32-bit
// element offset, so the address is formed by the load itself (no 64-bit vector adds).
template <typename S, typename C>
__device__ __forceinline__ void load_spinor(const S* __restrict__ f, uint32_t V, uint32_t s, bool g5, cpx<C> p[12]) {
#pragma unroll
    for (int c = 0; c < 12; c++) {
        p[c] = ld_c<C>(at(f, c * V + s));
        if (g5 && c >= 6) {
            p[c].x = -p[c].x;
            p[c].y = -p[c].y;
        }
    }
}

// Um = the links of direction mu ([ab][V] block, uniform base)
template <typename S, typename C>
__device__ __forceinline__ void load_link(const S* __restrict__ Um, uint32_t V, uint32_t s, cpx<C> u[9]) {
#pragma unroll
    for (int i = 0; i < 9; i++) u[i] = ld_c<C>(at(Um, i * V + s));
}

// hop for one direction: acc[r] += (1 - g) U(x) psi(x+mu) + (1 + g) U(x-mu)^+ psi(x-mu)
// (projector signs swap for the adjoint)
template <int MU, bool DAG, int R, typename S, typename C>
__device__ __forceinline__ void hop_dir(const S* __restrict__ U, const S* const inb[R], uint32_t V, uint32_t s,
                                        uint32_t sf, uint32_t sb, bool g5in, cpx<C> acc[R][12]) {
    // the R neighbour spinors of a direction are loaded (as stored) before any of them is
    // used; a group's unused right-hand sides read a valid field and are never stored
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    cpx<C> u[9], p[12], h0[3], h1[3], o0[3], o1[3];
    S raw[R][12];
    const S* Um = U + (long long)MU * 9 * V;
    load_link<S, C>(Um, V, s, u);
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 12; c++) raw[r][c] = *at(inb[r], c * V + sf);
#pragma unroll
    for (int r = 0; r < R; r++) {
#pragma unroll
        for (int c = 0; c < 12; c++) {
            p[c] = ld_c<C>(&raw[r][c]);
            if (g5in && c >= 6) p[c] = {-p[c].x, -p[c].y};
        }
        project<MU, SF>(p, h0, h1);
        su3_mul<false>(u, h0, o0);
        su3_mul<false>(u, h1, o1);
        rebuild_add<MU, SF>(acc[r], o0, o1);
    }
    load_link<S, C>(Um, V, sb, u);
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 12; c++) raw[r][c] = *at(inb[r], c * V + sb);
#pragma unroll
    for (int r = 0; r < R; r++) {
#pragma unroll
        for (int c = 0; c < 12; c++) {
            p[c] = ld_c<C>(&raw[r][c]);
            if (g5in && c >= 6) p[c] = {-p[c].x, -p[c].y};
        }
        project<MU, SB>(p, h0, h1);
        su3_mul<true>(u, h0, o0);
        su3_mul<true>(u, h1, o1);
        rebuild_add<MU, SB>(acc[r], o0, o1);
    }
}

// ---- FP16 storage with packed half-precision arithmetic (kind 2 of the tuner)
// The spin projection h = p_a + c p_b (c = +-1, +-i) is one packed FP16 add per complex
// number (its result rounded to FP16), and each complex product with a link element is a
// pair of FP16 dot products accumulated in FP32: Re(U h) = U . (Re h, -Im h),
// Im(U h) = U . (Im h, Re h) with U = (Re U, Im U) as stored; for U^+ the pairs are
// (Re h, Im h) and (Im h, -Re h).  Links and neighbour spinors are used as loaded.
typedef _Float16 hv2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ hv2 ldh(const h2* base, uint32_t i) {
    return __builtin_bit_cast(hv2, *(const uint32_t*)((const char*)base + i * 4u));
}

// Buffer accesses of the packed FP16 kernels: a field (or the links) is one buffer resource;
// the word of component c at site s sits at byte voff = 4 s (per lane, one register shared
// by every component) + soff = 4 c V (uniform, a scalar register), so no per-component
// address arithmetic runs on the vector ALUs.  Every offset stays below 4 GiB (checked when a
// context is created), and the resources carry no range limit.
using brsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ brsrc mkrsrc(const void* p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)0xFFFFFFFFu, 0x00020000);
}
__device__ __forceinline__ hv2 bld(brsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(hv2, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
// stores are non-temporal (cache policy NT): outputs are not read again by the launch, so they
// should not evict the neighbour rows that other blocks are about to read from L2
__device__ __forceinline__ void bst(brsrc r, hv2 v, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 2);
}
// c q for c = CRE + i CIM in {+-1, +-i}
template <int CRE, int CIM>
__device__ __forceinline__ hv2 cmul_unit(hv2 q) {
    if constexpr (CRE == 1) return q;
    else if constexpr (CRE == -1) return -q;
    else if constexpr (CIM == 1) return hv2{-q.y, q.x};
    else return hv2{q.y, -q.x};
}
// the two operand forms of h = a + c b for the dot products: forward link (Re h, -Im h),
// (Im h, Re h); backward link (Re h, Im h), (Im h, -Re h)
template <bool BWD, int CRE, int CIM>
__device__ __forceinline__ void hforms(hv2 a, hv2 b, hv2& f0, hv2& f1) {
    const hv2 cb = cmul_unit<CRE, CIM>(b);
    if constexpr (!BWD) {
        f0 = hv2{a.x, -a.y} + hv2{cb.x, -cb.y};
        f1 = hv2{a.y, a.x} + hv2{cb.y, cb.x};
    } else {
        f0 = a + cb;
        f1 = hv2{a.y, -a.x} + hv2{cb.y, -cb.x};
    }
}
// coefficient c of the projection (1 + SG g_MU) rows h0 (k = 0) and h1 (k = 1), and the spin
// of p_b: the same rules as project<MU, SG>
template <int MU, int SG, int K>
struct pk_rule {
    static constexpr int pb = MU == 0 ? (K == 0 ? 3 : 2) : MU == 1 ? (K == 0 ? 3 : 2) : MU == 2 ? (K == 0 ? 2 : 3) : (K == 0 ? 2 : 3);
    static constexpr int cre = MU == 1 ? (K == 0 ? -SG : SG) : MU == 3 ? SG : 0;
    static constexpr int cim = MU == 0 ? SG : MU == 2 ? (K == 0 ? SG : -SG) : 0;
};

// x.y of two FP16 pairs accumulated in FP32 from zero, as one three-operand instruction: the
// compiler's tied-accumulator form of the dot product would first move 0 into the
// destination, one extra instruction per product chain (12 per hop and right-hand side)
__device__ __forceinline__ float dot2_from_zero(hv2 x, hv2 y) {
    float d;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(d) : "v"(__builtin_bit_cast(uint32_t, x)),
        "v"(__builtin_bit_cast(uint32_t, y)));
    return d;
}

template <int MU, int SG, bool BWD, int K>
__device__ __forceinline__ void pk_half(const hv2 u[9], const hv2 p[12], cpx<float> o[3]) {
    using Rl = pk_rule<MU, SG, K>;
    hv2 f0[3], f1[3];
#pragma unroll
    for (int b = 0; b < 3; b++) hforms<BWD, Rl::cre, Rl::cim>(p[3 * K + b], p[3 * Rl::pb + b], f0[b], f1[b]);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const hv2 l0 = BWD ? u[a] : u[3 * a];
        float re = dot2_from_zero(l0, f0[0]), im = dot2_from_zero(l0, f1[0]);
#pragma unroll
        for (int b = 1; b < 3; b++) {
            const hv2 l = BWD ? u[3 * b + a] : u[3 * a + b];
            re = __builtin_amdgcn_fdot2(l, f0[b], re, false);
            im = __builtin_amdgcn_fdot2(l, f1[b], im, false);
        }
        o[a] = {re, im};
    }
}

// All 8 hops of the packed FP16 operator with the loads of the next hop issued before the
// products of the current one (two buffers of one link and R neighbour spinors).  Loads and
// products run for all R right-hand sides: a group's unused ones read a valid field (the
// pointers are clamped) and are never stored.
template <int R>
struct PkBuf {
    hv2 u[9];
    hv2 p[R][12];
};
// The links of a block's sites staged in LDS by the staged-link operator: word i of
// direction mu of site s0 + j at [(9 mu + i) 256 + j] (dynamic shared memory, 36 KB).
extern __shared__ hv2 lqt_staged_links[];

// With LDSU the forward link (direction MU at the thread's own site sl) comes from the
// staged links; backward links (at a neighbour) are read from memory, where those of the
// block's own sites are in the lines the staging has just read.
template <int R, bool LDSU = false, int MU = 0, bool BWD = false>
__device__ __forceinline__ void pk_load(PkBuf<R>& b, brsrc rU, const brsrc inr[R], uint32_t V, uint32_t sl,
                                        uint32_t sn, bool g5in, uint32_t s0 = 0) {
    if constexpr (LDSU && !BWD) {
        const uint32_t li = (9 * MU) * 256 + (sl - s0);
#pragma unroll
        for (int i = 0; i < 9; i++) b.u[i] = lqt_staged_links[i * 256 + li];
    } else {
#pragma unroll
        for (int i = 0; i < 9; i++) b.u[i] = bld(rU, sl * 4u, (uint32_t)(9 * MU + i) * V * 4u);
    }
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 12; c++) {
            b.p[r][c] = bld(inr[r], sn * 4u, (uint32_t)c * V * 4u);
            if (g5in && c >= 6) b.p[r][c] = -b.p[r][c];
        }
}
template <int MU, int SG, bool BWD, int R>
__device__ __forceinline__ void pk_comp_up(const hv2 u[9], const hv2 p[R][12], cpx<float> acc[R][12]) {
    cpx<float> o0[3], o1[3];
#pragma unroll
    for (int r = 0; r < R; r++) {
        pk_half<MU, SG, BWD, 0>(u, p[r], o0);
        pk_half<MU, SG, BWD, 1>(u, p[r], o1);
        rebuild_add<MU, SG>(acc[r], o0, o1);
    }
}
template <int MU, int SG, bool BWD, int R>
__device__ __forceinline__ void pk_comp(const PkBuf<R>& b, cpx<float> acc[R][12]) {
    pk_comp_up<MU, SG, BWD, R>(b.u, b.p, acc);
}
template <bool DAG, int R, bool LDSU = false>
__device__ __forceinline__ void hop_all_pk(brsrc rU, const brsrc inr[R], uint32_t V, uint32_t s, const uint32_t nf[4],
                                           const uint32_t nb[4], bool g5in, cpx<float> acc[R][12], uint32_t s0 = 0) {
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    // with staged links the scheduler would pull every LDS read to the top (one hop's reads
    // in flight is the design): a scheduling fence after each hop's products
    auto fence = [] {
        if constexpr (LDSU) __builtin_amdgcn_sched_barrier(0);
    };
    PkBuf<R> A, B;
    pk_load<R, LDSU, 0>(A, rU, inr, V, s, nf[0], g5in, s0);
    pk_load<R, LDSU, 0, true>(B, rU, inr, V, nb[0], nb[0], g5in, s0);
    pk_comp<0, SF, false, R>(A, acc);
    fence();
    pk_load<R, LDSU, 1>(A, rU, inr, V, s, nf[1], g5in, s0);
    pk_comp<0, SB, true, R>(B, acc);
    fence();
    pk_load<R, LDSU, 1, true>(B, rU, inr, V, nb[1], nb[1], g5in, s0);
    pk_comp<1, SF, false, R>(A, acc);
    fence();
    pk_load<R, LDSU, 2>(A, rU, inr, V, s, nf[2], g5in, s0);
    pk_comp<1, SB, true, R>(B, acc);
    fence();
    pk_load<R, LDSU, 2, true>(B, rU, inr, V, nb[2], nb[2], g5in, s0);
    pk_comp<2, SF, false, R>(A, acc);
    fence();
    pk_load<R, LDSU, 3>(A, rU, inr, V, s, nf[3], g5in, s0);
    pk_comp<2, SB, true, R>(B, acc);
    fence();
    pk_load<R, LDSU, 3, true>(B, rU, inr, V, nb[3], nb[3], g5in, s0);
    pk_comp<3, SF, false, R>(A, acc);
    pk_comp<3, SB, true, R>(B, acc);
}

// ---- Streaming operator (kind 4 of the tuner): FP16 storage, packed half arithmetic.
// A block owns 256 consecutive sites of a time slice (one site per thread, R right-hand
// sides) and walks every slice of its right-hand-side group in turn.  The spinors of its
// sites at t-1, t and t+1 stay in registers, so the +-t neighbours are read from memory once
// per sweep instead of once per neighbouring site; U_t(x - t) is the previous step's forward
// link.  The +-x, +-y, +-z neighbours lie in the same slice: the blocks of one group run on
// one XCD (contiguous logical blocks) and advance together, so a slice's rows are read from
// HBM by their own block and found in L2 by the blocks next to it.  Single-lattice contexts
// whose slice holds a multiple of 256 sites.  Measured at 16^3x32 with 128 right-hand sides it
// fetches as many bytes as the site-block kernels: with one right-hand side per thread (two
// spill) every group reads all links again, which takes back what the rolling slices save.
template <int R>
struct Sp {
    hv2 p[R][12];
};

template <int R>
__device__ __forceinline__ void ld_sp(Sp<R>& d, const brsrc inr[R], uint32_t V, uint32_t s, bool g5in) {
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 12; c++) {
            d.p[r][c] = bld(inr[r], s * 4u, (uint32_t)c * V * 4u);
            if (g5in && c >= 6) d.p[r][c] = -d.p[r][c];
        }
}

// the 9 words of U_mu at site s
template <int MU>
__device__ __forceinline__ void ld_link9(hv2 u[9], brsrc rU, uint32_t V, uint32_t s) {
#pragma unroll
    for (int i = 0; i < 9; i++) u[i] = bld(rU, s * 4u, (uint32_t)(9 * MU + i) * V * 4u);
}

// one slice t of the streaming operator: prev/cur/next hold psi at t-1, t, t+1 of the
// thread's site; at the end psi(t + 2) is loading into prev's registers
template <int R, bool DAG, bool G5IN, bool G5OUT>
__device__ __forceinline__ void tstream_step(brsrc rU, const brsrc inr[R], const brsrc outr[R], Sp<R>& prev,
                                             const Sp<R>& cur, const Sp<R>& next, hv2 utp[9], uint32_t V,
                                             uint32_t S, int L3, int t, uint32_t s0, const uint32_t nf[3],
                                             const uint32_t nb[3], int nr, float diag, float hs) {
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const uint32_t st = (uint32_t)t * S;
    const uint32_t s = st + s0;
    cpx<float> acc[R][12];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 12; c++) acc[r][c] = {0.f, 0.f};
    // -t hop with the previous step's link, then prev's registers take psi(t + 2)
    pk_comp_up<3, SB, true, R>(utp, prev.p, acc);
    if (t + 2 <= L3) ld_sp<R>(prev, inr, V, (uint32_t)((t + 2) % L3) * S + s0, G5IN);
    // +t hop: U_t(s) is this step's forward link and the next step's backward one
    ld_link9<3>(utp, rU, V, s);
    pk_comp_up<3, SF, false, R>(utp, next.p, acc);
    // +-x, +-y, +-z hops, one link and its spinors at a time (the registers go to the three
    // rolling slices; the other waves of the SIMD hide the load latency)
    PkBuf<R> A;
    pk_load<R, false, 0>(A, rU, inr, V, s, st + nf[0], G5IN);
    pk_comp<0, SF, false, R>(A, acc);
    pk_load<R, false, 0, true>(A, rU, inr, V, st + nb[0], st + nb[0], G5IN);
    pk_comp<0, SB, true, R>(A, acc);
    pk_load<R, false, 1>(A, rU, inr, V, s, st + nf[1], G5IN);
    pk_comp<1, SF, false, R>(A, acc);
    pk_load<R, false, 1, true>(A, rU, inr, V, st + nb[1], st + nb[1], G5IN);
    pk_comp<1, SB, true, R>(A, acc);
    pk_load<R, false, 2>(A, rU, inr, V, s, st + nf[2], G5IN);
    pk_comp<2, SF, false, R>(A, acc);
    pk_load<R, false, 2, true>(A, rU, inr, V, st + nb[2], st + nb[2], G5IN);
    pk_comp<2, SB, true, R>(A, acc);
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (r < nr) {
#pragma unroll
            for (int c = 0; c < 12; c++) {
                const hv2 pc = cur.p[r][c];
                float vx = fmaf(diag, (float)pc.x, hs * acc[r][c].x);
                float vy = fmaf(diag, (float)pc.y, hs * acc[r][c].y);
                if (G5OUT && c >= 6) {
                    vx = -vx;
                    vy = -vy;
                }
                bst(outr[r], hv2{(_Float16)vx, (_Float16)vy}, s * 4u, (uint32_t)c * V * 4u);
            }
        }
    }
}

template <int R, int OPK>
__global__ __launch_bounds__(256, 2) void k_dslash_tstream(const h2* __restrict__ U, const h2* __restrict__ in,
                                                           h2* __restrict__ out, LatTab tab, int nrhs,
                                                           long long in_stride, long long out_stride, double shift,
                                                           double scale) {
    constexpr bool DAG = OPK == LQT_A_DAG;
    constexpr bool G5IN = OPK == LQT_A_G5, G5OUT = OPK == LQT_G5_A;
    const int L0 = tab.L[0][0], L1 = tab.L[0][1], L2 = tab.L[0][2], L3 = tab.L[0][3];
    const uint32_t S = (uint32_t)(L0 * L1 * L2);
    const uint32_t V = S * (uint32_t)L3;
    const int nsb = (int)(S >> 8);
    const int ngrp = (nrhs + R - 1) / R;
    const int lb = xcd_block(ngrp * nsb);
    if (lb < 0) return;
    const int grp = lb / nsb, sb = lb - grp * nsb;
    const uint32_t s0 = (uint32_t)sb * 256u + threadIdx.x;  // site within the slice
    const int x = s0 % L0, y = (s0 / L0) % L1, z = s0 / (L0 * L1);
    const uint32_t s1 = L0, s2 = L0 * L1;
    const uint32_t nf[3] = {x == L0 - 1 ? s0 - (L0 - 1) : s0 + 1, y == L1 - 1 ? s0 - (L1 - 1) * s1 : s0 + s1,
                            z == L2 - 1 ? s0 - (L2 - 1) * s2 : s0 + s2};
    const uint32_t nb[3] = {x == 0 ? s0 + (L0 - 1) : s0 - 1, y == 0 ? s0 + (L1 - 1) * s1 : s0 - s1,
                            z == 0 ? s0 + (L2 - 1) * s2 : s0 - s2};
    const int r0 = grp * R;
    const int nr = min(R, nrhs - r0);
    brsrc inr[R], outr[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int rr = min(r0 + r, nrhs - 1);
        inr[r] = mkrsrc(in + (long long)rr * in_stride);
        outr[r] = mkrsrc(out + (long long)rr * out_stride);
    }
    const brsrc rU = mkrsrc(U);
    const float diag = (float)((tab.diag[0] - shift) * scale);
    const float hs = (float)(-0.5 * scale);
    Sp<R> A, B, C;
    hv2 utp[9];
    ld_sp<R>(A, inr, V, (uint32_t)(L3 - 1) * S + s0, G5IN);
    ld_sp<R>(B, inr, V, s0, G5IN);
    ld_sp<R>(C, inr, V, S + s0, G5IN);
    ld_link9<3>(utp, rU, V, (uint32_t)(L3 - 1) * S + s0);
#pragma unroll 1
    for (int t = 0; t < L3; t += 3) {
        tstream_step<R, DAG, G5IN, G5OUT>(rU, inr, outr, A, B, C, utp, V, S, L3, t, s0, nf, nb, nr, diag, hs);
        if (t + 1 < L3)
            tstream_step<R, DAG, G5IN, G5OUT>(rU, inr, outr, B, C, A, utp, V, S, L3, t + 1, s0, nf, nb, nr, diag, hs);
        if (t + 2 < L3)
            tstream_step<R, DAG, G5IN, G5OUT>(rU, inr, outr, C, A, B, utp, V, S, L3, t + 2, s0, nf, nb, nr, diag, hs);
    }
}

// kind 4 applies: FP16 storage, one lattice, slices of a multiple of 256 sites
static bool tstream_fits(const Geom& g) {
    const long long S = (long long)g.lat.L[0][0] * g.lat.L[0][1] * g.lat.L[0][2];
    return g.lat.nlat == 1 && S % 256 == 0 && (long long)g.V == S * g.lat.L[0][3];
}

template <int R>
static void launch_tstream(lqt_ctx* c, int op, const void* in, void* out, int nrhs, long long is, long long os,
                           double shift, double scale) {
    const Geom& g = c->g;
    LQT_CHECK(tstream_fits(g), LQT_EINVAL, "streaming operator: one lattice with slices of a multiple of 256 sites");
    const long long S = (long long)g.lat.L[0][0] * g.lat.L[0][1] * g.lat.L[0][2];
    const int nl = (int)(S / 256) * ((nrhs + R - 1) / R);
    const h2* U = c->U[LQT_F16].as<h2>();
#define LQT_TSTREAM_OP(OPK)                                                                               \
    hipLaunchKernelGGL((k_dslash_tstream<R, OPK>), dim3(xcd_grid(nl)), dim3(256), 0, c->stream, U, (const h2*)in, \
                       (h2*)out, g.lat, nrhs, is, os, shift, scale)
    switch (op) {
        case LQT_A_DAG: LQT_TSTREAM_OP(LQT_A_DAG); break;
        case LQT_A_G5: LQT_TSTREAM_OP(LQT_A_G5); break;
        case LQT_G5_A: LQT_TSTREAM_OP(LQT_G5_A); break;
        default: LQT_TSTREAM_OP(LQT_A); break;
    }
#undef LQT_TSTREAM_OP
    LQT_HIP(hipGetLastError());
}

// EPI 0: out = op(in).  EPI 1 (FP64 only): out = b - A in, with per-block partial |out|^2.
// Right-hand side r of a group is field act[r0 + r] (act may be null: r0 + r) of in and b,
// and field r0 + r of out.  Sites of the lattice table tab; padding sites get zeros.
template <typename S, int R, int OPK, int EPI, bool PKH = false, int G = 1>
__global__ __launch_bounds__(256) void k_dslash(const S* __restrict__ U, const S* __restrict__ in, S* __restrict__ out,
                                                const S* __restrict__ bvec, double* __restrict__ part,
                                                const int* __restrict__ act, LatTab tab, int nrhs, long long in_stride,
                                                long long out_stride, int chunk, double shift, double scale) {
    constexpr bool DAG = OPK == LQT_A_DAG;
    constexpr bool g5in = OPK == LQT_A_G5, g5out = OPK == LQT_G5_A;
    using C = typename acc_of<S>::type;
    const uint32_t V = (uint32_t)tab.off[tab.nlat];
    static_assert(G == 1 || (PKH && EPI == 0), "groups looped in the block: packed FP16 operator only");
    const int nsb = (int)((V + blockDim.x - 1) / blockDim.x);
    const int ngrp = (nrhs + R - 1) / R;
    const int ngb = (ngrp + G - 1) / G;  // blocks of G groups
    const int lb = xcd_block(nsb * ngb);
    if (lb < 0) return;
    // Block order.  chunk = 0: site block major (a thread's R links serve every group in
    // turn).  chunk > 0: the sites are cut into chunks of `chunk` site blocks; each chunk is
    // swept once per right-hand-side group, so the +-t and +-z neighbours of a block are
    // read while they are still in the XCD's L2.
    int sblk, gblk;
    if (chunk <= 0) {
        sblk = lb / ngb;
        gblk = lb - sblk * ngb;
    } else {
        const int ch = lb / (chunk * ngb);
        const int cs = min(chunk, nsb - ch * chunk);
        const int rem = lb - ch * chunk * ngb;
        gblk = rem / cs;
        sblk = ch * chunk + (rem - gblk * cs);
    }
    // lattice of this block (uniform: blocks never straddle lattices)
    const uint32_t s0 = (uint32_t)sblk * blockDim.x;
    int k = 0;
#pragma unroll
    for (int i = 1; i < LQT_MAXLAT; i++)
        if (i < tab.nlat && s0 >= (uint32_t)tab.off[i]) k = i;
    const int L0 = tab.L[k][0], L1 = tab.L[k][1], L2 = tab.L[k][2], L3 = tab.L[k][3];
    const uint32_t base = (uint32_t)tab.off[k];
    const uint32_t Vk = (uint32_t)(L0 * L1 * L2 * L3);
    // out = scale * ((4 + m_k - shift) in - 1/2 hop(in)): shift 0, scale 1 is the operator itself
    const C diag = (C)((tab.diag[k] - shift) * scale);
    const C hs = (C)(-0.5 * scale);
    const uint32_t s_blk = s0 + threadIdx.x;
    // G > 1: the block's links (direction mu, element i at [mu][i][256]) are staged in LDS once
    // and serve the G groups of right-hand sides the block loops over
    if constexpr (G > 1) {
#pragma unroll 4
        for (int k = 0; k < 36; k++)
            lqt_staged_links[k * 256 + threadIdx.x] =
                s_blk < V ? bld(mkrsrc(U), s_blk * 4u, (uint32_t)k * V * 4u) : hv2{(_Float16)0, (_Float16)0};
        __syncthreads();
    }
    double nrm[R];
#pragma unroll
    for (int r = 0; r < R; r++) nrm[r] = 0;
#pragma unroll 1
    for (int gi = 0; gi < G; gi++) {
        const int grp = gblk * G + gi;
        if (grp >= ngrp) break;  // uniform over the block
        // the site index is made opaque per group so that no load is hoisted out of the loop
        // (hoisted, a site's 72 link words would live in registers across the groups)
        uint32_t s = s_blk;
        if constexpr (G > 1) asm volatile("" : "+v"(s));
        const int r0 = grp * R;
        const int nr = min(R, nrhs - r0);
        const S* inb[R];
        const S* bb[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int rr = min(r0 + r, nrhs - 1);
            const long long f = act ? act[rr] : rr;
            inb[r] = in + f * in_stride;
            bb[r] = (EPI == 1) ? bvec + f * in_stride : nullptr;
        }
        if (s < V) {
            const uint32_t sl = s - base;  // site within lattice k
            cpx<C> acc[R][12];
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int c = 0; c < 12; c++) acc[r][c] = {0, 0};
            const bool pad = sl >= Vk;
            if (!pad) {
                const int x = sl % L0;
                const int y = (sl / L0) % L1;
                const int z = (sl / (L0 * L1)) % L2;
                const int t = sl / (L0 * L1 * L2);
                const int s1 = L0, s2 = L0 * L1, s3 = L0 * L1 * L2;
                const uint32_t xf = (x == L0 - 1) ? s - (L0 - 1) : s + 1;
                const uint32_t xb = (x == 0) ? s + (L0 - 1) : s - 1;
                const uint32_t yf = (y == L1 - 1) ? s - (L1 - 1) * s1 : s + s1;
                const uint32_t yb = (y == 0) ? s + (L1 - 1) * s1 : s - s1;
                const uint32_t zf = (z == L2 - 1) ? s - (L2 - 1) * s2 : s + s2;
                const uint32_t zb = (z == 0) ? s + (L2 - 1) * s2 : s - s2;
                const uint32_t tf = (t == L3 - 1) ? s - (L3 - 1) * s3 : s + s3;
                const uint32_t tb = (t == 0) ? s + (L3 - 1) * s3 : s - s3;
                if constexpr (PKH) {
                    const uint32_t nf[4] = {xf, yf, zf, tf}, nbk[4] = {xb, yb, zb, tb};
                    brsrc inr[R];
#pragma unroll
                    for (int r = 0; r < R; r++) inr[r] = mkrsrc(inb[r]);
                    hop_all_pk<DAG, R, (G > 1)>(mkrsrc(U), inr, V, s, nf, nbk, g5in, acc, s0);
                } else {
                    hop_dir<0, DAG, R, S, C>(U, inb, V, s, xf, xb, g5in, acc);
                    hop_dir<1, DAG, R, S, C>(U, inb, V, s, yf, yb, g5in, acc);
                    hop_dir<2, DAG, R, S, C>(U, inb, V, s, zf, zb, g5in, acc);
                    hop_dir<3, DAG, R, S, C>(U, inb, V, s, tf, tb, g5in, acc);
                }
            }
#pragma unroll
            for (int r = 0; r < R; r++) {
                if (r < nr) {
                    cpx<C> p[12];
                    if (!pad) {
                        if constexpr (PKH) {
#pragma unroll
                            for (int c = 0; c < 12; c++) {
                                hv2 w = bld(mkrsrc(inb[r]), s * 4u, (uint32_t)c * V * 4u);
                                if (g5in && c >= 6) w = -w;
                                p[c] = {(C)(float)w.x, (C)(float)w.y};
                            }
                        } else {
                            load_spinor<S, C>(inb[r], V, s, g5in, p);
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < 12; c++) p[c] = {0, 0};
                    }
                    S* o = out + (long long)(r0 + r) * out_stride;  // uniform
#pragma unroll
                    for (int c = 0; c < 12; c++) {
                        cpx<C> v = {fm(diag, p[c].x, hs * acc[r][c].x), fm(diag, p[c].y, hs * acc[r][c].y)};
                        if (g5out && c >= 6) {
                            v.x = -v.x;
                            v.y = -v.y;
                        }
                        if (EPI == 1) {
                            const cpx<C> b = ld_c<C>(at(bb[r], c * V + s));
                            v.x = b.x - v.x;
                            v.y = b.y - v.y;
                            nrm[r] += (double)v.x * v.x + (double)v.y * v.y;
                        }
                        if constexpr (PKH)
                            bst(mkrsrc(o), hv2{(_Float16)v.x, (_Float16)v.y}, s * 4u, (uint32_t)c * V * 4u);
                        else
                            st_c<C>(at(o, c * V + s), v);
                    }
                }
            }
        }
    }  // groups of the block
    if (EPI == 1) {
        const int r0 = gblk * R;  // G == 1
        // deterministic block reduction of |r|^2 per right-hand side
        __shared__ double red[256];
#pragma unroll
        for (int r = 0; r < R; r++) {
            red[threadIdx.x] = nrm[r];
            __syncthreads();
            for (int w = blockDim.x / 2; w > 0; w >>= 1) {
                if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0 && r0 + r < nrhs) part[(long long)(r0 + r) * nsb + sblk] = red[0];
            __syncthreads();
        }
    }
}

template <typename S, int R, bool PKH = false, int G = 1>
static void launch_R(lqt_ctx* c, int op, const S* U, const S* in, S* out, int nrhs, long long is, long long os,
                     int bs, int chunk, double shift, double scale) {
    const Geom& g = c->g;
    int nsb = (g.V + bs - 1) / bs;
    int ngrp = (nrhs + R - 1) / R;
    int nl = nsb * ((ngrp + G - 1) / G);
    if (G > 1) LQT_CHECK(bs == 256, LQT_EINVAL, "staged-link operator: 256-site blocks only");
#define LQT_DSLASH_OP(OPK)                                                                                   \
    hipLaunchKernelGGL((k_dslash<S, R, OPK, 0, PKH, G>), dim3(xcd_grid(nl)), dim3(bs), G > 1 ? 36 * 256 * 4 : 0,     \
                       c->stream, U, in, out,                                                                    \
                       (const S*)nullptr, (double*)nullptr, (const int*)nullptr, g.lat, nrhs, is, os, chunk, shift,  \
                       scale)
    switch (op) {
        case LQT_A_DAG: LQT_DSLASH_OP(LQT_A_DAG); break;
        case LQT_A_G5: LQT_DSLASH_OP(LQT_A_G5); break;
        case LQT_G5_A: LQT_DSLASH_OP(LQT_G5_A); break;
        default: LQT_DSLASH_OP(LQT_A); break;
    }
#undef LQT_DSLASH_OP
    LQT_HIP(hipGetLastError());
}

template <typename S>
static const S* gauge_of(lqt_ctx* c);
template <>
const double2* gauge_of<double2>(lqt_ctx* c) {
    return c->U[LQT_F64].as<double2>();
}
template <>
const float2* gauge_of<float2>(lqt_ctx* c) {
    return c->U[LQT_F32].as<float2>();
}
template <>
const h2* gauge_of<h2>(lqt_ctx* c) {
    return c->U[LQT_F16].as<h2>();
}
template <>
const b2* gauge_of<b2>(lqt_ctx* c) {
    return c->U[LQT_BF16].as<b2>();
}

template <typename S>
static void launch_prec(lqt_ctx* c, int op, const void* in, void* out, int nrhs, long long is, long long os,
                        const Tuned& t, double shift, double scale) {
    const S* U = gauge_of<S>(c);
    switch (t.rhs_per_thread) {
        case 1: launch_R<S, 1>(c, op, U, (const S*)in, (S*)out, nrhs, is, os, t.block, t.chunk, shift, scale); break;
        case 2: launch_R<S, 2>(c, op, U, (const S*)in, (S*)out, nrhs, is, os, t.block, t.chunk, shift, scale); break;
        default: launch_R<S, 4>(c, op, U, (const S*)in, (S*)out, nrhs, is, os, t.block, t.chunk, shift, scale); break;
    }
}

long long tune_key(int prec, int nrhs) { return ((long long)prec << 32) | (unsigned)nrhs; }

static Tuned default_tile(int prec, int nrhs) {
    Tuned t;
    t.block = 256;
    t.chunk = 0;
    if (prec == LQT_F64)
        t.rhs_per_thread = nrhs >= 2 ? 2 : 1;
    else
        t.rhs_per_thread = nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1);
    return t;
}

template <int G>
static void launch_pkh(lqt_ctx* c, int op, const void* in, void* out, int nrhs, long long is, long long os,
                       const Tuned& t, double shift, double scale) {
    const h2* U = gauge_of<h2>(c);
    switch (t.rhs_per_thread) {
        case 1:
            launch_R<h2, 1, true, G>(c, op, U, (const h2*)in, (h2*)out, nrhs, is, os, t.block, t.chunk, shift, scale);
            break;
        case 2:
            launch_R<h2, 2, true, G>(c, op, U, (const h2*)in, (h2*)out, nrhs, is, os, t.block, t.chunk, shift, scale);
            break;
        default:
            launch_R<h2, 4, true, G>(c, op, U, (const h2*)in, (h2*)out, nrhs, is, os, t.block, t.chunk, shift, scale);
            break;
    }
}

static void dslash_cfg(lqt_ctx* c, int prec, int op, const void* in, void* out, int nrhs, long long is, long long os,
                       Tuned t, double shift = 0.0, double scale = 1.0) {
    if (t.kind == 1) {
        dslash_mf(c, prec, op, in, out, nrhs, is, os, t, shift, scale);
        return;
    }
    if (t.kind == 4) {
        LQT_CHECK(prec == LQT_F16, LQT_EINVAL, "streaming dslash: FP16 storage only");
        launch_tstream<1>(c, op, in, out, nrhs, is, os, shift, scale);
        return;
    }
    if (t.kind == 2 || t.kind == 3) {
        LQT_CHECK(prec == LQT_F16, LQT_EINVAL, "packed half-precision dslash: FP16 storage only");
        if (t.kind == 2)
            launch_pkh<1>(c, op, in, out, nrhs, is, os, t, shift, scale);
        else
            launch_pkh<8>(c, op, in, out, nrhs, is, os, t, shift, scale);
        return;
    }
    switch (prec) {
        case LQT_F64: launch_prec<double2>(c, op, in, out, nrhs, is, os, t, shift, scale); break;
        case LQT_F32: launch_prec<float2>(c, op, in, out, nrhs, is, os, t, shift, scale); break;
        case LQT_F16: launch_prec<h2>(c, op, in, out, nrhs, is, os, t, shift, scale); break;
        default: launch_prec<b2>(c, op, in, out, nrhs, is, os, t, shift, scale); break;
    }
}

// The tile for (prec, nrhs): the tuned one, else (a solve's active set shrinks as its systems
// converge) the tile tuned for the nearest larger batch of the same precision, else the nearest
// smaller one, narrowed to at most nrhs fields per thread; the default tile when none is tuned.
static Tuned tile_for(const lqt_ctx* c, int prec, int nrhs) {
    auto it = c->tuned.find(tune_key(prec, nrhs));
    if (it != c->tuned.end()) return it->second;
    const long long lo_key = tune_key(prec, 0), hi_key = tune_key(prec + 1, 0);
    const Tuned* pick = nullptr;
    auto up = c->tuned.lower_bound(tune_key(prec, nrhs));
    if (up != c->tuned.end() && up->first < hi_key) {
        pick = &up->second;
    } else if (up != c->tuned.begin()) {
        auto dn = std::prev(up);
        if (dn->first > lo_key && dn->first < hi_key) pick = &dn->second;
    }
    if (!pick) return default_tile(prec, nrhs);
    Tuned t = *pick;
    if (t.kind != 1 && t.kind != 4)
        while (t.rhs_per_thread > 1 && t.rhs_per_thread > nrhs) t.rhs_per_thread >>= 1;
    return t;
}

void dslash(lqt_ctx* c, int prec, int op, const void* in, void* out, int nrhs, long long in_stride,
            long long out_stride, double shift, double scale) {
    if (nrhs <= 0) return;
    const Tuned t = tile_for(c, prec, nrhs);
    c->timer.begin(c->stream, KT_DSLASH);
    dslash_cfg(c, prec, op, in, out, nrhs, in_stride, out_stride, t, shift, scale);
    const double b = (double)storage_bytes(prec) / 2;  // bytes per real
    c->timer.end(c->stream, (double)c->g.canon_sites * (72.0 * b + 48.0 * b * nrhs));
}

// Autotuner: time every (rhs per thread, block size, chunk) candidate on scratch fields and keep
// the fastest for this (precision, nrhs).
double dslash_tune(lqt_ctx* c, int prec, int nrhs, Tuned* chosen) {
    const size_t eb = storage_bytes(prec);
    const long long n = 12LL * c->g.V;
    DBuf a, b;
    a.ensure((size_t)n * nrhs * eb);
    b.ensure((size_t)n * nrhs * eb);
    LQT_HIP(hipMemsetAsync(a.p, 0, (size_t)n * nrhs * eb, c->stream));
    const int Rs[3] = {1, 2, 4};
    const int Bs[3] = {64, 128, 256};
    const int Cs[5] = {0, 16, 64, 256, 1024};  // 1024 site blocks: the whole of most lattices
    hipEvent_t e0, e1;
    LQT_HIP(hipEventCreate(&e0));
    LQT_HIP(hipEventCreate(&e1));
    double best = 1e30;
    Tuned bt = default_tile(prec, nrhs);
    // candidates: vector kernel (R right-hand sides per thread), for 16-bit storage the
    // matrix-core kernel (R groups of 4 right-hand sides per lane), for FP16 storage the
    // vector kernel with packed half-precision arithmetic (kind 2) and the same with the
    // block's links staged in LDS for 8 groups of right-hand sides (kind 3, 256-site blocks)
    std::vector<Tuned> cand;
    if (prec == LQT_F16 && tstream_fits(c->g)) {  // streaming kernel (kind 4), one rhs per thread
        Tuned t{1, 256, 0};
        t.kind = 4;
        cand.push_back(t);
    }
    for (int kind = 0; kind < 4; kind++)
        for (int ri = 0; ri < 3; ri++) {
            if (kind == 0 && (Rs[ri] > nrhs || (prec == LQT_F64 && Rs[ri] > 2))) continue;
            if ((kind == 2 || kind == 3) && (prec != LQT_F16 || Rs[ri] > nrhs)) continue;
            if (kind == 3 && nrhs <= Rs[ri]) continue;  // one group: nothing to share
            if (kind == 1 && (prec == LQT_F64 || prec == LQT_F32 || Rs[ri] > 2 || (Rs[ri] == 2 && nrhs <= 4) ||
                              !dslash_mf_fits(c->g, Rs[ri], n, n)))
                continue;
            for (int bi = 0; bi < 3; bi++)
                for (int ci = 0; ci < 5; ci++) {
                    if (kind == 3 && Bs[bi] != 256) continue;
                    Tuned t{Rs[ri], Bs[bi], Cs[ci]};
                    t.kind = kind;
                    cand.push_back(t);
                }
        }
    for (const Tuned& t : cand) {
        dslash_cfg(c, prec, LQT_A, a.p, b.p, nrhs, n, n, t);  // warm
        LQT_HIP(hipEventRecord(e0, c->stream));
        const int reps = 5;
        for (int k = 0; k < reps; k++) dslash_cfg(c, prec, LQT_A, a.p, b.p, nrhs, n, n, t);
        LQT_HIP(hipEventRecord(e1, c->stream));
        LQT_HIP(hipEventSynchronize(e1));
        float ms = 0;
        LQT_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms / reps < best) {
            best = ms / reps;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tuned[tune_key(prec, nrhs)] = bt;
    if (chosen) *chosen = bt;
    return best;
}

// r = b - A x for nrhs FP64 fields (device layout), rnorm2[r] = |r|^2 (device).
__global__ void k_sum_partials(const double* __restrict__ part, int nparts, int nrhs, double* __restrict__ out) {
    __shared__ double red[256];
    int r = blockIdx.x;
    double s = 0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[(long long)r * nparts + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && r < nrhs) out[r] = red[0];
}

// FP64 residual launch with R right-hand sides per thread and block order `chunk`
// (256-site blocks: the per-lattice norm sums need blocks aligned to the lattices).
static void residual_launch(lqt_ctx* c, const double2* b, const double2* x, double2* r, double* part, const int* act,
                            int nrhs, int R, int chunk) {
    const Geom& g = c->g;
    const int nsb = (g.V + 255) / 256;
    const long long n = 12LL * g.V;
    const int ngrp = (nrhs + R - 1) / R;
    if (R == 2)
        hipLaunchKernelGGL((k_dslash<double2, 2, LQT_A, 1>), dim3(xcd_grid(nsb * ngrp)), dim3(256), 0, c->stream,
                           c->U[LQT_F64].as<double2>(), x, r, b, part, act, g.lat, nrhs, n, n, chunk, 0.0, 1.0);
    else
        hipLaunchKernelGGL((k_dslash<double2, 1, LQT_A, 1>), dim3(xcd_grid(nsb * ngrp)), dim3(256), 0, c->stream,
                           c->U[LQT_F64].as<double2>(), x, r, b, part, act, g.lat, nrhs, n, n, chunk, 0.0, 1.0);
    LQT_HIP(hipGetLastError());
}

static long long resid_key(int nrhs) { return (100LL << 32) | (unsigned)nrhs; }

void residual64(lqt_ctx* c, const double2* b, const double2* x, double2* r, double* rnorm2, int nrhs,
                const int* act, double* rnorm2_lat) {
    if (nrhs <= 0) return;
    const Geom& g = c->g;
    const int nsb = (g.V + 255) / 256;
    c->scratch[7].ensure(sizeof(double) * (size_t)nsb * nrhs);
    double* part = c->scratch[7].as<double>();
    auto it = c->tuned.find(resid_key(nrhs));
    if (it == c->tuned.end()) it = c->tuned.find(resid_key(0));  // the last tuned batch size
    const Tuned t = it != c->tuned.end() ? it->second : Tuned{1, 256, 0};
    c->timer.begin(c->stream, KT_RESID);
    residual_launch(c, b, x, r, part, act, nrhs, t.rhs_per_thread, t.chunk);
    hipLaunchKernelGGL(k_sum_partials, dim3(nrhs), dim3(256), 0, c->stream, part, nsb, nrhs, rnorm2);
    LQT_HIP(hipGetLastError());
    if (rnorm2_lat) sum_partials_lattices(c, part, nsb, nrhs, rnorm2_lat);
    // links once; x, b read and r written per right-hand side (FP64)
    c->timer.end(c->stream, (double)g.canon_sites * (72.0 * 8 + 72.0 * 8 * nrhs));
}

// Autotuner of the FP64 residual for nrhs right-hand sides: (R, chunk) on scratch fields.
double residual_tune(lqt_ctx* c, int nrhs) {
    const long long n = 12LL * c->g.V;
    const int nsb = (c->g.V + 255) / 256;
    DBuf xb, bb, rb, pb;
    xb.ensure(sizeof(double2) * (size_t)n * nrhs);
    bb.ensure(sizeof(double2) * (size_t)n * nrhs);
    rb.ensure(sizeof(double2) * (size_t)n * nrhs);
    pb.ensure(sizeof(double) * (size_t)nsb * nrhs);
    LQT_HIP(hipMemsetAsync(xb.p, 0, sizeof(double2) * (size_t)n * nrhs, c->stream));
    LQT_HIP(hipMemsetAsync(bb.p, 0, sizeof(double2) * (size_t)n * nrhs, c->stream));
    hipEvent_t e0, e1;
    LQT_HIP(hipEventCreate(&e0));
    LQT_HIP(hipEventCreate(&e1));
    double best = 1e30;
    Tuned bt{1, 256, 0};
    const int Rs[2] = {1, 2}, Cs[5] = {0, 16, 64, 256, 1024};
    for (int R : Rs) {
        if (R > nrhs) continue;
        for (int ch : Cs) {
            residual_launch(c, bb.as<double2>(), xb.as<double2>(), rb.as<double2>(), pb.as<double>(), nullptr, nrhs, R,
                            ch);  // warm
            LQT_HIP(hipEventRecord(e0, c->stream));
            for (int k = 0; k < 3; k++)
                residual_launch(c, bb.as<double2>(), xb.as<double2>(), rb.as<double2>(), pb.as<double>(), nullptr,
                                nrhs, R, ch);
            LQT_HIP(hipEventRecord(e1, c->stream));
            LQT_HIP(hipEventSynchronize(e1));
            float ms = 0;
            LQT_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms / 3 < best) {
                best = ms / 3;
                bt = Tuned{R, 256, ch};
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tuned[resid_key(nrhs)] = bt;
    c->tuned[resid_key(0)] = bt;
    return best;
}

}  // namespace lqt
