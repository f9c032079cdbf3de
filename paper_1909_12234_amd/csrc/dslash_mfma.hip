// Wilson-Dirac operator on the matrix cores, for 16-bit storage (BF16 and FP16).
//
// The hopping term of A (the Wilson operator of the Dirac equation on the lattice) sums,
// over the 8 neighbours of a site, the spin matrix P_d = 1 + s g_mu (s = -1 forward, +1
// backward; swapped for A^+) times the 3x3 link W_d (U_mu(x) forward, U_mu(x-mu)^+ backward)
// applied to the neighbour spinor.  P_d couples each spin only to itself and to one partner:
// the pairs are (0,3), (1,2) for mu = x, y and (0,2), (1,3) for mu = z, t (DeGrand-Rossi
// matrices).  Restricted to one spin pair (s1, s2), one output colour a and one input colour b,
// the map from (Re, Im) psi(s1, b), psi(s2, b) to (Re, Im) out(s1, a), out(s2, a) is a real 4x4
// matrix whose entries are +-Re W[a][b] or +-Im W[a][b].  That is one block of the 16-block
// 4x4x4 matrix-core instruction: block i of the instruction is one lattice site, lane 4i+q
// holds row q of that site's block (A operand), column q of the neighbour data (B operand:
// right-hand side q) and column q of the sum.  A wave therefore covers 16 sites and 4
// right-hand sides per instruction; lanes stay on sites, so each load reads 64 contiguous
// bytes per right-hand side.  Per direction: 2 pairs x 3 x 3 colour blocks = 18 instructions.
//
// The A entries come from the stored link word w = (Re, Im) with one byte permute that picks
// the halves and their sign bytes out of w and w ^ 0x80008000 (no arithmetic), so the links
// enter the products exactly as stored.  Products are exact and sums are FP32.  The two
// direction classes (x,y and z,t) have different spin pairs and so separate accumulators,
// added in the epilogue together with the diagonal term (4 + m) psi(x).
#include "dslash_mfma.h"

#include <algorithm>
#include <type_traits>

namespace lqt {

typedef short mf_s4 __attribute__((ext_vector_type(4)));
typedef _Float16 mf_h4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef uint32_t mf_u2 __attribute__((ext_vector_type(2)));

template <typename S>
struct mf_core;
template <>
struct mf_core<b2> {
    __device__ __forceinline__ static mf_f4 mma(mf_u2 a, mf_u2 b, mf_f4 c) {
        return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(__builtin_bit_cast(mf_s4, a), __builtin_bit_cast(mf_s4, b), c,
                                                     0, 0, 0);
    }
    __device__ __forceinline__ static float lo(uint32_t w) { return __uint_as_float(w << 16); }
    __device__ __forceinline__ static float hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
};
template <>
struct mf_core<h2> {
    __device__ __forceinline__ static mf_f4 mma(mf_u2 a, mf_u2 b, mf_f4 c) {
        return __builtin_amdgcn_mfma_f32_4x4x4f16(__builtin_bit_cast(mf_h4, a), __builtin_bit_cast(mf_h4, b), c, 0, 0,
                                                 0);
    }
    __device__ __forceinline__ static float lo(uint32_t w) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
    }
    __device__ __forceinline__ static float hi(uint32_t w) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
    }
};

// ---------------------------------------------------------------- block entries
// coefficient P_d[row][col] of 1 + s g_mu as (re, im), for row and col in one spin pair
struct mf_cc {
    int re, im;
};
__host__ __device__ constexpr mf_cc mf_pcoef(int mu, int s, int row, int col) {
    if (row == col) return {1, 0};
    switch (mu) {
        case 0:  // g_x: [0][3] = [1][2] = i, [2][1] = [3][0] = -i
            return (row == 0 || row == 1) ? mf_cc{0, s} : mf_cc{0, -s};
        case 1:  // g_y: [0][3] = [3][0] = -1, [1][2] = [2][1] = 1
            return (row == 0 || row == 3) ? mf_cc{-s, 0} : mf_cc{s, 0};
        case 2:  // g_z: [0][2] = [3][1] = i, [1][3] = [2][0] = -i
            return (row == 0 || row == 3) ? mf_cc{0, s} : mf_cc{0, -s};
        default:  // g_t: [0][2] = [1][3] = [2][0] = [3][1] = 1
            return mf_cc{s, 0};
    }
}

// spin pair p of direction class cls (0: x,y; 1: z,t), member i
__host__ __device__ constexpr int mf_pair(int cls, int p, int i) {
    return cls == 0 ? (p == 0 ? (i == 0 ? 0 : 3) : (i == 0 ? 1 : 2)) : (p == 0 ? (i == 0 ? 0 : 2) : (i == 0 ? 1 : 3));
}

// Byte-permute selector giving, from S1 = w = (wr, wi) and S0 = w ^ 0x80008000, the two A
// entries of block row (spin row, reim) and column spin col: realrep(c W)[reim][0..1], where
// realrep(z) = [[Re z, -Im z], [Im z, Re z]], c = P_d[row][col], W = w (forward link) or
// conj(w) (w = U[b][a] of the backward link), times -1 for a column that gamma_5 negates.
__host__ __device__ constexpr uint32_t mf_sel(int mu, int s, bool dagger_link, bool negcol, int row, int col,
                                              int reim) {
    const mf_cc c = mf_pcoef(mu, s, row, col);
    // a real quantity is (component of w: 0 re / 1 im, negated)
    const int wr_c = 0, wr_n = 0, wi_c = 1, wi_n = dagger_link ? 1 : 0;
    int mr_c = 0, mr_n = 0, mi_c = 0, mi_n = 0;  // M = c W
    if (c.re == 1) {
        mr_c = wr_c, mr_n = wr_n, mi_c = wi_c, mi_n = wi_n;
    } else if (c.re == -1) {
        mr_c = wr_c, mr_n = !wr_n, mi_c = wi_c, mi_n = !wi_n;
    } else if (c.im == 1) {
        mr_c = wi_c, mr_n = !wi_n, mi_c = wr_c, mi_n = wr_n;
    } else {
        mr_c = wi_c, mr_n = wi_n, mi_c = wr_c, mi_n = !wr_n;
    }
    int lo_c = 0, lo_n = 0, hi_c = 0, hi_n = 0;
    if (reim == 0) {
        lo_c = mr_c, lo_n = mr_n, hi_c = mi_c, hi_n = !mi_n;
    } else {
        lo_c = mi_c, lo_n = mi_n, hi_c = mr_c, hi_n = mr_n;
    }
    if (negcol) lo_n = !lo_n, hi_n = !hi_n;
    // bytes 0-3 select from S1 = w, 4-7 from S0 = w with both sign bits flipped
    return (uint32_t)(2 * lo_c) | ((uint32_t)(2 * lo_c + 1 + 4 * lo_n) << 8) | ((uint32_t)(2 * hi_c) << 16) |
           ((uint32_t)(2 * hi_c + 1 + 4 * hi_n) << 24);
}

// the selector of this lane (q = lane & 3: row spin index q >> 1 of the pair, reim q & 1)
template <int MU, int SG, bool DAGL, bool G5IN, int CLS, int P, int J>
__device__ __forceinline__ uint32_t mf_lane_sel(bool qhi, bool qim) {
    constexpr int col = mf_pair(CLS, P, J);
    constexpr bool neg = G5IN && col >= 2;
    constexpr uint32_t s00 = mf_sel(MU, SG, DAGL, neg, mf_pair(CLS, P, 0), col, 0);
    constexpr uint32_t s01 = mf_sel(MU, SG, DAGL, neg, mf_pair(CLS, P, 0), col, 1);
    constexpr uint32_t s10 = mf_sel(MU, SG, DAGL, neg, mf_pair(CLS, P, 1), col, 0);
    constexpr uint32_t s11 = mf_sel(MU, SG, DAGL, neg, mf_pair(CLS, P, 1), col, 1);
    return qhi ? (qim ? s11 : s10) : (qim ? s01 : s00);
}

__device__ __forceinline__ uint32_t ld32(const void* base, uint32_t byte_off) {
    return *(const uint32_t*)((const char*)base + byte_off);
}

// one direction: A blocks from the link, then 18 products per group of 4 right-hand sides
template <typename S, int R, int MU, bool FWD, bool DAG, bool G5IN>
__device__ __forceinline__ void mf_hop(const S* __restrict__ Um, const S* __restrict__ inb, uint32_t V,
                                       uint32_t lsite, uint32_t nsite, const uint32_t roff[R], bool qhi, bool qim,
                                       mf_f4 (&acc)[R][2][3]) {
    constexpr int CLS = MU >= 2 ? 1 : 0;
    constexpr int SG = (FWD ? -1 : 1) * (DAG ? -1 : 1);
    constexpr bool DAGL = !FWD;
    uint32_t A[2][2][9];  // [pair][column member][a*3+b]
    {
        const uint32_t sel00 = mf_lane_sel<MU, SG, DAGL, G5IN, CLS, 0, 0>(qhi, qim);
        const uint32_t sel01 = mf_lane_sel<MU, SG, DAGL, G5IN, CLS, 0, 1>(qhi, qim);
        const uint32_t sel10 = mf_lane_sel<MU, SG, DAGL, G5IN, CLS, 1, 0>(qhi, qim);
        const uint32_t sel11 = mf_lane_sel<MU, SG, DAGL, G5IN, CLS, 1, 1>(qhi, qim);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                // forward: W[a][b] = U[a][b]; backward: W[a][b] = conj(U[b][a])
                const int e = FWD ? 3 * a + b : 3 * b + a;
                const uint32_t w = ld32(Um, ((uint32_t)e * V + lsite) * 4u);
                const uint32_t nw = w ^ 0x80008000u;
                A[0][0][3 * a + b] = __builtin_amdgcn_perm(nw, w, sel00);
                A[0][1][3 * a + b] = __builtin_amdgcn_perm(nw, w, sel01);
                A[1][0][3 * a + b] = __builtin_amdgcn_perm(nw, w, sel10);
                A[1][1][3 * a + b] = __builtin_amdgcn_perm(nw, w, sel11);
            }
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        uint32_t B[12];
#pragma unroll
        for (int c = 0; c < 12; c++) B[c] = ld32(inb, roff[r] + ((uint32_t)c * V + nsite) * 4u);
#pragma unroll
        for (int p = 0; p < 2; p++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                const mf_u2 bv = {B[3 * mf_pair(CLS, p, 0) + b], B[3 * mf_pair(CLS, p, 1) + b]};
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const mf_u2 av = {A[p][0][3 * a + b], A[p][1][3 * a + b]};
                    acc[r][p][a] = mf_core<S>::mma(av, bv, acc[r][p][a]);
                }
            }
    }
}

// out = scale ((4 + m - shift) in - 1/2 hop(in)) for op A, A^+, A g5, g5 A; right-hand sides
// grp*4R + 4r + (lane & 3); fields at in + f*in_stride, out + f*out_stride.  Padding sites
// of the lattice table get zeros.  Byte offsets of one group stay below 2^32 (checked by the
// host).
template <typename S, int R, int OPK>
__global__ __launch_bounds__(256) void k_dslash_mf(const S* __restrict__ U, const S* __restrict__ in,
                                                   S* __restrict__ out, LatTab tab, int nrhs, long long in_stride,
                                                   long long out_stride, int chunk, double shift, double scale) {
    constexpr bool DAG = OPK == LQT_A_DAG;
    constexpr bool G5IN = OPK == LQT_A_G5, G5OUT = OPK == LQT_G5_A;
    const uint32_t V = (uint32_t)tab.off[tab.nlat];
    const uint32_t spb = blockDim.x >> 2;  // sites per block: 16 per wave
    const int nsb = (int)((V + spb - 1) / spb);
    const int ngrp = (nrhs + 4 * R - 1) / (4 * R);
    const int lb = xcd_block(nsb * ngrp);
    if (lb < 0) return;
    int sblk, grp;
    if (chunk <= 0) {
        sblk = lb / ngrp;
        grp = lb - sblk * ngrp;
    } else {
        const int ch = lb / (chunk * ngrp);
        const int cs = min(chunk, nsb - ch * chunk);
        const int rem = lb - ch * chunk * ngrp;
        grp = rem / cs;
        sblk = ch * chunk + (rem - grp * cs);
    }
    const uint32_t s0 = (uint32_t)sblk * spb;
    int k = 0;
#pragma unroll
    for (int i = 1; i < LQT_MAXLAT; i++)
        if (i < tab.nlat && s0 >= (uint32_t)tab.off[i]) k = i;
    const int L0 = tab.L[k][0], L1 = tab.L[k][1], L2 = tab.L[k][2], L3 = tab.L[k][3];
    const uint32_t base = (uint32_t)tab.off[k];
    const uint32_t Vk = (uint32_t)(L0 * L1 * L2 * L3);
    const float diag = (float)((tab.diag[k] - shift) * scale);
    const float hs = (float)(-0.5 * scale);

    const int lane = threadIdx.x & 63;
    const int q = lane & 3;
    const bool qhi = (q & 2) != 0, qim = (q & 1) != 0;
    const uint32_t s = s0 + (threadIdx.x >> 6) * 16 + (lane >> 2);
    const bool inr = s < V;
    const uint32_t sc = inr ? s : V - 1;  // loads of lanes past the end stay in bounds
    const uint32_t sl = sc - base;
    const bool pad = !inr || sl >= Vk;
    uint32_t nf[4], nbk[4];
    if (!pad) {
        const int x = sl % L0;
        const int y = (sl / L0) % L1;
        const int z = (sl / (L0 * L1)) % L2;
        const int t = sl / (L0 * L1 * L2);
        const uint32_t s1 = L0, s2 = L0 * L1, s3 = L0 * L1 * L2;
        nf[0] = (x == L0 - 1) ? sc - (L0 - 1) : sc + 1;
        nbk[0] = (x == 0) ? sc + (L0 - 1) : sc - 1;
        nf[1] = (y == L1 - 1) ? sc - (L1 - 1) * s1 : sc + s1;
        nbk[1] = (y == 0) ? sc + (L1 - 1) * s1 : sc - s1;
        nf[2] = (z == L2 - 1) ? sc - (L2 - 1) * s2 : sc + s2;
        nbk[2] = (z == 0) ? sc + (L2 - 1) * s2 : sc - s2;
        nf[3] = (t == L3 - 1) ? sc - (L3 - 1) * s3 : sc + s3;
        nbk[3] = (t == 0) ? sc + (L3 - 1) * s3 : sc - s3;
    } else {
#pragma unroll
        for (int m = 0; m < 4; m++) nf[m] = nbk[m] = sc;
    }
    // right-hand sides of this lane: group base (uniform) plus a 32-bit byte offset
    const long long f0 = (long long)grp * 4 * R;
    const S* inb = in + f0 * in_stride;
    uint32_t roff[R], ooff[R];
    bool rok[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const long long f = f0 + 4 * r + q;
        rok[r] = f < nrhs;
        const long long fc = (rok[r] ? f : nrhs - 1) - f0;
        roff[r] = (uint32_t)(fc * in_stride * 4);
        ooff[r] = (uint32_t)((4 * r + q) * out_stride * 4);
    }
    mf_f4 ax[R][2][3], az[R][2][3];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int p = 0; p < 2; p++)
#pragma unroll
            for (int a = 0; a < 3; a++) ax[r][p][a] = az[r][p][a] = mf_f4{0.f, 0.f, 0.f, 0.f};
    const uint32_t V9 = 9u * V;
    mf_hop<S, R, 0, true, DAG, G5IN>(U, inb, V, sc, nf[0], roff, qhi, qim, ax);
    mf_hop<S, R, 0, false, DAG, G5IN>(U, inb, V, nbk[0], nbk[0], roff, qhi, qim, ax);
    mf_hop<S, R, 1, true, DAG, G5IN>(U + V9, inb, V, sc, nf[1], roff, qhi, qim, ax);
    mf_hop<S, R, 1, false, DAG, G5IN>(U + V9, inb, V, nbk[1], nbk[1], roff, qhi, qim, ax);
    mf_hop<S, R, 2, true, DAG, G5IN>(U + 2 * V9, inb, V, sc, nf[2], roff, qhi, qim, az);
    mf_hop<S, R, 2, false, DAG, G5IN>(U + 2 * V9, inb, V, nbk[2], nbk[2], roff, qhi, qim, az);
    mf_hop<S, R, 3, true, DAG, G5IN>(U + 3 * V9, inb, V, sc, nf[3], roff, qhi, qim, az);
    mf_hop<S, R, 3, false, DAG, G5IN>(U + 3 * V9, inb, V, nbk[3], nbk[3], roff, qhi, qim, az);

    if (!inr) return;
    S* ob = out + f0 * out_stride;
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (!rok[r]) continue;
#pragma unroll
        for (int sg = 0; sg < 4; sg++) {
            // spin sg in the x,y pairs (0,3),(1,2) and the z,t pairs (0,2),(1,3)
            const int px = (sg == 0 || sg == 3) ? 0 : 1, ix = (sg == 0 || sg == 1) ? 0 : 1;
            const int pz = (sg == 0 || sg == 2) ? 0 : 1, iz = (sg == 0 || sg == 1) ? 0 : 1;
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const int c = 3 * sg + a;
                float vr = 0.f, vi = 0.f;
                if (!pad) {
                    const uint32_t w = ld32(inb, roff[r] + ((uint32_t)c * V + sc) * 4u);
                    float pr = mf_core<S>::lo(w), pi = mf_core<S>::hi(w);
                    if (G5IN && sg >= 2) pr = -pr, pi = -pi;
                    const float hr = ax[r][px][a][2 * ix] + az[r][pz][a][2 * iz];
                    const float hi = ax[r][px][a][2 * ix + 1] + az[r][pz][a][2 * iz + 1];
                    vr = fmaf(diag, pr, hs * hr);
                    vi = fmaf(diag, pi, hs * hi);
                    if (G5OUT && sg >= 2) vr = -vr, vi = -vi;
                }
                io<S>::st((S*)((char*)ob + ooff[r] + ((uint32_t)c * V + s) * 4u), make_float2(vr, vi));
            }
        }
    }
}

bool dslash_mf_fits(const Geom& g, int R, long long in_stride, long long out_stride) {
    const double lim = 4294967295.0;
    return (double)(4 * R) * (double)std::max(in_stride, out_stride) * 4.0 + 12.0 * g.V * 4.0 < lim &&
           36.0 * g.V * 4.0 < lim;
}

template <typename S, int R>
static void launch_mf_R(lqt_ctx* c, int op, const S* U, const S* in, S* out, int nrhs, long long is, long long os,
                        int bs, int chunk, double shift, double scale) {
    const Geom& g = c->g;
    const int spb = bs / 4;
    const int nsb = (g.V + spb - 1) / spb;
    const int ngrp = (nrhs + 4 * R - 1) / (4 * R);
    const int nl = nsb * ngrp;
#define LQT_DSLASH_MF(OPK)                                                                                     \
    hipLaunchKernelGGL((k_dslash_mf<S, R, OPK>), dim3(xcd_grid(nl)), dim3(bs), 0, c->stream, U, in, out, g.lat, \
                       nrhs, is, os, chunk, shift, scale)
    switch (op) {
        case LQT_A_DAG: LQT_DSLASH_MF(LQT_A_DAG); break;
        case LQT_A_G5: LQT_DSLASH_MF(LQT_A_G5); break;
        case LQT_G5_A: LQT_DSLASH_MF(LQT_G5_A); break;
        default: LQT_DSLASH_MF(LQT_A); break;
    }
#undef LQT_DSLASH_MF
    LQT_HIP(hipGetLastError());
}

template <typename S>
static void launch_mf(lqt_ctx* c, int op, const void* in, void* out, int nrhs, long long is, long long os,
                      const Tuned& t, double shift, double scale) {
    const S* U = c->U[std::is_same<S, b2>::value ? LQT_BF16 : LQT_F16].template as<S>();
    switch (t.rhs_per_thread) {
        case 1: launch_mf_R<S, 1>(c, op, U, (const S*)in, (S*)out, nrhs, is, os, t.block, t.chunk, shift, scale); break;
        default: launch_mf_R<S, 2>(c, op, U, (const S*)in, (S*)out, nrhs, is, os, t.block, t.chunk, shift, scale); break;
    }
}

void dslash_mf(lqt_ctx* c, int prec, int op, const void* in, void* out, int nrhs, long long is, long long os,
               const Tuned& t, double shift, double scale) {
    LQT_CHECK(prec == LQT_F16 || prec == LQT_BF16, LQT_EINVAL, "matrix-core dslash: 16-bit storage only");
    LQT_CHECK(t.block == 64 || t.block == 128 || t.block == 256, LQT_EINVAL, "matrix-core dslash: bad block");
    LQT_CHECK(dslash_mf_fits(c->g, t.rhs_per_thread, is, os), LQT_EINVAL, "matrix-core dslash: fields too large");
    if (prec == LQT_BF16)
        launch_mf<b2>(c, op, in, out, nrhs, is, os, t, shift, scale);
    else
        launch_mf<h2>(c, op, in, out, nrhs, is, os, t, shift, scale);
}

}  // namespace lqt
