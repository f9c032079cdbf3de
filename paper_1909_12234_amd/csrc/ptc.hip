// Gauge-equivariant parallel-transport network used as a right preconditioner.
//
// A field with F features holds F colour 3-vectors per site, laid out like a spinor:
// [rhs][3f + colour][V] (so the 4 spin components of a spinor are its 4 input features).
// Layer l maps F_in -> F_out features:
//   out_f(x) = sum_{p=0..8} sum_g W[p][f][g] (T_p v_g)(x),
//   T_0 = 1, (T_{1+2mu} v)(x) = U_mu(x) v(x+mu), (T_{2+2mu} v)(x) = U_mu(x-mu)^+ v(x-mu),
// with the links of the operator (antiperiodic sign folded in), so the layer commutes with
// gauge transformations.  The adjoint of a layer is a layer with path-swapped (+mu <-> -mu),
// conjugate-transposed weights, which gives the backward pass.  Arithmetic is FP32: the
// transports on the vector units, the channel mixing on the matrix cores; the weights live
// on the device in BF16 (rounded once when set).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "blas.h"
#include "gemm.h"
#include "lqt_internal.h"
#include "ptc.h"
#include "solver.h"

namespace lqt {

template <typename S>
__device__ __forceinline__ float2 pld(const S* p) {
    if constexpr (sizeof(S) == 16) {
        double2 v = *(const double2*)p;
        return make_float2((float)v.x, (float)v.y);
    } else {
        return io<S>::ld(p);
    }
}
template <typename S>
__device__ __forceinline__ void pst(S* p, float2 v) {
    if constexpr (sizeof(S) == 16)
        *(double2*)p = make_double2(v.x, v.y);
    else
        io<S>::st(p, v);
}

typedef float pf4 __attribute__((ext_vector_type(4)));

// 4 x 4 transpose of 16-lane rows over four registers: on return r[t] holds, in lane row q,
// what r[q] held in lane row t (two 32-lane swaps, then two 16-lane swaps).
__device__ __forceinline__ void rows_transpose4(float (&r)[4]) {
    auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(r[0]), __float_as_uint(r[2]), false, false);
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(r[1]), __float_as_uint(r[3]), false, false);
    auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
    auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
    r[0] = __uint_as_float(c[0]);
    r[1] = __uint_as_float(c[1]);
    r[2] = __uint_as_float(d[0]);
    r[3] = __uint_as_float(d[1]);
}

// The A operand of the channel-mixing products of one layer, FI -> FO features:
// WA[p][h][lane] = (A of product 2h, A of product 2h + 1) for path p, input-feature group h
// (features 4h..4h+3) and the lane's matrix position (row lane % 16, K slot lane / 16).
// Row 2f + oc is output feature f, re (oc = 0) or im (oc = 1), zero for f >= FO; K slot q of
// product 2h + ic is input feature 4h + q, re (ic = 0) or im (ic = 1).  For the complex
// weight w = W[p][f][g]: (re, re) and (im, im) take Re w, (re, im) -Im w, (im, re) Im w.
template <int FI, int FO>
__global__ __launch_bounds__(256) void k_ptc_aprep(const float2* __restrict__ Wg, float2* __restrict__ WA) {
    constexpr int NH = FI / 4;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 9 * NH * 64) return;
    const int l = i % 64, h = (i / 64) % NH, p = i / (64 * NH);
    const int f = (l & 15) >> 1, oc = l & 1, g = 4 * h + (l >> 4);
    float a[2] = {0.f, 0.f};
    if (f < FO) {
        const float2 w = Wg[(p * FO + f) * FI + g];
        for (int ic = 0; ic < 2; ic++) a[ic] = (oc == ic) ? w.x : (oc ? w.y : -w.y);
    }
    WA[i] = make_float2(a[0], a[1]);
}

// element i of an array through a wave-uniform base and a 32-bit byte offset (the load takes
// a scalar base and a vector offset)
template <typename S>
__device__ __forceinline__ const S* ptc_at(const S* base, uint32_t i) {
    return (const S*)((const char*)base + i * (uint32_t)sizeof(S));
}

// Neighbour of the lane's site sc along path p (1 + 2 mu: +mu, 2 + 2 mu: -mu; 0: sc itself),
// from the boundary bits lo/hi (bit mu set where the coordinate is 0 / L_mu - 1).
__device__ __forceinline__ uint32_t ptc_nbr(int p, uint32_t sc, uint32_t lo, uint32_t hi, const uint32_t (&st)[4],
                                            const int (&Ls)[4]) {
    if (p == 0) return sc;
    const int mu = (p - 1) >> 1;
    const uint32_t wrap = (uint32_t)(Ls[mu] - 1) * st[mu];
    if (((p - 1) & 1) == 0) return ((hi >> mu) & 1u) ? sc - wrap : sc + st[mu];
    return ((lo >> mu) & 1u) ? sc + wrap : sc - st[mu];
}

// the link of path p (1..8) at the lane's site: U_mu(x) forward, U_mu(x - mu) backward
struct PtcLink {
    float2 u[9];
};
__device__ __forceinline__ void ptc_load_link(PtcLink& L, int p, const float2* __restrict__ U, uint32_t V,
                                              uint32_t sc, uint32_t ns) {
    const int mu = (p - 1) >> 1;
    const uint32_t ls = (((p - 1) & 1) == 0) ? sc : ns;
#pragma unroll
    for (int k = 0; k < 9; k++) L.u[k] = *ptc_at(U, (uint32_t)(mu * 9 + k) * V + ls);
}

// 4 input features (the group that vb points at) at the neighbour ns, and the A operands wa
// of the group's 2 products on path p
template <typename SI>
struct PtcVec {
    float2 v[4][3];
    float2 wa;
};
template <typename SI>
__device__ __forceinline__ void ptc_load_vec(PtcVec<SI>& B, const SI* __restrict__ vb, uint32_t qoff, uint32_t V,
                                             uint32_t ns, const float2* __restrict__ wa) {
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int b = 0; b < 3; b++) B.v[k][b] = pld<SI>(ptc_at(vb, qoff + (uint32_t)(3 * k + b) * V + ns));
    B.wa = *wa;
}

// Transport and mix one feature group on path p: colour by colour, the 4 transported
// features (path 0: the features themselves) go through the lane-row transpose into the 2
// products (re, im) of each of the 4 fields.
template <typename SI>
__device__ __forceinline__ void ptc_comp(const PtcLink& L, const PtcVec<SI>& B, int p, pf4 (&acc)[4][3]) {
    const bool fwd = ((p - 1) & 1) == 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        float2 tv[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (p == 0) {
                tv[k] = B.v[k][a];
            } else {
                float re = 0.f, im = 0.f;
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    // forward: U[a][b]; backward: conj(U[b][a])
                    const float lx = fwd ? L.u[3 * a + b].x : L.u[3 * b + a].x;
                    const float ly = fwd ? L.u[3 * a + b].y : -L.u[3 * b + a].y;
                    re = fmaf(lx, B.v[k][b].x, fmaf(-ly, B.v[k][b].y, re));
                    im = fmaf(lx, B.v[k][b].y, fmaf(ly, B.v[k][b].x, im));
                }
                tv[k] = make_float2(re, im);
            }
        }
#pragma unroll
        for (int c = 0; c < 2; c++) {
            float bt[4];
#pragma unroll
            for (int k = 0; k < 4; k++) bt[k] = c ? tv[k].y : tv[k].x;
            rows_transpose4(bt);
#pragma unroll
            for (int k = 0; k < 4; k++)
                acc[k][a] = __builtin_amdgcn_mfma_f32_16x16x4f32(c ? B.wa.y : B.wa.x, bt[k], acc[k][a], 0, 0, 0);
        }
    }
}

// One layer, FI -> FO features.  A wave takes 16 consecutive sites (matrix column c = lane
// % 16) of 4 fields (lane row q = lane / 16 is field 4 rg + q).  For each group of 4 input
// features and each path, every lane transports the group of its own (site, field) on the
// vector units (one link load serves the 4 fields); the channel mixing is a real matrix
// product on the matrix cores, 16 x 16 x 4 in FP32, with
//   rows 2f + c (output feature f, c = re/im; rows past 2 FO are zero),
//   columns the 16 sites, one product chain per field and colour,
//   K over (path, input feature, re/im): product 2h + c takes the features 4h + q in K slot q.
// A 4 x 4 transpose of lane rows turns the per-(site, field) values into the B operands of
// the 4 fields.  The accumulator of lane (c, q) for field t holds output features 2q, 2q + 1
// (re, im) of site c.  Lanes past the lattice or the last field load from a valid clamped
// (site, field): their values only reach matrix columns that are not stored.  Waves walk
// (site chunk, field group) with the chunk fastest, and the blocks are renumbered so each
// XCD takes a contiguous range: the neighbour rows a wave reads are those that concurrent
// waves on the same L2 read as their own.  The loads of the next step are issued before the
// current step computes.  FP32 links [mu][ab][V].  Byte offsets within 4
// fields are 32-bit (4 * 3 FI * V * sizeof(SI) < 4 GiB, checked by the caller).
// 4 waves per SIMD for the inference layers (FP32/16-bit fields: 128 registers, no spills);
// 3 for the FP64-activation training layers, which would spill at 4
template <int FI, int FO, typename SI, typename SO>
__global__ __launch_bounds__(256, (sizeof(SI) == 16 || sizeof(SO) == 16) ? 3 : 4) void k_ptc_layer(const float2* __restrict__ U, const SI* __restrict__ in,
                                                   SO* __restrict__ out, const float2* __restrict__ WA, int nrhs,
                                                   int L0, int L1, int L2, int L3) {
    static_assert(FI == 4 || FI == 8, "4 or 8 input features");
    static_assert(FO == 4 || FO == 8, "4 or 8 output features");
    constexpr int NH = FI / 4;  // input-feature groups
    const uint32_t V = (uint32_t)(L0 * L1 * L2 * L3);
    const int nchunk = (int)((V + 15) >> 4);
    const int lb = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);  // gridDim.x % 8 == 0
    const int task = __builtin_amdgcn_readfirstlane(lb * 4 + (int)(threadIdx.x >> 6));
    const int rg = task / nchunk, chunk = task - rg * nchunk;
    if (4 * rg >= nrhs) return;  // whole wave past the last field
    const int lane = threadIdx.x & 63, q = lane >> 4;
    const uint32_t s = (uint32_t)(chunk * 16 + (lane & 15));
    const bool site_ok = s < V;
    const uint32_t sc = site_ok ? s : 0u;
    const uint32_t qoff = (4 * rg + q < nrhs ? (uint32_t)q : 0u) * (uint32_t)(FI * 3) * V;
    const SI* vb = in + (long long)(4 * rg) * FI * 3 * V;
    const int Ls[4] = {L0, L1, L2, L3};
    const uint32_t st[4] = {1u, (uint32_t)L0, (uint32_t)(L0 * L1), (uint32_t)(L0 * L1 * L2)};
    // per-lane boundary bits: bit mu of lo/hi set where the coordinate is 0 / L_mu - 1
    uint32_t lo = 0, hi = 0;
    {
        uint32_t rem = sc;
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            const uint32_t cm = rem % (uint32_t)Ls[mu];
            rem /= (uint32_t)Ls[mu];
            lo |= (cm == 0u) << mu;
            hi |= (cm == (uint32_t)(Ls[mu] - 1)) << mu;
        }
    }
    pf4 acc[4][3];
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int a = 0; a < 3; a++) acc[k][a] = pf4{0.f, 0.f, 0.f, 0.f};
    // paths p = 0..8, each over the NH feature groups; the next (path, group)'s loads are in
    // flight while the current one computes, the links loaded once per path
    PtcLink L[2];
    PtcVec<SI> B[2];
    ptc_load_vec<SI>(B[0], vb, qoff, V, sc, WA + lane);
#pragma unroll
    for (int p = 0; p < 9; p++) {
        const PtcLink& Lc = L[p & 1];
        const uint32_t nn = ptc_nbr(p + 1 < 9 ? p + 1 : 0, sc, lo, hi, st, Ls);
        if (NH == 2) {
            ptc_load_vec<SI>(B[1], vb + 12 * V, qoff, V, ptc_nbr(p, sc, lo, hi, st, Ls), WA + (p * 2 + 1) * 64 + lane);
            ptc_comp<SI>(Lc, B[0], p, acc);
            if (p + 1 < 9) {
                ptc_load_link(L[(p + 1) & 1], p + 1, U, V, sc, nn);
                ptc_load_vec<SI>(B[0], vb, qoff, V, nn, WA + (p + 1) * 2 * 64 + lane);
            }
            ptc_comp<SI>(Lc, B[1], p, acc);
        } else {
            if (p + 1 < 9) {
                ptc_load_link(L[(p + 1) & 1], p + 1, U, V, sc, nn);
                ptc_load_vec<SI>(B[(p + 1) & 1], vb, qoff, V, nn, WA + (p + 1) * 64 + lane);
            }
            ptc_comp<SI>(Lc, B[p & 1], p, acc);
        }
    }
    if (2 * q < FO && site_ok) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (4 * rg + k >= nrhs) break;
            SO* vo = out + (long long)(4 * rg + k) * FO * 3 * V;
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int hh = 0; hh < 2; hh++)
                    pst<SO>(vo + (3 * (2 * q + hh) + a) * V + s, make_float2(acc[k][a][2 * hh], acc[k][a][2 * hh + 1]));
        }
    }
}

// Transport only, all nine paths: out[p][g] = T_p in_g (FP64 fields [g][colour][V] in,
// [p][g][colour][V] out; grid (site blocks, F, 9)), used for the weight gradients.
__global__ __launch_bounds__(256) void k_transport9(const double2* __restrict__ U, const double2* __restrict__ in,
                                                    double2* __restrict__ out, int F, int L0, int L1, int L2, int L3) {
    const int V = L0 * L1 * L2 * L3;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const int g = blockIdx.y, p = blockIdx.z;
    const int x = s % L0, y = (s / L0) % L1, z = (s / (L0 * L1)) % L2, t = s / (L0 * L1 * L2);
    const int st[4] = {1, L0, L0 * L1, L0 * L1 * L2};
    const int co[4] = {x, y, z, t};
    const int Ls[4] = {L0, L1, L2, L3};
    const double2* vin = in + (long long)3 * g * V;
    double2* vo = out + ((long long)p * F + g) * 3 * V;
    if (p == 0) {
        for (int a = 0; a < 3; a++) vo[(long long)a * V + s] = vin[(long long)a * V + s];
        return;
    }
    const int mu = (p - 1) >> 1;
    const bool fwd = ((p - 1) & 1) == 0;
    int ns;
    if (fwd)
        ns = (co[mu] == Ls[mu] - 1) ? s - (Ls[mu] - 1) * st[mu] : s + st[mu];
    else
        ns = (co[mu] == 0) ? s + (Ls[mu] - 1) * st[mu] : s - st[mu];
    const int ls = fwd ? s : ns;
    double2 u[9], v[3];
    for (int i = 0; i < 9; i++) u[i] = U[(long long)(mu * 9 + i) * V + ls];
    for (int b = 0; b < 3; b++) v[b] = vin[(long long)b * V + ns];
    for (int a = 0; a < 3; a++) {
        double re = 0, im = 0;
        for (int b = 0; b < 3; b++) {
            const double2 l = fwd ? u[3 * a + b] : make_double2(u[3 * b + a].x, -u[3 * b + a].y);
            re += l.x * v[b].x - l.y * v[b].y;
            im += l.x * v[b].y + l.y * v[b].x;
        }
        vo[(long long)a * V + s] = make_double2(re, im);
    }
}

// delta = (a - e) * wq[q] for pair q (grid (256, np)); part[q*256 + b] = partial |a - e|^2
__global__ __launch_bounds__(256) void k_ptc_delta(const double2* __restrict__ a, const double2* __restrict__ e,
                                                   const double* __restrict__ wq, long long n,
                                                   double2* __restrict__ del, double* __restrict__ part) {
    __shared__ double red[256];
    const int q = blockIdx.y;
    const double w = wq[q];
    double acc = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const double2 av = a[q * n + i], ev = e[q * n + i];
        const double dx = av.x - ev.x, dy = av.y - ev.y;
        acc += dx * dx + dy * dy;
        del[q * n + i] = make_double2(dx * w, dy * w);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)q * gridDim.x + blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- host side
// four layers, 12 -> 24 -> 24 -> 24 -> 12 complex channels (4 -> 8 -> 8 -> 8 -> 4 features)
const int FEATS[5] = {4, 8, 8, 8, 4};

int ptc_weight_count() {
    int n = 0;
    for (int l = 0; l < NL; l++) n += 9 * FEATS[l] * FEATS[l + 1];
    return n;  // complex entries
}

static float bf16_round(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

void ptc_set(lqt_ctx* c, const float* w, bool round_bf16) {
    const int nw = ptc_weight_count();
    c->net.w.assign(w, w + 2 * nw);
    std::vector<float> dev(2 * nw);
    for (int i = 0; i < 2 * nw; i++) dev[i] = round_bf16 ? bf16_round(w[i]) : w[i];
    c->net.wf.ensure(sizeof(float) * 2 * nw);
    LQT_HIP(hipMemcpyAsync(c->net.wf.p, dev.data(), sizeof(float) * 2 * nw, hipMemcpyHostToDevice, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    c->net.set = true;
}

template <int FI, int FO, typename SI, typename SO>
static void layer_launch(lqt_ctx* c, const float2* W, const SI* in, SO* out, int nrhs) {
    const Geom& g = c->g;
    constexpr int nwa = 9 * (FI / 4) * 64;
    c->net.wa.ensure(sizeof(float2) * 9 * 2 * 64);  // the largest layer: never reallocated between layers
    float2* WA = c->net.wa.as<float2>();
    hipLaunchKernelGGL((k_ptc_aprep<FI, FO>), dim3((nwa + 255) / 256), dim3(256), 0, c->stream, W, WA);
    LQT_HIP(hipGetLastError());
    // 4 waves per block, one wave per (16-site chunk, group of 4 fields); a multiple of 8 blocks
    const long long tasks = (long long)((g.V + 15) / 16) * ((nrhs + 3) / 4);
    const long long nb = ((tasks + 3) / 4 + 7) / 8 * 8;
    if (nb > 0x7fffffffLL) throw Error{LQT_EINVAL, "net layer launch too large"};
    if ((double)4 * 3 * FI * g.V * sizeof(SI) >= 4294967296.0)
        throw Error{LQT_EINVAL, "lattice too large for the net layer's 32-bit offsets"};
    hipLaunchKernelGGL((k_ptc_layer<FI, FO, SI, SO>), dim3((unsigned)nb), dim3(256), 0, c->stream,
                       c->U[LQT_F32].as<float2>(), in, out, (const float2*)WA, nrhs, g.L[0], g.L[1], g.L[2], g.L[3]);
    LQT_HIP(hipGetLastError());
}

template <typename S>
void ptc_apply(lqt_ctx* c, const S* in, S* out, int nrhs) {
    if (nrhs <= 0) return;
    const long long V = c->g.V;
    c->net.act.ensure(sizeof(float2) * (size_t)nrhs * 24 * V * 2);
    float2* a = c->net.act.as<float2>();
    float2* b = a + (size_t)nrhs * 24 * V;
    const float2* W = c->net.wf.as<float2>();
    c->timer.begin(c->stream, KT_NET);
    layer_launch<4, 8, S, float2>(c, W, in, a, nrhs);
    W += 9 * 4 * 8;
    layer_launch<8, 8, float2, float2>(c, W, a, b, nrhs);
    W += 9 * 8 * 8;
    layer_launch<8, 8, float2, float2>(c, W, b, a, nrhs);
    W += 9 * 8 * 8;
    layer_launch<8, 4, float2, S>(c, W, a, out, nrhs);
    // algorithmic bytes: input, output and the two intermediate FP32 fields, links per layer
    c->timer.end(c->stream, (double)V * nrhs * (12.0 * sizeof(S) * 2 + 24.0 * 8 * 4) + 4.0 * 72 * 4 * V);
}

template void ptc_apply<double2>(lqt_ctx*, const double2*, double2*, int);
template void ptc_apply<float2>(lqt_ctx*, const float2*, float2*, int);
template void ptc_apply<h2>(lqt_ctx*, const h2*, h2*, int);
template void ptc_apply<b2>(lqt_ctx*, const b2*, b2*, int);

// ---------------------------------------------------------------- training
// One FP64-activation pass: forward with stored activations, loss, backward through the
// adjoint layers and weight gradients G_l[p][f][g] = sum_x conj(T_p a_{l-1,g}) delta_{l,f}.

template <int FI, int FO>
static void layer64(lqt_ctx* c, const float2* W, const double2* in, double2* out, int nrhs) {
    layer_launch<FI, FO, double2, double2>(c, W, in, out, nrhs);
}

static void layer64_dyn(lqt_ctx* c, int fi, int fo, const float2* W, const double2* in, double2* out, int nrhs) {
    if (fi == 4 && fo == 8) layer64<4, 8>(c, W, in, out, nrhs);
    else if (fi == 8 && fo == 8) layer64<8, 8>(c, W, in, out, nrhs);
    else if (fi == 8 && fo == 4) layer64<8, 4>(c, W, in, out, nrhs);
    else throw Error{LQT_EINVAL, "unsupported layer shape"};
}

// adjoint weights: W'[p'][g][f] = conj(W[p][f][g]), p' = path with the opposite direction
static std::vector<float> adjoint_weights(const float* W, int fi, int fo) {
    std::vector<float> A(2 * 9 * fi * fo);
    for (int p = 0; p < 9; p++) {
        const int pa = (p == 0) ? 0 : (((p - 1) & 1) ? p - 1 : p + 1);
        for (int f = 0; f < fo; f++)
            for (int g = 0; g < fi; g++) {
                const float* w = W + 2 * ((p * fo + f) * fi + g);
                float* o = A.data() + 2 * ((pa * fi + g) * fo + f);
                o[0] = w[0];
                o[1] = -w[1];
            }
    }
    return A;
}

// Loss sum_pairs ||M r - e||^2 / ||e||^2 and its gradient with respect to conj(W) (FP64
// fields r, e: np spinors in device layout).  grad receives 2 * ptc_weight_count() doubles.
// Forward with stored activations a_1..a_4; delta_4 = (a_4 - e)/||e||^2; delta_{l-1} =
// L_l^+ delta_l (the adjoint layer); G_l[p][f][g] = sum_x conj(T_p a_{l-1,g}) . delta_{l,f}
// from one FP64 MFMA Gram product per (layer, pair); one device-to-host copy per call.
double ptc_loss_grad(lqt_ctx* c, const double2* r, const double2* e, int np, const float* Wh, std::vector<double>& grad,
                     const std::vector<double>& enorm2) {
    const long long V = c->g.V;
    const long long n = 12 * V;
    const int nw = ptc_weight_count();
    grad.assign(2 * nw, 0.0);
    DBuf* tw = c->net.train;  // workspace kept across calls
    // weights of this pass and their adjoints
    std::vector<float> adj;
    int woff[NL];
    for (int l = 0, off = 0; l < NL; l++) {
        woff[l] = off;
        std::vector<float> a = adjoint_weights(Wh + 2 * off, FEATS[l], FEATS[l + 1]);
        adj.insert(adj.end(), a.begin(), a.end());
        off += 9 * FEATS[l] * FEATS[l + 1];
    }
    tw[0].ensure(sizeof(float) * 2 * nw);
    tw[1].ensure(sizeof(float) * 2 * nw);
    LQT_HIP(hipMemcpyAsync(tw[0].p, Wh, sizeof(float) * 2 * nw, hipMemcpyHostToDevice, c->stream));
    LQT_HIP(hipMemcpyAsync(tw[1].p, adj.data(), sizeof(float) * 2 * nw, hipMemcpyHostToDevice, c->stream));
    // activations a_1..a_4 (FP64, [pair][3F][V]) in one buffer, two delta buffers, the
    // transported inputs of one pair, the Gram blocks of every (layer, pair), small vectors
    size_t aoff[NL + 2];
    aoff[1] = 0;
    for (int l = 1; l <= NL; l++) aoff[l + 1] = aoff[l] + (size_t)np * 3 * FEATS[l] * V;
    tw[2].ensure(sizeof(double2) * aoff[NL + 1]);
    tw[3].ensure(sizeof(double2) * (size_t)np * 24 * V);
    tw[4].ensure(sizeof(double2) * (size_t)np * 24 * V);
    tw[5].ensure(sizeof(double2) * (size_t)9 * 8 * 3 * V);
    tw[6].ensure(sizeof(double2) * (size_t)np * nw);
    const int nbl = 256;
    tw[7].ensure(sizeof(double) * ((size_t)np * nbl + np));
    auto act = [&](int l) { return tw[2].as<double2>() + aoff[l]; };
    double2* G = tw[6].as<double2>();
    double* lpart = tw[7].as<double>();
    double* wq = lpart + (size_t)np * nbl;
    std::vector<double> hw(np);
    for (int q = 0; q < np; q++) hw[q] = 1.0 / enorm2[q];
    LQT_HIP(hipMemcpyAsync(wq, hw.data(), sizeof(double) * np, hipMemcpyHostToDevice, c->stream));
    const float2* Wd = tw[0].as<float2>();
    const float2* Wa = tw[1].as<float2>();
    const double2* a_prev = r;
    for (int l = 0; l < NL; l++) {
        layer64_dyn(c, FEATS[l], FEATS[l + 1], Wd + woff[l], a_prev, act(l + 1), np);
        a_prev = act(l + 1);
    }
    hipLaunchKernelGGL(k_ptc_delta, dim3(nbl, np), dim3(256), 0, c->stream, act(NL), e, wq, n,
                       tw[3].as<double2>(), lpart);
    LQT_HIP(hipGetLastError());
    int cur = 3;
    for (int l = NL; l >= 1; l--) {
        const int fi = FEATS[l - 1], fo = FEATS[l];
        const double2* ain = (l == 1) ? r : act(l - 1);
        const double2* dl = tw[cur].as<double2>();
        for (int q = 0; q < np; q++) {
            dim3 grid((unsigned)((V + 255) / 256), fi, 9);
            hipLaunchKernelGGL(k_transport9, grid, dim3(256), 0, c->stream, c->U[LQT_F64].as<double2>(),
                               ain + (size_t)q * 3 * fi * V, tw[5].as<double2>(), fi, c->g.L[0], c->g.L[1],
                               c->g.L[2], c->g.L[3]);
            LQT_HIP(hipGetLastError());
            // C[p*fi + g][f] = sum_x conj(T_p a_g) . delta_f   (vectors of length 3V)
            gemm_gram(c, tw[5].as<double2>(), 9 * fi, dl + (size_t)q * 3 * fo * V, fo,
                      G + (size_t)q * nw + woff[l - 1], 3LL * V);
        }
        if (l > 1) {  // delta_{l-1} = L_l^+ delta_l
            const int nxt = (cur == 3) ? 4 : 3;
            layer64_dyn(c, fo, fi, Wa + woff[l - 1], dl, tw[nxt].as<double2>(), np);
            cur = nxt;
        }
    }
    std::vector<double2> hG((size_t)np * nw);
    std::vector<double> hl((size_t)np * nbl);
    LQT_HIP(hipMemcpyAsync(hG.data(), G, sizeof(double2) * hG.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipMemcpyAsync(hl.data(), lpart, sizeof(double) * hl.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    double loss = 0;
    for (int q = 0; q < np; q++) {
        double lq = 0;
        for (int b = 0; b < nbl; b++) lq += hl[(size_t)q * nbl + b];
        loss += lq * hw[q];
    }
    for (int q = 0; q < np; q++)
        for (int l = 0; l < NL; l++) {
            const int fi = FEATS[l], fo = FEATS[l + 1];
            const double2* Gq = hG.data() + (size_t)q * nw + woff[l];
            for (int p = 0; p < 9; p++)
                for (int g = 0; g < fi; g++)
                    for (int f = 0; f < fo; f++) {
                        const double2 v = Gq[(p * fi + g) * fo + f];
                        double* gw = grad.data() + 2 * (woff[l] + (p * fo + f) * fi + g);
                        gw[0] += v.x;
                        gw[1] += v.y;
                    }
        }
    return loss;
}

// r = A e (FP64) for np error fields e (device layout), then the summed loss and gradient.
double ptc_pairs_loss_grad(lqt_ctx* c, const double2* e, double2* r, int np, const float* Wh,
                           std::vector<double>& grad) {
    const long long n = 12LL * c->g.V;
    dslash(c, LQT_F64, LQT_A, e, r, np, n, n);
    c->scratch[9].ensure(sizeof(double) * np);
    std::vector<double> en(np);
    norm2_fields(c, e, np, c->scratch[9].as<double>());
    LQT_HIP(hipMemcpyAsync(en.data(), c->scratch[9].p, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    for (int q = 0; q < np; q++) LQT_CHECK(en[q] > 0, LQT_EINVAL, "an error field is zero");
    return ptc_loss_grad(c, r, e, np, Wh, grad, en);
}

}  // namespace lqt

namespace {

template <typename F>
int guard(lqt_ctx* c, F&& f) {
    try {
        f();
        return LQT_OK;
    } catch (const lqt::Error& e) {
        if (c) c->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        return LQT_ENOMEM;
    } catch (...) {
        if (c) c->err = "unexpected exception";
        return LQT_EINVAL;
    }
}

}  // namespace

extern "C" {

int lqt_precond_set(lqt_ctx* c, const void* w, size_t nbytes) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(w && nbytes == sizeof(float) * 2 * (size_t)lqt::ptc_weight_count(), LQT_EINVAL,
                  "weights must be " + std::to_string(8 * lqt::ptc_weight_count()) + " bytes of complex FP32");
        const float* f = (const float*)w;
        for (int i = 0; i < 2 * lqt::ptc_weight_count(); i++) LQT_CHECK(std::isfinite(f[i]), LQT_ENAN, "weight is NaN");
        lqt::ptc_set(c, f, true);
    });
}

int lqt_precond_get(lqt_ctx* c, void* w, size_t nbytes) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->net.set, LQT_ESTATE, "no preconditioner weights");
        LQT_CHECK(w && nbytes == sizeof(float) * c->net.w.size(), LQT_EINVAL, "bad weight buffer");
        std::memcpy(w, c->net.w.data(), nbytes);
    });
}

int lqt_precond_apply(lqt_ctx* c, const double* in, double* out, int nrhs) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        LQT_CHECK(c->net.set, LQT_ESTATE, "no preconditioner weights");
        LQT_CHECK(nrhs >= 0 && (nrhs == 0 || (in && out)), LQT_EINVAL, "bad fields");
        if (nrhs == 0) return;
        const long long n = 12LL * c->g.V;
        lqt::DBuf a, b;
        a.ensure(sizeof(double2) * (size_t)nrhs * n);
        b.ensure(sizeof(double2) * (size_t)nrhs * n);
        lqt::to_device_layout(c, (const double2*)in, a.as<double2>(), nrhs);
        lqt::ptc_apply<double2>(c, a.as<double2>(), b.as<double2>(), nrhs);
        lqt::from_device_layout(c, b.as<double2>(), (double2*)out, nrhs);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

int lqt_precond_loss_grad(lqt_ctx* c, const double* e, int npairs, double* loss, double* grad) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        LQT_CHECK(c->net.set, LQT_ESTATE, "no preconditioner weights");
        LQT_CHECK(npairs >= 1 && e && loss && grad, LQT_EINVAL, "bad arguments");
        const long long n = 12LL * c->g.V;
        const int nw = lqt::ptc_weight_count();
        const int chunk = 4;
        lqt::DBuf E, R;
        E.ensure(sizeof(double2) * (size_t)chunk * n);
        R.ensure(sizeof(double2) * (size_t)chunk * n);
        std::vector<double> gsum(2 * nw, 0.0), g;
        double lsum = 0;
        for (int p0 = 0; p0 < npairs; p0 += chunk) {
            const int np = std::min(chunk, npairs - p0);
            lqt::to_device_layout(c, (const double2*)e + (size_t)p0 * n, E.as<double2>(), np);
            lsum += lqt::ptc_pairs_loss_grad(c, E.as<double2>(), R.as<double2>(), np, c->net.w.data(), g);
            for (int i = 0; i < 2 * nw; i++) gsum[i] += g[i];
        }
        *loss = lsum / npairs;
        for (int i = 0; i < 2 * nw; i++) grad[i] = gsum[i] / npairs;
    });
}

int lqt_precond_train(lqt_ctx* c, int npairs, uint64_t seed, const lqt_train_opts* opts, double* final_loss) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        LQT_CHECK(npairs >= 1, LQT_EINVAL, "npairs must be >= 1");
        LQT_CHECK(!opts || (opts->epochs >= 0 && opts->batch >= 0 && opts->lr >= 0 && opts->pair_xi >= 0 &&
                            opts->pair_xi < 1),
                  LQT_EINVAL, "bad options");
        const int epochs = (opts && opts->epochs > 0) ? opts->epochs : 4;
        const double lr = (opts && opts->lr > 0) ? opts->lr : 1e-3;
        const int batch = (opts && opts->batch > 0) ? opts->batch : 4;  // pairs per optimiser step
        const double pair_xi = opts ? opts->pair_xi : 0.0;
        const int nw = lqt::ptc_weight_count();
        const long long n = 12LL * c->g.V;
        // the training set stays resident: npairs error fields e (FP64)
        size_t fr = 0, tot = 0;
        LQT_HIP(hipMemGetInfo(&fr, &tot));
        const size_t need = sizeof(double2) * (size_t)npairs * n;
        LQT_CHECK(need <= fr / 2, LQT_ENOMEM, "training set does not fit in half of the free device memory");
        lqt::DBuf E, R, G;
        E.ensure(need);
        R.ensure(sizeof(double2) * (size_t)batch * n);
        // errors: Gaussian g, or the solver's own output e = A^{-1}_{pair_xi} g (r = A e exactly)
        const int gchunk = 16;
        if (pair_xi > 0) G.ensure(sizeof(double2) * (size_t)gchunk * n);
        for (int p0 = 0; p0 < npairs; p0 += gchunk) {
            const int np = std::min(gchunk, npairs - p0);
            double2* Ep = E.as<double2>() + (size_t)p0 * n;
            const uint64_t s0 = seed ^ (0x9E3779B97F4A7C15ull * (uint64_t)(p0 + 1));
            if (pair_xi > 0) {
                lqt::gaussian_fields(c, s0, n, np, G.as<double2>());
                lqt::SolveOpts so;
                so.prec = LQT_F32;
                lqt::solve_fields(c, G.as<double2>(), Ep, np, pair_xi, so, nullptr);
            } else {
                lqt::gaussian_fields(c, s0, n, np, Ep);
            }
        }
        // start: the identity scaled by |4+m|^{-1/4} per layer (M = 1/(4+m)) unless set
        std::vector<float> W(2 * nw, 0.0f);
        if (c->net.set) {
            W = c->net.w;
        } else {
            const float s = (float)std::pow(1.0 / std::fabs(4.0 + c->mass), 0.25);
            for (int l = 0, off = 0; l < lqt::NL; l++) {
                const int fi = lqt::FEATS[l], fo = lqt::FEATS[l + 1];
                for (int f = 0; f < std::min(fi, fo); f++) W[2 * (off + f * fi + f)] = s;  // p = 0
                off += 9 * fi * fo;
            }
        }
        std::vector<double> m1(2 * nw, 0.0), m2(2 * nw, 0.0), grad;
        const double b1 = 0.9, b2 = 0.999, eps = 1e-12;
        double loss = 0;
        long long t = 0;
        for (int ep = 0; ep < epochs; ep++) {
            double eloss = 0;
            for (int p0 = 0; p0 < npairs; p0 += batch) {
                const int np = std::min(batch, npairs - p0);
                eloss += lqt::ptc_pairs_loss_grad(c, E.as<double2>() + (size_t)p0 * n, R.as<double2>(), np,
                                                  W.data(), grad);
                t++;
                for (int i = 0; i < 2 * nw; i++) {  // Adam on the real and imaginary parts
                    const double gi = grad[i] / np;
                    m1[i] = b1 * m1[i] + (1 - b1) * gi;
                    m2[i] = b2 * m2[i] + (1 - b2) * gi * gi;
                    const double mh = m1[i] / (1 - std::pow(b1, (double)t)), vh = m2[i] / (1 - std::pow(b2, (double)t));
                    W[i] -= (float)(lr * mh / (std::sqrt(vh) + eps));
                }
            }
            loss = eloss / npairs;
            if (opts && opts->verbose) {
                fprintf(stderr, "[lqtrace] train epoch %d: mean loss %.5e\n", ep, loss);
                fflush(stderr);
            }
        }
        lqt::ptc_set(c, W.data(), true);
        if (final_loss) *final_loss = loss;
    });
}

}  // extern "C"
