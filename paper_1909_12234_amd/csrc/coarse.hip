// Explicit coarse operator D_c = W^+ A W of a multigrid prolongator (Section 2: the coarse
// operator of the blocking; Algorithm 2 works with g5^W D_c).
//
// A couples a site only to itself and its 8 neighbours, so D_c couples an aggregate only to
// itself and to the aggregates one block away in +-mu: a 9-point stencil of nb x nb complex
// blocks, nb = 2 nv (chirality x near-null vector).  Stored FP64 as
//   Dc[a][slot][i][j],  slot 0: the aggregate itself, slot 1 + 2 mu: +mu, slot 2 + 2 mu: -mu,
// where slot 1 + d collects the hops of direction d that leave the aggregate and slot 0 the
// mass term and the hops that stay inside it.  (With one or two blocks along mu, several slots
// point at the same aggregate; applying the stencil sums them, which is what A does.)
//
// Build: D_c[a][slot](i, j) = sum_x W_{a,i}(x)^+ (A W_{b,j})(x), one workgroup per aggregate and
// hop direction, the hop matrix -1/2 (1 -+ g_mu) (x) U applied to the 6 non-zero entries of a
// chirality-split column; the mass term adds (4 + m) W_a^+ W_a.  Apply: per aggregate and group
// of right-hand sides, the 9 block products with the stencil blocks and the inputs staged in LDS.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>

#include "lqt_internal.h"
#include "prolong.h"

namespace lqt {

// DeGrand-Rossi gamma matrices g_mu (mu = 0..3 <-> x, y, z, t), complex 4 x 4, row-major.
__constant__ double2 kGamma[4][16] = {
    {{0, 0}, {0, 0}, {0, 0}, {0, 1}, {0, 0}, {0, 0}, {0, 1}, {0, 0},
     {0, 0}, {0, -1}, {0, 0}, {0, 0}, {0, -1}, {0, 0}, {0, 0}, {0, 0}},
    {{0, 0}, {0, 0}, {0, 0}, {-1, 0}, {0, 0}, {0, 0}, {1, 0}, {0, 0},
     {0, 0}, {1, 0}, {0, 0}, {0, 0}, {-1, 0}, {0, 0}, {0, 0}, {0, 0}},
    {{0, 0}, {0, 0}, {0, 1}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, -1},
     {0, -1}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 1}, {0, 0}, {0, 0}},
    {{0, 0}, {0, 0}, {1, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {1, 0},
     {1, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {1, 0}, {0, 0}, {0, 0}}};

constexpr int CB_MAXNB = 64;           // largest nb = 2 nv of the explicit operator
constexpr int CB_OUT = 16;             // nb^2 / 256 outputs per thread at nb = 64
constexpr int CA_R = 64;               // right-hand sides per workgroup of the apply (16 x 4)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cjmul(double2 a, double2 b) {  // conj(a) b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ void agg_coords(const PG& p, int a, int c[4]) {
    c[0] = a % p.n0;
    c[1] = (a / p.n0) % p.n1;
    c[2] = (a / (p.n0 * p.n1)) % p.n2;
    c[3] = a / (p.n0 * p.n1 * p.n2);
}
// aggregate in stencil slot `slot` of aggregate a (periodic)
__device__ __forceinline__ int agg_nbr(const PG& p, int a, int slot) {
    if (slot == 0) return a;
    int c[4];
    agg_coords(p, a, c);
    const int n[4] = {p.n0, p.n1, p.n2, p.n3};
    const int mu = (slot - 1) >> 1;
    c[mu] = ((slot - 1) & 1) ? (c[mu] + n[mu] - 1) % n[mu] : (c[mu] + 1) % n[mu];
    return c[0] + p.n0 * (c[1] + p.n1 * (c[2] + p.n2 * c[3]));
}

// One workgroup per (aggregate a, hop direction d = 2 mu + back): the hops of direction d
// from every site of a.  Hops that leave the aggregate add to Dc[a][1 + d], the others to the
// partial self block Ps[a][d].  U: FP64 links [mu][ab][V] (antiperiodic sign folded in).
__global__ __launch_bounds__(256) void k_coarse_hops(const double2* __restrict__ W, const double2* __restrict__ U,
                                                     PG p, double2* __restrict__ Dc, double2* __restrict__ Ps) {
    const int a = blockIdx.x, d = blockIdx.y;
    const int mu = d >> 1;
    const bool back = d & 1;
    const int nv = p.nv, nb = 2 * nv;
    const int tid = threadIdx.x;
    __shared__ double2 A[CB_MAXNB][6], B[CB_MAXNB][6], UW[CB_MAXNB][6], T[CB_MAXNB][12];
    __shared__ double2 L[9], P4[16];
    const int bl[4] = {p.b0, p.b1, p.b2, p.b3};
    const int Ls[4] = {p.L0, p.L1, p.L2, p.L3};
    const int bstride[4] = {1, p.b0, p.b0 * p.b1, p.b0 * p.b1 * p.b2};
    // projector -1/2 (1 - s g_mu), s = +1 forward, -1 backward
    if (tid < 16) {
        const double2 g = kGamma[mu][tid];
        const double sg = back ? -1.0 : 1.0;
        const double id = (tid % 5 == 0) ? 1.0 : 0.0;
        P4[tid] = make_double2(-0.5 * (id - sg * g.x), 0.5 * sg * g.y);
    }
    double2 acc_x[CB_OUT], acc_s[CB_OUT];
#pragma unroll
    for (int q = 0; q < CB_OUT; q++) acc_x[q] = acc_s[q] = make_double2(0, 0);
    int ac[4];
    agg_coords(p, a, ac);
    const int b_out = agg_nbr(p, a, 1 + d);
    for (int bs = 0; bs < p.bsites; bs++) {
        const int lmu = (bs / bstride[mu]) % bl[mu];
        const bool cross = back ? (lmu == 0) : (lmu == bl[mu] - 1);
        // neighbour site y and its place (aggregate, local index)
        int lc[4];
        for (int k = 0; k < 4; k++) lc[k] = (bs / bstride[k]) % bl[k];
        int g[4];
        for (int k = 0; k < 4; k++) g[k] = ac[k] * bl[k] + lc[k];
        const int x = g[0] + p.L0 * (g[1] + p.L1 * (g[2] + p.L2 * g[3]));
        g[mu] = back ? (g[mu] + Ls[mu] - 1) % Ls[mu] : (g[mu] + 1) % Ls[mu];
        const int y = g[0] + p.L0 * (g[1] + p.L1 * (g[2] + p.L2 * g[3]));
        lc[mu] = back ? (lc[mu] + bl[mu] - 1) % bl[mu] : (lc[mu] + 1) % bl[mu];
        const int bsy = lc[0] + bstride[1] * lc[1] + bstride[2] * lc[2] + bstride[3] * lc[3];
        const int by = cross ? b_out : a;
        __syncthreads();  // previous site's LDS reads are done
        // columns of W at x (aggregate a) and y (aggregate by): 6 entries per column
        for (int t = tid; t < nb * 6; t += 256) {
            const int i = t / 6, e = t % 6;
            const int ch = i / nv, v = i % nv;
            A[i][e] = W[(((long long)a * 2 + ch) * nv + v) * p.d + bs * 6 + e];
            B[i][e] = W[(((long long)by * 2 + ch) * nv + v) * p.d + bsy * 6 + e];
        }
        // link: U_mu(x) forward, U_mu(y)^+ backward
        if (tid < 9) {
            const int r = tid / 3, cc = tid % 3;
            if (!back) {
                L[tid] = U[((long long)mu * 9 + tid) * p.V + x];
            } else {
                const double2 u = U[((long long)mu * 9 + cc * 3 + r) * p.V + y];
                L[tid] = make_double2(u.x, -u.y);
            }
        }
        __syncthreads();
        // UW[j][s2'][alpha] = sum_beta L[alpha][beta] B[j][s2'][beta]
        for (int t = tid; t < nb * 6; t += 256) {
            const int j = t / 6, e = t % 6, s2 = e / 3, al = e % 3;
            double2 s = make_double2(0, 0);
            for (int be = 0; be < 3; be++) {
                const double2 q = cmul(L[al * 3 + be], B[j][s2 * 3 + be]);
                s.x += q.x;
                s.y += q.y;
            }
            UW[j][e] = s;
        }
        __syncthreads();
        // T[j][sigma][alpha] = sum_{s2'} P4[sigma][2 c_j + s2'] UW[j][s2'][alpha]
        for (int t = tid; t < nb * 12; t += 256) {
            const int j = t / 12, e = t % 12, sg = e / 3, al = e % 3;
            const int cj = j / nv;
            double2 s = make_double2(0, 0);
            for (int s2 = 0; s2 < 2; s2++) {
                const double2 q = cmul(P4[sg * 4 + 2 * cj + s2], UW[j][s2 * 3 + al]);
                s.x += q.x;
                s.y += q.y;
            }
            T[j][e] = s;
        }
        __syncthreads();
        // D(i, j) += sum_{s2, alpha} conj(A[i][s2][alpha]) T[j][2 c_i + s2][alpha]
#pragma unroll
        for (int q = 0; q < CB_OUT; q++) {
            const int o = tid + 256 * q;
            if (o < nb * nb) {
                const int i = o / nb, j = o % nb;
                const int ci = i / nv;
                double2 s = make_double2(0, 0);
                for (int e = 0; e < 6; e++) {
                    const double2 r = cjmul(A[i][e], T[j][6 * ci + e]);
                    s.x += r.x;
                    s.y += r.y;
                }
                if (cross) {
                    acc_x[q].x += s.x;
                    acc_x[q].y += s.y;
                } else {
                    acc_s[q].x += s.x;
                    acc_s[q].y += s.y;
                }
            }
        }
    }
    const long long nb2 = (long long)nb * nb;
#pragma unroll
    for (int q = 0; q < CB_OUT; q++) {
        const int o = tid + 256 * q;
        if (o < nb * nb) {
            Dc[((long long)a * 9 + 1 + d) * nb2 + o] = acc_x[q];
            Ps[((long long)a * 8 + d) * nb2 + o] = acc_s[q];
        }
    }
}

// Dc[a][0] = (4 + m) W_a^+ W_a + sum_d Ps[a][d]; one workgroup per aggregate
__global__ __launch_bounds__(256) void k_coarse_self(const double2* __restrict__ W, PG p, double diag,
                                                     const double2* __restrict__ Ps, double2* __restrict__ Dc) {
    const int a = blockIdx.x;
    const int nv = p.nv, nb = 2 * nv;
    const long long nb2 = (long long)nb * nb;
    for (int o = threadIdx.x; o < nb * nb; o += 256) {
        const int i = o / nb, j = o % nb;
        double2 s = make_double2(0, 0);
        if (i / nv == j / nv) {  // chirality blocks of W_a^+ W_a
            const double2* wi = W + (((long long)a * 2 + i / nv) * nv + i % nv) * p.d;
            const double2* wj = W + (((long long)a * 2 + j / nv) * nv + j % nv) * p.d;
            for (int e = 0; e < p.d; e++) {
                const double2 r = cjmul(wi[e], wj[e]);
                s.x += r.x;
                s.y += r.y;
            }
            s.x *= diag;
            s.y *= diag;
        }
        for (int d = 0; d < 8; d++) {
            const double2 q = Ps[((long long)a * 8 + d) * nb2 + o];
            s.x += q.x;
            s.y += q.y;
        }
        Dc[(long long)a * 9 * nb2 + o] = s;
    }
}

// out[r][a] = sum_slot Dc[a][slot] in[r][nbr(a, slot)]  (g5^W applied to the result when
// HERM); grid (nagg, ceil(nrhs / CA_R)).  The block D^T and the inputs of the slot are staged
// in LDS; thread t owns a micro-tile of up to 4 rows i (i = ib + 16 q, ib = t % 16) and 4
// right-hand sides (r = rb + 16 w, rb = t / 16), so every LDS value read feeds 4 products.
template <bool HERM>
__global__ __launch_bounds__(256) void k_coarse_apply(const double2* __restrict__ Dc, PG p,
                                                      const double2* __restrict__ in, double2* __restrict__ out,
                                                      int nrhs) {
    extern __shared__ double2 cl[];  // Dt[nb][nb], X[CA_R][nb + 1] (padded against bank conflicts)
    const int a = blockIdx.x;
    const int r0 = blockIdx.y * CA_R;
    const int nr = min(CA_R, nrhs - r0);
    const int nv = p.nv, nb = 2 * nv;
    const long long nc = (long long)p.nagg * nb;
    const long long nb2 = (long long)nb * nb;
    double2* Dt = cl;
    double2* X = cl + nb2;
    const int ib = threadIdx.x & 15, rb = threadIdx.x >> 4;
    double2 acc[4][4];
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
        for (int w = 0; w < 4; w++) acc[q][w] = make_double2(0, 0);
    for (int slot = 0; slot < 9; slot++) {
        const int b = agg_nbr(p, a, slot);
        __syncthreads();
        const double2* D = Dc + ((long long)a * 9 + slot) * nb2;
        for (int t = threadIdx.x; t < nb * nb; t += 256) {
            const int i = t / nb, j = t % nb;
            Dt[j * nb + i] = D[t];
        }
        for (int t = threadIdx.x; t < CA_R * nb; t += 256) {
            const int r = t / nb, j = t % nb;
            X[r * (nb + 1) + j] = r < nr ? in[(long long)(r0 + r) * nc + (long long)b * nb + j] : make_double2(0, 0);
        }
        __syncthreads();
        for (int j = 0; j < nb; j++) {
            double2 dv[4], xv[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int i = ib + 16 * q;
                dv[q] = i < nb ? Dt[j * nb + i] : make_double2(0, 0);
            }
#pragma unroll
            for (int w = 0; w < 4; w++) xv[w] = X[(rb + 16 * w) * (nb + 1) + j];
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int w = 0; w < 4; w++) {
                    acc[q][w].x = fma(dv[q].x, xv[w].x, fma(-dv[q].y, xv[w].y, acc[q][w].x));
                    acc[q][w].y = fma(dv[q].x, xv[w].y, fma(dv[q].y, xv[w].x, acc[q][w].y));
                }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int i = ib + 16 * q;
        if (i >= nb) continue;
#pragma unroll
        for (int w = 0; w < 4; w++) {
            const int r = rb + 16 * w;
            if (r < nr) {
                double2 v = acc[q][w];
                if (HERM && i >= nv) v = make_double2(-v.x, -v.y);
                out[(long long)(r0 + r) * nc + (long long)a * nb + i] = v;
            }
        }
    }
}

void coarse_explicit_build(lqt_ctx* c, lqt_basis* B) {
    if (B->Dc.p) return;
    PG p = pg_of(B);
    const int nb = 2 * p.nv;
    LQT_CHECK(nb <= CB_MAXNB, LQT_EINVAL, "explicit coarse operator: nv must be at most 32");
    LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "explicit coarse operator: one lattice");
    const size_t nb2 = (size_t)nb * nb;
    auto t0 = std::chrono::steady_clock::now();
    B->Dc.ensure(sizeof(double2) * (size_t)p.nagg * 9 * nb2);
    DBuf Ps;
    Ps.ensure(sizeof(double2) * (size_t)p.nagg * 8 * nb2);
    hipLaunchKernelGGL(k_coarse_hops, dim3(p.nagg, 8), dim3(256), 0, c->stream, B->W.as<double2>(),
                       c->U[LQT_F64].as<double2>(), p, B->Dc.as<double2>(), Ps.as<double2>());
    LQT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_coarse_self, dim3(p.nagg), dim3(256), 0, c->stream, B->W.as<double2>(), p,
                       c->g.lat.diag[0], Ps.as<double2>(), B->Dc.as<double2>());
    LQT_HIP(hipGetLastError());
    LQT_HIP(hipStreamSynchronize(c->stream));
    B->coarse_build_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void coarse_explicit_apply(lqt_ctx* c, const lqt_basis* B, const double2* in, double2* out, int nrhs, bool herm) {
    if (nrhs <= 0) return;
    LQT_CHECK(B->Dc.p, LQT_ESTATE, "explicit coarse operator not built");
    coarse_stencil_apply(c, pg_of(B), B->Dc.as<double2>(), in, out, nrhs, herm);
}

void coarse_stencil_apply(lqt_ctx* c, const PG& p, const double2* Dc, const double2* in, double2* out, int nrhs,
                          bool herm) {
    if (nrhs <= 0) return;
    const int nb = 2 * p.nv;
    LQT_CHECK(nb <= CB_MAXNB, LQT_EINVAL, "stencil blocks larger than 64");
    const size_t lds = sizeof(double2) * ((size_t)nb * nb + (size_t)CA_R * (nb + 1));  // <= 129 KiB
    static bool lds_ok = false;  // allow more than 64 KiB of dynamic LDS per workgroup
    if (!lds_ok) {
        LQT_HIP(hipFuncSetAttribute((const void*)k_coarse_apply<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(130 * 1024)));
        LQT_HIP(hipFuncSetAttribute((const void*)k_coarse_apply<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(130 * 1024)));
        lds_ok = true;
    }
    dim3 grid(p.nagg, (nrhs + CA_R - 1) / CA_R);
    c->timer.begin(c->stream, KT_PR);
    if (herm)
        hipLaunchKernelGGL(k_coarse_apply<true>, grid, dim3(256), lds, c->stream, Dc, p, in, out, nrhs);
    else
        hipLaunchKernelGGL(k_coarse_apply<false>, grid, dim3(256), lds, c->stream, Dc, p, in, out, nrhs);
    LQT_HIP(hipGetLastError());
    // stencil blocks once per group of right-hand sides, inputs (9 slots) and outputs once
    c->timer.end(c->stream, 16.0 * ((double)p.nagg * 9 * nb * nb * grid.y + (double)nrhs * p.nagg * nb * 10));
}

}  // namespace lqt
