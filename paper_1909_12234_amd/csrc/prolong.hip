// Multigrid prolongator W and the coarse-space deflation of Algorithm 2.
//
// Aggregates are disjoint blocks of b0 x b1 x b2 x b3 sites.  For aggregate a and chirality
// c (c = 0: spins {0,1}, c = 1: spins {2,3}; g5 = +1 / -1) the block W_{a,c} holds nv
// orthonormal columns of length d = 6 * (sites per block), the restrictions of nv near-null
// vectors to that block and chirality (Section 2: blocking; g5 W = W g5^W by construction).
//   W layout     [a][c][v][bs][s2][colour] complex128, bs = site inside the block, x fastest
//   coarse       [rhs][a][c][v]            complex128, length nc = 2 * nagg * nv
// Near-null vectors follow the paper's adaptive setup: approximate solutions of A y = 0 from
// random starts y0, i.e. y = y0 - e with A e = A y0 solved to null_xi or null_maxit steps.
// The coarse operator g5^W W^+ A W is applied implicitly (prolong, Wilson operator, restrict).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>

#include "blas.h"
#include "gemm.h"
#include "hostla.h"
#include "lqt_internal.h"
#include "devla.h"
#include "eigcheb.h"
#include "prolong.h"
#include "twogrid.h"
#include "solver.h"

using lqt::DBuf;
using lqt::Error;
using lqt::zd;

namespace lqt {

__device__ __forceinline__ double pwsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint64_t psm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------- W from near-null vectors
// W[a][c][v][e] = y_v(comp, site) with e = bs*6 + s2*3 + col, comp = (2c + s2)*3 + col
__global__ void k_gather_null(const double2* __restrict__ Y, PG p, double2* __restrict__ W) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)p.nagg * 2 * p.nv * p.d;
    if (i >= tot) return;
    const int e = (int)(i % p.d);
    long long r = i / p.d;
    const int v = (int)(r % p.nv);
    r /= p.nv;
    const int ch = (int)(r % 2), agg = (int)(r / 2);
    const int bs = e / 6, s2 = (e % 6) / 3, col = e % 3;
    const int comp = (2 * ch + s2) * 3 + col;
    W[i] = Y[(long long)v * 12 * p.V + (long long)comp * p.V + site_of(p, agg, bs)];
}

// Modified Gram-Schmidt (two passes) on the nv columns of each block W_{a,c}; one workgroup
// per block.  A column that vanishes stays zero.
__global__ __launch_bounds__(256) void k_block_mgs(double2* __restrict__ W, PG p) {
    __shared__ double red[4][2];
    __shared__ double bc[2];
    double2* Wb = W + (long long)blockIdx.x * p.nv * p.d;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int pass = 0; pass < 2; pass++)
        for (int v = 0; v < p.nv; v++) {
            double2* wv = Wb + (long long)v * p.d;
            for (int u = 0; u < v; u++) {
                const double2* wu = Wb + (long long)u * p.d;
                double a = 0, b = 0;
                for (int e = threadIdx.x; e < p.d; e += 256) {
                    double2 x = wu[e], y = wv[e];
                    a += x.x * y.x + x.y * y.y;
                    b += x.x * y.y - x.y * y.x;
                }
                a = pwsum(a);
                b = pwsum(b);
                if (lane == 0) red[wave][0] = a, red[wave][1] = b;
                __syncthreads();
                if (threadIdx.x == 0) {
                    bc[0] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
                    bc[1] = red[0][1] + red[1][1] + red[2][1] + red[3][1];
                }
                __syncthreads();
                const double hr = bc[0], hi = bc[1];
                for (int e = threadIdx.x; e < p.d; e += 256) {
                    double2 x = wu[e], y = wv[e];
                    wv[e] = make_double2(y.x - (hr * x.x - hi * x.y), y.y - (hr * x.y + hi * x.x));
                }
                __syncthreads();
            }
            double a = 0;
            for (int e = threadIdx.x; e < p.d; e += 256) {
                double2 y = wv[e];
                a += y.x * y.x + y.y * y.y;
            }
            a = pwsum(a);
            if (lane == 0) red[wave][0] = a;
            __syncthreads();
            if (threadIdx.x == 0) bc[0] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
            __syncthreads();
            const double nrm = sqrt(bc[0]);
            const double s = nrm > 1e-300 ? 1.0 / nrm : 0.0;
            for (int e = threadIdx.x; e < p.d; e += 256) {
                double2 y = wv[e];
                wv[e] = make_double2(s * y.x, s * y.y);
            }
            __syncthreads();
        }
}

void block_mgs(lqt_ctx* c, double2* W, const PG& p, int nblocks) {
    hipLaunchKernelGGL(k_block_mgs, dim3(nblocks), dim3(256), 0, c->stream, W, p);
    LQT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- restrict / prolong
constexpr int RB = 8;  // right-hand sides per workgroup: each W entry is read once per RB

// coarse[r][(a*2 + c)*nv + v] = sum_e conj(W[a][c][v][e]) y_r(e); grid (nagg*2, ceil(nrhs/RB))
__global__ __launch_bounds__(256) void k_restrict(const double2* __restrict__ W, PG p, const double2* __restrict__ y,
                                                  int nrhs, double2* __restrict__ out) {
    extern __shared__ double lds[];  // [nv][RB][4 waves][2]
    const int blk = blockIdx.x, agg = blk >> 1, ch = blk & 1;
    const int r0 = blockIdx.y * RB;
    const int nr = min(RB, nrhs - r0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double2* Wb = W + (long long)blk * p.nv * p.d;
    const long long n = 12LL * p.V;
    for (int v = 0; v < p.nv; v++) {
        double ar[RB], ai[RB];
#pragma unroll
        for (int r = 0; r < RB; r++) ar[r] = ai[r] = 0;
        for (int e = threadIdx.x; e < p.d; e += 256) {
            const double2 w = Wb[(long long)v * p.d + e];
            const int bs = e / 6, s2 = (e % 6) / 3, col = e % 3;
            const int comp = (2 * ch + s2) * 3 + col;
            const int site = site_of(p, agg, bs);
#pragma unroll
            for (int r = 0; r < RB; r++) {
                if (r < nr) {
                    const double2 yv = y[(long long)(r0 + r) * n + (long long)comp * p.V + site];
                    ar[r] += w.x * yv.x + w.y * yv.y;
                    ai[r] += w.x * yv.y - w.y * yv.x;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RB; r++) {
            double a = pwsum(ar[r]), b = pwsum(ai[r]);
            if (lane == 0) {
                lds[((v * RB + r) * 4 + wave) * 2] = a;
                lds[((v * RB + r) * 4 + wave) * 2 + 1] = b;
            }
        }
    }
    __syncthreads();
    const long long nc = 2LL * p.nagg * p.nv;
    for (int t = threadIdx.x; t < p.nv * RB; t += 256) {
        const int v = t / RB, r = t % RB;
        if (r >= nr) continue;
        double a = 0, b = 0;
        for (int w = 0; w < 4; w++) {
            a += lds[((v * RB + r) * 4 + w) * 2];
            b += lds[((v * RB + r) * 4 + w) * 2 + 1];
        }
        out[(long long)(r0 + r) * nc + (long long)blk * p.nv + v] = make_double2(a, b);
    }
}

// Restriction of Rademacher probes for the deflation projections (Algorithm 2, last step):
// out_up / out_dn [r][(a*2 + c)*nv + v] = sum_e conj(W[a][c][v][e]) z_r(e) for the block of
// chirality c (zero in the other array), z_r the probe j0 + r.  One workgroup per (block, RBP
// probes); thread (r = t mod RBP, q = t / RBP) sums the entries e = q (mod 256 / RBP) of a tile
// for probe r.  A tile's signs are hashed once into LDS as bit masks (bit r set: z_r(e) = -1)
// and each row of W is staged in LDS, so W streams from HBM once per RBP probes and the real
// +-1 probe turns the products into signed additions.
constexpr int RBP = 32;
constexpr int RP_TILE = 1536;  // W row entries per tile (one chirality half of a 4^4 block)

__global__ __launch_bounds__(256) void k_restrict_probes(const double2* __restrict__ W, PG p, int nrhs, uint64_t seed,
                                                         long long j0, double2* __restrict__ out_up,
                                                         double2* __restrict__ out_dn) {
    __shared__ uint32_t sg[RP_TILE];
    __shared__ double2 row[RP_TILE];
    __shared__ double2 red[256 / RBP][RBP];
    const int blk = blockIdx.x, agg = blk >> 1, ch = blk & 1;
    const int r0 = blockIdx.y * RBP;
    const int nr = min(RBP, nrhs - r0);
    const int r = threadIdx.x % RBP, q = threadIdx.x / RBP;
    const double2* Wb = W + (long long)blk * p.nv * p.d;
    const long long nc = 2LL * p.nagg * p.nv;
    const int ntiles = (p.d + RP_TILE - 1) / RP_TILE;
    for (int v = 0; v < p.nv; v++) {
        double ar = 0, ai = 0;
        for (int tl = 0; tl < ntiles; tl++) {
            const int e0 = tl * RP_TILE, ne = min(RP_TILE, p.d - e0);
            __syncthreads();  // readers of the previous tile and of red are done
            if (v == 0 || ntiles > 1) {
                for (int e = threadIdx.x; e < ne; e += 256) {
                    const int ee = e0 + e;
                    const int bs = ee / 6, s2 = (ee % 6) / 3, col = ee % 3;
                    const uint64_t hi = psm64((uint64_t)(12LL * site_of(p, agg, bs) + (2 * ch + s2) * 3 + col));
                    uint32_t bits = 0;
                    for (int rr = 0; rr < nr; rr++)
                        bits |= (uint32_t)(psm64(seed ^ psm64((uint64_t)(j0 + r0 + rr) ^ hi)) >> 63) << rr;
                    sg[e] = bits;
                }
            }
            for (int e = threadIdx.x; e < ne; e += 256) row[e] = Wb[(long long)v * p.d + e0 + e];
            __syncthreads();
            for (int e = q; e < ne; e += 256 / RBP) {
                const double2 w = row[e];
                const bool neg = (sg[e] >> r) & 1u;
                ar += neg ? -w.x : w.x;  // Re conj(w) z
                ai += neg ? w.y : -w.y;  // Im conj(w) z
            }
        }
        red[q][r] = make_double2(ar, ai);
        __syncthreads();
        if (threadIdx.x < nr) {
            double a = 0, b = 0;
            for (int qq = 0; qq < 256 / RBP; qq++) a += red[qq][threadIdx.x].x, b += red[qq][threadIdx.x].y;
            const long long o = (long long)(r0 + threadIdx.x) * nc + (long long)blk * p.nv + v;
            out_up[o] = ch == 0 ? make_double2(a, b) : make_double2(0, 0);
            out_dn[o] = ch == 1 ? make_double2(a, b) : make_double2(0, 0);
        }
    }
}

// y_r(e) = sum_v W[a][c][v][e] coarse[r][(a*2 + c)*nv + v]; grid (nagg*2, ceil(nrhs/RB))
__global__ __launch_bounds__(256) void k_prolong(const double2* __restrict__ W, PG p, const double2* __restrict__ cin,
                                                 int nrhs, double2* __restrict__ y) {
    extern __shared__ double2 cv[];  // [RB][nv]
    const int blk = blockIdx.x, agg = blk >> 1, ch = blk & 1;
    const int r0 = blockIdx.y * RB;
    const int nr = min(RB, nrhs - r0);
    const long long nc = 2LL * p.nagg * p.nv;
    const long long n = 12LL * p.V;
    for (int t = threadIdx.x; t < RB * p.nv; t += 256) {
        const int r = t / p.nv, v = t % p.nv;
        cv[t] = r < nr ? cin[(long long)(r0 + r) * nc + (long long)blk * p.nv + v] : make_double2(0, 0);
    }
    __syncthreads();
    const double2* Wb = W + (long long)blk * p.nv * p.d;
    for (int e = threadIdx.x; e < p.d; e += 256) {
        double ar[RB], ai[RB];
#pragma unroll
        for (int r = 0; r < RB; r++) ar[r] = ai[r] = 0;
        for (int v = 0; v < p.nv; v++) {
            const double2 w = Wb[(long long)v * p.d + e];
#pragma unroll
            for (int r = 0; r < RB; r++) {
                const double2 cc = cv[r * p.nv + v];
                ar[r] += w.x * cc.x - w.y * cc.y;
                ai[r] += w.x * cc.y + w.y * cc.x;
            }
        }
        const int bs = e / 6, s2 = (e % 6) / 3, col = e % 3;
        const int comp = (2 * ch + s2) * 3 + col;
        const int site = site_of(p, agg, bs);
#pragma unroll
        for (int r = 0; r < RB; r++)
            if (r < nr) y[(long long)(r0 + r) * n + (long long)comp * p.V + site] = make_double2(ar[r], ai[r]);
    }
}

// coarse g5^W: negate the chirality-1 entries
__global__ void k_g5c(double2* __restrict__ x, long long nc, int nv, long long total) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    long long e = i % nc;
    if ((e / nv) & 1) {
        double2 v = x[i];
        x[i] = make_double2(-v.x, -v.y);
    }
}

// y = y0 - e (near-null vectors from A e = A y0)
__global__ void k_sub(const double2* __restrict__ a, double2* __restrict__ b, long long total) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    double2 x = a[i], y = b[i];
    b[i] = make_double2(x.x - y.x, x.y - y.y);
}

static dim3 g1(long long n) { return dim3((unsigned)((n + 255) / 256)); }

void restrict_fields(lqt_ctx* c, const lqt_basis* B, const double2* fine, double2* coarse, int nrhs) {
    if (nrhs <= 0) return;
    PG p = pg_of(B);
    dim3 grid(p.nagg * 2, (nrhs + RB - 1) / RB);
    size_t lds = sizeof(double) * p.nv * RB * 4 * 2;
    c->timer.begin(c->stream, KT_PR);
    hipLaunchKernelGGL(k_restrict, grid, dim3(256), lds, c->stream, B->W.as<double2>(), p, fine, nrhs, coarse);
    LQT_HIP(hipGetLastError());
    // algorithmic bytes: W once, the fine and the coarse fields once each
    c->timer.end(c->stream, 16.0 * ((double)p.nv * 12 * p.V + (double)nrhs * 12 * p.V + (double)nrhs * 2 * p.nagg * p.nv));
}

void prolong_fields(lqt_ctx* c, const lqt_basis* B, const double2* coarse, double2* fine, int nrhs) {
    if (nrhs <= 0) return;
    PG p = pg_of(B);
    dim3 grid(p.nagg * 2, (nrhs + RB - 1) / RB);
    size_t lds = sizeof(double2) * RB * p.nv;
    c->timer.begin(c->stream, KT_PR);
    hipLaunchKernelGGL(k_prolong, grid, dim3(256), lds, c->stream, B->W.as<double2>(), p, coarse, nrhs, fine);
    LQT_HIP(hipGetLastError());
    // algorithmic bytes: W once, the fine and the coarse fields once each
    c->timer.end(c->stream, 16.0 * ((double)p.nv * 12 * p.V + (double)nrhs * 12 * p.V + (double)nrhs * 2 * p.nagg * p.nv));
}

// out_f = g5^W W^+ A W in_f (FP64), nf coarse vectors: with the explicit stencil when it has
// been built, else prolong, Wilson operator, restrict, in chunks that bound the fine memory
static void coarse_herm(lqt_ctx* c, const lqt_basis* B, const double2* in, double2* out, int nf) {
    if (B->Dc.p) {
        coarse_explicit_apply(c, B, in, out, nf, true);
        return;
    }
    const long long n = 12LL * c->g.V;
    const long long nc = 2LL * B->nagg * B->nv;
    const int chunk = (int)std::max<long long>(1, std::min<long long>(nf, (8LL << 30) / (2 * n * 16)));
    c->scratch[10].ensure(sizeof(double2) * (size_t)chunk * n);
    c->scratch[11].ensure(sizeof(double2) * (size_t)chunk * n);
    for (int f0 = 0; f0 < nf; f0 += chunk) {
        const int cs = std::min(chunk, nf - f0);
        prolong_fields(c, B, in + (size_t)f0 * nc, c->scratch[10].as<double2>(), cs);
        dslash(c, LQT_F64, LQT_A, c->scratch[10].p, c->scratch[11].p, cs, n, n);
        restrict_fields(c, B, c->scratch[11].as<double2>(), out + (size_t)f0 * nc, cs);
    }
    long long tot = nc * nf;
    hipLaunchKernelGGL(k_g5c, g1(tot), dim3(256), 0, c->stream, out, nc, B->nv, tot);
    LQT_HIP(hipGetLastError());
}

void prolong_project_probes(lqt_ctx* c, const lqt_basis* B, uint64_t seed, long long j0, int s, double2* cup,
                            double2* cdn) {
    PG p = pg_of(B);
    const long long nc = 2LL * p.nagg * p.nv;
    DBuf rz;
    rz.ensure(sizeof(double2) * (size_t)s * nc * 2);
    double2* up = rz.as<double2>();
    double2* dn = up + (size_t)s * nc;
    dim3 grid(p.nagg * 2, (s + RBP - 1) / RBP);
    c->timer.begin(c->stream, KT_PR);
    hipLaunchKernelGGL(k_restrict_probes, grid, dim3(256), 0, c->stream, B->W.as<double2>(), p, s, seed, j0, up, dn);
    LQT_HIP(hipGetLastError());
    // algorithmic bytes: W once, both coarse outputs
    c->timer.end(c->stream, 16.0 * ((double)p.nv * 12 * p.V + 2.0 * s * nc));
    gemm_gram(c, B->Uc.as<double2>(), B->k, up, s, cup, nc);
    gemm_gram(c, B->Uc.as<double2>(), B->k, dn, s, cdn, nc);
}

// cm = U_c^+ W^+ Z and cg = U_c^+ g5^W W^+ Z (= u_i^+ g5 z for the chirality-split W) for s
// fine fields Z, k x s each (device)
void prolong_project_fields(lqt_ctx* c, const lqt_basis* B, const double2* Z, int s, double2* cm, double2* cg) {
    PG p = pg_of(B);
    const long long nc = 2LL * p.nagg * p.nv;
    DBuf rz;
    rz.ensure(sizeof(double2) * (size_t)s * nc);
    restrict_fields(c, B, Z, rz.as<double2>(), s);
    gemm_gram(c, B->Uc.as<double2>(), B->k, rz.as<double2>(), s, cm, nc);
    const long long tot = nc * s;
    hipLaunchKernelGGL(k_g5c, g1(tot), dim3(256), 0, c->stream, rz.as<double2>(), nc, p.nv, tot);
    LQT_HIP(hipGetLastError());
    gemm_gram(c, B->Uc.as<double2>(), B->k, rz.as<double2>(), s, cg, nc);
}

__global__ void k_sub_from(double2* __restrict__ z, const double2* __restrict__ y, long long total) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    double2 a = z[i], b = y[i];
    z[i] = make_double2(a.x - b.x, a.y - b.y);
}

// Z <- Z - W U_c C for s fine fields Z and the k x s coefficients C (device); tmp: s fine fields
void prolong_subtract(lqt_ctx* c, const lqt_basis* B, const double2* C, int s, double2* Z, double2* tmp) {
    PG p = pg_of(B);
    const long long nc = 2LL * p.nagg * p.nv;
    DBuf cc;
    cc.ensure(sizeof(double2) * (size_t)s * nc);
    gemm_combine(c, B->Uc.as<double2>(), B->k, C, s, 0.0, 1.0, cc.as<double2>(), nc);
    prolong_fields(c, B, cc.as<double2>(), tmp, s);
    const long long tot = 12LL * p.V * s;
    hipLaunchKernelGGL(k_sub_from, g1(tot), dim3(256), 0, c->stream, Z, tmp, tot);
    LQT_HIP(hipGetLastError());
}

// The orthogonal projector W U_c U_c^+ W^+ needs orthonormal coarse vectors (W is orthonormal
// by construction): LQT_EINVAL unless max |U_c^+ U_c - I| <= 1e-10.
void prolong_check_orthonormal(lqt_ctx* c, const lqt_basis* B) {
    const int k = B->k;
    if (k == 0) return;
    const long long nc = 2LL * B->nagg * B->nv;
    DBuf G;
    G.ensure(sizeof(double2) * (size_t)k * k);
    gemm_gram(c, B->Uc.as<double2>(), k, B->Uc.as<double2>(), k, G.as<double2>(), nc);
    std::vector<zd> h((size_t)k * k);
    LQT_HIP(hipMemcpyAsync(h.data(), G.p, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    double dev = 0;
    for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++) dev = std::max(dev, std::abs(h[(size_t)i * k + j] - zd(i == j ? 1.0 : 0.0)));
    LQT_CHECK(dev <= 1e-10, LQT_EINVAL,
              "the orthogonal projector needs orthonormal coarse vectors (max |U_c^+ U_c - I| = " + std::to_string(dev) +
                  ")");
}

// Coarse oblique data from coarse vectors Ubar (k, device): M = Ubar^+ g5^W W^+ A W Ubar,
// eigh, Uc = Ubar U_hat, u_i^+ g5 u_i = Uc_i^+ g5^W Uc_i.
static void coarse_oblique_setup(lqt_ctx* c, lqt_basis* B, const double2* Ubar, int k) {
    const long long nc = 2LL * B->nagg * B->nv;
    DBuf HU, G5U, Md;
    HU.ensure(sizeof(double2) * (size_t)k * nc);
    coarse_herm(c, B, Ubar, HU.as<double2>(), k);
    Md.ensure(sizeof(double2) * (size_t)k * k);
    gemm_gram(c, Ubar, k, HU.as<double2>(), k, Md.as<double2>(), nc);
    std::vector<zd> M((size_t)k * k);
    LQT_HIP(hipMemcpyAsync(M.data(), Md.p, sizeof(double2) * M.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    std::vector<double> lam;
    std::vector<zd> Uh;
    heev_any(c, k, M, lam, Uh, true);
    LQT_HIP(hipMemcpyAsync(Md.p, Uh.data(), sizeof(double2) * Uh.size(), hipMemcpyHostToDevice, c->stream));
    B->Uc.ensure(sizeof(double2) * (size_t)k * nc);
    gemm_combine(c, Ubar, k, Md.as<double2>(), k, 0.0, 1.0, B->Uc.as<double2>(), nc);
    G5U.ensure(sizeof(double2) * (size_t)k * nc);
    LQT_HIP(hipMemcpyAsync(G5U.p, B->Uc.p, sizeof(double2) * (size_t)k * nc, hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(k_g5c, g1(nc * k), dim3(256), 0, c->stream, G5U.as<double2>(), nc, B->nv, nc * k);
    LQT_HIP(hipGetLastError());
    gemm_gram(c, B->Uc.as<double2>(), k, G5U.as<double2>(), k, Md.as<double2>(), nc);
    std::vector<zd> D((size_t)k * k);
    LQT_HIP(hipMemcpyAsync(D.data(), Md.p, sizeof(double2) * D.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    B->k = k;
    B->lambda.assign(2 * k, 0.0);
    B->ug5u.assign(2 * k, 0.0);
    for (int i = 0; i < k; i++) {
        B->lambda[2 * i] = lam[i];
        B->ug5u[2 * i] = D[(size_t)i * k + i].real();
        B->ug5u[2 * i + 1] = D[(size_t)i * k + i].imag();
    }
}

static void check_block(const lqt_ctx* c, const int* block, int nv) {
    LQT_CHECK(block, LQT_EINVAL, "null block");
    for (int i = 0; i < 4; i++)
        LQT_CHECK(block[i] >= 1 && c->g.L[i] % block[i] == 0, LQT_EINVAL, "block extents must divide the lattice");
    const int bs = block[0] * block[1] * block[2] * block[3];
    LQT_CHECK(nv >= 1 && nv <= 64 && nv <= 6 * bs, LQT_EINVAL, "nv must be in 1..min(64, 6 * block sites)");
}

}  // namespace lqt

namespace {

template <typename F>
int guard(lqt_ctx* c, F&& f) {
    try {
        f();
        return LQT_OK;
    } catch (const Error& e) {
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

lqt_basis* new_prolongator(lqt_ctx* c, const int* block, int nv) {
    lqt_basis* B = new lqt_basis();
    B->ctx = c;
    B->kind = 1;
    for (int i = 0; i < 4; i++) B->block[i] = block[i];
    B->nv = nv;
    lqt::PG p = lqt::make_pg(c, block, nv);
    B->nagg = p.nagg;
    B->W.ensure(sizeof(double2) * (size_t)nv * 12 * c->g.V);
    return B;
}

}  // namespace

extern "C" {

int lqt_basis_prolongator(lqt_ctx* c, const int block[4], int nv, int k, double null_xi, int null_maxit,
                          const lqt_solver_opts* opts, lqt_basis** out) {
    if (!c || !out) return LQT_EINVAL;
    *out = nullptr;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        lqt::check_block(c, block, nv);
        LQT_CHECK(null_xi > 0 && null_xi < 1 && null_maxit >= 1, LQT_EINVAL, "bad null-vector tolerance");
        const long long n = 12LL * c->g.V;
        {
            const long long nc0 = 2LL * lqt::make_pg(c, block, nv).nagg * nv;
            LQT_CHECK(k >= 0 && k <= nc0 / 8, LQT_EINVAL, "k must be in 0..nc/8");
        }
        lqt_basis* B = new_prolongator(c, block, nv);
        const long long nc = 2LL * B->nagg * nv;
        try {
            lqt::SolveOpts o = lqt::make_opts(opts);
            // near-null vectors: y = y0 - e, A e = A y0 to null_xi or null_maxit steps
            lqt::SolveOpts on = o;
            on.maxit = null_maxit;
            DBuf Y0, AY, E;
            Y0.ensure(sizeof(double2) * (size_t)nv * n);
            AY.ensure(sizeof(double2) * (size_t)nv * n);
            E.ensure(sizeof(double2) * (size_t)nv * n);
            lqt::gaussian_fields(c, 0x4E554C4Cull, n, nv, Y0.as<double2>());
            lqt::dslash(c, LQT_F64, LQT_A, Y0.p, AY.p, nv, n, n);
            std::vector<lqt_solve_stats> st(nv);
            lqt::solve_fields(c, AY.as<double2>(), E.as<double2>(), nv, null_xi, on, st.data());
            hipLaunchKernelGGL(lqt::k_sub, lqt::g1((long long)nv * n), dim3(256), 0, c->stream, Y0.as<double2>(),
                               E.as<double2>(), (long long)nv * n);
            LQT_HIP(hipGetLastError());
            if (o.verbose) {
                fprintf(stderr, "[lqtrace] prolongator: %d near-null vectors, %d steps each\n", nv, st[0].iters);
                fflush(stderr);
            }
            // block, split by chirality, orthonormalise
            lqt::PG p = lqt::make_pg(c, block, nv);
            long long tot = (long long)p.nagg * 2 * nv * p.d;
            hipLaunchKernelGGL(lqt::k_gather_null, lqt::g1(tot), dim3(256), 0, c->stream, E.as<double2>(), p,
                               B->W.as<double2>());
            hipLaunchKernelGGL(lqt::k_block_mgs, dim3(p.nagg * 2), dim3(256), 0, c->stream, B->W.as<double2>(), p);
            LQT_HIP(hipGetLastError());
            if (k > 0) {
                // the coarse operator as an explicit 9-point block stencil (nv <= 32), which the
                // eigensolver applies to its whole block at once
                if (2 * nv <= 64) {
                    lqt::coarse_explicit_build(c, B);
                    if (o.verbose) {
                        fprintf(stderr, "[lqtrace] prolongator: coarse operator W^+ A W built in %.2f s\n",
                                B->coarse_build_s);
                        fflush(stderr);
                    }
                }
                // Algorithm 2, second step: k eigenpairs of g5^W W^+ A W with smallest |lambda|
                lqt::HermOp H = [c, B](const double2* in, double2* o2, int nf) { lqt::coarse_herm(c, B, in, o2, nf); };
                DBuf Qb;
                std::vector<double> theta, resT;
                const double exi = o.eig_xi > 0 ? o.eig_xi : null_xi;
                int conv = lqt::eig_chebyshev(c, nc, H, nullptr, lqt::wilson_norm_bound(c), k, exi, o.outer_maxit,
                                              o.eig_degree, o.verbose, Qb, theta, resT);
                // third step: rotate so that U^+ g5^W W^+ A W U is diagonal
                lqt::coarse_oblique_setup(c, B, Qb.as<double2>(), k);
                B->theta.assign(theta.begin(), theta.begin() + k);
                B->resid.assign(resT.begin(), resT.begin() + k);
                LQT_HIP(hipStreamSynchronize(c->stream));
                *out = B;
                if (conv < k) {
                    c->err = "coarse eigensolver: " + std::to_string(conv) + " of " + std::to_string(k) +
                             " pairs converged";
                    throw Error{LQT_ENOTCONV, c->err};
                }
                return;
            }
            LQT_HIP(hipStreamSynchronize(c->stream));
        } catch (const Error& e) {
            if (*out == nullptr) delete B;
            throw;
        }
        *out = B;
    });
}

int lqt_coarse_apply(lqt_ctx* c, lqt_basis* B, const double* d_in, double* d_out, int nrhs, int herm) {
    if (!c || !B) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(B->kind == 1, LQT_EINVAL, "not a prolongator basis");
        LQT_CHECK(nrhs >= 0 && (nrhs == 0 || (d_in && d_out)), LQT_EINVAL, "bad coarse apply arguments");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        lqt::coarse_explicit_build(c, B);
        lqt::coarse_explicit_apply(c, B, (const double2*)d_in, (double2*)d_out, nrhs, herm != 0);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

int lqt_basis_prolongator_from(lqt_ctx* c, const int block[4], int nv, const double* d_w, const double* d_coarse,
                               int k, lqt_basis** out) {
    if (!c || !out) return LQT_EINVAL;
    *out = nullptr;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge || k == 0, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        lqt::check_block(c, block, nv);
        LQT_CHECK(d_w, LQT_EINVAL, "null prolongator");
        LQT_CHECK(k >= 0 && (k == 0 || d_coarse), LQT_EINVAL, "coarse vectors missing");
        lqt_basis* B = new_prolongator(c, block, nv);
        try {
            LQT_HIP(hipMemcpyAsync(B->W.p, d_w, sizeof(double2) * (size_t)nv * 12 * c->g.V, hipMemcpyDeviceToDevice,
                                   c->stream));
            if (k > 0) lqt::coarse_oblique_setup(c, B, (const double2*)d_coarse, k);
            LQT_HIP(hipStreamSynchronize(c->stream));
        } catch (...) {
            delete B;
            throw;
        }
        *out = B;
    });
}

int lqt_restrict(lqt_ctx* c, const lqt_basis* B, const double* fine, double* coarse, int nrhs) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(B && B->kind == 1 && B->ctx == c, LQT_EINVAL, "not a prolongator basis of this context");
        LQT_CHECK(nrhs >= 0 && (nrhs == 0 || (fine && coarse)), LQT_EINVAL, "bad fields");
        if (nrhs == 0) return;
        const long long n = 12LL * c->g.V;
        DBuf f;
        f.ensure(sizeof(double2) * (size_t)nrhs * n);
        lqt::to_device_layout(c, (const double2*)fine, f.as<double2>(), nrhs);
        lqt::restrict_fields(c, B, f.as<double2>(), (double2*)coarse, nrhs);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

int lqt_prolong(lqt_ctx* c, const lqt_basis* B, const double* coarse, double* fine, int nrhs) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(B && B->kind == 1 && B->ctx == c, LQT_EINVAL, "not a prolongator basis of this context");
        LQT_CHECK(nrhs >= 0 && (nrhs == 0 || (fine && coarse)), LQT_EINVAL, "bad fields");
        if (nrhs == 0) return;
        const long long n = 12LL * c->g.V;
        DBuf f;
        f.ensure(sizeof(double2) * (size_t)nrhs * n);
        lqt::prolong_fields(c, B, (const double2*)coarse, f.as<double2>(), nrhs);
        lqt::from_device_layout(c, f.as<double2>(), (double2*)fine, nrhs);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

// ---- second multigrid level
static void check_level2(const lqt_basis* B, const int* block2, int nv2) {
    LQT_CHECK(block2, LQT_EINVAL, "null level-2 block");
    const lqt::PG p = lqt::pg_of(B);
    const int n[4] = {p.n0, p.n1, p.n2, p.n3};
    for (int i = 0; i < 4; i++)
        LQT_CHECK(block2[i] >= 1 && n[i] % block2[i] == 0, LQT_EINVAL,
                  "level-2 block extents must divide the coarse lattice");
    const int bs2 = block2[0] * block2[1] * block2[2] * block2[3];
    LQT_CHECK(2 * B->nv <= 64, LQT_EINVAL, "the second level needs the explicit coarse operator (nv <= 32)");
    LQT_CHECK(nv2 >= 1 && nv2 <= 32 && nv2 <= bs2 * B->nv, LQT_EINVAL, "nv2 must be in 1..min(32, level-2 block entries)");
}

static void level2_setup(lqt_ctx* c, lqt_basis* B, const int* block2, int nv2) {
    for (int i = 0; i < 4; i++) B->block2[i] = block2[i];
    B->nv2 = nv2;
}

// Algorithm 2's second and third steps on the level-2 operator: the k eigenpairs of
// g5^{W2} D_cc with smallest |lambda|, prolongated to the level-1 coarse space, then the
// rotation of the coarse vectors.  Returns the number of pairs that passed.
static int level2_eig(lqt_ctx* c, lqt_basis* B, int k, double xi, const lqt::SolveOpts& o) {
    const lqt::PG q = lqt::pg2_of(B);
    const long long nc1 = 2LL * B->nagg * B->nv, nc2 = 2LL * q.nagg * q.nv;
    lqt::HermOp H = [c, B](const double2* in, double2* o2, int nf) { lqt::level2_apply(c, B, in, o2, nf, true); };
    DBuf Qb;
    std::vector<double> theta, resT;
    const int conv = lqt::eig_chebyshev(c, nc2, H, nullptr, lqt::wilson_norm_bound(c), k, xi, o.outer_maxit,
                                        o.eig_degree, o.verbose, Qb, theta, resT);
    DBuf Ub;
    Ub.ensure(sizeof(double2) * (size_t)k * nc1);
    lqt::prolong2_fields(c, B, Qb.as<double2>(), Ub.as<double2>(), k);
    lqt::coarse_oblique_setup(c, B, Ub.as<double2>(), k);
    B->theta.assign(theta.begin(), theta.begin() + k);
    B->resid.assign(resT.begin(), resT.begin() + k);
    return conv;
}

int lqt_basis_prolongator2(lqt_ctx* c, const int block[4], int nv, const int block2[4], int nv2, int k,
                           double null_xi, int null_maxit, const lqt_solver_opts* opts, lqt_basis** out) {
    if (!c || !out) return LQT_EINVAL;
    *out = nullptr;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        lqt::check_block(c, block, nv);
        LQT_CHECK(null_xi > 0 && null_xi < 1 && null_maxit >= 1, LQT_EINVAL, "bad null-vector tolerance");
        lqt_basis* B = new_prolongator(c, block, nv);
        try {
            check_level2(B, block2, nv2);
            level2_setup(c, B, block2, nv2);
            const lqt::PG q = lqt::pg2_of(B);
            const long long nc2 = 2LL * q.nagg * nv2;
            LQT_CHECK(k >= 0 && k <= nc2 / 8, LQT_EINVAL, "k must be in 0..nc2/8");
            lqt::SolveOpts o = lqt::make_opts(opts);
            const long long n = 12LL * c->g.V;
            const long long nc1 = 2LL * B->nagg * nv;
            // level 1: near-null vectors of A, W, the explicit coarse operator
            {
                lqt::SolveOpts on = o;
                on.maxit = null_maxit;
                DBuf Y0, AY, E;
                Y0.ensure(sizeof(double2) * (size_t)nv * n);
                AY.ensure(sizeof(double2) * (size_t)nv * n);
                E.ensure(sizeof(double2) * (size_t)nv * n);
                lqt::gaussian_fields(c, 0x4E554C4Cull, n, nv, Y0.as<double2>());
                lqt::dslash(c, LQT_F64, LQT_A, Y0.p, AY.p, nv, n, n);
                std::vector<lqt_solve_stats> st(nv);
                lqt::solve_fields(c, AY.as<double2>(), E.as<double2>(), nv, null_xi, on, st.data());
                hipLaunchKernelGGL(lqt::k_sub, lqt::g1((long long)nv * n), dim3(256), 0, c->stream, Y0.as<double2>(),
                                   E.as<double2>(), (long long)nv * n);
                LQT_HIP(hipGetLastError());
                lqt::PG p = lqt::make_pg(c, block, nv);
                long long tot = (long long)p.nagg * 2 * nv * p.d;
                hipLaunchKernelGGL(lqt::k_gather_null, lqt::g1(tot), dim3(256), 0, c->stream, E.as<double2>(), p,
                                   B->W.as<double2>());
                lqt::block_mgs(c, B->W.as<double2>(), p, p.nagg * 2);
                lqt::coarse_explicit_build(c, B);
            }
            // level 2: near-null vectors of D_c (coarse GMRES to null_xi or null_maxit steps), W2,
            // the level-2 operator
            {
                DBuf Y0, AY, E;
                Y0.ensure(sizeof(double2) * (size_t)nv2 * nc1);
                AY.ensure(sizeof(double2) * (size_t)nv2 * nc1);
                E.ensure(sizeof(double2) * (size_t)nv2 * nc1);
                lqt::gaussian_fields(c, 0x4E554C32ull, nc1, nv2, Y0.as<double2>());
                lqt::coarse_explicit_apply(c, B, Y0.as<double2>(), AY.as<double2>(), nv2, false);
                const double rel = lqt::coarse_gmres(c, B, AY.as<double2>(), E.as<double2>(), nv2, null_xi, null_maxit);
                hipLaunchKernelGGL(lqt::k_sub, lqt::g1((long long)nv2 * nc1), dim3(256), 0, c->stream, Y0.as<double2>(),
                                   E.as<double2>(), (long long)nv2 * nc1);
                LQT_HIP(hipGetLastError());
                lqt::level2_blocks(c, B, E.as<double2>());
                lqt::level2_build(c, B);
                if (o.verbose) {
                    fprintf(stderr,
                            "[lqtrace] prolongator: level 1 operator built in %.2f s; %d level-2 near-null vectors "
                            "(coarse relative residual %.2e); level-2 operator built in %.2f s\n",
                            B->coarse_build_s, nv2, rel, B->level2_build_s);
                    fflush(stderr);
                }
            }
            if (k > 0) {
                const double exi = o.eig_xi > 0 ? o.eig_xi : null_xi;
                const int conv = level2_eig(c, B, k, exi, o);
                LQT_HIP(hipStreamSynchronize(c->stream));
                *out = B;
                if (conv < k) {
                    c->err = "level-2 eigensolver: " + std::to_string(conv) + " of " + std::to_string(k) +
                             " pairs converged";
                    throw Error{LQT_ENOTCONV, c->err};
                }
                return;
            }
            LQT_HIP(hipStreamSynchronize(c->stream));
        } catch (const Error& e) {
            if (*out == nullptr) delete B;
            throw;
        }
        *out = B;
    });
}

int lqt_basis_prolongator2_from(lqt_ctx* c, const int block[4], int nv, const double* d_w, const int block2[4],
                                int nv2, const double* d_w2, const double* d_coarse2, int k, lqt_basis** out) {
    if (!c || !out) return LQT_EINVAL;
    *out = nullptr;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        lqt::check_block(c, block, nv);
        LQT_CHECK(d_w && d_w2, LQT_EINVAL, "null prolongator");
        LQT_CHECK(k >= 0 && (k == 0 || d_coarse2), LQT_EINVAL, "level-2 coarse vectors missing");
        lqt_basis* B = new_prolongator(c, block, nv);
        try {
            check_level2(B, block2, nv2);
            level2_setup(c, B, block2, nv2);
            const lqt::PG q = lqt::pg2_of(B);
            const long long nc1 = 2LL * B->nagg * nv, nc2 = 2LL * q.nagg * nv2;
            LQT_CHECK(k <= nc2, LQT_EINVAL, "k must be at most nc2");
            LQT_HIP(hipMemcpyAsync(B->W.p, d_w, sizeof(double2) * (size_t)nv * 12 * c->g.V, hipMemcpyDeviceToDevice,
                                   c->stream));
            lqt::coarse_explicit_build(c, B);
            const size_t w2 = (size_t)q.nagg * 2 * nv2 * q.d;
            B->W2.ensure(sizeof(double2) * w2);
            LQT_HIP(hipMemcpyAsync(B->W2.p, d_w2, sizeof(double2) * w2, hipMemcpyDeviceToDevice, c->stream));
            lqt::level2_build(c, B);
            if (k > 0) {
                DBuf Ub;
                Ub.ensure(sizeof(double2) * (size_t)k * nc1);
                lqt::prolong2_fields(c, B, (const double2*)d_coarse2, Ub.as<double2>(), k);
                lqt::coarse_oblique_setup(c, B, Ub.as<double2>(), k);
            }
            (void)nc2;
            LQT_HIP(hipStreamSynchronize(c->stream));
        } catch (...) {
            delete B;
            throw;
        }
        *out = B;
    });
}

int lqt_coarse2_apply(lqt_ctx* c, lqt_basis* B, const double* d_in, double* d_out, int nrhs, int herm) {
    if (!c || !B) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(B->kind == 1 && B->nv2 > 0 && B->Dc2.p, LQT_EINVAL, "not a two-level prolongator basis");
        LQT_CHECK(nrhs >= 0 && (nrhs == 0 || (d_in && d_out)), LQT_EINVAL, "bad level-2 apply arguments");
        lqt::level2_apply(c, B, (const double2*)d_in, (double2*)d_out, nrhs, herm != 0);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

int lqt_prolongator2_get(const lqt_basis* B, double* d_w2, long long* nc2) {
    if (!B || B->kind != 1 || B->nv2 == 0) return LQT_EINVAL;
    const lqt::PG q = lqt::pg2_of(B);
    if (nc2) *nc2 = 2LL * q.nagg * q.nv;
    if (d_w2) {
        if (hipMemcpyAsync(d_w2, B->W2.p, sizeof(double2) * (size_t)q.nagg * 2 * q.nv * q.d, hipMemcpyDeviceToDevice,
                           B->ctx->stream) != hipSuccess)
            return LQT_EHIP;
        if (hipStreamSynchronize(B->ctx->stream) != hipSuccess) return LQT_EHIP;
    }
    return LQT_OK;
}

int lqt_prolongator_get(const lqt_basis* B, double* d_w, long long* nc) {
    if (!B || B->kind != 1) return LQT_EINVAL;
    if (nc) *nc = 2LL * B->nagg * B->nv;
    if (d_w) {
        if (hipMemcpyAsync(d_w, B->W.p, sizeof(double2) * (size_t)B->nv * 12 * B->ctx->g.V, hipMemcpyDeviceToDevice,
                           B->ctx->stream) != hipSuccess)
            return LQT_EHIP;
        if (hipStreamSynchronize(B->ctx->stream) != hipSuccess) return LQT_EHIP;
    }
    return LQT_OK;
}

}  // extern "C"
