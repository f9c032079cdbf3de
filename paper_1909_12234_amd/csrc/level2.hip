// Second multigrid level (Table 2: the coarse lattice blocked again).  The level-1 coarse
// lattice has one site per aggregate (x fastest) and 2 nv1 entries per site, index
// (a1 * 2 + c) * nv1 + v1.  A level-2 block (A, c) gathers the chirality-c entries of its
// level-1 sites, local index e = ls * nv1 + v1 (ls = site inside the block, x fastest), so
//   W2[A][c][v2][e],  v2 < nv2,
// is block-diagonal in chirality like W and g5^{W1} W2 = W2 g5^{W2}.  The level-2 operator
// D_cc = W2^+ D_c W2 couples a level-2 block only to itself and its +-mu neighbours (D_c is
// a nearest-neighbour stencil on the level-1 lattice), so it is stored as the same 9-point
// block stencil as D_c and applied by the same kernel.
//
// D_cc is assembled by coloured probing: the level-2 blocks are coloured by their coordinates
// modulo q_mu (q_mu = the extent when it is at most 4, else 4 or 3, whichever divides it), so
// that no block has two blocks of one colour among itself and its +-mu neighbours.  For each
// colour and each column j = (c, v2) the columns of all blocks of that colour are prolongated
// together, D_c is applied, and the restriction to every block A is its stencil column for
// the one neighbour of that colour.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>

#include "lqt_internal.h"
#include "prolong.h"

namespace lqt {

PG pg2_of(const lqt_basis* B) {
    const PG p = pg_of(B);
    PG q;
    q.L0 = p.n0, q.L1 = p.n1, q.L2 = p.n2, q.L3 = p.n3;
    q.b0 = B->block2[0], q.b1 = B->block2[1], q.b2 = B->block2[2], q.b3 = B->block2[3];
    q.n0 = q.L0 / q.b0, q.n1 = q.L1 / q.b1, q.n2 = q.L2 / q.b2, q.n3 = q.L3 / q.b3;
    q.bsites = q.b0 * q.b1 * q.b2 * q.b3;
    q.nagg = p.nagg / q.bsites;
    q.d = q.bsites * B->nv;  // entries per block and chirality
    q.nv = B->nv2;
    q.V = p.nagg;  // level-1 coarse sites
    return q;
}

// level-1 coarse index of entry e of level-2 block (A, c)
__device__ __forceinline__ long long idx1(const PG& q, int nv1, int A, int c, int e) {
    const int ls = e / nv1, v1 = e - ls * nv1;
    return ((long long)site_of(q, A, ls) * 2 + c) * nv1 + v1;
}

// W2[A][c][v][e] = Y[v][idx1(A, c, e)] for the nv2 level-1 coarse vectors Y
__global__ void k_gather2(const double2* __restrict__ Y, PG q, int nv1, double2* __restrict__ W2) {
    const long long tot = (long long)q.nagg * 2 * q.nv * q.d;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tot) return;
    const int e = (int)(i % q.d);
    const long long r = i / q.d;
    const int v = (int)(r % q.nv);
    const long long ac = r / q.nv;
    const int c = (int)(ac & 1), A = (int)(ac >> 1);
    const long long nc1 = 2LL * q.V * nv1;
    W2[i] = Y[(long long)v * nc1 + idx1(q, nv1, A, c, e)];
}

// out[r][(A*2 + c)*nv2 + v] = sum_e conj(W2[A][c][v][e]) y[r][idx1(A, c, e)]; grid (nagg2*2, nrhs)
__global__ __launch_bounds__(256) void k_restrict2(const double2* __restrict__ W2, PG q, int nv1,
                                                   const double2* __restrict__ y, double2* __restrict__ out) {
    __shared__ double red[4][2];
    const int blk = blockIdx.x, A = blk >> 1, c = blk & 1, r = blockIdx.y;
    const long long nc1 = 2LL * q.V * nv1, nc2 = 2LL * q.nagg * q.nv;
    const double2* yr = y + (long long)r * nc1;
    const double2* Wb = W2 + (long long)blk * q.nv * q.d;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int v = 0; v < q.nv; v++) {
        double a = 0, b = 0;
        for (int e = threadIdx.x; e < q.d; e += 256) {
            const double2 w = Wb[(long long)v * q.d + e], x = yr[idx1(q, nv1, A, c, e)];
            a += w.x * x.x + w.y * x.y;
            b += w.x * x.y - w.y * x.x;
        }
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o);
            b += __shfl_xor(b, o);
        }
        if (lane == 0) red[wave][0] = a, red[wave][1] = b;
        __syncthreads();
        if (threadIdx.x == 0)
            out[(long long)r * nc2 + (long long)blk * q.nv + v] =
                make_double2(red[0][0] + red[1][0] + red[2][0] + red[3][0], red[0][1] + red[1][1] + red[2][1] + red[3][1]);
        __syncthreads();
    }
}

// y[r][idx1(A, c, e)] = sum_v W2[A][c][v][e] x[r][(A*2 + c)*nv2 + v]; grid (nagg2*2, nrhs)
__global__ __launch_bounds__(256) void k_prolong2(const double2* __restrict__ W2, PG q, int nv1,
                                                  const double2* __restrict__ x, double2* __restrict__ y) {
    const int blk = blockIdx.x, A = blk >> 1, c = blk & 1, r = blockIdx.y;
    const long long nc1 = 2LL * q.V * nv1, nc2 = 2LL * q.nagg * q.nv;
    const double2* xr = x + (long long)r * nc2 + (long long)blk * q.nv;
    const double2* Wb = W2 + (long long)blk * q.nv * q.d;
    for (int e = threadIdx.x; e < q.d; e += 256) {
        double a = 0, b = 0;
        for (int v = 0; v < q.nv; v++) {
            const double2 w = Wb[(long long)v * q.d + e], s = xr[v];
            a += w.x * s.x - w.y * s.y;
            b += w.x * s.y + w.y * s.x;
        }
        y[(long long)r * nc1 + idx1(q, nv1, A, c, e)] = make_double2(a, b);
    }
}

struct Colours {
    int q[4];
    int n;
};

static Colours colours_of(const PG& q) {
    Colours k;
    const int n[4] = {q.n0, q.n1, q.n2, q.n3};
    k.n = 1;
    for (int mu = 0; mu < 4; mu++) {
        int m = n[mu];
        if (m > 4) m = (n[mu] % 4 == 0) ? 4 : ((n[mu] % 3 == 0) ? 3 : n[mu]);
        k.q[mu] = m;
        k.n *= m;
    }
    return k;
}

__device__ __forceinline__ int colour_of(const PG& q, const Colours& k, int A) {
    const int x = A % q.n0, y = (A / q.n0) % q.n1, z = (A / (q.n0 * q.n1)) % q.n2, t = A / (q.n0 * q.n1 * q.n2);
    return (x % k.q[0]) + k.q[0] * ((y % k.q[1]) + k.q[1] * ((z % k.q[2]) + k.q[2] * (t % k.q[3])));
}

// level-2 block in stencil slot `slot` of block A (periodic)
__device__ __forceinline__ int blk_nbr(const PG& q, int A, int slot) {
    if (slot == 0) return A;
    int cc[4] = {A % q.n0, (A / q.n0) % q.n1, (A / (q.n0 * q.n1)) % q.n2, A / (q.n0 * q.n1 * q.n2)};
    const int n[4] = {q.n0, q.n1, q.n2, q.n3};
    const int mu = (slot - 1) >> 1;
    cc[mu] = ((slot - 1) & 1) ? (cc[mu] + n[mu] - 1) % n[mu] : (cc[mu] + 1) % n[mu];
    return cc[0] + q.n0 * (cc[1] + q.n1 * (cc[2] + q.n2 * cc[3]));
}

// probe r of colour `col` (r = column j = c * nv2 + v2 of every block of that colour):
// y[r] = the prolongation of those columns, a level-1 coarse field
__global__ void k_probe2(const double2* __restrict__ W2, PG q, int nv1, Colours k, int col, int ncols,
                         double2* __restrict__ y) {
    const long long nc1 = 2LL * q.V * nv1;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc1 * ncols) return;
    const int r = (int)(i / nc1);
    const long long e1 = i - (long long)r * nc1;
    // level-1 entry (a1, c1, v1) -> level-2 block and local entry
    const int v1 = (int)(e1 % nv1);
    const long long ac = e1 / nv1;
    const int c1 = (int)(ac & 1), a1 = (int)(ac >> 1);
    const int x = a1 % q.L0, yy = (a1 / q.L0) % q.L1, z = (a1 / (q.L0 * q.L1)) % q.L2, t = a1 / (q.L0 * q.L1 * q.L2);
    const int A = x / q.b0 + q.n0 * (yy / q.b1 + q.n1 * (z / q.b2 + q.n2 * (t / q.b3)));
    const int ls = x % q.b0 + q.b0 * (yy % q.b1 + q.b1 * (z % q.b2 + q.b2 * (t % q.b3)));
    const int c = r / q.nv, v2 = r - c * q.nv;
    double2 val = make_double2(0, 0);
    if (c1 == c && colour_of(q, k, A) == col) val = W2[(((long long)A * 2 + c) * q.nv + v2) * q.d + ls * nv1 + v1];
    y[i] = val;
}

// Dc2[A][slot][i][j] = R[j][(A*2 + ci)*nv2 + vi] for the first slot whose block has colour col
// (i = ci*nv2 + vi, j = the probe's column); grid over nagg2 * nb2 rows, one thread per (A, i)
// and column
__global__ void k_scatter2(const double2* __restrict__ R, PG q, Colours k, int col, int ncols,
                           double2* __restrict__ Dc2) {
    const int nb = 2 * q.nv;
    const long long nc2 = 2LL * q.nagg * q.nv;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)q.nagg * nb * ncols) return;
    const int j = (int)(t % ncols);
    const long long ai = t / ncols;
    const int i = (int)(ai % nb), A = (int)(ai / nb);
    int slot = -1;
    for (int s = 0; s < 9 && slot < 0; s++)
        if (colour_of(q, k, blk_nbr(q, A, s)) == col) slot = s;
    if (slot < 0) return;
    // the first slot that reaches this block holds the column; the other slots that reach
    // the same block (extents 1 and 2) stay zero, so the stencil's sum is the column
    Dc2[(((long long)A * 9 + slot) * nb + i) * nb + j] = R[(long long)j * nc2 + (long long)A * 2 * q.nv + i];
}

void restrict2_fields(lqt_ctx* c, const lqt_basis* B, const double2* y1, double2* x2, int nrhs) {
    if (nrhs <= 0) return;
    const PG q = pg2_of(B);
    for (int r0 = 0; r0 < nrhs; r0 += 65535) {
        const int nr = std::min(65535, nrhs - r0);
        hipLaunchKernelGGL(k_restrict2, dim3(q.nagg * 2, nr), dim3(256), 0, c->stream, B->W2.as<double2>(), q, B->nv,
                           y1 + (size_t)r0 * 2 * q.V * B->nv, x2 + (size_t)r0 * 2 * q.nagg * q.nv);
        LQT_HIP(hipGetLastError());
    }
}

void prolong2_fields(lqt_ctx* c, const lqt_basis* B, const double2* x2, double2* y1, int nrhs) {
    if (nrhs <= 0) return;
    const PG q = pg2_of(B);
    for (int r0 = 0; r0 < nrhs; r0 += 65535) {
        const int nr = std::min(65535, nrhs - r0);
        hipLaunchKernelGGL(k_prolong2, dim3(q.nagg * 2, nr), dim3(256), 0, c->stream, B->W2.as<double2>(), q, B->nv,
                           x2 + (size_t)r0 * 2 * q.nagg * q.nv, y1 + (size_t)r0 * 2 * q.V * B->nv);
        LQT_HIP(hipGetLastError());
    }
}

void level2_blocks(lqt_ctx* c, lqt_basis* B, const double2* Y) {
    const PG q = pg2_of(B);
    const long long tot = (long long)q.nagg * 2 * q.nv * q.d;
    B->W2.ensure(sizeof(double2) * (size_t)tot);
    hipLaunchKernelGGL(k_gather2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, Y, q, B->nv,
                       B->W2.as<double2>());
    LQT_HIP(hipGetLastError());
    block_mgs(c, B->W2.as<double2>(), q, q.nagg * 2);
}

void level2_build(lqt_ctx* c, lqt_basis* B) {
    LQT_CHECK(B->Dc.p && B->W2.p, LQT_ESTATE, "level-2 operator needs D_c and W2");
    const auto t0 = std::chrono::steady_clock::now();
    const PG q = pg2_of(B);
    const Colours k = colours_of(q);
    const int nb = 2 * q.nv;
    const long long nc1 = 2LL * q.V * B->nv, nc2 = 2LL * q.nagg * q.nv;
    B->Dc2.ensure(sizeof(double2) * (size_t)q.nagg * 9 * nb * nb);
    LQT_HIP(hipMemsetAsync(B->Dc2.p, 0, sizeof(double2) * (size_t)q.nagg * 9 * nb * nb, c->stream));
    DBuf Y, AY, R;
    Y.ensure(sizeof(double2) * (size_t)nc1 * nb);
    AY.ensure(sizeof(double2) * (size_t)nc1 * nb);
    R.ensure(sizeof(double2) * (size_t)nc2 * nb);
    for (int col = 0; col < k.n; col++) {
        const long long tot = nc1 * nb;
        hipLaunchKernelGGL(k_probe2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream,
                           B->W2.as<double2>(), q, B->nv, k, col, nb, Y.as<double2>());
        LQT_HIP(hipGetLastError());
        coarse_explicit_apply(c, B, Y.as<double2>(), AY.as<double2>(), nb, false);
        restrict2_fields(c, B, AY.as<double2>(), R.as<double2>(), nb);
        const long long ts = (long long)q.nagg * nb * nb;
        hipLaunchKernelGGL(k_scatter2, dim3((unsigned)((ts + 255) / 256)), dim3(256), 0, c->stream, R.as<double2>(), q, k,
                           col, nb, B->Dc2.as<double2>());
        LQT_HIP(hipGetLastError());
    }
    LQT_HIP(hipStreamSynchronize(c->stream));
    B->level2_build_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void level2_apply(lqt_ctx* c, const lqt_basis* B, const double2* in, double2* out, int nrhs, bool herm) {
    LQT_CHECK(B->Dc2.p, LQT_ESTATE, "level-2 operator not built");
    coarse_stencil_apply(c, pg2_of(B), B->Dc2.as<double2>(), in, out, nrhs, herm);
}

}  // namespace lqt
