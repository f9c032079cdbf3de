// Batched MINRES (Paige and Saunders) for a Hermitian indefinite operator, FP64.
//
// Used for the inexact inverses of the eigensolvers: (A g5)^{-1}_xi on the fine lattice and
// (g5^W W^+ A W)^{-1}_xi on the coarse space of a prolongator.  A short recurrence with no
// restart, so right-hand sides made of near-null modes (what inverse iteration produces) do
// not stall it the way restarted GMRES stalls.  The Lanczos coefficients of a Hermitian
// operator are real; the scalar recurrences run on the host, vectors are generic FP64
// complex arrays of length n, one batch of vector kernels per step.
#include <cmath>
#include <vector>

#include "blas.h"
#include "lqt_internal.h"
#include "minres.h"

namespace lqt {

__device__ __forceinline__ double msum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void mr_block_store(double a, double* part) {
    __shared__ double red[4];
    a = msum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// y_f <- y_f - c_f r1_f ; partial Re(v_f^+ y_f)     grid (nblk, nf)
__global__ __launch_bounds__(256) void k_mr_step1(double2* __restrict__ y, const double2* __restrict__ r1,
                                                  const double2* __restrict__ v, const double* __restrict__ cf,
                                                  long long n, double* __restrict__ part) {
    const int f = blockIdx.y;
    const long long o = f * n;
    const double c = cf[f];
    double a = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        double2 yy = y[o + i], rr = r1[o + i], vv = v[o + i];
        yy.x -= c * rr.x;
        yy.y -= c * rr.y;
        y[o + i] = yy;
        a += vv.x * yy.x + vv.y * yy.y;
    }
    mr_block_store(a, part);
}

// y_f <- y_f - c_f r2_f ; partial |y_f|^2
__global__ __launch_bounds__(256) void k_mr_step2(double2* __restrict__ y, const double2* __restrict__ r2,
                                                  const double* __restrict__ cf, long long n,
                                                  double* __restrict__ part) {
    const int f = blockIdx.y;
    const long long o = f * n;
    const double c = cf[f];
    double a = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        double2 yy = y[o + i], rr = r2[o + i];
        yy.x -= c * rr.x;
        yy.y -= c * rr.y;
        y[o + i] = yy;
        a += yy.x * yy.x + yy.y * yy.y;
    }
    mr_block_store(a, part);
}

// w_new = (v - e_f w1 - d_f w2) g_f (written over w1), x += p_f w_new, v = s_f r2 for the next
// step; co[f] = {e, d, g, p, s}
__global__ __launch_bounds__(256) void k_mr_update(double2* __restrict__ x, double2* __restrict__ w1,
                                                   const double2* __restrict__ w2, double2* __restrict__ v,
                                                   const double2* __restrict__ r2, const double* __restrict__ co,
                                                   long long n) {
    const int f = blockIdx.y;
    const long long o = f * n;
    const double e = co[5 * f], d = co[5 * f + 1], g = co[5 * f + 2], p = co[5 * f + 3], sn = co[5 * f + 4];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        double2 vv = v[o + i], a = w1[o + i], b = w2[o + i];
        double2 w = make_double2((vv.x - e * a.x - d * b.x) * g, (vv.y - e * a.y - d * b.y) * g);
        w1[o + i] = w;
        double2 xx = x[o + i];
        x[o + i] = make_double2(xx.x + p * w.x, xx.y + p * w.y);
        double2 rr = r2[o + i];
        v[o + i] = make_double2(sn * rr.x, sn * rr.y);
    }
}

// partial |b_f|^2
__global__ __launch_bounds__(256) void k_mr_norm(const double2* __restrict__ b, long long n,
                                                 double* __restrict__ part) {
    const int f = blockIdx.y;
    const long long o = f * n;
    double a = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        double2 v = b[o + i];
        a += v.x * v.x + v.y * v.y;
    }
    mr_block_store(a, part);
}

__global__ void k_mr_sum(const double* __restrict__ part, int nparts, double* __restrict__ out) {
    const int f = blockIdx.x;
    double a = 0;
    for (int k = threadIdx.x; k < nparts; k += 64) a += part[(long long)f * nparts + k];
    a = msum(a);
    if (threadIdx.x == 0) out[f] = a;
}

__global__ void k_mr_scale(const double2* __restrict__ src, double2* __restrict__ dst, const double* __restrict__ sf,
                           long long n) {
    const int f = blockIdx.y;
    const long long o = f * n;
    const double c = sf[f];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        double2 a = src[o + i];
        dst[o + i] = make_double2(c * a.x, c * a.y);
    }
}

int minres(lqt_ctx* c, long long n, const HermOp& H, const double2* b, double2* x, int nf, double tol, int maxit,
           std::vector<int>* iters) {
    const int nblk = (int)std::min<long long>(1024, (n + 255) / 256);
    const size_t fb = sizeof(double2) * (size_t)nf * n;
    DBuf bufs[6];
    for (auto& d : bufs) d.ensure(fb);
    double2 *r1 = bufs[0].as<double2>(), *r2 = bufs[1].as<double2>(), *y = bufs[2].as<double2>(),
            *v = bufs[3].as<double2>(), *w1 = bufs[4].as<double2>(), *w2 = bufs[5].as<double2>();
    DBuf part, sc;
    part.ensure(sizeof(double) * (size_t)nblk * nf);
    sc.ensure(sizeof(double) * 8 * (size_t)nf);
    double* dsc = sc.as<double>();
    const dim3 g2(nblk, nf);
    LQT_HIP(hipMemsetAsync(x, 0, fb, c->stream));
    LQT_HIP(hipMemsetAsync(w1, 0, fb, c->stream));
    LQT_HIP(hipMemsetAsync(w2, 0, fb, c->stream));
    LQT_HIP(hipMemcpyAsync(r1, b, fb, hipMemcpyDeviceToDevice, c->stream));
    LQT_HIP(hipMemcpyAsync(r2, b, fb, hipMemcpyDeviceToDevice, c->stream));
    std::vector<double> h(8 * (size_t)nf);
    hipLaunchKernelGGL(k_mr_norm, g2, dim3(256), 0, c->stream, b, n, part.as<double>());
    hipLaunchKernelGGL(k_mr_sum, dim3(nf), dim3(64), 0, c->stream, part.as<double>(), nblk, dsc);
    LQT_HIP(hipGetLastError());
    LQT_HIP(hipMemcpyAsync(h.data(), dsc, sizeof(double) * nf, hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    std::vector<double> beta1(nf), beta(nf), oldb(nf, 0.0), dbar(nf, 0.0), epsln(nf, 0.0), phibar(nf), cs(nf, -1.0),
        sn(nf, 0.0), alfa(nf);
    std::vector<int> its(nf, 0), done(nf, 0);
    for (int f = 0; f < nf; f++) {
        beta1[f] = std::sqrt(h[f]);
        beta[f] = beta1[f];
        phibar[f] = beta1[f];
        done[f] = beta1[f] == 0;
        h[f] = beta1[f] > 0 ? 1.0 / beta1[f] : 0.0;
    }
    LQT_HIP(hipMemcpyAsync(dsc, h.data(), sizeof(double) * nf, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_mr_scale, g2, dim3(256), 0, c->stream, b, v, dsc, n);  // v = b / beta1
    LQT_HIP(hipGetLastError());
    int nact = 0;
    for (int f = 0; f < nf; f++) nact += !done[f];
    std::vector<double> co(5 * (size_t)nf, 0.0);
    for (int it = 1; it <= maxit && nact > 0; it++) {
        H(v, y, nf);  // y = H v
        // y -= (beta/oldb) r1 ; alfa = v^+ y
        for (int f = 0; f < nf; f++) h[f] = (it >= 2 && oldb[f] > 0) ? beta[f] / oldb[f] : 0.0;
        LQT_HIP(hipMemcpyAsync(dsc, h.data(), sizeof(double) * nf, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_mr_step1, g2, dim3(256), 0, c->stream, y, r1, v, dsc, n, part.as<double>());
        hipLaunchKernelGGL(k_mr_sum, dim3(nf), dim3(64), 0, c->stream, part.as<double>(), nblk, dsc + nf);
        LQT_HIP(hipGetLastError());
        LQT_HIP(hipMemcpyAsync(h.data() + nf, dsc + nf, sizeof(double) * nf, hipMemcpyDeviceToHost, c->stream));
        LQT_HIP(hipStreamSynchronize(c->stream));
        for (int f = 0; f < nf; f++) alfa[f] = h[nf + f];
        // y -= (alfa/beta) r2 ; new beta = |y|
        for (int f = 0; f < nf; f++) h[f] = beta[f] > 0 ? alfa[f] / beta[f] : 0.0;
        LQT_HIP(hipMemcpyAsync(dsc, h.data(), sizeof(double) * nf, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_mr_step2, g2, dim3(256), 0, c->stream, y, r2, dsc, n, part.as<double>());
        hipLaunchKernelGGL(k_mr_sum, dim3(nf), dim3(64), 0, c->stream, part.as<double>(), nblk, dsc + nf);
        LQT_HIP(hipGetLastError());
        LQT_HIP(hipMemcpyAsync(h.data() + nf, dsc + nf, sizeof(double) * nf, hipMemcpyDeviceToHost, c->stream));
        LQT_HIP(hipStreamSynchronize(c->stream));
        std::swap(r1, r2);  // r1 <- r2, r2 <- y
        std::swap(r2, y);
        nact = 0;
        for (int f = 0; f < nf; f++) {
            double* cf = co.data() + 5 * f;
            if (done[f]) {  // finished: x stays, directions and v become zero
                cf[0] = cf[1] = cf[2] = cf[3] = cf[4] = 0;
                continue;
            }
            oldb[f] = beta[f];
            beta[f] = std::sqrt(std::max(h[nf + f], 0.0));
            const double oldeps = epsln[f];
            const double delta = cs[f] * dbar[f] + sn[f] * alfa[f];
            const double gbar = sn[f] * dbar[f] - cs[f] * alfa[f];
            epsln[f] = sn[f] * beta[f];
            dbar[f] = -cs[f] * beta[f];
            double gamma = std::max(std::sqrt(gbar * gbar + beta[f] * beta[f]), 1e-300);
            cs[f] = gbar / gamma;
            sn[f] = beta[f] / gamma;
            const double phi = cs[f] * phibar[f];
            phibar[f] = sn[f] * phibar[f];
            cf[0] = oldeps;
            cf[1] = delta;
            cf[2] = 1.0 / gamma;
            cf[3] = phi;
            cf[4] = beta[f] > 0 ? 1.0 / beta[f] : 0.0;
            its[f] = it;
            if (phibar[f] <= tol * beta1[f] || !(beta[f] > 0)) done[f] = 1;
            nact += !done[f];
        }
        LQT_HIP(hipMemcpyAsync(dsc, co.data(), sizeof(double) * 5 * nf, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_mr_update, g2, dim3(256), 0, c->stream, x, w1, w2, v, r2, dsc, n);
        LQT_HIP(hipGetLastError());
        std::swap(w1, w2);  // w2 now holds the newest direction
        LQT_HIP(hipStreamSynchronize(c->stream));
    }
    int nfail = 0;
    for (int f = 0; f < nf; f++) nfail += (phibar[f] > tol * beta1[f]) ? 1 : 0;
    if (iters) *iters = its;
    return nfail;
}

}  // namespace lqt
