// Two-grid preconditioner from the prolongator W (Section 2, the two-grid method), as the
// right preconditioner of flexible GMRES.  One application to v, from x = 0:
//   coarse grid correction  x_c = W D_c^{-1} W^+ v with the explicit coarse operator
//                           D_c = W^+ A W (9-point block stencil), solved by batched FP64
//                           GMRES(TG_M) to the relative tolerance tg_coarse_tol (at most
//                           tg_coarse_maxit steps);
//   smoothing               tg_smooth minimal-residual steps on A from x_c: s = v - A x_c,
//                           p = A s, a = p^+ s / p^+ p, x += a s, s -= a p.
// Everything runs in FP64 on the device; the Krylov vectors of the outer solver are converted
// from and to their storage precision at the two ends.  The coarse solve and the smoothing
// depend on v (a nonlinear preconditioner), which flexible GMRES allows.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "hostla.h"
#include "krylov.h"
#include "lqt_internal.h"
#include "prolong.h"
#include "solver.h"
#include "twogrid.h"

namespace lqt {

constexpr int TG_M = 16;        // coarse GMRES restart length
constexpr int TG_CHUNK = 4096;  // vector entries per workgroup of the batched dot products

// element access in FP64 for every storage type
template <typename T>
__device__ __forceinline__ double2 ldd(const T* p) {
    if constexpr (sizeof(T) == 16) {
        return *(const double2*)p;
    } else {
        const float2 v = io<T>::ld(p);
        return make_double2(v.x, v.y);
    }
}
template <typename T>
__device__ __forceinline__ void std_(T* p, double2 v) {
    if constexpr (sizeof(T) == 16)
        *(double2*)p = v;
    else
        io<T>::st(p, make_float2((float)v.x, (float)v.y));
}

// part[(f * nchunk + blk) * ni + i] = sum over the block's entries of conj(V_i,f) w_f, for
// i < ni; vector i of field f at V + i * vstride + f * len, w_f at w + f * len (FP64 sums)
template <typename T>
__global__ __launch_bounds__(256) void k_mdot_part(const T* __restrict__ V, long long vstride,
                                                   const T* __restrict__ w, long long len, int ni,
                                                   double2* __restrict__ part) {
    __shared__ double red[4][2];
    const int f = blockIdx.y, blk = blockIdx.x, nchunk = gridDim.x;
    const long long e0 = (long long)blk * TG_CHUNK;
    const long long e1 = (e0 + TG_CHUNK < len) ? e0 + TG_CHUNK : len;
    const T* wf = w + (long long)f * len;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = 0; i < ni; i++) {
        const T* vi = V + (long long)i * vstride + (long long)f * len;
        double a = 0, b = 0;
        for (long long e = e0 + threadIdx.x; e < e1; e += 256) {
            const double2 x = ldd(vi + e), y = ldd(wf + e);
            a += x.x * y.x + x.y * y.y;
            b += x.x * y.y - x.y * y.x;
        }
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o);
            b += __shfl_xor(b, o);
        }
        if (lane == 0) red[wave][0] = a, red[wave][1] = b;
        __syncthreads();
        if (threadIdx.x == 0)
            part[((long long)f * nchunk + blk) * ni + i] =
                make_double2(red[0][0] + red[1][0] + red[2][0] + red[3][0], red[0][1] + red[1][1] + red[2][1] + red[3][1]);
        __syncthreads();
    }
}

// out[i * nf + f] = sum over the chunks of part
__global__ void k_mdot_sum(const double2* __restrict__ part, int nchunk, int ni, int nf, double2* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ni * nf) return;
    const int i = t / nf, f = t % nf;
    double a = 0, b = 0;
    for (int q = 0; q < nchunk; q++) {
        const double2 p = part[((long long)f * nchunk + q) * ni + i];
        a += p.x;
        b += p.y;
    }
    out[t] = make_double2(a, b);
}

// y_f = sc[f] (w_f + sgn * sum_{i < ni} coef[i * nf + f] V_i,f)  (coefficients on the device;
// sc = nullptr: no scaling; y may be w)
template <typename T>
__global__ __launch_bounds__(256) void k_maxpy(T* y, const T* w, const T* __restrict__ V,
                                               long long vstride, long long len, int ni, int nf,
                                               const double2* __restrict__ coef, double sgn,
                                               const double* __restrict__ sc) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    const int f = blockIdx.y;
    if (e >= len) return;
    double2 acc = ldd(w + (long long)f * len + e);
    for (int i = 0; i < ni; i++) {
        const double2 h = coef[i * nf + f];
        const double2 v = ldd(V + (long long)i * vstride + (long long)f * len + e);
        acc.x += sgn * (h.x * v.x - h.y * v.y);
        acc.y += sgn * (h.x * v.y + h.y * v.x);
    }
    if (sc) acc = make_double2(sc[f] * acc.x, sc[f] * acc.y);
    std_(y + (long long)f * len + e, acc);
}

// r = b - w over total entries
template <typename T>
__global__ void k_diff(T* __restrict__ r, const T* __restrict__ b, const T* __restrict__ w, long long total) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const double2 x = ldd(b + i), y = ldd(w + i);
    std_(r + i, make_double2(x.x - y.x, x.y - y.y));
}

template <typename S, typename T>
__global__ void k_convert(const S* __restrict__ in, T* __restrict__ out, long long total) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    std_(out + i, ldd(in + i));
}

namespace {

struct Work {
    DBuf part, out, coef, sc;
};

// out (host) [i * nf + f] = V_i,f^+ w_f for i < ni
template <typename T>
void mdot(lqt_ctx* c, Work& wk, const T* V, long long vstride, const T* w, long long len, int ni, int nf,
          std::vector<zd>& out) {
    const int nchunk = (int)((len + TG_CHUNK - 1) / TG_CHUNK);
    wk.part.ensure(sizeof(double2) * (size_t)nf * nchunk * ni);
    wk.out.ensure(sizeof(double2) * (size_t)nf * ni);
    hipLaunchKernelGGL(k_mdot_part<T>, dim3(nchunk, nf), dim3(256), 0, c->stream, V, vstride, w, len, ni,
                       wk.part.as<double2>());
    LQT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mdot_sum, dim3((ni * nf + 255) / 256), dim3(256), 0, c->stream, wk.part.as<double2>(), nchunk,
                       ni, nf, wk.out.as<double2>());
    LQT_HIP(hipGetLastError());
    out.resize((size_t)ni * nf);
    LQT_HIP(hipMemcpyAsync(out.data(), wk.out.p, sizeof(double2) * out.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
}

// y_f = scale_f (w_f + sgn sum_i coef[i][f] V_i,f); scale empty: none
template <typename T>
void maxpy(lqt_ctx* c, Work& wk, T* y, const T* w, const T* V, long long vstride, long long len, int ni, int nf,
           const std::vector<zd>& coef, double sgn, const std::vector<double>& scale) {
    wk.coef.ensure(sizeof(double2) * std::max<size_t>(1, coef.size()));
    if (!coef.empty())
        LQT_HIP(hipMemcpyAsync(wk.coef.p, coef.data(), sizeof(double2) * coef.size(), hipMemcpyHostToDevice, c->stream));
    const double* sc = nullptr;
    if (!scale.empty()) {
        wk.sc.ensure(sizeof(double) * scale.size());
        LQT_HIP(hipMemcpyAsync(wk.sc.p, scale.data(), sizeof(double) * scale.size(), hipMemcpyHostToDevice, c->stream));
        sc = wk.sc.as<double>();
    }
    hipLaunchKernelGGL(k_maxpy<T>, dim3((unsigned)((len + 255) / 256), nf), dim3(256), 0, c->stream, y, w, V, vstride,
                       len, ni, nf, wk.coef.as<double2>(), sgn, sc);
    LQT_HIP(hipGetLastError());
}

template <typename T>
void diff(lqt_ctx* c, T* r, const T* b, const T* w, long long total) {
    hipLaunchKernelGGL(k_diff<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, r, b, w, total);
    LQT_HIP(hipGetLastError());
}

template <typename S, typename T>
void convert(lqt_ctx* c, const S* in, T* out, long long total) {
    hipLaunchKernelGGL((k_convert<S, T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, in, out,
                       total);
    LQT_HIP(hipGetLastError());
}

}  // namespace

double coarse_gmres(lqt_ctx* c, const lqt_basis* B, const double2* b, double2* x, int nf, double tol, int maxit) {
    const long long nc = 2LL * B->nagg * B->nv;
    const int m = TG_M;
    const long long vs = (long long)nf * nc;  // stride between basis vectors
    Work wk;
    DBuf Vb, wb, rb;
    Vb.ensure(sizeof(double2) * (size_t)(m + 1) * vs);
    wb.ensure(sizeof(double2) * (size_t)vs);
    rb.ensure(sizeof(double2) * (size_t)vs);
    double2* V = Vb.as<double2>();
    double2* w = wb.as<double2>();
    double2* r = rb.as<double2>();
    const std::vector<double> none;
    LQT_HIP(hipMemsetAsync(x, 0, sizeof(double2) * (size_t)vs, c->stream));
    LQT_HIP(hipMemcpyAsync(r, b, sizeof(double2) * (size_t)vs, hipMemcpyDeviceToDevice, c->stream));
    std::vector<zd> d;
    mdot(c, wk, r, 0, r, nc, 1, nf, d);
    std::vector<double> bn(nf), beta(nf);
    for (int f = 0; f < nf; f++) bn[f] = beta[f] = std::sqrt(std::max(0.0, d[f].real()));
    auto worst = [&]() {
        double mx = 0;
        for (int f = 0; f < nf; f++) mx = std::max(mx, bn[f] > 0 ? beta[f] / bn[f] : 0.0);
        return mx;
    };
    int its = 0;
    std::vector<zd> H((size_t)nf * (m + 1) * m), g((size_t)nf * (m + 1)), sn((size_t)nf * m);
    std::vector<double> cs((size_t)nf * m), inv(nf);
    while (worst() > tol && its < maxit) {
        for (int f = 0; f < nf; f++) inv[f] = beta[f] > 0 ? 1.0 / beta[f] : 0.0;
        maxpy<double2>(c, wk, V, r, V, 0, nc, 0, nf, {}, 0.0, inv);  // V_0 = r / beta
        std::fill(H.begin(), H.end(), zd(0));
        std::fill(g.begin(), g.end(), zd(0));
        for (int f = 0; f < nf; f++) g[(size_t)f * (m + 1)] = beta[f];
        int jend = 0;
        for (int j = 0; j < m && its < maxit; j++) {
            double2* wj = V + (size_t)(j + 1) * vs;  // A v_j is formed in place of v_{j+1}
            coarse_explicit_apply(c, B, V + (size_t)j * vs, wj, nf, false);
            // classical Gram-Schmidt with the new vector's own norm in the same pass:
            // |w - V h|^2 = |w|^2 - |h|^2 for orthonormal V; a second pass when that loses
            // more than 90 % of |w| to cancellation
            std::vector<zd> hp;
            mdot(c, wk, V, vs, wj, nc, j + 2, nf, hp);
            std::vector<zd> h(hp.begin(), hp.begin() + (size_t)(j + 1) * nf);
            std::vector<double> hn(nf);
            bool again = false;
            for (int f = 0; f < nf; f++) {
                double hh = 0;
                for (int i = 0; i <= j; i++) hh += std::norm(h[(size_t)i * nf + f]);
                const double ww = hp[(size_t)(j + 1) * nf + f].real();
                const double rem = ww - hh;
                if (!(rem > 0.01 * ww)) again = true;
                hn[f] = std::sqrt(std::max(0.0, rem));
            }
            if (again) {
                maxpy<double2>(c, wk, wj, wj, V, vs, nc, j + 1, nf, h, -1.0, none);
                std::vector<zd> h2;
                mdot(c, wk, V, vs, wj, nc, j + 2, nf, h2);
                std::vector<zd> h2v(h2.begin(), h2.begin() + (size_t)(j + 1) * nf);
                for (int f = 0; f < nf; f++) {
                    double hh = 0;
                    for (int i = 0; i <= j; i++) hh += std::norm(h2v[(size_t)i * nf + f]);
                    hn[f] = std::sqrt(std::max(0.0, h2[(size_t)(j + 1) * nf + f].real() - hh));
                }
                for (size_t e = 0; e < h.size(); e++) h[e] += h2v[e];
                for (int f = 0; f < nf; f++) inv[f] = hn[f] > 0 ? 1.0 / hn[f] : 0.0;
                maxpy<double2>(c, wk, wj, wj, V, vs, nc, j + 1, nf, h2v, -1.0, inv);
            } else {
                for (int f = 0; f < nf; f++) inv[f] = hn[f] > 0 ? 1.0 / hn[f] : 0.0;
                maxpy<double2>(c, wk, wj, wj, V, vs, nc, j + 1, nf, h, -1.0, inv);
            }
            for (int f = 0; f < nf; f++) {
                zd* Hf = H.data() + (size_t)f * (m + 1) * m;
                for (int i = 0; i <= j; i++) Hf[(size_t)i * m + j] = h[(size_t)i * nf + f];
                Hf[(size_t)(j + 1) * m + j] = hn[f];
                // Givens rotations of column j
                zd* gf = g.data() + (size_t)f * (m + 1);
                for (int i = 0; i < j; i++) {
                    const double cc = cs[(size_t)f * m + i];
                    const zd ss = sn[(size_t)f * m + i];
                    const zd a = Hf[(size_t)i * m + j], bb = Hf[(size_t)(i + 1) * m + j];
                    Hf[(size_t)i * m + j] = cc * a + ss * bb;
                    Hf[(size_t)(i + 1) * m + j] = -std::conj(ss) * a + cc * bb;
                }
                const zd a = Hf[(size_t)j * m + j], bb = Hf[(size_t)(j + 1) * m + j];
                const double den = std::sqrt(std::norm(a) + std::norm(bb));
                double cc = 1.0;
                zd ss = 0;
                if (den > 0) {
                    if (std::abs(a) > 0) {
                        cc = std::abs(a) / den;
                        ss = (a / std::abs(a)) * std::conj(bb) / den;
                    } else {
                        cc = 0;
                        ss = 1;
                    }
                }
                cs[(size_t)f * m + j] = cc;
                sn[(size_t)f * m + j] = ss;
                Hf[(size_t)j * m + j] = cc * a + ss * bb;
                Hf[(size_t)(j + 1) * m + j] = 0;
                const zd gj = gf[j];
                gf[j] = cc * gj;
                gf[j + 1] = -std::conj(ss) * gj;
            }
            its++;
            jend = j + 1;
            double mx = 0;
            for (int f = 0; f < nf; f++)
                mx = std::max(mx, bn[f] > 0 ? std::abs(g[(size_t)f * (m + 1) + j + 1]) / bn[f] : 0.0);
            if (mx <= tol) break;
        }
        // y = R^{-1} g per system, x += V y
        std::vector<zd> y((size_t)jend * nf, zd(0));
        for (int f = 0; f < nf; f++) {
            const zd* Hf = H.data() + (size_t)f * (m + 1) * m;
            const zd* gf = g.data() + (size_t)f * (m + 1);
            for (int i = jend - 1; i >= 0; i--) {
                zd acc = gf[i];
                for (int l = i + 1; l < jend; l++) acc -= Hf[(size_t)i * m + l] * y[(size_t)l * nf + f];
                const zd dgl = Hf[(size_t)i * m + i];
                y[(size_t)i * nf + f] = std::abs(dgl) > 0 ? acc / dgl : zd(0);
            }
        }
        maxpy<double2>(c, wk, x, x, V, vs, nc, jend, nf, y, 1.0, none);
        // true coarse residual
        coarse_explicit_apply(c, B, x, w, nf, false);
        diff<double2>(c, r, b, w, vs);
        mdot(c, wk, r, 0, r, nc, 1, nf, d);
        for (int f = 0; f < nf; f++) beta[f] = std::sqrt(std::max(0.0, d[f].real()));
    }
    return worst();
}

template <typename S>
void twogrid_apply(lqt_ctx* c, const S* v, S* z, int nf, const SolveOpts& o) {
    lqt_basis* B = c->tg;
    LQT_CHECK(B && B->Dc.p, LQT_ESTATE, "no two-grid prolongator set (lqt_precond_twogrid)");
    const long long n = 12LL * c->g.V;
    const long long nc = 2LL * B->nagg * B->nv;
    const long long tot = (long long)nf * n;
    // FP64 fine field for restriction and prolongation; the smoother's fields in the outer
    // storage S (the operator of the solve's precision)
    c->tg_work[0].ensure(sizeof(double2) * (size_t)tot + sizeof(S) * (size_t)tot * 2);
    c->tg_work[1].ensure(sizeof(double2) * (size_t)nf * nc * 2);
    double2* f64 = c->tg_work[0].as<double2>();
    S* s = (S*)(f64 + tot);
    S* p = s + tot;
    double2* rc = c->tg_work[1].as<double2>();
    double2* ec = rc + (size_t)nf * nc;
    convert<S, double2>(c, v, f64, tot);
    // coarse grid correction x_c = W D_c^{-1} W^+ v, into z
    restrict_fields(c, B, f64, rc, nf);
    coarse_gmres(c, B, rc, ec, nf, o.tg_coarse_tol, o.tg_coarse_maxit);
    prolong_fields(c, B, ec, f64, nf);
    convert<double2, S>(c, f64, z, tot);
    // smoothing: minimal-residual steps on A in the storage precision
    if (o.tg_smooth > 0) {
        Work wk;
        const std::vector<double> none;
        dslash(c, o.prec, LQT_A, z, p, nf, n, n);
        diff<S>(c, s, v, p, tot);
        std::vector<zd> ps, a(nf), na(nf);
        for (int it = 0; it < o.tg_smooth; it++) {
            dslash(c, o.prec, LQT_A, s, p, nf, n, n);
            mdot<S>(c, wk, p, 0, s, n, 1, nf, ps);
            std::vector<zd> pp;
            mdot<S>(c, wk, p, 0, p, n, 1, nf, pp);
            for (int f = 0; f < nf; f++) {
                a[f] = pp[f].real() > 0 ? ps[f] / pp[f].real() : zd(0);
                na[f] = -a[f];
            }
            maxpy<S>(c, wk, z, z, s, 0, n, 1, nf, a, 1.0, none);
            if (it + 1 < o.tg_smooth) maxpy<S>(c, wk, s, s, p, 0, n, 1, nf, na, 1.0, none);
        }
    }
}

template void twogrid_apply<double2>(lqt_ctx*, const double2*, double2*, int, const SolveOpts&);
template void twogrid_apply<float2>(lqt_ctx*, const float2*, float2*, int, const SolveOpts&);
template void twogrid_apply<h2>(lqt_ctx*, const h2*, h2*, int, const SolveOpts&);
template void twogrid_apply<b2>(lqt_ctx*, const b2*, b2*, int, const SolveOpts&);

}  // namespace lqt

using lqt::Error;

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

}  // namespace

int lqt_precond_twogrid(lqt_ctx* c, lqt_basis* B) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        if (!B) {
            c->tg = nullptr;
            return;
        }
        LQT_CHECK(B->ctx == c && B->kind == 1, LQT_EINVAL, "the two-grid preconditioner needs a prolongator basis "
                                                           "of this context");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "the two-grid preconditioner serves single-lattice contexts");
        lqt::coarse_explicit_build(c, B);
        c->tg = B;
    });
}

int lqt_precond_twogrid_apply(lqt_ctx* c, const double* d_in, double* d_out, int nrhs, const lqt_solver_opts* opts) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(nrhs >= 0 && (nrhs == 0 || (d_in && d_out)), LQT_EINVAL, "bad two-grid apply arguments");
        LQT_CHECK(c->tg, LQT_ESTATE, "no two-grid prolongator set (lqt_precond_twogrid)");
        if (nrhs == 0) return;
        lqt::SolveOpts o = lqt::make_opts(opts);
        const long long n = 12LL * c->g.V;
        lqt::DBuf in, out;
        in.ensure(sizeof(double2) * (size_t)nrhs * n);
        out.ensure(sizeof(double2) * (size_t)nrhs * n);
        lqt::to_device_layout(c, (const double2*)d_in, in.as<double2>(), nrhs);
        o.prec = LQT_F64;
        lqt::twogrid_apply<double2>(c, in.as<double2>(), out.as<double2>(), nrhs, o);
        lqt::from_device_layout(c, out.as<double2>(), (double2*)d_out, nrhs);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}
