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

// part[(f * nchunk + blk) * ni + i] = sum over the block's entries of conj(V_i,f) w_f, for
// i < ni; vector i of field f at V + i * vstride + f * len, w_f at w + f * len
__global__ __launch_bounds__(256) void k_mdot_part(const double2* __restrict__ V, long long vstride,
                                                   const double2* __restrict__ w, long long len, int ni,
                                                   double2* __restrict__ part) {
    __shared__ double red[4][2];
    const int f = blockIdx.y, blk = blockIdx.x, nchunk = gridDim.x;
    const long long e0 = (long long)blk * TG_CHUNK;
    const long long e1 = (e0 + TG_CHUNK < len) ? e0 + TG_CHUNK : len;
    const double2* wf = w + (long long)f * len;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = 0; i < ni; i++) {
        const double2* vi = V + (long long)i * vstride + (long long)f * len;
        double a = 0, b = 0;
        for (long long e = e0 + threadIdx.x; e < e1; e += 256) {
            const double2 x = vi[e], y = wf[e];
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

// w_f += sgn * sum_{i < ni} coef[i * nf + f] V_i,f  (coef on the device)
__global__ __launch_bounds__(256) void k_maxpy(double2* __restrict__ w, const double2* __restrict__ V,
                                               long long vstride, long long len, int ni, int nf,
                                               const double2* __restrict__ coef, double sgn) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    const int f = blockIdx.y;
    if (e >= len) return;
    double2 acc = w[(long long)f * len + e];
    for (int i = 0; i < ni; i++) {
        const double2 h = coef[i * nf + f];
        const double2 v = V[(long long)i * vstride + (long long)f * len + e];
        acc.x += sgn * (h.x * v.x - h.y * v.y);
        acc.y += sgn * (h.x * v.y + h.y * v.x);
    }
    w[(long long)f * len + e] = acc;
}

// y_f = a_f x_f (a real, on the device)
__global__ __launch_bounds__(256) void k_scale_into(double2* __restrict__ y, const double2* __restrict__ x,
                                                    long long len, const double* __restrict__ a) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    const int f = blockIdx.y;
    if (e >= len) return;
    const double2 v = x[(long long)f * len + e];
    y[(long long)f * len + e] = make_double2(a[f] * v.x, a[f] * v.y);
}

// r = b - w over total entries
__global__ void k_diff(double2* __restrict__ r, const double2* __restrict__ b, const double2* __restrict__ w,
                       long long total) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    r[i] = make_double2(b[i].x - w[i].x, b[i].y - w[i].y);
}

namespace {

struct Work {
    DBuf part, out, coef;
};

// out (host) [i * nf + f] = V_i,f^+ w_f for i < ni
void mdot(lqt_ctx* c, Work& wk, const double2* V, long long vstride, const double2* w, long long len, int ni, int nf,
          std::vector<zd>& out) {
    const int nchunk = (int)((len + TG_CHUNK - 1) / TG_CHUNK);
    wk.part.ensure(sizeof(double2) * (size_t)nf * nchunk * ni);
    wk.out.ensure(sizeof(double2) * (size_t)nf * ni);
    hipLaunchKernelGGL(k_mdot_part, dim3(nchunk, nf), dim3(256), 0, c->stream, V, vstride, w, len, ni,
                       wk.part.as<double2>());
    LQT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mdot_sum, dim3((ni * nf + 255) / 256), dim3(256), 0, c->stream, wk.part.as<double2>(), nchunk,
                       ni, nf, wk.out.as<double2>());
    LQT_HIP(hipGetLastError());
    out.resize((size_t)ni * nf);
    LQT_HIP(hipMemcpyAsync(out.data(), wk.out.p, sizeof(double2) * out.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
}

void maxpy(lqt_ctx* c, Work& wk, double2* w, const double2* V, long long vstride, long long len, int ni, int nf,
           const std::vector<zd>& coef, double sgn) {
    wk.coef.ensure(sizeof(double2) * coef.size());
    LQT_HIP(hipMemcpyAsync(wk.coef.p, coef.data(), sizeof(double2) * coef.size(), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_maxpy, dim3((unsigned)((len + 255) / 256), nf), dim3(256), 0, c->stream, w, V, vstride, len,
                       ni, nf, wk.coef.as<double2>(), sgn);
    LQT_HIP(hipGetLastError());
}

void scale_into(lqt_ctx* c, Work& wk, double2* y, const double2* x, long long len, int nf, const std::vector<double>& a) {
    wk.coef.ensure(sizeof(double) * a.size());
    LQT_HIP(hipMemcpyAsync(wk.coef.p, a.data(), sizeof(double) * a.size(), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_scale_into, dim3((unsigned)((len + 255) / 256), nf), dim3(256), 0, c->stream, y, x, len,
                       wk.coef.as<double>());
    LQT_HIP(hipGetLastError());
}

void diff(lqt_ctx* c, double2* r, const double2* b, const double2* w, long long total) {
    hipLaunchKernelGGL(k_diff, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, r, b, w, total);
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
        scale_into(c, wk, V, r, nc, nf, inv);
        std::fill(H.begin(), H.end(), zd(0));
        std::fill(g.begin(), g.end(), zd(0));
        for (int f = 0; f < nf; f++) g[(size_t)f * (m + 1)] = beta[f];
        int jend = 0;
        for (int j = 0; j < m && its < maxit; j++) {
            coarse_explicit_apply(c, B, V + (size_t)j * vs, w, nf, false);
            std::vector<zd> h((size_t)(j + 1) * nf, zd(0));
            for (int pass = 0; pass < 2; pass++) {  // classical Gram-Schmidt, twice
                std::vector<zd> hp;
                mdot(c, wk, V, vs, w, nc, j + 1, nf, hp);
                maxpy(c, wk, w, V, vs, nc, j + 1, nf, hp, -1.0);
                for (size_t e = 0; e < h.size(); e++) h[e] += hp[e];
            }
            std::vector<zd> wn;
            mdot(c, wk, w, 0, w, nc, 1, nf, wn);
            for (int f = 0; f < nf; f++) {
                const double hn = std::sqrt(std::max(0.0, wn[f].real()));
                inv[f] = hn > 0 ? 1.0 / hn : 0.0;
                zd* Hf = H.data() + (size_t)f * (m + 1) * m;
                for (int i = 0; i <= j; i++) Hf[(size_t)i * m + j] = h[(size_t)i * nf + f];
                Hf[(size_t)(j + 1) * m + j] = hn;
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
            scale_into(c, wk, V + (size_t)(j + 1) * vs, w, nc, nf, inv);
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
        maxpy(c, wk, x, V, vs, nc, jend, nf, y, 1.0);
        // true coarse residual
        coarse_explicit_apply(c, B, x, w, nf, false);
        diff(c, r, b, w, vs);
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
    c->tg_work[0].ensure(sizeof(double2) * (size_t)tot * 4);
    c->tg_work[1].ensure(sizeof(double2) * (size_t)nf * nc * 2);
    double2* r = c->tg_work[0].as<double2>();
    double2* x = r + tot;
    double2* s = x + tot;
    double2* p = s + tot;
    double2* rc = c->tg_work[1].as<double2>();
    double2* ec = rc + (size_t)nf * nc;
    fields_to_f64<S>(c, v, r, tot);
    // coarse grid correction
    restrict_fields(c, B, r, rc, nf);
    coarse_gmres(c, B, rc, ec, nf, o.tg_coarse_tol, o.tg_coarse_maxit);
    prolong_fields(c, B, ec, x, nf);
    // smoothing: minimal-residual steps on A
    if (o.tg_smooth > 0) {
        Work wk;
        dslash(c, LQT_F64, LQT_A, x, p, nf, n, n);
        diff(c, s, r, p, tot);
        std::vector<zd> ps, pp;
        std::vector<zd> a(nf), na(nf);
        for (int it = 0; it < o.tg_smooth; it++) {
            dslash(c, LQT_F64, LQT_A, s, p, nf, n, n);
            mdot(c, wk, p, 0, s, n, 1, nf, ps);
            mdot(c, wk, p, 0, p, n, 1, nf, pp);
            for (int f = 0; f < nf; f++) {
                a[f] = pp[f].real() > 0 ? ps[f] / pp[f].real() : zd(0);
                na[f] = -a[f];
            }
            maxpy(c, wk, x, s, 0, n, 1, nf, a, 1.0);
            maxpy(c, wk, s, p, 0, n, 1, nf, na, 1.0);
        }
    }
    fields_from_f64<S>(c, x, z, tot);
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
        lqt::twogrid_apply<double2>(c, in.as<double2>(), out.as<double2>(), nrhs, o);
        lqt::from_device_layout(c, out.as<double2>(), (double2*)d_out, nrhs);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}
