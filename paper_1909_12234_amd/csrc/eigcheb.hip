// Eigenpairs of a Hermitian indefinite operator H with the smallest |lambda| (the first step
// of Algorithm 1 for H = A g5, whose eigenvectors are left singular vectors of A; the
// coarse eigensolve of Algorithm 2 for H = g5^W W^+ A W).
//
// Chebyshev-filtered subspace iteration on H^2 with harmonic Rayleigh-Ritz extraction:
//   - the wanted eigenvectors of H are the lowest of the positive semi-definite H^2, so a
//     Chebyshev polynomial of H^2 that is bounded by 1 on [a, b] (b >= ||H||^2, a the
//     largest Ritz value of H^2 in the block) and grows below a enriches the block in
//     them; the filter needs only operator applications on the whole block (one multi-RHS
//     launch per application), no solves and no orthogonalisation;
//   - the smallest |lambda| of H are interior, so ordinary Rayleigh-Ritz with H would give
//     spurious Ritz values near 0; harmonic Ritz pairs with target 0 (the Ritz pairs of
//     H^{-1} on H V, through the Gram matrices (HV)^+ HV and V^+ HV) are not affected;
//   - a pair (theta, q) is accepted when ||H q - theta q|| <= xi |theta|.  Then
//     ||H^{-1} q - q / theta|| <= ||H q - theta q|| / (|theta| sigma_min) <= xi ||H^{-1}||,
//     i.e. the convergence test of the paper's Table 1 holds for the exact inverse.
// The filter runs in FP32 storage and arithmetic when an FP32 operator is given (the
// block's vectors only need to point in the right directions; residuals, Gram matrices and
// the small eigenproblems are FP64).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>

#include "blas.h"
#include "devla.h"
#include "eigcheb.h"
#include "gemm.h"
#include "hostla.h"
#include "lqt_internal.h"

namespace lqt {

template <typename S>
struct acc2;
template <>
struct acc2<double2> {
    using R = double;
};
template <>
struct acc2<float2> {
    using R = float;
};

// out = a u + b v + w_c w (real coefficients) over m complex entries; w may be null
template <typename S>
__global__ __launch_bounds__(256) void k_lincomb(S* __restrict__ out, const S* __restrict__ u,
                                                 const S* __restrict__ v, const S* __restrict__ w, double a, double b,
                                                 double wc, long long m) {
    using R = typename acc2<S>::R;
    const R ra = (R)a, rb = (R)b, rc = (R)wc;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < m; i += (long long)gridDim.x * 256) {
        const S x = u[i], y = v[i];
        S o;
        o.x = ra * x.x + rb * y.x;
        o.y = ra * x.y + rb * y.y;
        if (w) {
            const S z = w[i];
            o.x += rc * z.x;
            o.y += rc * z.y;
        }
        out[i] = o;
    }
}

__global__ __launch_bounds__(256) void k_to_f32(const double2* __restrict__ in, float2* __restrict__ out,
                                                long long m) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < m; i += (long long)gridDim.x * 256)
        out[i] = make_float2((float)in[i].x, (float)in[i].y);
}
__global__ __launch_bounds__(256) void k_to_f64(const float2* __restrict__ in, double2* __restrict__ out,
                                                long long m) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < m; i += (long long)gridDim.x * 256)
        out[i] = make_double2((double)in[i].x, (double)in[i].y);
}

static dim3 grid_of(long long m) { return dim3((unsigned)std::min<long long>((m + 255) / 256, 8192)); }

template <typename S>
static void lincomb(lqt_ctx* c, S* out, const S* u, const S* v, const S* w, double a, double b, double wc,
                    long long m) {
    hipLaunchKernelGGL(k_lincomb<S>, grid_of(m), dim3(256), 0, c->stream, out, u, v, w, a, b, wc, m);
    LQT_HIP(hipGetLastError());
}

// Y = p(H^2) X for the scaled Chebyshev polynomial of degree `deg` that is bounded by 1 in
// modulus on [a, b] and equals 1 at the lower bound 0 of the spectrum of H^2 (the scaling
// keeps the vectors' size near that of their lowest components).  Three-term recurrence
//   Y_1 = (s1/e)(H^2 - c) X,  Y_{j+1} = (2 s_{j+1}/e)(H^2 - c) Y_j - s_j s_{j+1} Y_{j-1},
//   e = (b - a)/2, c = (b + a)/2, s1 = e/(0 - c), s_{j+1} = 1/(2/s1 - s_j).
// buf holds 4 blocks of nf vectors of n entries; the result is returned as a pointer into it.
template <typename S>
static S* cheb_filter(lqt_ctx* c, const std::function<void(const S*, S*, int)>& H, long long n, int nf, int deg,
                      double a, double b, S* buf) {
    const long long m = (long long)nf * n;
    S* X = buf;          // Y_{j-1}, holds the input
    S* Y = buf + m;      // Y_j
    S* T1 = buf + 2 * m;
    S* T2 = buf + 3 * m;
    const double e = 0.5 * (b - a), cc = 0.5 * (b + a);
    const double s1 = e / (0.0 - cc);
    double s = s1;
    H(X, T1, nf);
    H(T1, T2, nf);
    lincomb<S>(c, Y, T2, X, nullptr, s1 / e, -cc * s1 / e, 0.0, m);
    for (int j = 2; j <= deg; j++) {
        const double sn = 1.0 / (2.0 / s1 - s);
        H(Y, T1, nf);
        H(T1, T2, nf);
        // T1 <- (2 sn / e)(T2 - cc Y) - s sn X
        lincomb<S>(c, T1, T2, Y, X, 2.0 * sn / e, -2.0 * sn * cc / e, -s * sn, m);
        S* old = X;
        X = Y;
        Y = T1;
        T1 = old;
        s = sn;
    }
    return Y;
}

// C = X^+ Y (ka x kb) on the host
static std::vector<zd> gram_h(lqt_ctx* c, const double2* X, int ka, const double2* Y, int kb, long long n) {
    c->scratch[9].ensure(sizeof(double2) * (size_t)ka * kb);
    gemm_gram(c, X, ka, Y, kb, c->scratch[9].as<double2>(), n);
    std::vector<zd> h((size_t)ka * kb);
    LQT_HIP(hipMemcpyAsync(h.data(), c->scratch[9].p, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    return h;
}

// Y = X C (C host ka x kb, row-major); Y must not overlap X
static void combine_h(lqt_ctx* c, const double2* X, int ka, const std::vector<zd>& C, int kb, double2* Y,
                      long long n) {
    c->scratch[9].ensure(sizeof(double2) * (size_t)ka * kb);
    LQT_HIP(hipMemcpyAsync(c->scratch[9].p, C.data(), sizeof(double2) * (size_t)ka * kb, hipMemcpyHostToDevice,
                           c->stream));
    gemm_combine(c, X, ka, c->scratch[9].as<double2>(), kb, 0.0, 1.0, Y, n);
    LQT_HIP(hipStreamSynchronize(c->stream));
}

// X (nf vectors) <- an orthonormal basis of its span, two passes (Cholesky of the Gram
// matrix, or its eigen-decomposition with directions below 1e-13 of the largest dropped when
// the Cholesky meets a pivot below 1e-14 of the largest diagonal).  tmp: nf vectors.  Returns
// the rank.
static int orth_block(lqt_ctx* c, double2* X, int nf, double2* tmp, long long n) {
    int r = nf;
    for (int pass = 0; pass < 2; pass++) {
        std::vector<zd> G = gram_h(c, X, r, X, r, n);
        std::vector<zd> T;
        const int r2 = chol_inverse(r, G, T) ? r : orthonormalizer_any(c, r, G, T, 1e-13);
        combine_h(c, X, r, T, r2, tmp, n);
        LQT_HIP(hipMemcpyAsync(X, tmp, sizeof(double2) * (size_t)r2 * n, hipMemcpyDeviceToDevice, c->stream));
        r = r2;
    }
    return r;
}

// Orthonormal block of exactly kk vectors: fills directions lost to rank deficiency with
// fresh Gaussian vectors (seeded by the iteration) and orthonormalises again.
static void orth_full(lqt_ctx* c, double2* X, int kk, double2* tmp, long long n, uint64_t seed) {
    for (int tries = 0; tries < 4; tries++) {
        const int r = orth_block(c, X, kk, tmp, n);
        if (r == kk) return;
        gaussian_fields(c, seed + 0x9E37ull * (tries + 1), n, kk - r, X + (size_t)r * n);
    }
    throw Error{LQT_ENOTCONV, "eigensolver: block lost rank"};
}

// `steps` Lanczos steps on H^2 (full re-orthogonalisation) from a Gaussian start: returns the
// largest Ritz value, and in *bound that value plus the norm of the last residual vector,
// which bounds the spectrum from above once the largest Ritz value has settled (Zhou and
// Li, 2011).
double lanczos_h2(lqt_ctx* c, long long n, const HermOp& H, int steps, double* bound) {
    DBuf Vb, Tb;
    Vb.ensure(sizeof(double2) * (size_t)(steps + 1) * n);
    Tb.ensure(sizeof(double2) * (size_t)n);
    double2* V = Vb.as<double2>();
    double2* w = Tb.as<double2>();
    gaussian_fields(c, 0x1A2C05ull, n, 1, V);
    std::vector<zd> g = gram_h(c, V, 1, V, 1, n);
    lincomb<double2>(c, V, V, V, nullptr, 1.0 / std::sqrt(g[0].real()), 0.0, 0.0, n);
    std::vector<double> al, be;
    for (int j = 0; j < steps; j++) {
        H(V + (size_t)j * n, V + (size_t)(j + 1) * n, 1);
        H(V + (size_t)(j + 1) * n, w, 1);
        double aj = 0;
        for (int pass = 0; pass < 2; pass++) {  // w -= V_j (V_j^+ w)
            std::vector<zd> h = gram_h(c, V, j + 1, w, 1, n);
            aj += h[j].real();
            c->scratch[9].ensure(sizeof(double2) * (size_t)(j + 1));
            LQT_HIP(hipMemcpyAsync(c->scratch[9].p, h.data(), sizeof(double2) * (j + 1), hipMemcpyHostToDevice,
                                   c->stream));
            gemm_combine(c, V, j + 1, c->scratch[9].as<double2>(), 1, 1.0, -1.0, w, n);
        }
        std::vector<zd> nn = gram_h(c, w, 1, w, 1, n);
        const double bj = std::sqrt(std::max(0.0, nn[0].real()));
        al.push_back(aj);
        be.push_back(bj);
        if (!(bj > 0)) break;
        lincomb<double2>(c, V + (size_t)(j + 1) * n, w, w, nullptr, 1.0 / bj, 0.0, 0.0, n);
    }
    const int m = (int)al.size();
    std::vector<zd> T((size_t)m * m, zd(0));
    for (int i = 0; i < m; i++) {
        T[(size_t)i * m + i] = al[i];
        if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = be[i];
    }
    std::vector<double> th;
    std::vector<zd> E;
    heev(m, T, th, E, false);
    *bound = th[m - 1] + be[m - 1];
    return th[m - 1];
}

int eig_chebyshev(lqt_ctx* c, long long n, const HermOp& H, const HermOp32* H32, double hbound, int k, double xi,
                  int maxit, int degree, int verbose, DBuf& Qout, std::vector<double>& theta,
                  std::vector<double>& resid) {
    const int kk = (int)std::min<long long>(n / 4, 2LL * k);
    LQT_CHECK(kk >= k, LQT_EINVAL, "eigensolver: operator too small for k");
    const long long m = (long long)kk * n;
    DBuf Vb, Wb, Fb;
    Vb.ensure(sizeof(double2) * (size_t)m);
    Wb.ensure(sizeof(double2) * (size_t)m);
    const bool f32 = H32 != nullptr;
    Fb.ensure((f32 ? sizeof(float2) : sizeof(double2)) * (size_t)m * 4);
    Qout.ensure(sizeof(double2) * (size_t)kk * n);
    double2* V = Vb.as<double2>();
    double2* W = Wb.as<double2>();
    gaussian_fields(c, 0xC4EB5EEDull, n, kk, V);
    orth_full(c, V, kk, W, n, 0xC4EB0000ull);
    double b = 0;
    lanczos_h2(c, n, H, 24, &b);
    b = std::min(1.02 * b, hbound * hbound);
    double a = b;
    int conv = 0;
    std::vector<zd> Y;     // harmonic Ritz coefficients (kk x kk, columns), |mu| descending
    std::vector<double> rho(kk), res(kk);
    auto t0 = std::chrono::steady_clock::now();
    long long napp = 0;
    for (int it = 0; it <= maxit; it++) {
        if (it > 0) {
            // degree of this filter: at most `degree`, and low enough that the growth at the
            // bottom of the spectrum, T_d((b + a)/(b - a)), stays below 1e4, so the block keeps
            // every wanted direction above the orthonormalisation's rank threshold (the first
            // iterations, whose cut lies far above the wanted eigenvalues, get short filters)
            const double x0 = (b + a) / (b - a);
            const int deg = (int)std::min<double>(degree, std::max(4.0, std::acosh(1e4) / std::acosh(x0)));
            // filter the block (FP32 when an FP32 operator is given), then orthonormalise
            if (f32) {
                float2* F = Fb.as<float2>();
                hipLaunchKernelGGL(k_to_f32, grid_of(m), dim3(256), 0, c->stream, V, F, m);
                LQT_HIP(hipGetLastError());
                float2* out = cheb_filter<float2>(c, *H32, n, kk, deg, a, b, F);
                hipLaunchKernelGGL(k_to_f64, grid_of(m), dim3(256), 0, c->stream, out, V, m);
                LQT_HIP(hipGetLastError());
            } else {
                double2* F = Fb.as<double2>();
                LQT_HIP(hipMemcpyAsync(F, V, sizeof(double2) * (size_t)m, hipMemcpyDeviceToDevice, c->stream));
                double2* out = cheb_filter<double2>(c, H, n, kk, deg, a, b, F);
                LQT_HIP(hipMemcpyAsync(V, out, sizeof(double2) * (size_t)m, hipMemcpyDeviceToDevice, c->stream));
            }
            napp += 2LL * deg * kk;
            orth_full(c, V, kk, W, n, 0xC4EB0000ull + 97ull * it);
        }
        H(V, W, kk);
        napp += kk;
        std::vector<zd> G2 = gram_h(c, W, kk, W, kk, n);  // V^+ H^2 V
        std::vector<zd> G1 = gram_h(c, V, kk, W, kk, n);  // V^+ H V
        // cut of the next filter: the largest Ritz value of H^2 in the block (power iteration
        // on the positive semi-definite G2; 60 steps settle its largest eigenvalue well enough
        // for a filter bound)
        {
            std::vector<zd> v(kk, zd(1.0)), w(kk);
            double nu = 0;
            for (int pit = 0; pit < 60; pit++) {
                double nw = 0;
                for (int i = 0; i < kk; i++) {
                    zd sacc = 0;
                    for (int l = 0; l < kk; l++) sacc += G2[(size_t)i * kk + l] * v[l];
                    w[i] = sacc;
                    nw += std::norm(sacc);
                }
                double nv2 = 0;
                for (int i = 0; i < kk; i++) nv2 += std::norm(v[i]);
                nu = std::sqrt(nw / nv2);
                for (int i = 0; i < kk; i++) v[i] = w[i] / std::sqrt(nw);
            }
            a = std::min(nu, 0.5 * b);
        }
        // harmonic Ritz pairs with target 0: G1 y = (1/mu) G2 y  ->  T^+ G1 T z = mu z with
        // T^+ G2 T = 1 (Cholesky of G2), y = T z; |mu| descending = |theta| ascending
        std::vector<zd> T;
        if (!chol_inverse(kk, G2, T)) throw Error{LQT_ENOTCONV, "eigensolver: (HV)^+ HV is singular"};
        std::vector<zd> K((size_t)kk * kk, zd(0)), TK((size_t)kk * kk, zd(0));
        for (int i = 0; i < kk; i++)  // TK = G1 T
            for (int l = 0; l < kk; l++) {
                zd s = 0;
                for (int p = 0; p <= l; p++) s += G1[(size_t)i * kk + p] * T[(size_t)p * kk + l];
                TK[(size_t)i * kk + l] = s;
            }
        for (int i = 0; i < kk; i++)  // K = T^+ G1 T
            for (int l = 0; l < kk; l++) {
                zd s = 0;
                for (int p = 0; p <= i; p++) s += std::conj(T[(size_t)p * kk + i]) * TK[(size_t)p * kk + l];
                K[(size_t)i * kk + l] = s;
            }
        std::vector<double> mu;
        std::vector<zd> Z;
        heev_any(c, kk, K, mu, Z, true);  // ascending |mu|
        Y.assign((size_t)kk * kk, zd(0));
        for (int j = 0; j < kk; j++) {  // column j of Y: T z_(kk-1-j), |mu| descending
            const int src = kk - 1 - j;
            for (int i = 0; i < kk; i++) {
                zd s = 0;
                for (int p = i; p < kk; p++) s += T[(size_t)i * kk + p] * Z[(size_t)p * kk + src];
                Y[(size_t)i * kk + j] = s;
            }
        }
        // Rayleigh quotients from the Gram matrices (V orthonormal): rho = y^+ G1 y / y^+ y;
        // residual norms of the first k from the vectors themselves (the Gram form
        // ||H u||^2 - rho^2 ||u||^2 cancels below about 1e-8 |rho|): U = V Y_k, HU = W Y_k
        std::vector<double> yy(kk, 0.0);
        for (int j = 0; j < kk; j++) {
            zd q1 = 0;
            for (int i = 0; i < kk; i++) {
                const zd yi = Y[(size_t)i * kk + j];
                yy[j] += std::norm(yi);
                zd g1 = 0;
                for (int l = 0; l < kk; l++) g1 += G1[(size_t)i * kk + l] * Y[(size_t)l * kk + j];
                q1 += std::conj(yi) * g1;
            }
            rho[j] = q1.real() / yy[j];
        }
        {
            std::vector<zd> Yk((size_t)kk * k);
            for (int i = 0; i < kk; i++)
                for (int j = 0; j < k; j++) Yk[(size_t)i * k + j] = Y[(size_t)i * kk + j];
            double2* Uk = Qout.as<double2>();
            double2* HUk = (double2*)Fb.p;  // the filter buffers hold at least 2 kk FP64 vectors
            combine_h(c, V, kk, Yk, k, Uk, n);
            combine_h(c, W, kk, Yk, k, HUk, n);
            c->scratch[9].ensure(sizeof(double) * 2 * k);
            double* thd = c->scratch[9].as<double>();
            LQT_HIP(hipMemcpyAsync(thd, rho.data(), sizeof(double) * k, hipMemcpyHostToDevice, c->stream));
            eig_residual_norms(c, HUk, Uk, thd, n, k, thd + k);
            LQT_HIP(hipMemcpyAsync(res.data(), thd + k, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
            LQT_HIP(hipStreamSynchronize(c->stream));
        }
        conv = 0;
        for (int j = 0; j < k; j++) {
            res[j] = std::sqrt(res[j] / yy[j]);
            if (res[j] <= xi * std::fabs(rho[j])) conv++;
        }
        if (verbose && it == 0) {
            fprintf(stderr, "[lqtrace] eig: block %d, ||H||^2 <= %.4e (rigorous bound %.4e), filter degree %d%s\n", kk,
                    b, hbound * hbound, degree, f32 ? " (FP32)" : "");
            fflush(stderr);
        }
        if (verbose) {
            double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            double worst = 0;
            for (int j = 0; j < k; j++) worst = std::max(worst, res[j] / std::fabs(rho[j]));
            fprintf(stderr,
                    "[lqtrace] eig it %d: %d/%d pass, |theta| %.3e..%.3e, max |r|/|theta| %.2e, filter cut %.3e, "
                    "%lld applications, %.1f s\n",
                    it, conv, k, std::fabs(rho[0]), std::fabs(rho[k - 1]), worst, std::sqrt(a), napp, el);
            fflush(stderr);
        }
        if (conv >= k) break;
    }
    // the k harmonic Ritz vectors with the largest |mu| (in Qout from the last iteration),
    // orthonormalised, then Rayleigh-Ritz with H inside their span (an accurate invariant
    // subspace: no spurious values)
    double2* Q = Qout.as<double2>();
    const int r = orth_block(c, Q, k, W, n);
    LQT_CHECK(r == k, LQT_ENOTCONV, "eigensolver: Ritz vectors lost rank");
    H(Q, W, k);
    std::vector<zd> M = gram_h(c, Q, k, W, k, n);
    std::vector<double> th;
    std::vector<zd> E;
    heev_any(c, k, M, th, E, true);  // ascending |theta|
    combine_h(c, Q, k, E, k, V, n);
    LQT_HIP(hipMemcpyAsync(Q, V, sizeof(double2) * (size_t)k * n, hipMemcpyDeviceToDevice, c->stream));
    H(Q, W, k);
    theta.assign(th.begin(), th.end());
    c->scratch[9].ensure(sizeof(double) * 2 * k);
    double* thd = c->scratch[9].as<double>();
    LQT_HIP(hipMemcpyAsync(thd, theta.data(), sizeof(double) * k, hipMemcpyHostToDevice, c->stream));
    eig_residual_norms(c, W, Q, thd, n, k, thd + k);
    resid.assign(k, 0.0);
    LQT_HIP(hipMemcpyAsync(resid.data(), thd + k, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    conv = 0;
    for (int i = 0; i < k; i++) {
        resid[i] = std::sqrt(resid[i]);
        if (resid[i] <= xi * std::fabs(theta[i])) conv++;
    }
    if (verbose) {
        fprintf(stderr, "[lqtrace] eig final: %d/%d pairs meet |r| <= %.1e |theta|, |theta| %.4e..%.4e\n", conv, k, xi,
                std::fabs(theta[0]), std::fabs(theta[k - 1]));
        fflush(stderr);
    }
    return conv;
}

}  // namespace lqt
