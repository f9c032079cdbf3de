// Deflated Hutchinson estimation of trace(A^{-1}) and the deflation bases.
//
// Estimator (Eq. 1 with the split of Section 2; real Rademacher probes z_j):
//   oblique, K = g5 (Section 2.1, Algorithm 2 form):
//     t_j = z_j^T y_j - (z_j^T U) Lambda^{-1} (U^+ g5 z_j),  y_j = A^{-1}_xi z_j
//     t0  = sum_i lambda_i^{-1} u_i^+ g5 u_i,  U = X U_hat,  U_hat Lambda U_hat^+ = X^+ g5 A X
//   orthogonal (Algorithm 1):
//     t_j = z_j^T A^{-1}_xi (z_j - U U^+ z_j),  t0 = sum_i u_i^+ A^{-1}_xi u_i
// Only the k x s products U^+ z and U^+ g5 z are kept, which is what lets the estimate be
// recomputed for every deflation rank after the solves (Section 2.2).
//
// Bases: from caller vectors, or the k eigenpairs of A g5 with the smallest |lambda| (the
// largest of (A g5)^{-1} = g5 A^{-1}: Algorithm 1, first step; the eigenvectors of A g5 are
// left singular vectors of A), by Chebyshev-filtered subspace iteration (eigcheb.hip).
// For the oblique projector an A g5 eigenbasis Q enters as X = g5 Q, for which the oblique
// projector is Q Q^+ when Q is exact.
#include <algorithm>
#include <cmath>
#include <complex>
#include <chrono>
#include <cstdio>
#include <new>

#include "blas.h"
#include "gemm.h"
#include "hostla.h"
#include "lqt_internal.h"
#include "devla.h"
#include "eigcheb.h"
#include "prolong.h"
#include "solver.h"

using lqt::DBuf;
using lqt::Error;
using lqt::zd;

namespace lqt {

// Host -> device from pageable memory; waits, so the host buffer may be released at once.
static void h2d(lqt_ctx* c, void* d, const void* h, size_t bytes) {
    LQT_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
}
static void d2h(lqt_ctx* c, void* h, const void* d, size_t bytes) {
    LQT_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
}

// C = X^+ Y on the device, copied to a host vector (ka x kb row-major)
static std::vector<zd> gram_host(lqt_ctx* c, const double2* X, int ka, const double2* Y, int kb, long long n = -1) {
    c->scratch[9].ensure(sizeof(double2) * (size_t)ka * kb);
    gemm_gram(c, X, ka, Y, kb, c->scratch[9].as<double2>(), n);
    std::vector<zd> h((size_t)ka * kb);
    d2h(c, h.data(), c->scratch[9].p, sizeof(double2) * h.size());
    return h;
}

// Y = X C with a host matrix C (ka x kb row-major)
static void combine_host(lqt_ctx* c, const double2* X, int ka, const std::vector<zd>& C, int kb, double beta,
                         double alpha, double2* Y, long long n = -1) {
    c->scratch[9].ensure(sizeof(double2) * (size_t)ka * kb);
    h2d(c, c->scratch[9].p, C.data(), sizeof(double2) * (size_t)ka * kb);
    gemm_combine(c, X, ka, c->scratch[9].as<double2>(), kb, beta, alpha, Y, n);
}

// In place: X (k vectors) <- an orthonormal basis of span X (r <= k vectors). tmp: k vectors.
static int orthonormalize(lqt_ctx* c, double2* X, int k, double2* tmp, long long n = -1) {
    if (n < 0) n = 12LL * c->g.V;
    int r = k;
    for (int pass = 0; pass < 2; pass++) {
        std::vector<zd> G = gram_host(c, X, r, X, r, n);
        std::vector<zd> T;
        int r2 = orthonormalizer_any(c, r, G, T, 1e-13);
        combine_host(c, X, r, T, r2, 0.0, 1.0, tmp, n);
        LQT_HIP(hipMemcpyAsync(X, tmp, sizeof(double2) * (size_t)r2 * n, hipMemcpyDeviceToDevice, c->stream));
        r = r2;
    }
    return r;
}

// Oblique-projector data for fine vectors X: M = X^+ g5 A X, eigh, U = X U_hat.
void fine_oblique_setup(lqt_ctx* c, lqt_basis* B, const double2* X, int k) {
    const long long n = 12LL * c->g.V;
    DBuf AX;
    AX.ensure(sizeof(double2) * (size_t)k * n);
    dslash(c, LQT_F64, LQT_A, X, AX.p, k, n, n);
    gamma5_fields(c, AX.as<double2>(), k);
    std::vector<zd> M = gram_host(c, X, k, AX.as<double2>(), k);
    std::vector<double> lam;
    std::vector<zd> Uh;
    heev_any(c, k, M, lam, Uh, true);
    B->U.ensure(sizeof(double2) * (size_t)k * n);
    combine_host(c, X, k, Uh, k, 0.0, 1.0, B->U.as<double2>());
    LQT_HIP(hipMemcpyAsync(AX.p, B->U.p, sizeof(double2) * (size_t)k * n, hipMemcpyDeviceToDevice, c->stream));
    gamma5_fields(c, AX.as<double2>(), k);
    c->scratch[9].ensure(sizeof(double2) * (size_t)k);
    dot_fields(c, B->U.as<double2>(), AX.as<double2>(), k, c->scratch[9].as<double2>());
    std::vector<zd> d(k);
    d2h(c, d.data(), c->scratch[9].p, sizeof(double2) * k);
    B->k = k;
    B->lambda.assign(2 * k, 0.0);
    B->ug5u.assign(2 * k, 0.0);
    for (int i = 0; i < k; i++) {
        B->lambda[2 * i] = lam[i];
        B->ug5u[2 * i] = d[i].real();
        B->ug5u[2 * i + 1] = d[i].imag();
    }
}

// Upper bound of ||A|| (and of ||A g5||, ||g5^W W^+ A W|| for orthonormal W): each
// direction's hop 2 (P- U psi(x+mu) + P+ U^+ psi(x-mu)) with the orthogonal spin projectors
// P-+ = (1 -+ g_mu)/2 has norm <= 2 sqrt(2), so ||A|| <= |4 + m| + (1/2) 4 (2 sqrt(2)).
double wilson_norm_bound(const lqt_ctx* c) {
    double d = 0;
    for (int l = 0; l < c->g.lat.nlat; l++) d = std::max(d, std::fabs(c->g.lat.diag[l]));
    return d + 4.0 * std::sqrt(2.0);
}

// Largest singular value of A: the square root of the largest Ritz value of 40 Lanczos
// steps on (A g5)^2 = A A^+ (accurate to well below a percent for the extreme eigenvalue).
double sigma_max(lqt_ctx* c) {
    if (c->sigma_max > 0) return c->sigma_max;
    const long long n = 12LL * c->g.V;
    HermOp H = [c, n](const double2* in, double2* outv, int nf) { dslash(c, LQT_F64, LQT_A_G5, in, outv, nf, n, n); };
    double bound = 0;
    const double ritz = lanczos_h2(c, n, H, 40, &bound);
    c->sigma_max = std::sqrt(ritz);
    return c->sigma_max;
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

void need_gauge(lqt_ctx* c) { LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)"); }

struct Stats {
    zd mean;
    double var = 0, var_re = 0, jk = 0;
};

Stats summarize(const std::vector<zd>& t) {
    Stats s;
    const int m = (int)t.size();
    zd sum = 0;
    for (auto& x : t) sum += x;
    s.mean = m ? sum / (double)m : zd(0);
    if (m > 1) {
        double v = 0, vr = 0;
        for (auto& x : t) {
            v += std::norm(x - s.mean);
            vr += (x.real() - s.mean.real()) * (x.real() - s.mean.real());
        }
        s.var = v / (m - 1);
        s.var_re = vr / (m - 1);
        std::vector<zd> loo(m);
        zd lm = 0;
        for (int j = 0; j < m; j++) {
            loo[j] = (sum - t[j]) / (double)(m - 1);
            lm += loo[j];
        }
        lm /= (double)m;
        double a = 0;
        for (auto& x : loo) a += std::norm(x - lm);
        s.jk = std::sqrt((m - 1.0) / m * a);
    }
    return s;
}

}  // namespace

extern "C" {

int lqt_basis_from_vectors(lqt_ctx* c, const double* vectors, int k, lqt_basis** out) {
    if (!c || !out) return LQT_EINVAL;
    *out = nullptr;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(vectors && k >= 1, LQT_EINVAL, "need k >= 1 vectors");
        need_gauge(c);
        const long long n = 12LL * c->g.V;
        LQT_CHECK(!lqt::has_nonfinite(c, vectors, (size_t)(2 * n * k)), LQT_ENAN, "basis vectors hold NaN or Inf");
        lqt_basis* B = new lqt_basis();
        B->ctx = c;
        try {
            DBuf X;
            X.ensure(sizeof(double2) * (size_t)k * n);
            lqt::to_device_layout(c, (const double2*)vectors, X.as<double2>(), k);
            lqt::fine_oblique_setup(c, B, X.as<double2>(), k);
            LQT_HIP(hipStreamSynchronize(c->stream));
        } catch (...) {
            delete B;
            throw;
        }
        *out = B;
    });
}

int lqt_basis_eig(lqt_ctx* c, int k, double xi, double tau, const lqt_solver_opts* opts, lqt_basis** out) {
    if (!c || !out) return LQT_EINVAL;
    *out = nullptr;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(k >= 1, LQT_EINVAL, "k must be >= 1");
        LQT_CHECK(xi > 0 && xi < 1, LQT_EINVAL, "xi must be in (0, 1)");
        // the shift i tau g5 leaves the eigenvectors of A g5 and their order unchanged (the
        // filter takes no inverse, where the shift would condition the solves)
        LQT_CHECK(std::isfinite(tau), LQT_EINVAL, "tau must be finite");
        need_gauge(c);
        const long long n = 12LL * c->g.V;
        LQT_CHECK(k <= n / 8, LQT_EINVAL, "k too large for the lattice");
        lqt::SolveOpts o = lqt::make_opts(opts);
        // Algorithm 1, first step: eigenpairs of g5 A^{-1} = (A g5)^{-1} of largest magnitude,
        // i.e. the smallest |lambda| of the Hermitian A g5
        lqt::HermOp H = [c, n](const double2* in, double2* outv, int nf) {
            lqt::dslash(c, LQT_F64, LQT_A_G5, in, outv, nf, n, n);
        };
        lqt::HermOp32 H32 = [c, n](const float2* in, float2* outv, int nf) {
            lqt::dslash(c, LQT_F32, LQT_A_G5, in, outv, nf, n, n);
        };
        const int kk = (int)std::min<long long>(n / 4, 2LL * k);
        if (xi >= 1e-5 && c->tuned.find(lqt::tune_key(LQT_F32, kk)) == c->tuned.end()) lqt::dslash_tune(c, LQT_F32, kk);
        DBuf Qb;
        std::vector<double> theta, resid;
        // the FP32 filter suffices while the accepted residuals are well above FP32 rounding
        const int conv = lqt::eig_chebyshev(c, n, H, xi >= 1e-5 ? &H32 : nullptr, lqt::wilson_norm_bound(c), k, xi,
                                            o.outer_maxit, o.eig_degree, o.verbose, Qb, theta, resid);
        double2* Q = Qb.as<double2>();
        lqt_basis* B = new lqt_basis();
        B->ctx = c;
        try {
            // orthonormal Ritz vectors Q (Algorithm 1) and X = g5 Q for the oblique form
            B->Q.ensure(sizeof(double2) * (size_t)k * n);
            LQT_HIP(hipMemcpyAsync(B->Q.p, Q, sizeof(double2) * (size_t)k * n, hipMemcpyDeviceToDevice, c->stream));
            B->orthonormal = true;
            B->theta.assign(theta.begin(), theta.begin() + k);
            B->resid.assign(resid.begin(), resid.begin() + k);
            lqt::gamma5_fields(c, Q, k);  // X = g5 Q (B->Q keeps Q)
            lqt::fine_oblique_setup(c, B, Q, k);
            LQT_HIP(hipStreamSynchronize(c->stream));
        } catch (...) {
            delete B;
            throw;
        }
        *out = B;
        if (conv < k) {
            c->err = "eigensolver: " + std::to_string(conv) + " of " + std::to_string(k) + " pairs converged";
            throw Error{LQT_ENOTCONV, c->err};
        }
    });
}

int lqt_sigma_max(lqt_ctx* c, double* h_sigma) {
    if (!c || !h_sigma) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        need_gauge(c);
        *h_sigma = lqt::sigma_max(c);
    });
}

int lqt_basis_eigenvalues(const lqt_basis* B, double* lambda, int* k) {
    if (!B || !k) return LQT_EINVAL;
    *k = B->k;
    if (lambda)
        for (int i = 0; i < 2 * B->k; i++) lambda[i] = B->lambda[i];
    return LQT_OK;
}

int lqt_basis_vectors(const lqt_basis* B, double* out) {
    if (!B || !out) return LQT_EINVAL;
    lqt_ctx* c = B->ctx;
    return guard(c, [&] {
        if (B->kind == 0) {
            lqt::from_device_layout(c, B->U.as<double2>(), (double2*)out, B->k);
        } else {  // U = W U_c
            DBuf f;
            f.ensure(sizeof(double2) * (size_t)B->k * 12 * c->g.V);
            lqt::prolong_fields(c, B, B->Uc.as<double2>(), f.as<double2>(), B->k);
            lqt::from_device_layout(c, f.as<double2>(), (double2*)out, B->k);
        }
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

void lqt_basis_free(lqt_basis* B) {
    if (!B) return;
    if (B->ctx) (void)hipStreamSynchronize(B->ctx->stream);
    if (B->ctx && B->ctx->tg == B) B->ctx->tg = nullptr;
    delete B;
}

int lqt_trace_lattices(lqt_ctx* c, int nprobes, uint64_t seed, double xi, const lqt_solver_opts* opts,
                       lqt_trace_result* res, double* samples) {
    if (!c) return LQT_EINVAL;
    int nfail_total = 0;
    int rc = guard(c, [&] {
        LQT_CHECK(res, LQT_EINVAL, "null result");
        LQT_CHECK(nprobes >= 1, LQT_EINVAL, "nprobes must be >= 1");
        LQT_CHECK(xi > 0 && xi < 1, LQT_EINVAL, "xi must be in (0, 1)");
        need_gauge(c);
        lqt::SolveOpts o = lqt::make_opts(opts);
        LQT_CHECK(!o.use_net, LQT_EINVAL, "the network preconditioner serves single-lattice contexts");
        const int nlat = c->g.lat.nlat;
        const long long n = 12LL * c->g.V;
        const int s = nprobes;
        size_t fr = 0, tot = 0;
        LQT_HIP(hipMemGetInfo(&fr, &tot));
        size_t per = (size_t)n * 16 * 2 + (size_t)(o.restart + 1) * n * lqt::storage_bytes(o.prec) + (size_t)n * 32;
        int fit = (int)std::max<size_t>(1, (size_t)(0.6 * (double)(fr + c->scratch[0].n + c->scratch[10].n +
                                                                     c->scratch[11].n)) / per);
        int chunk = std::min(s, o.max_batch > 0 ? o.max_batch : s);
        chunk = std::max(1, std::min(chunk, fit));
        c->scratch[10].ensure(sizeof(double2) * (size_t)chunk * n);
        c->scratch[11].ensure(sizeof(double2) * (size_t)chunk * n);
        double2* Z = c->scratch[10].as<double2>();
        double2* Y = c->scratch[11].as<double2>();
        std::vector<zd> t((size_t)s * nlat);  // [probe][lattice]
        std::vector<lqt_solve_stats> st(s);
        hipEvent_t e0, e1;
        LQT_HIP(hipEventCreate(&e0));
        LQT_HIP(hipEventCreate(&e1));
        double t_solve = 0;
        for (int j0 = 0; j0 < s; j0 += chunk) {
            const int cs = std::min(chunk, s - j0);
            lqt::probes_gen(c, seed, j0, cs, Z);
            LQT_HIP(hipEventRecord(e0, c->stream));
            nfail_total += lqt::solve_fields(c, Z, Y, cs, xi, o, st.data() + j0);
            LQT_HIP(hipEventRecord(e1, c->stream));
            c->scratch[9].ensure(sizeof(double2) * (size_t)cs * nlat);
            lqt::probe_dots(c, seed, j0, Y, cs, c->scratch[9].as<double2>(), true);
            lqt::d2h(c, t.data() + (size_t)j0 * nlat, c->scratch[9].p, sizeof(double2) * cs * nlat);
            float a = 0;
            LQT_HIP(hipEventElapsedTime(&a, e0, e1));
            t_solve += a * 1e-3;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        long long iters = 0;
        int nf = 0, nfb = 0;
        for (auto& x : st) {
            iters += x.iters;
            nf += x.converged ? 0 : 1;
            nfb += x.fallback > 0 ? 1 : 0;
        }
        for (int l = 0; l < nlat; l++) {
            std::vector<zd> tl(s);
            for (int j = 0; j < s; j++) tl[j] = t[(size_t)j * nlat + l];
            Stats S = summarize(tl);
            lqt_trace_result& R = res[l];
            R.trace_re = S.mean.real();
            R.trace_im = S.mean.imag();
            R.t0_re = R.t0_im = 0;
            R.var_sample = S.var;
            R.var_mean = S.var / s;
            R.jackknife_err = S.jk;
            R.var_re_only = S.var_re;
            R.nsolves = s;
            R.nfailed = nf;
            R.nfallback = nfb;
            R.iters_total = iters;
            R.seconds_solve = t_solve;
            R.seconds_setup = 0;
            if (samples)
                for (int j = 0; j < s; j++) {
                    samples[2 * ((size_t)l * s + j)] = tl[j].real();
                    samples[2 * ((size_t)l * s + j) + 1] = tl[j].imag();
                }
        }
    });
    if (rc == LQT_OK && nfail_total > 0) {
        c->err = std::to_string(nfail_total) + " probe solves missed the tolerance";
        return LQT_ENOTCONV;
    }
    return rc;
}

int lqt_trace(lqt_ctx* c, const lqt_basis* B, int projector, int nprobes, uint64_t seed, double xi,
              const lqt_solver_opts* opts, lqt_trace_result* res, double* rank_curve, double* samples) {
    return lqt_trace_probing(c, B, projector, nprobes, seed, xi, 1, 0, opts, res, rank_curve, samples);
}

// The trace of lqt_trace_probing; with_t0 = false skips the deterministic part (the k extra
// solves of the orthogonal projector), for the correction runs of lqt_trace_tsm.
static int trace_impl(lqt_ctx* c, const lqt_basis* B, int projector, int nprobes, uint64_t seed, double xi,
                      int hp_vectors, int dilute, const lqt_solver_opts* opts, lqt_trace_result* res,
                      double* rank_curve, double* samples, bool with_t0) {
    if (!c) return LQT_EINVAL;
    int nfail_total = 0;
    int rc = guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "several lattices: use lqt_trace_lattices");
        LQT_CHECK(res, LQT_EINVAL, "null result");
        LQT_CHECK(nprobes >= 1, LQT_EINVAL, "nprobes must be >= 1");
        LQT_CHECK(xi > 0 && xi < 1, LQT_EINVAL, "xi must be in (0, 1)");
        LQT_CHECK(projector == LQT_OBLIQUE_G5 || projector == LQT_ORTH, LQT_EINVAL, "bad projector");
        lqt::check_partition(c, hp_vectors, dilute);
        LQT_CHECK(!B || B->ctx == c, LQT_EINVAL, "basis belongs to another context");
        LQT_CHECK(!(B && projector == LQT_ORTH && B->kind == 0 && !B->orthonormal), LQT_EINVAL,
                  "the orthogonal projector needs an orthonormal fine basis (lqt_basis_eig)");
        need_gauge(c);
        if (B && projector == LQT_ORTH && B->kind == 1) lqt::prolong_check_orthonormal(c, B);
        lqt::SolveOpts o = lqt::make_opts(opts);
        LQT_CHECK(!o.use_net || c->net.set, LQT_ESTATE, "use_net without preconditioner weights");
        const long long n = 12LL * c->g.V;
        const int k = B ? B->k : 0;
        const int s = nprobes;
        // solves per draw: the probing vectors, each split into the 12 components with dilution
        const int nd = dilute ? 12 : 1;
        const int q = hp_vectors * nd;
        const bool part = q > 1;
        LQT_CHECK((long long)s * q <= (1LL << 31) - 1, LQT_EINVAL, "too many probe vectors");
        const int nvec = s * q;
        // vector chunk: the caller's batch, else what fits (Z and Y FP64 + the Krylov basis)
        size_t fr = 0, tot = 0;
        LQT_HIP(hipMemGetInfo(&fr, &tot));
        size_t per = (size_t)n * 16 * 2 + (size_t)(o.restart + 1) * n * lqt::storage_bytes(o.prec) + (size_t)n * 32;
        if (o.use_net) per += (size_t)o.restart * n * lqt::storage_bytes(o.prec);
        if (o.twogrid) per += (size_t)o.restart * n * lqt::storage_bytes(o.prec) + (size_t)n * 16 * 4;
        int fit = (int)std::max<size_t>(1, (size_t)(0.6 * (double)(fr + c->scratch[0].n + c->scratch[10].n +
                                                                     c->scratch[11].n)) / per);
        int chunk = std::min(nvec, o.max_batch > 0 ? o.max_batch : nvec);
        chunk = std::max(1, std::min({chunk, fit, 65535}));
        c->scratch[10].ensure(sizeof(double2) * (size_t)chunk * n);
        c->scratch[11].ensure(sizeof(double2) * (size_t)chunk * n);
        double2* Z = c->scratch[10].as<double2>();
        double2* Y = c->scratch[11].as<double2>();
        // per draw: the undeflated sample t_j and the per-mode oblique terms
        // term[i][j] = (1/hp) sum over the vectors v of draw j of (v^T u_i)(u_i^+ g5 v)
        std::vector<zd> t(s, zd(0)), term((size_t)k * s, zd(0));
        std::vector<lqt_solve_stats> st(nvec);
        hipEvent_t e0, e1, e2;
        LQT_HIP(hipEventCreate(&e0));
        LQT_HIP(hipEventCreate(&e1));
        LQT_HIP(hipEventCreate(&e2));
        double t_setup = 0, t_solve = 0;
        const double wgt = 1.0 / hp_vectors;
        DBuf small;
        std::vector<zd> tv(chunk);
        for (int p0 = 0; p0 < nvec; p0 += chunk) {
            const int cs = std::min(chunk, nvec - p0);
            LQT_HIP(hipEventRecord(e0, c->stream));
            if (part)
                lqt::partition_probes_gen(c, seed, p0, cs, hp_vectors, dilute, Z);
            else
                lqt::probes_gen(c, seed, p0, cs, Z);
            std::vector<zd> hm, hg;  // u_i^+ v and u_i^+ g5 v of the chunk, k x cs
            if (B) {
                small.ensure(sizeof(double2) * (size_t)k * cs * 2);
                double2* cm = small.as<double2>();
                double2* cg = cm + (size_t)k * cs;
                hm.resize((size_t)k * cs);
                hg.resize((size_t)k * cs);
                const double2* Ub = (projector == LQT_ORTH) ? B->Q.as<double2>() : B->U.as<double2>();
                if (!part) {
                    // the probes are regenerated inside the projection kernels
                    double2* cup = cm;
                    double2* cdn = cg;
                    if (B->kind == 0)
                        lqt::gemm_probes(c, Ub, k, seed, p0, cs, cup, cdn);
                    else
                        lqt::prolong_project_probes(c, B, seed, p0, cs, cup, cdn);
                    std::vector<zd> hu((size_t)k * cs), hd((size_t)k * cs);
                    lqt::d2h(c, hu.data(), cup, sizeof(double2) * hu.size());
                    lqt::d2h(c, hd.data(), cdn, sizeof(double2) * hd.size());
                    for (size_t e = 0; e < hu.size(); e++) hm[e] = hu[e] + hd[e], hg[e] = hu[e] - hd[e];
                } else {
                    if (B->kind == 0) {
                        lqt::gemm_gram(c, Ub, k, Z, cs, cm);
                        if (projector == LQT_OBLIQUE_G5) {
                            LQT_HIP(hipMemcpyAsync(Y, Z, sizeof(double2) * (size_t)cs * n, hipMemcpyDeviceToDevice,
                                                   c->stream));
                            lqt::gamma5_fields(c, Y, cs);
                            lqt::gemm_gram(c, Ub, k, Y, cs, cg);
                        }
                    } else {
                        lqt::prolong_project_fields(c, B, Z, cs, cm, cg);
                    }
                    lqt::d2h(c, hm.data(), cm, sizeof(double2) * hm.size());
                    if (projector == LQT_OBLIQUE_G5) lqt::d2h(c, hg.data(), cg, sizeof(double2) * hg.size());
                }
                if (projector == LQT_OBLIQUE_G5) {
                    for (int i = 0; i < k; i++)
                        for (int pl = 0; pl < cs; pl++) {
                            const int j = (p0 + pl) / q;
                            // v real: v^T u_i = conj(u_i^+ v)
                            term[(size_t)i * s + j] += wgt * std::conj(hm[(size_t)i * cs + pl]) * hg[(size_t)i * cs + pl];
                        }
                } else if (B->kind == 0) {  // v <- v - Q (Q^+ v)
                    lqt::combine_host(c, B->Q.as<double2>(), k, hm, cs, 1.0, -1.0, Z);
                } else {  // v <- v - W U_c (U_c^+ W^+ v), Y as the fine work space
                    lqt::h2d(c, cm, hm.data(), sizeof(double2) * hm.size());
                    lqt::prolong_subtract(c, B, cm, cs, Z, Y);
                }
            }
            LQT_HIP(hipEventRecord(e1, c->stream));
            nfail_total += lqt::solve_fields(c, Z, Y, cs, xi, o, st.data() + p0);
            LQT_HIP(hipEventRecord(e2, c->stream));
            c->scratch[9].ensure(sizeof(double2) * (size_t)cs);
            if (part) {
                // v^T y with the unprojected v (regenerated: the orthogonal projector changed Z)
                if (B && projector == LQT_ORTH) lqt::partition_probes_gen(c, seed, p0, cs, hp_vectors, dilute, Z);
                lqt::dot_fields(c, Z, Y, cs, c->scratch[9].as<double2>());
            } else {
                lqt::probe_dots(c, seed, p0, Y, cs, c->scratch[9].as<double2>());
            }
            lqt::d2h(c, tv.data(), c->scratch[9].p, sizeof(double2) * cs);
            for (int pl = 0; pl < cs; pl++) t[(p0 + pl) / q] += wgt * tv[pl];
            float a = 0, b = 0;
            LQT_HIP(hipEventElapsedTime(&a, e0, e1));
            LQT_HIP(hipEventElapsedTime(&b, e1, e2));
            t_setup += a * 1e-3;
            t_solve += b * 1e-3;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
        // deterministic part
        zd t0 = 0;
        if (B && projector == LQT_OBLIQUE_G5) {
            for (int i = 0; i < k; i++) t0 += zd(B->ug5u[2 * i], B->ug5u[2 * i + 1]) / B->lambda[2 * i];
        } else if (B && with_t0 && B->kind == 0) {  // Algorithm 1: t0 = sum_i u_i^+ A^{-1}_xi u_i (k extra solves)
            DBuf Yu;
            Yu.ensure(sizeof(double2) * (size_t)k * n);
            std::vector<lqt_solve_stats> su(k);
            nfail_total += lqt::solve_fields(c, B->Q.as<double2>(), Yu.as<double2>(), k, xi, o, su.data());
            c->scratch[9].ensure(sizeof(double2) * (size_t)k);
            lqt::dot_fields(c, B->Q.as<double2>(), Yu.as<double2>(), k, c->scratch[9].as<double2>());
            std::vector<zd> d(k);
            lqt::d2h(c, d.data(), c->scratch[9].p, sizeof(double2) * k);
            for (auto& x : d) t0 += x;
        } else if (B && with_t0) {  // the same with u_i = W U_c e_i, prolongated a chunk at a time
            const long long nc = 2LL * B->nagg * B->nv;
            const int ck = std::min(k, chunk);
            std::vector<lqt_solve_stats> su(ck);
            std::vector<zd> d(ck);
            for (int i0 = 0; i0 < k; i0 += ck) {
                const int cnt = std::min(ck, k - i0);
                lqt::prolong_fields(c, B, B->Uc.as<double2>() + (size_t)i0 * nc, Z, cnt);
                nfail_total += lqt::solve_fields(c, Z, Y, cnt, xi, o, su.data());
                c->scratch[9].ensure(sizeof(double2) * (size_t)cnt);
                lqt::dot_fields(c, Z, Y, cnt, c->scratch[9].as<double2>());
                lqt::d2h(c, d.data(), c->scratch[9].p, sizeof(double2) * cnt);
                for (int i = 0; i < cnt; i++) t0 += d[i];
            }
        }
        // samples
        std::vector<zd> base = t, ts = t;
        if (B && projector == LQT_OBLIQUE_G5)
            for (int j = 0; j < s; j++) {
                zd corr = 0;
                for (int i = 0; i < k; i++) corr += term[(size_t)i * s + j] / B->lambda[2 * i];
                ts[j] = t[j] - corr;
            }
        Stats S = summarize(ts);
        res->trace_re = (t0 + S.mean).real();
        res->trace_im = (t0 + S.mean).imag();
        res->t0_re = t0.real();
        res->t0_im = t0.imag();
        res->var_sample = S.var;
        res->var_mean = S.var / s;
        res->jackknife_err = S.jk;
        res->var_re_only = S.var_re;
        res->nsolves = nvec;
        res->nfailed = 0;
        res->nfallback = 0;
        res->iters_total = 0;
        for (auto& x : st) {
            res->iters_total += x.iters;
            res->nfailed += x.converged ? 0 : 1;
            res->nfallback += x.fallback > 0 ? 1 : 0;
        }
        res->seconds_solve = t_solve;
        res->seconds_setup = t_setup;
        if (samples)
            for (int j = 0; j < s; j++) {
                samples[2 * j] = ts[j].real();
                samples[2 * j + 1] = ts[j].imag();
            }
        if (rank_curve) {
            for (int kp = 0; kp <= k; kp++) {
                double* row = rank_curve + 3 * kp;
                if (!(B && projector == LQT_OBLIQUE_G5)) {
                    row[0] = row[1] = row[2] = 0;
                    continue;
                }
                std::vector<zd> tk(s);
                zd t0k = 0;
                for (int i = 0; i < kp; i++) t0k += zd(B->ug5u[2 * i], B->ug5u[2 * i + 1]) / B->lambda[2 * i];
                for (int j = 0; j < s; j++) {
                    zd corr = 0;
                    for (int i = 0; i < kp; i++) corr += term[(size_t)i * s + j] / B->lambda[2 * i];
                    tk[j] = base[j] - corr;
                }
                Stats Sk = summarize(tk);
                row[0] = (t0k + Sk.mean).real();
                row[1] = Sk.var;
                row[2] = Sk.jk;
            }
        }
    });
    if (rc == LQT_OK && nfail_total) return LQT_ENOTCONV;
    return rc;
}

int lqt_trace_probing(lqt_ctx* c, const lqt_basis* B, int projector, int nprobes, uint64_t seed, double xi,
                      int hp_vectors, int dilute, const lqt_solver_opts* opts, lqt_trace_result* res,
                      double* rank_curve, double* samples) {
    return trace_impl(c, B, projector, nprobes, seed, xi, hp_vectors, dilute, opts, res, rank_curve, samples, true);
}

int lqt_trace_tsm(lqt_ctx* c, const lqt_basis* B, int projector, int nprobes, uint64_t seed, double xi_loose,
                  int ncorr, uint64_t seed_corr, double xi_tight, int hp_vectors, int dilute,
                  const lqt_solver_opts* opts, lqt_trace_result* main, lqt_tsm_result* out, double* corr_samples) {
    if (!c) return LQT_EINVAL;
    if (!main || !out || ncorr < 2 || seed_corr == seed || !(xi_tight > 0 && xi_tight < xi_loose)) {
        c->err = "tsm: needs results, ncorr >= 2, seed_corr != seed and 0 < xi_tight < xi_loose";
        return LQT_EINVAL;
    }
    int rc = trace_impl(c, B, projector, nprobes, seed, xi_loose, hp_vectors, dilute, opts, main, nullptr, nullptr,
                        true);
    if (rc != LQT_OK && rc != LQT_ENOTCONV) return rc;
    int worst = rc;
    // the correction probes at both tolerances: the deflation terms of a draw do not depend on
    // the solves, so the difference of its two samples is (1/hp) sum_v v^T (y_tight - y_loose)
    std::vector<double> sl(2 * (size_t)ncorr), st(2 * (size_t)ncorr);
    lqt_trace_result rl{}, rt{};
    rc = trace_impl(c, B, projector, ncorr, seed_corr, xi_loose, hp_vectors, dilute, opts, &rl, nullptr, sl.data(),
                    false);
    if (rc != LQT_OK && rc != LQT_ENOTCONV) return rc;
    if (rc != LQT_OK) worst = rc;
    rc = trace_impl(c, B, projector, ncorr, seed_corr, xi_tight, hp_vectors, dilute, opts, &rt, nullptr, st.data(),
                    false);
    if (rc != LQT_OK && rc != LQT_ENOTCONV) return rc;
    if (rc != LQT_OK) worst = rc;
    std::vector<zd> d(ncorr);
    for (int j = 0; j < ncorr; j++) d[j] = zd(st[2 * j] - sl[2 * j], st[2 * j + 1] - sl[2 * j + 1]);
    Stats S = summarize(d);
    out->trace_re = main->trace_re + S.mean.real();
    out->trace_im = main->trace_im + S.mean.imag();
    out->err = std::sqrt(main->var_mean + S.var / ncorr);
    out->corr_re = S.mean.real();
    out->corr_im = S.mean.imag();
    out->corr_var_sample = S.var;
    out->corr_jackknife_err = S.jk;
    out->nsolves_loose = main->nsolves + rl.nsolves;
    out->nsolves_tight = rt.nsolves;
    out->iters_loose = main->iters_total + rl.iters_total;
    out->iters_tight = rt.iters_total;
    out->nfailed = main->nfailed + rl.nfailed + rt.nfailed;
    if (corr_samples)
        for (int j = 0; j < ncorr; j++) {
            corr_samples[2 * j] = d[j].real();
            corr_samples[2 * j + 1] = d[j].imag();
        }
    return worst;
}

int lqt_gram(lqt_ctx* c, const double* x, int ka, const double* y, int kb, double* h_c) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(ka >= 1 && kb >= 1 && x && y && h_c, LQT_EINVAL, "bad gram arguments");
        const long long n = 12LL * c->g.V;
        DBuf X, Yd;
        X.ensure(sizeof(double2) * (size_t)ka * n);
        Yd.ensure(sizeof(double2) * (size_t)kb * n);
        lqt::to_device_layout(c, (const double2*)x, X.as<double2>(), ka);
        lqt::to_device_layout(c, (const double2*)y, Yd.as<double2>(), kb);
        std::vector<zd> C = lqt::gram_host(c, X.as<double2>(), ka, Yd.as<double2>(), kb);
        std::copy((double*)C.data(), (double*)C.data() + 2 * C.size(), h_c);
    });
}

int lqt_project_probes(lqt_ctx* c, const double* x, int ka, uint64_t seed, long long j0, int s, double* h_cup,
                       double* h_cdn) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(ka >= 1 && s >= 1 && j0 >= 0 && x && h_cup && h_cdn, LQT_EINVAL, "bad projection arguments");
        const long long n = 12LL * c->g.V;
        DBuf X, out;
        X.ensure(sizeof(double2) * (size_t)ka * n);
        out.ensure(sizeof(double2) * (size_t)ka * s * 2);
        lqt::to_device_layout(c, (const double2*)x, X.as<double2>(), ka);
        lqt::gemm_probes(c, X.as<double2>(), ka, seed, j0, s, out.as<double2>(), out.as<double2>() + (size_t)ka * s);
        lqt::d2h(c, h_cup, out.p, sizeof(double2) * (size_t)ka * s);
        lqt::d2h(c, h_cdn, out.as<double2>() + (size_t)ka * s, sizeof(double2) * (size_t)ka * s);
    });
}

int lqt_combine(lqt_ctx* c, const double* x, int ka, const double* h_c, int kb, double beta, double alpha,
                double* y) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(ka >= 1 && kb >= 1 && x && h_c && y, LQT_EINVAL, "bad combine arguments");
        const long long n = 12LL * c->g.V;
        DBuf X, Yd;
        X.ensure(sizeof(double2) * (size_t)ka * n);
        Yd.ensure(sizeof(double2) * (size_t)kb * n);
        lqt::to_device_layout(c, (const double2*)x, X.as<double2>(), ka);
        lqt::to_device_layout(c, (const double2*)y, Yd.as<double2>(), kb);
        std::vector<zd> C((size_t)ka * kb);
        std::copy(h_c, h_c + 2 * C.size(), (double*)C.data());
        lqt::combine_host(c, X.as<double2>(), ka, C, kb, beta, alpha, Yd.as<double2>());
        lqt::from_device_layout(c, Yd.as<double2>(), (double2*)y, kb);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

}  // extern "C"
