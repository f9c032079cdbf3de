// Dense Hermitian eigenproblems of the setup (Rayleigh-Ritz and harmonic Ritz matrices of the
// eigensolvers, the k x k matrices M = X^+ g5 A X of the oblique projector) on the device:
// rocSOLVER's divide-and-conquer zheevd for n > 64, the host Jacobi routine (hostla) below.
// The cyclic Jacobi sweeps grow as n^3 per sweep with many sweeps (51 s at n = 512 on one host
// core), which the 2k-vector blocks of a k = 256 coarse eigensolve cannot afford.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <numeric>

#include "devla.h"
#include "hostla.h"
#include "lqt_internal.h"

namespace lqt {

static rocblas_handle blas_of(lqt_ctx* c) {
    if (!c->blas) {
        rocblas_handle h = nullptr;
        LQT_CHECK(rocblas_create_handle(&h) == rocblas_status_success, LQT_EHIP, "rocblas_create_handle failed");
        c->blas = h;
    }
    rocblas_handle h = (rocblas_handle)c->blas;
    LQT_CHECK(rocblas_set_stream(h, c->stream) == rocblas_status_success, LQT_EHIP, "rocblas_set_stream failed");
    return h;
}

void blas_release(lqt_ctx* c) {
    if (c->blas) (void)rocblas_destroy_handle((rocblas_handle)c->blas);
    c->blas = nullptr;
}

void heev_any(lqt_ctx* c, int n, const std::vector<zd>& A, std::vector<double>& w, std::vector<zd>& V, bool by_abs) {
    if (n <= 64) {
        heev(n, A, w, V, by_abs);
        return;
    }
    rocblas_handle h = blas_of(c);
    // column-major copy of the Hermitian part (row-major A: element (i, j) at i n + j)
    std::vector<zd> col((size_t)n * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            col[(size_t)j * n + i] = 0.5 * (A[(size_t)i * n + j] + std::conj(A[(size_t)j * n + i]));
    DBuf dA, dD;
    dA.ensure(sizeof(zd) * (size_t)n * n);
    dD.ensure(sizeof(double) * (size_t)2 * n + 64);
    double* D = dD.as<double>();
    double* E = D + n;
    rocblas_int* info = (rocblas_int*)(E + n);
    LQT_HIP(hipMemcpyAsync(dA.p, col.data(), sizeof(zd) * col.size(), hipMemcpyHostToDevice, c->stream));
    LQT_CHECK(rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, n,
                               (rocblas_double_complex*)dA.p, n, D, E, info) == rocblas_status_success,
              LQT_EHIP, "rocsolver_zheevd failed");
    std::vector<double> wa(n);
    rocblas_int hinfo = 0;
    LQT_HIP(hipMemcpyAsync(col.data(), dA.p, sizeof(zd) * col.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipMemcpyAsync(wa.data(), D, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    LQT_CHECK(hinfo == 0, LQT_ENOTCONV, "rocsolver_zheevd did not converge");
    // ascending w (as returned) or ascending |w|; V row-major, eigenvectors in columns
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    if (by_abs) std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return std::fabs(wa[a]) < std::fabs(wa[b]); });
    w.resize(n);
    V.assign((size_t)n * n, zd(0));
    for (int j = 0; j < n; j++) {
        w[j] = wa[ord[j]];
        for (int i = 0; i < n; i++) V[(size_t)i * n + j] = col[(size_t)ord[j] * n + i];
    }
}

int orthonormalizer_any(lqt_ctx* c, int n, const std::vector<zd>& G, std::vector<zd>& T, double rtol) {
    if (n <= 64) return orthonormalizer(n, G, T, rtol);
    std::vector<double> w;
    std::vector<zd> V;
    heev_any(c, n, G, w, V, false);  // ascending
    double mx = 0;
    for (double x : w) mx = std::max(mx, x);
    std::vector<int> keep;
    for (int j = n - 1; j >= 0; j--)  // largest first
        if (w[j] > rtol * mx && w[j] > 0) keep.push_back(j);
    const int r = (int)keep.size();
    T.assign((size_t)n * r, zd(0, 0));
    for (int cidx = 0; cidx < r; cidx++) {
        const double f = 1.0 / std::sqrt(w[keep[cidx]]);
        for (int i = 0; i < n; i++) T[(size_t)i * r + cidx] = V[(size_t)i * n + keep[cidx]] * f;
    }
    return r;
}

}  // namespace lqt
