// The small FP64 part of an s-step cycle (host and device): Cholesky of the Gram matrix of
// the cycle's vectors, the small Hessenberg matrix and its least-squares problem.  Kept in a
// header of its own so that the host compiler can build it for tests of its edge cases.
#pragma once
#include <math.h>

namespace lqt {

// The small FP64 part of an s-step cycle for one system: G (NV x NV Hermitian Gram matrix
// of k_0..k_s), nr = |r|.  Cholesky G = R^+ R truncated at the first pivot below 1e-12 G_00 or not finite
// (the basis then stops at that column), H = R T R^{-1}, Givens least squares; writes
// beta[0..m] and returns the steps used (kdim, 0 when fewer than two columns survive: a
// rank-one Gram matrix or a non-finite one) and *est.
template <int NV>
__host__ __device__ int sstep_small_solve(const double2 (&G)[NV][NV], double nr, double theta, double sigma,
                                          double sqrtN, int m, double2* beta, double* est) {
    constexpr int S = NV - 1;
    // Cholesky G = R^+ R, R upper triangular
    double2 R[NV][NV];
    for (int i = 0; i < NV; i++)
        for (int j = 0; j < NV; j++) R[i][j] = make_double2(0, 0);
    int kk = NV;
    const double floor = 1e-12 * G[0][0].x;
    for (int j = 0; j < NV; j++) {
        double d = G[j][j].x;
        for (int k = 0; k < j; k++) d -= R[k][j].x * R[k][j].x + R[k][j].y * R[k][j].y;
        if (!(d > floor && d < HUGE_VAL)) {  // tiny, negative or not finite
            kk = j;
            break;
        }
        const double rd = sqrt(d);
        R[j][j] = make_double2(rd, 0);
        for (int l = j + 1; l < NV; l++) {
            double2 t = G[j][l];
            for (int k = 0; k < j; k++) {  // t -= conj(R[k][j]) R[k][l]
                const double2 a = R[k][j], b = R[k][l];
                t.x -= a.x * b.x + a.y * b.y;
                t.y -= a.x * b.y - a.y * b.x;
            }
            R[j][l] = make_double2(t.x / rd, t.y / rd);
        }
    }
    const int ss = kk - 1;  // usable steps
    for (int i = 0; i <= m; i++) beta[i] = make_double2(0, 0);
    if (ss < 1 || !(nr > 0)) {
        *est = nr;
        return 0;
    }
    // Rinv = R_ss^{-1} (upper triangular)
    double2 Ri[S][S];
    for (int i = 0; i < ss; i++)
        for (int j = 0; j < ss; j++) Ri[i][j] = make_double2(0, 0);
    for (int j = 0; j < ss; j++) {
        Ri[j][j] = make_double2(1.0 / R[j][j].x, 0);
        for (int i = j - 1; i >= 0; i--) {
            double2 t = make_double2(0, 0);
            for (int k = i + 1; k <= j; k++) {  // t += R[i][k] Ri[k][j]
                const double2 a = R[i][k], b = Ri[k][j];
                t.x += a.x * b.x - a.y * b.y;
                t.y += a.x * b.y + a.y * b.x;
            }
            Ri[i][j] = make_double2(-t.x / R[i][i].x, -t.y / R[i][i].x);
        }
    }
    // H = R[0..ss][0..ss] T Rinv, with (T Rinv)[k][j] = theta Rinv[k][j] + Rinv[k-1][j] / sigma
    double2 H[NV][S];
    for (int i = 0; i <= ss; i++)
        for (int j = 0; j < ss; j++) {
            double2 h = make_double2(0, 0);
            for (int k = i; k <= ss; k++) {
                double2 tr = make_double2(0, 0);
                if (k < ss) tr = make_double2(theta * Ri[k][j].x, theta * Ri[k][j].y);
                if (k >= 1) {
                    tr.x += Ri[k - 1][j].x / sigma;
                    tr.y += Ri[k - 1][j].y / sigma;
                }
                const double2 a = R[i][k];
                h.x += a.x * tr.x - a.y * tr.y;
                h.y += a.x * tr.y + a.y * tr.x;
            }
            H[i][j] = h;
        }
    // Givens QR of H against g = rho R_00 e_1
    double2 g[NV];
    for (int i = 0; i <= ss; i++) g[i] = make_double2(0, 0);
    g[0] = make_double2(nr / sqrtN * R[0][0].x, 0);
    for (int j = 0; j < ss; j++) {
        const double2 a = H[j][j], b = H[j + 1][j];
        const double absa = sqrt(a.x * a.x + a.y * a.y), absb = sqrt(b.x * b.x + b.y * b.y);
        const double r = sqrt(absa * absa + absb * absb);
        double c;
        double2 sn;
        if (r == 0) {
            c = 1;
            sn = make_double2(0, 0);
        } else if (absa == 0) {
            c = 0;
            sn = make_double2(b.x / absb, -b.y / absb);  // conj(b)/|b|
        } else {
            c = absa / r;
            // s = (a/|a|) conj(b) / r
            const double ux = a.x / absa, uy = a.y / absa;
            sn = make_double2((ux * b.x + uy * b.y) / r, (uy * b.x - ux * b.y) / r);
        }
        for (int l = j; l < ss; l++) {  // rows j, j+1: [c s; -conj(s) c]
            const double2 h0 = H[j][l], h1 = H[j + 1][l];
            H[j][l] = make_double2(c * h0.x + sn.x * h1.x - sn.y * h1.y, c * h0.y + sn.x * h1.y + sn.y * h1.x);
            H[j + 1][l] = make_double2(-(sn.x * h0.x + sn.y * h0.y) + c * h1.x, -(sn.x * h0.y - sn.y * h0.x) + c * h1.y);
        }
        const double2 g0 = g[j], g1 = g[j + 1];
        g[j] = make_double2(c * g0.x + sn.x * g1.x - sn.y * g1.y, c * g0.y + sn.x * g1.y + sn.y * g1.x);
        g[j + 1] = make_double2(-(sn.x * g0.x + sn.y * g0.y) + c * g1.x, -(sn.x * g0.y - sn.y * g0.x) + c * g1.y);
    }
    double2 y[S];
    for (int i = ss - 1; i >= 0; i--) {
        double2 t = g[i];
        for (int l = i + 1; l < ss; l++) {
            const double2 h = H[i][l];
            t.x -= h.x * y[l].x - h.y * y[l].y;
            t.y -= h.x * y[l].y + h.y * y[l].x;
        }
        const double2 d = H[i][i];
        const double den = d.x * d.x + d.y * d.y;
        y[i] = den > 0 ? make_double2((t.x * d.x + t.y * d.y) / den, (t.y * d.x - t.x * d.y) / den)
                       : make_double2(0, 0);
    }
    for (int i = 0; i < ss; i++) {  // beta = Rinv y
        double2 t = make_double2(0, 0);
        for (int k = i; k < ss; k++) {
            const double2 a = Ri[i][k], b = y[k];
            t.x += a.x * b.x - a.y * b.y;
            t.y += a.x * b.y + a.y * b.x;
        }
        beta[i] = t;
    }
    *est = sqrt(g[ss].x * g[ss].x + g[ss].y * g[ss].y) * sqrtN / R[0][0].x;
    return ss;
}

}  // namespace lqt
