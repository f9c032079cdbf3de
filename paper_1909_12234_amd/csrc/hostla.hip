// Host FP64 dense linear algebra: complex Hermitian Jacobi eigensolver and a Gram-matrix
// orthonormaliser.  Sizes are the deflation rank (tens to hundreds).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "hostla.h"

namespace lqt {

void heev(int n, const std::vector<zd>& A0, std::vector<double>& w, std::vector<zd>& V, bool by_abs) {
    std::vector<zd> A(A0.size());
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) A[i * n + j] = 0.5 * (A0[i * n + j] + std::conj(A0[j * n + i]));
    V.assign((size_t)n * n, zd(0, 0));
    for (int i = 0; i < n; i++) V[i * n + i] = 1.0;
    double fro = 0;
    for (auto& a : A) fro += std::norm(a);
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) off += std::norm(A[p * n + q]);
        if (std::sqrt(off) <= 1e-15 * fro || off == 0) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                zd apq = A[p * n + q];
                double b = std::abs(apq);
                if (b <= 1e-300 || b <= 1e-18 * fro) continue;
                // phase making the pair real: with ph = apq / |apq|, G = diag(1, conj(ph)) R
                zd ph = apq / b;
                double app = A[p * n + p].real(), aqq = A[q * n + q].real();
                double tau = (aqq - app) / (2 * b);
                double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
                double c = 1 / std::sqrt(1 + t * t), s = t * c;
                // G = [[c, s], [-s conj(ph), c conj(ph)]]
                zd g00 = c, g01 = s, g10 = -s * std::conj(ph), g11 = c * std::conj(ph);
                for (int k = 0; k < n; k++) {  // A <- A G (columns p, q)
                    zd akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = akp * g00 + akq * g10;
                    A[k * n + q] = akp * g01 + akq * g11;
                }
                for (int k = 0; k < n; k++) {  // A <- G^+ A (rows p, q)
                    zd apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = std::conj(g00) * apk + std::conj(g10) * aqk;
                    A[q * n + k] = std::conj(g01) * apk + std::conj(g11) * aqk;
                }
                A[p * n + q] = A[q * n + p] = 0;
                for (int k = 0; k < n; k++) {  // V <- V G
                    zd vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = vkp * g00 + vkq * g10;
                    V[k * n + q] = vkp * g01 + vkq * g11;
                }
            }
    }
    std::vector<double> d(n);
    for (int i = 0; i < n; i++) d[i] = A[i * n + i].real();
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        return by_abs ? std::fabs(d[a]) < std::fabs(d[b]) : d[a] < d[b];
    });
    w.resize(n);
    std::vector<zd> Vs((size_t)n * n);
    for (int j = 0; j < n; j++) {
        w[j] = d[idx[j]];
        for (int i = 0; i < n; i++) Vs[i * n + j] = V[i * n + idx[j]];
    }
    V.swap(Vs);
}

int orthonormalizer(int n, const std::vector<zd>& G, std::vector<zd>& T, double rtol) {
    std::vector<double> w;
    std::vector<zd> V;
    heev(n, G, w, V, false);  // ascending
    double mx = 0;
    for (double x : w) mx = std::max(mx, x);
    std::vector<int> keep;
    for (int j = n - 1; j >= 0; j--)  // largest first
        if (w[j] > rtol * mx && w[j] > 0) keep.push_back(j);
    int r = (int)keep.size();
    T.assign((size_t)n * r, zd(0, 0));
    for (int c = 0; c < r; c++) {
        double f = 1.0 / std::sqrt(w[keep[c]]);
        for (int i = 0; i < n; i++) T[i * r + c] = V[i * n + keep[c]] * f;
    }
    return r;
}

bool chol_inverse(int n, const std::vector<zd>& G, std::vector<zd>& T) {
    std::vector<zd> R((size_t)n * n, zd(0, 0));
    double dmax = 0;
    for (int i = 0; i < n; i++) dmax = std::max(dmax, G[i * n + i].real());
    for (int i = 0; i < n; i++) {
        zd s = G[i * n + i];
        for (int k = 0; k < i; k++) s -= std::conj(R[k * n + i]) * R[k * n + i];
        if (!(s.real() > 1e-14 * dmax)) return false;
        double d = std::sqrt(s.real());
        R[i * n + i] = d;
        for (int j = i + 1; j < n; j++) {
            zd t = G[i * n + j];
            for (int k = 0; k < i; k++) t -= std::conj(R[k * n + i]) * R[k * n + j];
            R[i * n + j] = t / d;
        }
    }
    // T = R^{-1} by back substitution, column by column
    T.assign((size_t)n * n, zd(0, 0));
    for (int j = 0; j < n; j++) {
        T[j * n + j] = 1.0 / R[j * n + j];
        for (int i = j - 1; i >= 0; i--) {
            zd s = 0;
            for (int k = i + 1; k <= j; k++) s += R[i * n + k] * T[k * n + j];
            T[i * n + j] = -s / R[i * n + i];
        }
    }
    return true;
}

}  // namespace lqt
