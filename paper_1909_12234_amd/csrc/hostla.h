// Small dense FP64 linear algebra on the host (k x k problems, k <= a few hundred).
#pragma once
#include <complex>
#include <vector>

namespace lqt {

using zd = std::complex<double>;

// Eigen-decomposition of a Hermitian n x n matrix (row-major A, only its Hermitian part is
// used) by cyclic complex Jacobi rotations: A = V diag(w) V^+.  V is row-major with the
// eigenvectors in its columns.  Eigenpairs are ordered by increasing |w| when by_abs,
// else by increasing w.
void heev(int n, const std::vector<zd>& A, std::vector<double>& w, std::vector<zd>& V, bool by_abs);

// Orthonormalising transform of a Gram matrix G = X^+ X (n x n): returns T (n x r,
// row-major) with X T orthonormal, r = numerical rank (eigenvalues above rtol * max).
int orthonormalizer(int n, const std::vector<zd>& G, std::vector<zd>& T, double rtol);

// Cholesky G = R^+ R of a Hermitian positive definite n x n matrix; on success T = R^{-1}
// (upper triangular, row-major) so that X R^{-1} is orthonormal when G = X^+ X.  Returns
// false when a pivot is not positive (G numerically singular).
bool chol_inverse(int n, const std::vector<zd>& G, std::vector<zd>& T);

}  // namespace lqt
