// Dense Hermitian eigenproblems of the setup: rocSOLVER on the device for n > 64, the host
// Jacobi routine for smaller ones (same interface and ordering as hostla.h).
#pragma once
#include <vector>

#include "hostla.h"
#include "lqt_internal.h"

namespace lqt {

// A = V diag(w) V^+ (row-major A, its Hermitian part; V row-major, eigenvectors in columns),
// ascending |w| when by_abs, else ascending w
void heev_any(lqt_ctx* c, int n, const std::vector<zd>& A, std::vector<double>& w, std::vector<zd>& V, bool by_abs);
// orthonormalising transform of a Gram matrix (as hostla's orthonormalizer)
int orthonormalizer_any(lqt_ctx* c, int n, const std::vector<zd>& G, std::vector<zd>& T, double rtol);
// destroy the context's rocBLAS handle (created on first use)
void blas_release(lqt_ctx* c);

}  // namespace lqt
