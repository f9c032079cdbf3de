// Batched MINRES for Hermitian indefinite operators, FP64, on generic complex vectors.
#pragma once
#include <functional>
#include <vector>

#include "lqt_internal.h"

namespace lqt {

// out_f = H in_f for f < nf; vectors of the operator's length, contiguous per vector.
using HermOp = std::function<void(const double2* in, double2* out, int nf)>;

// x_f = H^{-1} b_f for f < nf (vectors of length n), x0 = 0, until the MINRES residual
// estimate is <= tol ||b_f|| or maxit steps.  Returns the number of systems that missed
// tol; iters (may be null) receives the steps per system.
int minres(lqt_ctx* c, long long n, const HermOp& H, const double2* b, double2* x, int nf, double tol, int maxit,
           std::vector<int>* iters);

// Subspace iteration with Rayleigh-Ritz on T = H^{-1}_xi for the k eigenpairs of the
// Hermitian H with the smallest |theta| (largest |1/theta|); inner solves by MINRES to
// xi/10.  On return Q (device, at least kk vectors of length n) holds the Ritz vectors in
// its first k slots with |theta| ascending, theta[0..k) their Ritz values of H.  A pair
// passes when ||T q - q/theta|| <= xi ||T|| (the test of the paper's Table 1).  Returns the
// number of pairs that pass.  kk (output) = block size used.
int eig_subspace(lqt_ctx* c, long long n, const HermOp& H, int k, double xi, int maxit, int inner_maxit,
                 int verbose, DBuf& Q, std::vector<double>& theta, std::vector<double>& resid_T);

}  // namespace lqt
