// Smallest-|lambda| eigenpairs of a Hermitian indefinite operator (Chebyshev-filtered
// subspace iteration on H^2, harmonic Rayleigh-Ritz extraction).
#pragma once
#include <functional>
#include <vector>

#include "lqt_internal.h"

namespace lqt {

// out_f = H in_f for f < nf; vectors of the operator's length, contiguous per vector.
using HermOp = std::function<void(const double2* in, double2* out, int nf)>;
// the same operator on FP32 vectors (used by the filter only)
using HermOp32 = std::function<void(const float2* in, float2* out, int nf)>;

// Upper bound of ||A|| for the context's operator (also of ||A g5|| and, for an
// orthonormal prolongator W, of ||g5^W W^+ A W||).
double wilson_norm_bound(const lqt_ctx* c);

// `steps` Lanczos steps on H^2: the largest Ritz value; *bound = that value plus the last
// residual norm (an upper bound of the spectrum of H^2 once the Ritz value has settled).
double lanczos_h2(lqt_ctx* c, long long n, const HermOp& H, int steps, double* bound);

// The k eigenpairs of H with the smallest |theta|, for H of length-n vectors with
// ||H|| <= hbound.  Block of 2k vectors (at most n/4); at most `degree` applications of H^2
// per filter (fewer while the filter's growth at 0 would exceed 1e4); at most maxit filtered iterations.  On return Q (device) holds k orthonormal
// vectors, theta their Ritz values (ascending |theta|) and resid ||H q - theta q||.  A pair
// passes when resid <= xi |theta|; returns the number of pairs that pass.  H32 (may be null)
// runs the filter in FP32.
int eig_chebyshev(lqt_ctx* c, long long n, const HermOp& H, const HermOp32* H32, double hbound, int k, double xi,
                  int maxit, int degree, int verbose, DBuf& Q, std::vector<double>& theta,
                  std::vector<double>& resid);

}  // namespace lqt
