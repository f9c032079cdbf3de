// Two-grid preconditioner from the prolongator W (Section 2): coarse grid correction with the
// explicit coarse operator, then minimal-residual smoothing.
#pragma once
#include "lqt_internal.h"
#include "solver.h"

namespace lqt {

// z = M(v) for nf fields in storage S (device layout), with the context's two-grid basis
template <typename S>
void twogrid_apply(lqt_ctx* c, const S* v, S* z, int nf, const SolveOpts& o);
// x = D_c^{-1} b by batched FP64 GMRES on the explicit coarse operator (nf coarse vectors,
// x from zero) until every relative residual is <= tol or maxit steps; returns the largest
// relative residual
double coarse_gmres(lqt_ctx* c, const lqt_basis* B, const double2* b, double2* x, int nf, double tol, int maxit);

}  // namespace lqt
