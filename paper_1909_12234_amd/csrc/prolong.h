// Multigrid prolongator W (Algorithm 2): blocked, chirality-split near-null vectors.
#pragma once
#include "lqt_internal.h"

namespace lqt {

// C_up[i][j] = u_i^+ P_+ z_j and C_dn[i][j] = u_i^+ P_- z_j for the basis U = W U_c of a
// prolongator basis and the probes j0 .. j0+s-1 (device outputs, k x s).
void prolong_project_probes(lqt_ctx* c, const lqt_basis* B, uint64_t seed, long long j0, int s, double2* cup,
                            double2* cdn);
// coarse = W^+ fine and fine = W coarse for nrhs fields (fine: device layout FP64)
void restrict_fields(lqt_ctx* c, const lqt_basis* B, const double2* fine, double2* coarse, int nrhs);
void prolong_fields(lqt_ctx* c, const lqt_basis* B, const double2* coarse, double2* fine, int nrhs);

}  // namespace lqt
