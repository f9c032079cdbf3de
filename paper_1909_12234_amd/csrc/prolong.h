// Multigrid prolongator W (Algorithm 2): blocked, chirality-split near-null vectors.
#pragma once
#include "lqt_internal.h"

namespace lqt {

// C_up[i][j] = u_i^+ P_+ z_j and C_dn[i][j] = u_i^+ P_- z_j for the basis U = W U_c of a
// prolongator basis and the probes j0 .. j0+s-1 (device outputs, k x s).
void prolong_project_probes(lqt_ctx* c, const lqt_basis* B, uint64_t seed, long long j0, int s, double2* cup,
                            double2* cdn);

}  // namespace lqt
