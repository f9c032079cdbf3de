// Multigrid prolongator W (Algorithm 2): blocked, chirality-split near-null vectors.
#pragma once
#include "lqt_internal.h"

namespace lqt {

// Aggregate geometry: blocks of b0 x b1 x b2 x b3 sites, n0 x n1 x n2 x n3 of them, numbered
// x fastest like the sites; bs = site inside a block, x fastest.
struct PG {
    int L0, L1, L2, L3;  // lattice
    int b0, b1, b2, b3;  // block
    int n0, n1, n2, n3;  // blocks per direction (x, y, z, t)
    int nagg, bsites, d, nv;
    int V;
};

inline PG make_pg(const lqt_ctx* c, const int* b, int nv) {
    PG p;
    p.L0 = c->g.L[0], p.L1 = c->g.L[1], p.L2 = c->g.L[2], p.L3 = c->g.L[3];
    p.b0 = b[0], p.b1 = b[1], p.b2 = b[2], p.b3 = b[3];
    p.n0 = p.L0 / p.b0, p.n1 = p.L1 / p.b1, p.n2 = p.L2 / p.b2, p.n3 = p.L3 / p.b3;
    p.bsites = p.b0 * p.b1 * p.b2 * p.b3;
    p.nagg = c->g.V / p.bsites;
    p.d = 6 * p.bsites;
    p.nv = nv;
    p.V = c->g.V;
    return p;
}

inline PG pg_of(const lqt_basis* B) {
    PG p = make_pg(B->ctx, B->block, B->nv);
    return p;
}

__device__ __forceinline__ int site_of(const PG& p, int agg, int bs) {
    const int ax = agg % p.n0, ay = (agg / p.n0) % p.n1, az = (agg / (p.n0 * p.n1)) % p.n2,
              at = agg / (p.n0 * p.n1 * p.n2);
    const int bx = bs % p.b0, by = (bs / p.b0) % p.b1, bz = (bs / (p.b0 * p.b1)) % p.b2,
              bt = bs / (p.b0 * p.b1 * p.b2);
    const int x = ax * p.b0 + bx, y = ay * p.b1 + by, z = az * p.b2 + bz, t = at * p.b3 + bt;
    return x + p.L0 * (y + p.L1 * (z + p.L2 * t));
}

// coarse = W^+ A W (explicit 9-point block stencil, built on first use) and out = g5^W of it
void coarse_explicit_build(lqt_ctx* c, lqt_basis* B);
void coarse_explicit_apply(lqt_ctx* c, const lqt_basis* B, const double2* in, double2* out, int nrhs, bool herm);

// C_up[i][j] = u_i^+ P_+ z_j and C_dn[i][j] = u_i^+ P_- z_j for the basis U = W U_c of a
// prolongator basis and the probes j0 .. j0+s-1 (device outputs, k x s).
void prolong_project_probes(lqt_ctx* c, const lqt_basis* B, uint64_t seed, long long j0, int s, double2* cup,
                            double2* cdn);
// coarse = W^+ fine and fine = W coarse for nrhs fields (fine: device layout FP64)
void restrict_fields(lqt_ctx* c, const lqt_basis* B, const double2* fine, double2* coarse, int nrhs);
// cm = U_c^+ W^+ Z, cg = U_c^+ g5^W W^+ Z for s fine fields (k x s, device)
void prolong_project_fields(lqt_ctx* c, const lqt_basis* B, const double2* Z, int s, double2* cm, double2* cg);
// Z <- Z - W U_c C (C: k x s device coefficients; tmp: s fine fields of work space)
void prolong_subtract(lqt_ctx* c, const lqt_basis* B, const double2* C, int s, double2* Z, double2* tmp);
// LQT_EINVAL unless the coarse vectors U_c are orthonormal (orthogonal projector W U_c U_c^+ W^+)
void prolong_check_orthonormal(lqt_ctx* c, const lqt_basis* B);
// block modified Gram-Schmidt of nblocks blocks of p.nv vectors of p.d entries
void block_mgs(lqt_ctx* c, double2* W, const PG& p, int nblocks);
// a 9-point block stencil [agg][slot][nb][nb] (nb = 2 p.nv) on the lattice of aggregates of p
void coarse_stencil_apply(lqt_ctx* c, const PG& p, const double2* Dc, const double2* in, double2* out, int nrhs,
                          bool herm);
// second level (level2.hip): geometry, W2 from nv2 level-1 coarse vectors Y, the level-2
// operator, restriction / prolongation between level-1 and level-2 coarse fields
PG pg2_of(const lqt_basis* B);
void level2_blocks(lqt_ctx* c, lqt_basis* B, const double2* Y);
void level2_build(lqt_ctx* c, lqt_basis* B);
void level2_apply(lqt_ctx* c, const lqt_basis* B, const double2* in, double2* out, int nrhs, bool herm);
void restrict2_fields(lqt_ctx* c, const lqt_basis* B, const double2* y1, double2* x2, int nrhs);
void prolong2_fields(lqt_ctx* c, const lqt_basis* B, const double2* x2, double2* y1, int nrhs);
void prolong_fields(lqt_ctx* c, const lqt_basis* B, const double2* coarse, double2* fine, int nrhs);

}  // namespace lqt
