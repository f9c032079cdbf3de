"""Two-grid preconditioner from the prolongator W (Section 2, the two-grid method), written out
in numpy (oracle).

TEST INFRASTRUCTURE ONLY: used by tests/ and never by the product library.

One application to a residual r, from x = 0, takes the method's two steps in order:
  coarse grid correction  x_c = P (P^+ A P)^{-1} P^+ r   (P = W: restriction, exact coarse
                                                            solve, prolongation)
  smoothing               x = x_c + M^{-1}(r - A x_c),  M^{-1} = nu minimal-residual steps
                          on A (the paper's smoother is a few iterations of a Krylov solver
                          such as GCR; one minimal-residual step is GCR(1) without memory):
                          s = r - A x_c;  repeat nu times: p = A s, a = p^+ s / p^+ p,
                          x += a s, s -= a p.
Rows are vectors: r has shape (nrhs, N).
"""
import numpy as np

from . import core
from . import prolongator as pr


def coarse_operator(U, dims, mass, W, block):
    """D_c = P^+ A P (dense, nc x nc) with A applied column by column by the oracle operator."""
    P = pr.dense_prolongator(W, dims, block)
    AP = core.apply(U, dims, mass, core.OP_A, P.T.copy()).T
    return P.conj().T @ AP


def mr_smooth(U, dims, mass, r, x, nu):
    """nu minimal-residual steps on A for A x = r from x (rows); a step with p = 0 (the
    residual already zero) changes nothing."""
    x = x.copy()
    s = r - core.apply(U, dims, mass, core.OP_A, x)
    for _ in range(nu):
        p = core.apply(U, dims, mass, core.OP_A, s)
        for f in range(r.shape[0]):
            pp = np.vdot(p[f], p[f]).real
            a = np.vdot(p[f], s[f]) / pp if pp > 0 else 0.0
            x[f] += a * s[f]
            s[f] -= a * p[f]
    return x


def apply(U, dims, mass, W, block, r, nu, Dc=None):
    """One two-grid application to the rows of r: exact coarse grid correction, then nu
    minimal-residual smoothing steps."""
    if Dc is None:
        Dc = coarse_operator(U, dims, mass, W, block)
    rc = pr.restrict(W, r, dims, block)
    ec = np.linalg.solve(Dc, rc.T).T
    xc = pr.prolong(W, ec, dims, block)
    return mr_smooth(U, dims, mass, r, xc, nu)
