"""Locate the left edge of the Wilson spectrum with the CPU oracle, to choose the mass.

TEST INFRASTRUCTURE / configuration tool: calls only the oracle and the seeded input
generator.  Usage:
    python -m oracle.tune_mass --dims 16 16 16 32 --eps 0.5 --seed 1

The eigenvalues of A(m) are those of A(0) shifted by m.  For the random links of the
benchmark workloads the left edge of the spectrum of A(0) is made of complex-conjugate
pairs; once m moves that edge across the imaginary axis the spectrum surrounds the
origin and restarted GMRES stagnates, so the most ill-conditioned usable operator has
m slightly above -min Re lambda(A(0)).  The script prints the leftmost eigenvalues
(implicitly restarted Arnoldi on A(0), which scipy's ARPACK binding performs; the
oracle supplies the matrix-vector product).
"""
import argparse
import json
import sys
import time

import numpy as np
from scipy.sparse.linalg import LinearOperator, eigs

from . import core


def leftmost_eigenvalues(links, dims, k=6, tol=1e-7, antiperiodic=True):
    N = 12 * core.volume(dims)
    op = LinearOperator(
        (N, N), dtype=np.complex128,
        matvec=lambda v: core.apply(links, dims, 0.0, core.OP_A, v.astype(np.complex128), antiperiodic),
    )
    w = eigs(op, k=k, which="SR", return_eigenvectors=False, tol=tol, maxiter=100000, ncv=max(4 * k, 40))
    return w[np.argsort(w.real)]


def main(argv=None):
    sys.path.insert(0, ".")
    import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, nargs=4, default=[16, 16, 16, 32])
    ap.add_argument("--eps", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--norm", type=float, default=1.0)
    ap.add_argument("--k", type=int, default=6)
    a = ap.parse_args(argv)
    t0 = time.time()
    U = synth.su3_links(a.dims, a.eps, a.seed, norm=a.norm)
    w = leftmost_eigenvalues(U, a.dims, k=a.k)
    rec = {
        "dims": a.dims, "eps": a.eps, "seed": a.seed, "norm": a.norm,
        "leftmost_eigenvalues_m0": [[float(z.real), float(z.imag)] for z in w],
        "min_real_part": float(w.real.min()),
        "seconds": time.time() - t0,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
