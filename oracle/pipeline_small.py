"""The whole deflated estimator on the 4^4 workload with the FP64 CPU oracle, timed.

TEST INFRASTRUCTURE / measurement tool: calls only the oracle and the seeded input
generator.  Usage:
    python -m oracle.pipeline_small [--threads T]

Steps (Section 1 and Section 2.1 of the paper, Algorithm 1's basis with exact eigenvectors):
  1. the dense operator A (3072 x 3072) and the exact trace of A^{-1} by LU;
  2. 64 real Rademacher probes solved one by one with FP64 GMRES(32) to 1e-10;
  3. the 16 eigenvectors Q of the Hermitian A g5 with the smallest |lambda| (the smallest
     singular vectors of A) by a dense eigen-decomposition, entering as X = g5 Q;
  4. the samples, t0 and the oblique K = g5 corrections for every rank 0..16;
  5. the exact one-probe variances (Eq. (2) on the symmetrised operator) of A^{-1} and of
     the deflated A^{-1}(I - P), also for bases of 64, 256 and 1024 such vectors.
Prints one JSON line: the estimates against the exact trace, the exact and sample variances,
and the wall time of each step.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import core, dense, estimator


def main(argv=None):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=None, help="OMP_NUM_THREADS of the C oracle")
    a = ap.parse_args(argv)
    if a.threads:
        os.environ["OMP_NUM_THREADS"] = str(a.threads)
    dims, eps, seed, mass, s, k, xi = (4, 4, 4, 4), 0.3, 1, 0.1, 64, 16, 1e-10
    t = {}

    t0 = time.perf_counter()
    U = synth.su3_links(dims, eps, seed)
    A = dense.dense_operator(U, dims, mass)
    Ai = np.linalg.inv(A)
    exact = np.trace(Ai)
    t["dense_lu_s"] = time.perf_counter() - t0

    t0 = time.perf_counter()
    N = A.shape[0]
    Z = core.probes(1000, s, N)
    Y = np.empty((s, N), dtype=np.complex128)
    steps = 0
    for j in range(s):
        Y[j], conv, its, rel = core.gmres(U, dims, mass, Z[j], xi)
        assert conv, (j, rel)
        steps += its
    t["solves_s"] = time.perf_counter() - t0

    t0 = time.perf_counter()
    g5 = estimator.g5_vec(N)
    w, Q = np.linalg.eigh(A * g5[None, :])  # A g5 is Hermitian
    idx = np.argsort(np.abs(w))[:k]
    X = g5 * Q[:, idx].T  # X = g5 Q: the oblique projector is then Q Q^+ (Section 2.1, K = g5)
    Ub, lam, ug5u, tzero = estimator.oblique_setup(X, (A @ X.T).T)
    t["basis_s"] = time.perf_counter() - t0

    t0 = time.perf_counter()
    curve = estimator.rank_curve(Z, Y, Ub, lam, ug5u)
    t["estimate_s"] = time.perf_counter() - t0

    P = estimator.oblique_projector_dense(A, Ub, lam)
    v0 = estimator.exact_variances(Ai)["exact"]
    vk = estimator.exact_variances(Ai @ (np.eye(N) - P))["exact"]
    # the exact variance for larger bases of the same kind
    by_rank = {0: v0, k: vk}
    for kk in (64, 256, 1024):
        Xk = g5 * Q[:, np.argsort(np.abs(w))[:kk]].T
        Uk, lamk, _, _ = estimator.oblique_setup(Xk, (A @ Xk.T).T)
        Pk = estimator.oblique_projector_dense(A, Uk, lamk)
        by_rank[kk] = estimator.exact_variances(Ai @ (np.eye(N) - Pk))["exact"]
    out = {
        "workload": "Wilson-Dirac 4^4, eps=0.3, m=0.1, 64 Rademacher probes, FP64 GMRES(32) to 1e-10, "
                    "k=16 smallest |lambda(A g5)|, oblique g5 projector",
        "trace_exact": [exact.real, exact.imag],
        "estimate_undeflated": {"trace": curve[0, 0], "var_sample": curve[0, 1], "jackknife_err": curve[0, 2]},
        "estimate_deflated": {"trace": curve[k, 0], "var_sample": curve[k, 1], "jackknife_err": curve[k, 2]},
        "var_exact_undeflated": v0,
        "var_exact_deflated": vk,
        "var_exact_by_rank": {str(r): v for r, v in by_rank.items()},
        "smallest_abs_lambda": float(np.abs(lam[0])),
        "gmres_steps_per_probe": steps / s,
        "seconds": {f: round(v, 3) for f, v in t.items()},
        "omp_threads": os.environ.get("OMP_NUM_THREADS", str(os.cpu_count())),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
