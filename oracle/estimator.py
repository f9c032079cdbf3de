"""Deflated Hutchinson estimator written from the paper, FP64 numpy (oracle).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's CPU leg.

Paper: Romero, Stathopoulos, Orginos, "Multigrid deflation for Lattice QCD".
  Eq. (1)          t = (1/s) sum_j x_j^+ A^{-1} x_j for probes with E[x_i^* x_j] = delta_ij
                   (the printed E[x^+ A x] is read as E[x^+ A^{-1} x]).
  Eq. (2)          Var = (2/s)||A^{-1}||_F^2 - (2/s) sum_i |A^{-1}_ii|^2, exact for real
                   +-1 probes only when A^{-1} is complex-symmetric; the exact variance for
                   real probes replaces A^{-1} by S = (A^{-1} + A^{-T})/2, the symmetrised
                   operator of Section 2.1 (same trace, no larger variance).
  Section 2.1      trace A^{-1} = trace A^{-1}(I - A V (V^+ K A V)^{-1} V^+ K)
                                 + trace V^+ K V (V^+ K A V)^{-1},  here K = g5.
  Section 2.2      the deflated samples need only the k x s products Z^T U and U^+ g5 Z, so
                   the estimate can be recomputed for every rank after the solves.
  Algorithm 2      factor U_hat Lambda U_hat^+ = X^+ g5 A X, U = X U_hat,
                   t0 = sum_i lambda_i^{-1} u_i^+ g5 u_i.
  Algorithm 1      orthogonal projector U U^+: t0 = sum_i u_i^+ A^{-1} u_i and the
                   stochastic part on A^{-1}(I - U U^+).
  Section 1        Truncated Solver Method: the samples of A_xi^{-1} (solves stopped at a loose
                   xi) are biased; an independent set of probes solved both loosely and tightly
                   estimates the trace of the difference, which is added.
Vectors are rows: X has shape (k, N), probes Z (s, N) real, solutions Y (s, N).
"""
import numpy as np


def g5_vec(N):
    """Diagonal of g5 in the spinor index order 12*site + 3*spin + colour."""
    return np.tile(np.array([1.0] * 6 + [-1.0] * 6), N // 12)


def hutchinson_samples(Z, Y):
    """t_j = z_j^T y_j (Eq. 1 with real probes)."""
    return np.einsum("jn,jn->j", Z, Y)


def oblique_setup(X, AX):
    """From rows X (k, N) and AX = A X: M = X^+ g5 A X, eigen-decomposition of the Hermitian
    M = U_hat diag(lambda) U_hat^+, U = U_hat^T X (rows u_i), t0 = sum_i u_i^+ g5 u_i / lambda_i.
    Eigenpairs are ordered by increasing |lambda| (Algorithm 2, third and fourth steps)."""
    N = X.shape[1]
    g5 = g5_vec(N)
    M = np.conj(X) @ (g5 * AX).T  # M[a, b] = x_a^+ g5 A x_b
    M = 0.5 * (M + M.conj().T)    # Hermitian up to rounding
    lam, Uh = np.linalg.eigh(M)
    order = np.argsort(np.abs(lam), kind="stable")
    lam, Uh = lam[order], Uh[:, order]
    U = Uh.T @ X                  # u_i = sum_a Uh[a, i] x_a
    ug5u = np.einsum("in,n,in->i", np.conj(U), g5, U)
    t0 = np.sum(ug5u / lam)
    return U, lam, ug5u, t0


def oblique_correction_terms(Z, U, lam):
    """(s, k) array of the per-mode terms (z_j^T u_i) lambda_i^{-1} (u_i^+ g5 z_j) of each
    probe's correction; summing the first k' columns gives the rank-k' correction."""
    N = Z.shape[1]
    g5 = g5_vec(N)
    ZU = Z @ U.T                    # (s, k): z_j^T u_i
    UgZ = np.conj(U) @ (g5 * Z).T   # (k, s): u_i^+ g5 z_j
    return ZU * (UgZ.T / lam[None, :])


def oblique_corrections(Z, U, lam, rank=None):
    """c_j = (z_j^T U) Lambda^{-1} (U^+ g5 z_j) for the first `rank` basis vectors."""
    k = U.shape[0] if rank is None else rank
    return oblique_correction_terms(Z, U[:k], lam[:k]).sum(axis=1)


def summarize(t, t0=0.0):
    """Estimate t0 + mean(t), one-probe variance (s-1 denominator, complex modulus), variance
    of the mean, leave-one-out jackknife error, and the one-probe variance of Re t."""
    t = np.asarray(t, dtype=np.complex128)
    s = t.size
    mean = t.mean()
    var = np.sum(np.abs(t - mean) ** 2) / (s - 1) if s > 1 else 0.0
    var_re = np.sum((t.real - mean.real) ** 2) / (s - 1) if s > 1 else 0.0
    if s > 1:
        loo = (t.sum() - t) / (s - 1)
        jk = np.sqrt((s - 1) / s * np.sum(np.abs(loo - loo.mean()) ** 2))
    else:
        jk = 0.0
    return {"estimate": t0 + mean, "t0": t0, "var_sample": var, "var_mean": var / s if s else 0.0,
            "jackknife_err": jk, "var_re_only": var_re}


def rank_curve(Z, Y, U, lam, ug5u):
    """Estimate, one-probe variance and jackknife error for every rank k' = 0..k."""
    base = hutchinson_samples(Z, Y)
    out = []
    for kk in range(U.shape[0] + 1):
        if kk == 0:
            r = summarize(base, 0.0)
        else:
            c = oblique_corrections(Z, U, lam, kk)
            r = summarize(base - c, np.sum(ug5u[:kk] / lam[:kk]))
        out.append((r["estimate"].real, r["var_sample"], r["jackknife_err"]))
    return np.array(out)


def exact_variances(Binv):
    """Exact one-probe variances of z^T B z for real +-1 probes (B = A^{-1} or deflated):
    'printed' = Eq. (2) as printed with s = 1; 'exact' = the same form on the symmetrised
    S = (B + B^T)/2 (the true variance for real probes); 're' = variance of Re(z^T B z)."""
    S = 0.5 * (Binv + Binv.T)
    d = np.diag(Binv)
    printed = 2 * np.sum(np.abs(Binv) ** 2) - 2 * np.sum(np.abs(d) ** 2)
    exact = 2 * np.sum(np.abs(S) ** 2) - 2 * np.sum(np.abs(np.diag(S)) ** 2)
    Sr = S.real
    re = 2 * np.sum(Sr ** 2) - 2 * np.sum(np.diag(Sr) ** 2)
    return {"printed": float(printed), "exact": float(exact), "re": float(re)}


def oblique_projector_dense(A, U, lam):
    """P = A U^T Lambda^{-1} U^* g5 (Section 2.1 with K = g5) as a dense N x N matrix."""
    N = A.shape[0]
    g5 = g5_vec(N)
    return (A @ U.T) @ np.diag(1.0 / lam) @ (np.conj(U) * g5[None, :])


def tsm_combine(t_main, t0, corr_loose, corr_tight):
    """Truncated Solver Method (Section 1): estimate t0 + mean(t_main) + mean(d) with the
    corrections d_j = corr_tight_j - corr_loose_j of an independent probe set solved at both
    tolerances; the two means are independent, so the variance of the estimate is
    var(t_main)/s + var(d)/n_c (one-draw variances with the (n-1) denominator)."""
    main = summarize(t_main, t0)
    d = np.asarray(corr_tight, dtype=np.complex128) - np.asarray(corr_loose, dtype=np.complex128)
    corr = summarize(d)
    return {"estimate": main["estimate"] + corr["estimate"], "err": np.sqrt(main["var_mean"] + corr["var_mean"]),
            "corr_mean": corr["estimate"], "corr_var_sample": corr["var_sample"]}

