"""GPU deflation projections, bases and trace estimates (through the C-ABI) against the oracle."""
import numpy as np
import pytest
import torch

import synth
from eigcheck import check_smallest_abs_pairs
from oracle import core, dense, estimator

pytestmark = pytest.mark.gpu


def crand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.fixture(scope="module")
def cfg0():
    """The 4^4 workload: m = 0.1, eps = 0.3, seed 1; dense inverse by LU."""
    dims, m = (4, 4, 4, 4), 0.1
    U = synth.su3_links(dims, 0.3, 1)
    A = dense.dense_operator(U, dims, m)
    Ai = np.linalg.inv(A)
    return dims, m, U, A, Ai


@pytest.mark.parametrize("dims", [(3, 5, 4, 6), (8, 8, 8, 8)])
@pytest.mark.parametrize("ka,kb", [(5, 3), (19, 37), (64, 1)])
def test_gram_and_combine_match_numpy(gpu, dims, ka, kb):
    lq = gpu
    print(f"gram/combine dims={dims} ka={ka} kb={kb}", flush=True)
    c = lq.Context(dims, 0.1)
    N = 12 * int(np.prod(dims))
    X, Y = crand((ka, N), 1), crand((kb, N), 2)
    G = c.gram(torch.as_tensor(X).cuda(), torch.as_tensor(Y).cuda()).numpy()
    ref = np.conj(X) @ Y.T
    assert np.max(np.abs(G - ref)) <= 1e-13 * np.max(np.abs(ref)) * np.sqrt(N)
    C = crand((ka, kb), 3)
    Y0 = crand((kb, N), 4)
    out = c.combine(torch.as_tensor(X).cuda(), C, torch.as_tensor(Y0).cuda(), beta=-1.0, alpha=0.5).cpu().numpy()
    refc = -Y0 + 0.5 * (C.T @ X)
    assert np.max(np.abs(out - refc)) <= 1e-13 * np.max(np.abs(refc)) * ka
    c.close()


# V = 81 (3^4) is not a multiple of 4: a contraction step straddles the spin split at 6V
@pytest.mark.parametrize("dims,ka,s", [((3, 5, 4, 6), 7, 5), ((8, 8, 8, 8), 16, 70), ((3, 3, 3, 3), 5, 19)])
def test_project_probes_match_oracle(gpu, dims, ka, s):
    lq = gpu
    c = lq.Context(dims, 0.1)
    N = 12 * int(np.prod(dims))
    X = crand((ka, N), 5)
    cup, cdn = c.project_probes(torch.as_tensor(X).cuda(), 1003, 11, s)
    Z = core.probes(1003, s, N, j0=11)
    g5 = estimator.g5_vec(N)
    Zu, Zd = Z * (g5 > 0), Z * (g5 < 0)
    ru, rd = np.conj(X) @ Zu.T, np.conj(X) @ Zd.T
    tol = 1e-13 * np.sqrt(N) * np.max(np.abs(X))
    assert np.max(np.abs(cup.numpy() - ru)) <= tol
    assert np.max(np.abs(cdn.numpy() - rd)) <= tol
    c.close()


def test_undeflated_trace_matches_oracle_samples(gpu, cfg0):
    lq = gpu
    dims, m, U, A, Ai = cfg0
    N = A.shape[0]
    c = lq.Context(dims, m)
    c.set_gauge(U)
    s, seed, xi = 64, 1000, 1e-10
    r = c.trace(s, seed, xi, samples=True)
    Z = core.probes(seed, s, N)
    t_ref = estimator.hutchinson_samples(Z, (Ai @ Z.T).T)
    kappa = np.linalg.cond(A)
    bound = N * kappa * xi * np.linalg.norm(Ai, 2)
    assert np.max(np.abs(r["samples"].numpy() - t_ref)) <= bound
    ref = estimator.summarize(t_ref)
    assert abs(complex(r["trace_re"], r["trace_im"]) - ref["estimate"]) <= bound
    assert abs(r["var_sample"] - ref["var_sample"]) <= 1e-6 * ref["var_sample"]
    assert abs(r["jackknife_err"] - ref["jackknife_err"]) <= 1e-6 * ref["jackknife_err"]
    assert r["nsolves"] == s and r["nfailed"] == 0 and r["iters_total"] > 0
    # the estimate is within 4 sigma of the exact trace
    assert abs(r["trace_re"] - np.trace(Ai).real) <= 4 * np.sqrt(r["var_mean"])
    c.close()


def test_deflated_trace_matches_oracle(gpu, cfg0):
    """16 lowest |lambda| eigenvectors of A g5 (dense), entered as X = g5 Q (oblique, K = g5)."""
    lq = gpu
    dims, m, U, A, Ai = cfg0
    N = A.shape[0]
    g5 = estimator.g5_vec(N)
    w, Q = np.linalg.eigh(A * g5[None, :])
    idx = np.argsort(np.abs(w))[:16]
    X = (g5[:, None] * Q[:, idx]).T.copy()
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_from_vectors(torch.as_tensor(X).cuda())
    Ub, lam, ug5u, t0 = estimator.oblique_setup(X, (A @ X.T).T)
    assert np.allclose(np.sort(np.abs(B.eigenvalues().numpy().real)), np.sort(np.abs(lam)), rtol=1e-10)
    s, seed, xi = 64, 1000, 1e-10
    r = c.trace(s, seed, xi, basis=B, samples=True, rank_curve=True)
    Z = core.probes(seed, s, N)
    Y = (Ai @ Z.T).T
    t_ref = estimator.hutchinson_samples(Z, Y) - estimator.oblique_corrections(Z, Ub, lam)
    ref = estimator.summarize(t_ref, t0)
    bound = N * np.linalg.cond(A) * xi * np.linalg.norm(Ai, 2)
    assert abs(complex(r["t0_re"], r["t0_im"]) - t0) <= 1e-10 * abs(t0)
    assert np.max(np.abs(r["samples"].numpy() - t_ref)) <= bound + 1e-9 * np.max(np.abs(t_ref))
    assert abs(r["var_sample"] - ref["var_sample"]) <= 1e-5 * ref["var_sample"]
    curve_ref = estimator.rank_curve(Z, Y, Ub, lam, ug5u)
    assert np.allclose(r["rank_curve"].numpy(), curve_ref, rtol=1e-6, atol=1e-6)
    # exact eigenvectors: deflation removes their contribution, variance cannot grow
    assert r["var_sample"] <= r["rank_curve"][0, 1].item() * 1.0000001
    assert abs(r["trace_re"] - np.trace(Ai).real) <= 4 * np.sqrt(r["var_mean"])
    B.close()
    c.close()


def test_eigensolver_basis(gpu, cfg0):
    """Chebyshev-filtered eigensolver of A g5, xi = 1e-2, k = 16: every pair meets
    ||A g5 q - theta q|| <= xi |theta| (which implies the Table 1 test for the exact
    inverse), and the deflated estimates stay unbiased."""
    lq = gpu
    dims, m, U, A, Ai = cfg0
    N = A.shape[0]
    g5 = estimator.g5_vec(N)
    H = A * g5[None, :]
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_eig(16, xi=1e-2, require_converged=True)
    lam = B.eigenvalues().numpy().real
    Uv = B.vectors().cpu().numpy()  # U = g5 Q U_hat: rows
    Q = g5[None, :] * Uv
    th = np.einsum("in,in->i", Q.conj(), (H @ Q.T).T).real
    check_smallest_abs_pairs(H, th, Q, xi=1e-2, tight=False)
    assert np.allclose(np.sort(th), np.sort(lam), rtol=1e-9)
    # Table 1 test with the exact inverse: ||H^{-1} q - q / theta|| <= xi ||H^{-1}||
    Hi = np.linalg.inv(H)
    t1 = np.linalg.norm((Hi @ Q.T).T - Q / th[:, None], axis=1)
    assert np.all(t1 <= 1e-2 * np.linalg.norm(Hi, 2))
    # the deflated estimate stays unbiased
    r = c.trace(64, 1000, 1e-10, basis=B)
    assert abs(r["trace_re"] - np.trace(Ai).real) <= 4 * np.sqrt(r["var_mean"])
    ro = c.trace(64, 1000, 1e-10, basis=B, projector=lq.ORTH)
    assert abs(ro["trace_re"] - np.trace(Ai).real) <= 4 * np.sqrt(ro["var_mean"]) + 1e-6 * abs(np.trace(Ai))
    B.close()
    c.close()


@pytest.mark.parametrize("k", [16, 64])
def test_eigensolver_returns_smallest_pairs(gpu, cfg0, k):
    """Tight tolerance on 4^4: the k returned pairs are the k smallest |lambda| of A g5 (each
    Ritz value within ||R|| of one of them, no other eigenvalue that close) and span the exact
    eigenspace up to the Davis-Kahan bound ||R|| / gap."""
    lq = gpu
    dims, m, U, A, Ai = cfg0
    N = A.shape[0]
    g5 = estimator.g5_vec(N)
    H = A * g5[None, :]
    print(f"eigensolver k={k} at 1e-9 on 4^4", flush=True)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_eig(k, xi=1e-9, require_converged=True, outer_maxit=200)
    Uv = B.vectors().cpu().numpy()
    # U = (g5 Q) U_hat with U_hat unitary (M = Q^+ A g5 Q is diagonal up to the residuals)
    X = g5[None, :] * Uv
    M = X.conj() @ (H @ X.T)
    th, E = np.linalg.eigh(0.5 * (M + M.conj().T))
    Q = E.T @ X
    r2, sin, delta = check_smallest_abs_pairs(H, th, Q, xi=2e-9)
    print(f"||R|| {r2:.2e} sin angle {sin:.2e} gap {delta:.2e}", flush=True)
    assert np.allclose(np.sort(np.abs(B.eigenvalues().numpy().real)), np.sort(np.abs(th)), rtol=1e-8)
    B.close()
    c.close()


def test_estimator_statistics_match_exact_variance(gpu):
    """2^3 x 4 lattice, 2000 probes: sample variance vs the exact symmetrised form."""
    lq = gpu
    dims, m = (2, 2, 2, 4), 0.1
    U = synth.su3_links(dims, 0.3, 2)
    A = dense.dense_operator(U, dims, m)
    Ai = np.linalg.inv(A)
    v = estimator.exact_variances(Ai)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    r = c.trace(2000, 77, 1e-12)
    assert abs(r["trace_re"] - np.trace(Ai).real) <= 4 * np.sqrt(v["exact"] / 2000)
    assert abs(r["var_sample"] / v["exact"] - 1) < 0.15
    assert abs(r["var_re_only"] / v["re"] - 1) < 0.15
    c.close()


def test_trace_error_paths(gpu, cfg0):
    lq = gpu
    dims, m, U, A, Ai = cfg0
    c = lq.Context(dims, m)
    c.set_gauge(U)
    X = crand((4, A.shape[0]), 9)
    B = c.basis_from_vectors(torch.as_tensor(X).cuda())
    with pytest.raises(lq.LqtError) as e:  # orthogonal projector needs an orthonormal eigenbasis
        c.trace(8, 1, 1e-8, basis=B, projector=lq.ORTH)
    assert e.value.code == -1
    with pytest.raises(lq.LqtError) as e:
        c.trace(0, 1, 1e-8)
    assert e.value.code == -1
    r = c.trace(4, 1, 1e-12, raise_on_fail=False, maxit=2, restart=2)
    assert r["rc"] == -4 and r["nfailed"] == 4
    B.close()
    c.close()


def test_tau_shift_leaves_the_basis_unchanged(gpu, cfg0):
    """Algorithm 1's target g5 (A + i tau g5)^{-1} = (A g5 + i tau)^{-1} has the eigenvectors
    of A g5, ordered by |lambda + i tau|, i.e. by |lambda|: the basis for tau = 0.3 is the
    basis for tau = 0 (the filter applies A g5 itself), and a non-finite tau is refused."""
    lq = gpu
    dims, m, U, A, Ai = cfg0
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B0 = c.basis_eig(16, xi=1e-2, tau=0.0)
    B1 = c.basis_eig(16, xi=1e-2, tau=0.3)
    assert np.array_equal(B0.eigenvalues().numpy(), B1.eigenvalues().numpy())
    assert torch.equal(B0.vectors(), B1.vectors())
    with pytest.raises(lq.LqtError):
        c.basis_eig(16, xi=1e-2, tau=float("inf"))
    B0.close()
    B1.close()
    c.close()
