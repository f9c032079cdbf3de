"""GPU prolongator restrict/prolong and the Algorithm 2 estimator against the oracle."""
import numpy as np
import pytest
import torch

import synth
from eigcheck import check_smallest_abs_pairs
from oracle import core, dense, estimator, prolongator as pr

pytestmark = pytest.mark.gpu


def _W(dims, block, nv, seed=3):
    rng = np.random.default_rng(seed)
    N = 12 * int(np.prod(dims))
    Y = rng.standard_normal((nv, N)) + 1j * rng.standard_normal((nv, N))
    return pr.block_orthonormalize(Y, dims, block)


@pytest.mark.parametrize("dims,block,nv", [((4, 4, 4, 4), (2, 2, 2, 2), 6), ((4, 4, 2, 8), (4, 4, 2, 2), 5),
                                           ((8, 4, 4, 4), (4, 4, 4, 4), 12)])
@pytest.mark.parametrize("nrhs", [1, 9])
def test_restrict_prolong_match_oracle(gpu, dims, block, nv, nrhs):
    lq = gpu
    print(f"P/R dims={dims} block={block} nv={nv} nrhs={nrhs}", flush=True)
    W = _W(dims, block, nv)
    c = lq.Context(dims, 0.1)
    B = c.basis_prolongator_from(block, nv, torch.as_tensor(W.reshape(-1)).cuda())
    N = 12 * int(np.prod(dims))
    rng = np.random.default_rng(7)
    y = rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N))
    cg = B.restrict(torch.as_tensor(y).cuda()).cpu().numpy()
    cr = pr.restrict(W, y, dims, block)
    assert np.max(np.abs(cg - cr)) <= 1e-13 * np.max(np.abs(cr))
    yg = B.prolong(torch.as_tensor(cr).cuda()).cpu().numpy()
    yr = pr.prolong(W, cr, dims, block)
    assert np.max(np.abs(yg - yr)) <= 1e-13 * np.max(np.abs(yr))
    assert np.array_equal(B.prolongator().cpu().numpy(), W.reshape(-1))
    B.close()
    c.close()


def test_algorithm2_estimator_matches_oracle(gpu):
    """W and the coarse eigenvectors U_bar from the oracle; the GPU forms M, Lambda, U_c,
    t0 and the deflated samples, compared with the oracle estimator on X = W U_bar."""
    lq = gpu
    dims, block, nv, m = (4, 4, 4, 4), (2, 2, 2, 2), 6, 0.1
    U = synth.su3_links(dims, 0.3, 1)
    A = dense.dense_operator(U, dims, m)
    Ai = np.linalg.inv(A)
    W = _W(dims, block, nv)
    P = pr.dense_prolongator(W, dims, block)
    g5c = pr.coarse_g5(W.shape[0], nv)
    Hc = g5c[:, None] * (P.conj().T @ A @ P)
    w, Ub = np.linalg.eigh(Hc)
    idx = np.argsort(np.abs(w))[:12]
    Ubar = Ub[:, idx].T.copy()  # rows
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator_from(block, nv, torch.as_tensor(W.reshape(-1)).cuda(), torch.as_tensor(Ubar).cuda())
    X = (P @ Ubar.T).T
    Uo, lam, ug5u, t0 = estimator.oblique_setup(X, (A @ X.T).T)
    assert np.allclose(np.sort(np.abs(B.eigenvalues().numpy().real)), np.sort(np.abs(lam)), rtol=1e-9)
    Uf = B.vectors().cpu().numpy()
    assert np.allclose(np.abs(np.conj(Uf) @ Uo.T).max(axis=1), 1.0, atol=1e-8)  # same vectors up to phase
    s, seed, xi = 48, 1005, 1e-10
    r = c.trace(s, seed, xi, basis=B, samples=True, rank_curve=True)
    Z = core.probes(seed, s, A.shape[0])
    Y = (Ai @ Z.T).T
    t_ref = estimator.hutchinson_samples(Z, Y) - estimator.oblique_corrections(Z, Uo, lam)
    bound = A.shape[0] * np.linalg.cond(A) * xi * np.linalg.norm(Ai, 2)
    assert abs(complex(r["t0_re"], r["t0_im"]) - t0) <= 1e-9 * abs(t0)
    assert np.max(np.abs(r["samples"].numpy() - t_ref)) <= bound + 1e-8 * np.max(np.abs(t_ref))
    curve = estimator.rank_curve(Z, Y, Uo, lam, ug5u)
    assert np.allclose(r["rank_curve"].numpy(), curve, rtol=1e-6, atol=1e-6)
    assert abs(r["trace_re"] - np.trace(Ai).real) <= 4 * np.sqrt(r["var_mean"])
    B.close()
    c.close()


def test_prolongator_basis_from_near_null_vectors(gpu):
    """lqt_basis_prolongator end to end (near-null vectors, blocking, coarse eigensolve):
    check what is unique or must hold for any valid result."""
    lq = gpu
    dims, block, nv, m, k = (4, 4, 4, 4), (2, 2, 2, 2), 6, 0.1, 8
    U = synth.su3_links(dims, 0.3, 1)
    A = dense.dense_operator(U, dims, m)
    Ai = np.linalg.inv(A)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator(block, nv, k, null_xi=1e-2, null_maxit=200, require_converged=True)
    W = B.prolongator().cpu().numpy().reshape(-1, 2, nv, 6 * 16)
    for a in range(W.shape[0]):  # orthonormal blocks
        for ch in range(2):
            assert np.allclose(W[a, ch].conj() @ W[a, ch].T, np.eye(nv), atol=1e-12)
    # the near-null vectors are smooth: A W is smaller than A on random blocks of the same shape
    P = pr.dense_prolongator(W, dims, block)
    Wr = _W(dims, block, nv)
    Pr = pr.dense_prolongator(Wr, dims, block)
    assert np.linalg.norm(A @ P) < 0.9 * np.linalg.norm(A @ Pr)
    # coarse eigenpairs: the returned coarse vectors U_c = W^+ U are orthonormal, each pair
    # meets ||H_c u - theta u|| <= xi |theta| on the dense coarse operator
    g5c = pr.coarse_g5(W.shape[0], nv)
    Hc = g5c[:, None] * (P.conj().T @ A @ P)
    lam = B.eigenvalues().numpy().real
    Uc = B.restrict(B.vectors()).cpu().numpy()
    thc = np.einsum("in,in->i", Uc.conj(), (Hc @ Uc.T).T).real
    assert np.allclose(thc, lam, rtol=1e-8, atol=1e-12)
    check_smallest_abs_pairs(Hc, thc, Uc, xi=1e-2, tight=False)
    r = c.trace(64, 1000, 1e-10, basis=B)
    assert abs(r["trace_re"] - np.trace(Ai).real) <= 4 * np.sqrt(r["var_mean"])
    B.close()
    c.close()


def test_coarse_eigensolver_returns_smallest_pairs(gpu):
    """The coarse eigensolve of Algorithm 2 at a tight tolerance on 4^4 (2^4 aggregates,
    nv = 6, nc = 192, k = 12): the k smallest |lambda| of the dense g5^W W^+ A W, with the
    sin-theta bound on the subspace."""
    lq = gpu
    dims, block, nv, m, k = (4, 4, 4, 4), (2, 2, 2, 2), 6, 0.1, 12
    U = synth.su3_links(dims, 0.3, 1)
    A = dense.dense_operator(U, dims, m)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator(block, nv, k, null_xi=1e-2, null_maxit=200, require_converged=True, eig_xi=1e-9, outer_maxit=200)
    W = B.prolongator().cpu().numpy().reshape(-1, 2, nv, 6 * 16)
    P = pr.dense_prolongator(W, dims, block)
    g5c = pr.coarse_g5(W.shape[0], nv)
    Hc = g5c[:, None] * (P.conj().T @ A @ P)
    Uc = B.restrict(B.vectors()).cpu().numpy()
    thc = np.einsum("in,in->i", Uc.conj(), (Hc @ Uc.T).T).real
    r2, sin, delta = check_smallest_abs_pairs(Hc, thc, Uc, xi=2e-9)
    print(f"coarse ||R|| {r2:.2e} sin angle {sin:.2e} gap {delta:.2e}", flush=True)
    B.close()
    c.close()


@pytest.mark.parametrize("dims,block,nv,s", [((8, 8, 8, 8), (8, 4, 4, 4), 3, 37), ((4, 4, 4, 8), (4, 4, 2, 2), 4, 70)])
def test_deflation_corrections_match_oracle(gpu, dims, block, nv, s):
    """The deflation corrections of Algorithm 2's estimator (undeflated minus deflated samples
    of the same probes, whose solves are bitwise identical) against the oracle on X = W U_bar,
    for blocks with more entries than one tile of the probe restriction (8 x 4 x 4 x 4 sites:
    3072 entries per chirality) and more probes than one workgroup restricts (32)."""
    lq = gpu
    m, seed = 0.2, 1011
    print(f"Algorithm 2 corrections dims={dims} block={block} nv={nv} probes={s}", flush=True)
    U = synth.su3_links(dims, 0.3, 2)
    W = _W(dims, block, nv)
    nc = W.shape[0] * 2 * nv
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((nc, 5)) + 1j * rng.standard_normal((nc, 5)))
    Ubar = Q.T.copy()
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator_from(block, nv, torch.as_tensor(W.reshape(-1)).cuda(), torch.as_tensor(Ubar).cuda())
    r0 = c.trace(s, seed, 1e-10, samples=True)
    rB = c.trace(s, seed, 1e-10, basis=B, samples=True)
    B.close()
    c.close()
    X = pr.prolong(W, Ubar, dims, block)
    Uo, lam, ug5u, t0 = estimator.oblique_setup(X, core.apply(U, dims, m, core.OP_A, X))
    assert abs(complex(rB["t0_re"], rB["t0_im"]) - t0) <= 1e-9 * abs(t0)
    Z = core.probes(seed, s, X.shape[1])
    corr = estimator.oblique_corrections(Z, Uo, lam)
    corr_gpu = r0["samples"].numpy() - rB["samples"].numpy()
    assert np.max(np.abs(corr_gpu - corr)) <= 1e-9 * np.max(np.abs(corr)) + 1e-9 * np.max(np.abs(r0["samples"].numpy()))
