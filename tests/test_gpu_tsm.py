"""Truncated Solver Method (lqt_trace_tsm, Section 1) and the orthogonal projector on a
prolongator basis (the variance lower bound of Section 2.1) against the oracle on 4^4."""
import numpy as np
import pytest
import torch

import synth
from oracle import core, dense, estimator, probing, prolongator as pr

pytestmark = pytest.mark.gpu

DIMS, M = (4, 4, 4, 4), 0.1


@pytest.fixture(scope="module")
def op():
    U = synth.su3_links(DIMS, 0.3, 1)
    A = dense.dense_operator(U, DIMS, M)
    return U, A, np.linalg.inv(A)


def _bound(A, Ai, xi):
    return A.shape[0] * np.linalg.cond(A) * xi * np.linalg.norm(Ai, 2)


@pytest.mark.parametrize("hp,dilute", [(1, False), (2, True)])
def test_tsm_matches_oracle_combination(gpu, op, hp, dilute):
    """The three runs are the library's deterministic traces (fixed reduction orders, same
    batches), so the main and correction samples are recomputed by separate lqt_trace calls;
    the oracle's TSM combination of them gives the returned estimate and error, the tight
    samples match the exact z^T A^-1 z, and the estimate is within 4 errors of tr A^-1."""
    lq = gpu
    U, A, Ai = op
    s, seed, nc, seed_c, xl, xt = 48, 1030, 12, 1031, 1e-2, 1e-10
    print(f"TSM hp={hp} dilute={dilute}", flush=True)
    c = lq.Context(DIMS, M)
    c.set_gauge(U)
    main, t = c.trace_tsm(s, seed, xl, nc, seed_c, xt, hp_vectors=hp, dilute=dilute)
    rm = c.trace(s, seed, xl, samples=True, hp_vectors=hp, dilute=dilute)
    rl = c.trace(nc, seed_c, xl, samples=True, hp_vectors=hp, dilute=dilute)
    rt = c.trace(nc, seed_c, xt, samples=True, hp_vectors=hp, dilute=dilute)
    with pytest.raises(lq.LqtError):
        c.trace_tsm(s, seed, xl, nc, seed, xt)  # the correction probes must be independent
    with pytest.raises(lq.LqtError):
        c.trace_tsm(s, seed, xt, nc, seed_c, xl)  # tight above loose
    c.close()
    q = hp * (12 if dilute else 1)
    assert t["nsolves_loose"] == (s + nc) * q and t["nsolves_tight"] == nc * q and t["nfailed"] == 0
    assert main["trace_re"] == rm["trace_re"]
    d = rt["samples"].numpy() - rl["samples"].numpy()
    assert np.array_equal(t["corr_samples"].numpy(), d)
    ref = estimator.tsm_combine(rm["samples"].numpy(), 0.0, rl["samples"].numpy(), rt["samples"].numpy())
    assert abs(complex(t["trace_re"], t["trace_im"]) - ref["estimate"]) <= 1e-12 * abs(ref["estimate"])
    assert abs(t["err"] - ref["err"]) <= 1e-9 * ref["err"]
    assert abs(t["corr_var_sample"] - ref["corr_var_sample"]) <= 1e-9 * ref["corr_var_sample"]
    exact = probing.estimator_samples(lambda X: X @ Ai.T, seed_c, nc, DIMS, hp, dilute)
    assert np.max(np.abs(rt["samples"].numpy() - exact)) <= _bound(A, Ai, xt)
    assert np.max(np.abs(rl["samples"].numpy() - exact)) <= _bound(A, Ai, xl)
    assert abs(complex(t["trace_re"], t["trace_im"]) - np.trace(Ai)) <= 4 * t["err"]


def _mg(U, A, orthonormal=True):
    block, nv = (2, 2, 2, 2), 6
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((nv, A.shape[0])) + 1j * rng.standard_normal((nv, A.shape[0]))
    W = pr.block_orthonormalize(Y, DIMS, block)
    P = pr.dense_prolongator(W, DIMS, block)
    Hc = pr.coarse_g5(W.shape[0], nv)[:, None] * (P.conj().T @ A @ P)
    w, Ub = np.linalg.eigh(Hc)
    Ubar = Ub[:, np.argsort(np.abs(w))[:10]].T.copy()
    if not orthonormal:
        Ubar = Ubar + 0.1 * Ubar[::-1]
    return block, nv, W, Ubar, P


@pytest.mark.parametrize("hp,dilute", [(1, False), (2, True)])
def test_orthogonal_projector_on_prolongator_basis(gpu, op, hp, dilute):
    """Solves on (1 - Q Q^+) v with Q = W U_c applied through restriction and prolongation;
    t0 = tr Q^+ A^-1 Q from k prolongated solves."""
    lq = gpu
    U, A, Ai = op
    s, seed, xi = 3, 1032, 1e-10
    block, nv, W, Ubar, P = _mg(U, A)
    c = lq.Context(DIMS, M)
    c.set_gauge(U)
    B = c.basis_prolongator_from(block, nv, torch.as_tensor(W.reshape(-1)).cuda(), torch.as_tensor(Ubar).cuda())
    r = c.trace(s, seed, xi, basis=B, projector=lq.ORTH, samples=True, hp_vectors=hp, dilute=dilute)
    B.close()
    c.close()
    Qm = P @ Ubar.T  # N x k, orthonormal columns
    ref = []
    for j in range(s):
        Vj = probing.partition_vectors(seed, j, DIMS, hp, dilute)
        R = Vj - (Qm @ (Qm.conj().T @ Vj.T)).T
        ref.append(np.einsum("pn,pn->", Vj, R @ Ai.T) / hp)
    assert np.max(np.abs(r["samples"].numpy() - np.array(ref))) <= _bound(A, Ai, xi)
    t0 = np.trace(Qm.conj().T @ Ai @ Qm)
    assert abs(complex(r["t0_re"], r["t0_im"]) - t0) <= 10 * np.linalg.cond(A) * xi * np.linalg.norm(Ai, 2)


def test_orthogonal_projector_needs_orthonormal_coarse_vectors(gpu, op):
    lq = gpu
    U, A, Ai = op
    block, nv, W, Ubar, P = _mg(U, A, orthonormal=False)
    c = lq.Context(DIMS, M)
    c.set_gauge(U)
    B = c.basis_prolongator_from(block, nv, torch.as_tensor(W.reshape(-1)).cuda(), torch.as_tensor(Ubar).cuda())
    with pytest.raises(lq.LqtError):
        c.trace(2, 1, 1e-8, basis=B, projector=lq.ORTH)
    r = c.trace(2, 1, 1e-8, basis=B)  # the oblique projector takes any basis
    assert r["nfailed"] == 0
    B.close()
    c.close()


def test_orthogonal_bound_below_oblique_for_prolongator_basis(gpu, op):
    """The variance of the orthogonal projector's samples, reported as the rough lower bound
    of Section 2.1, against the exact variances of both deflated operators on this basis (the
    oracle's formula with the symmetrised operators): the library's sample variances over 400
    probes fall within a chi^2 band of the exact ones."""
    lq = gpu
    U, A, Ai = op
    block, nv, W, Ubar, P = _mg(U, A)
    c = lq.Context(DIMS, M)
    c.set_gauge(U)
    B = c.basis_prolongator_from(block, nv, torch.as_tensor(W.reshape(-1)).cuda(), torch.as_tensor(Ubar).cuda())
    s = 400
    ro = c.trace(s, 1033, 1e-10, basis=B, projector=lq.ORTH)
    rb = c.trace(s, 1033, 1e-10, basis=B)
    B.close()
    c.close()
    Qm = P @ Ubar.T
    N = A.shape[0]
    B_orth = Ai @ (np.eye(N) - Qm @ Qm.conj().T)
    X = Qm.T
    Uo, lam, _, _ = estimator.oblique_setup(X, (A @ X.T).T)
    Pobl = estimator.oblique_projector_dense(A, Uo, lam)
    B_obl = Ai @ (np.eye(N) - Pobl)
    ones = np.ones((N, N))
    v_orth = probing.exact_variance(B_orth, ones)
    v_obl = probing.exact_variance(B_obl, ones)
    assert 0.75 * v_orth <= ro["var_sample"] <= 1.3 * v_orth
    assert 0.75 * v_obl <= rb["var_sample"] <= 1.3 * v_obl
    print(f"one-probe variance: orthogonal {v_orth:.4e}, oblique {v_obl:.4e}", flush=True)
