"""Second multigrid level (Table 2; lqt_basis_prolongator2) against the oracle: the level-2
operator W2^+ D_c W2 assembled by coloured probing against the oracle's P2^+ (P1^+ A P1) P2,
for level-2 lattices with extents 1, 2, 3 and 4 along a direction (the colourings' cases);
Algorithm 2's estimator on X = P1 P2 U2 against the oracle; and the full two-level build
(near-null vectors of both levels, the level-2 eigensolve) returning the smallest pairs of
the level-2 operator."""
import numpy as np
import pytest
import torch

import synth
from eigcheck import check_smallest_abs_pairs
from oracle import core, dense, estimator, prolongator as pr

pytestmark = pytest.mark.gpu


def _levels(dims, block1, nv1, block2, nv2, seed=4):
    rng = np.random.default_rng(seed)
    N = 12 * int(np.prod(dims))
    W1 = pr.block_orthonormalize(rng.standard_normal((nv1, N)) + 1j * rng.standard_normal((nv1, N)), dims, block1)
    P1 = pr.dense_prolongator(W1, dims, block1)
    cdims = tuple(L // b for L, b in zip(dims, block1))
    idx2 = pr.coarse_fine_index(cdims, block2, nv1)
    nc1 = P1.shape[1]
    W2 = pr.block_orthonormalize(rng.standard_normal((nv2, nc1)) + 1j * rng.standard_normal((nv2, nc1)), cdims, block2,
                                 idx=idx2)
    P2 = pr.dense_prolongator(W2, cdims, block2, idx=idx2, N=nc1)
    return W1, P1, W2, P2


CASES = [
    ((8, 4, 4, 4), (2, 2, 2, 2), 4, (2, 2, 2, 2), 3, 0.1),   # level 2: 2 x 1 x 1 x 1
    ((12, 4, 4, 4), (2, 2, 2, 2), 4, (2, 2, 2, 2), 3, -0.2),  # 3 x 1 x 1 x 1
    ((16, 4, 4, 8), (2, 2, 2, 2), 3, (2, 2, 2, 2), 4, 0.3),   # 4 x 1 x 1 x 2
    ((8, 8, 8, 8), (4, 4, 4, 4), 6, (1, 1, 2, 2), 5, 0.0),    # 2 x 2 x 1 x 1, non-cubic level-2 blocks
]


@pytest.mark.parametrize("dims,block1,nv1,block2,nv2,m", CASES)
def test_level2_operator_matches_oracle(gpu, dims, block1, nv1, block2, nv2, m):
    lq = gpu
    print(f"level-2 operator dims={dims} block1={block1} nv1={nv1} block2={block2} nv2={nv2}", flush=True)
    U = synth.su3_links(dims, 0.4, 3)
    W1, P1, W2, P2 = _levels(dims, block1, nv1, block2, nv2)
    Dc = P1.conj().T @ core.apply(U, dims, m, core.OP_A, P1.T.copy()).T
    Dcc = P2.conj().T @ Dc @ P2
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator2_from(block1, nv1, torch.as_tensor(W1.reshape(-1)).cuda(), block2, nv2,
                                  torch.as_tensor(W2.reshape(-1)).cuda())
    assert np.array_equal(B.prolongator2().cpu().numpy(), W2.reshape(-1))
    rng = np.random.default_rng(9)
    x = rng.standard_normal((5, Dcc.shape[0])) + 1j * rng.standard_normal((5, Dcc.shape[0]))
    y = B.coarse2_apply(torch.as_tensor(x).cuda()).cpu().numpy()
    ref = (Dcc @ x.T).T
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
    g2 = pr.coarse_g5(W2.shape[0], nv2)
    yh = B.coarse2_apply(torch.as_tensor(x[:2]).cuda(), herm=True).cpu().numpy()
    assert np.max(np.abs(yh - g2[None, :] * ref[:2])) <= 1e-12 * np.max(np.abs(ref))
    B.close()
    c.close()


def test_two_level_estimator_matches_oracle(gpu):
    """W1, W2 and the level-2 eigenvectors from the oracle; the library forms W2 U2, M, t0 and
    the deflated samples, compared with the oracle estimator on X = P1 P2 U2."""
    lq = gpu
    dims, block1, nv1, block2, nv2, m = (8, 4, 4, 4), (2, 2, 2, 2), 4, (2, 2, 2, 2), 3, 0.1
    U = synth.su3_links(dims, 0.3, 1)
    A = dense.dense_operator(U, dims, m)
    Ai = np.linalg.inv(A)
    W1, P1, W2, P2 = _levels(dims, block1, nv1, block2, nv2)
    P = P1 @ P2
    g2 = pr.coarse_g5(W2.shape[0], nv2)
    Hc = g2[:, None] * (P.conj().T @ A @ P)
    w, Ub = np.linalg.eigh(Hc)
    U2 = Ub[:, np.argsort(np.abs(w))[:5]].T.copy()
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator2_from(block1, nv1, torch.as_tensor(W1.reshape(-1)).cuda(), block2, nv2,
                                  torch.as_tensor(W2.reshape(-1)).cuda(), torch.as_tensor(U2).cuda())
    X = (P @ U2.T).T
    Uo, lam, ug5u, t0 = estimator.oblique_setup(X, (A @ X.T).T)
    assert np.allclose(np.sort(np.abs(B.eigenvalues().numpy().real)), np.sort(np.abs(lam)), rtol=1e-9)
    s, seed, xi = 24, 1060, 1e-10
    r = c.trace(s, seed, xi, basis=B, samples=True)
    B.close()
    c.close()
    Z = core.probes(seed, s, A.shape[0])
    t_ref = estimator.hutchinson_samples(Z, (Ai @ Z.T).T) - estimator.oblique_corrections(Z, Uo, lam)
    bound = A.shape[0] * np.linalg.cond(A) * xi * np.linalg.norm(Ai, 2)
    assert abs(complex(r["t0_re"], r["t0_im"]) - t0) <= 1e-9 * abs(t0)
    assert np.max(np.abs(r["samples"].numpy() - t_ref)) <= bound + 1e-8 * np.max(np.abs(t_ref))


def test_two_level_build_returns_the_smallest_level2_pairs(gpu):
    """The full two-level build on 8^4 (level 1: 2^4 aggregates, 6 vectors per chirality;
    level 2: 2^4 blocks of the 4^4 coarse lattice, 8 vectors): W2 orthonormal and
    chirality-split, and the coarse eigenvalues the k smallest |lambda| of the oracle's
    g5^{W2} P2^+ P1^+ A P1 P2 built from the library's W and W2."""
    lq = gpu
    dims, block1, nv1, block2, nv2, m, k = (8, 8, 8, 8), (2, 2, 2, 2), 6, (2, 2, 2, 2), 8, -0.3, 8
    U = synth.su3_links(dims, 0.4, 2)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator2(block1, nv1, block2, nv2, k, null_xi=1e-2, null_maxit=200, eig_xi=1e-9, outer_maxit=300,
                             require_converged=True)
    W1 = B.prolongator().cpu().numpy()
    W2 = B.prolongator2().cpu().numpy()
    lam_gpu = B.eigenvalues().numpy().real
    B.close()
    c.close()
    N = 12 * 4096
    nagg1 = 4 ** 4
    W1 = W1.reshape(nagg1, 2, nv1, -1)
    cdims = (4, 4, 4, 4)
    idx2 = pr.coarse_fine_index(cdims, block2, nv1)
    W2 = W2.reshape(16, 2, nv2, -1)
    for a in range(16):
        for ch in range(2):
            assert np.allclose(W2[a, ch].conj() @ W2[a, ch].T, np.eye(nv2), atol=1e-12)
    P1 = pr.dense_prolongator(W1, dims, block1)
    P2 = pr.dense_prolongator(W2, cdims, block2, idx=idx2, N=P1.shape[1])
    Dc = P1.conj().T @ core.apply(U, dims, m, core.OP_A, P1.T.copy()).T
    Dcc = P2.conj().T @ Dc @ P2
    Hc = pr.coarse_g5(16, nv2)[:, None] * Dcc
    w = np.linalg.eigvalsh(0.5 * (Hc + Hc.conj().T))
    exact = np.sort(np.abs(w))[:k]
    # the rotated Ritz values of M = U^+ g5^W D_c U equal those of g5^{W2} D_cc on span(U2)
    assert np.allclose(np.sort(np.abs(lam_gpu)), exact, rtol=1e-6)
    assert N == P1.shape[0]
