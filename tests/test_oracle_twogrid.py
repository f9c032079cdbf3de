"""Pins of the oracle's two-grid preconditioner (Section 2): the coarse grid correction is
exact on span(W) and its error propagation I - P D_c^{-1} P^+ A is a projector; with one
site per aggregate and 6 vectors per chirality W is unitary and the correction is A^{-1};
each minimal-residual step leaves a residual orthogonal to A s and no larger."""
import numpy as np

import synth
from oracle import core, dense, prolongator as pr, twogrid


def _W(dims, block, nv, seed=3):
    rng = np.random.default_rng(seed)
    N = 12 * int(np.prod(dims))
    Y = rng.standard_normal((nv, N)) + 1j * rng.standard_normal((nv, N))
    return pr.block_orthonormalize(Y, dims, block)


DIMS, BLOCK, NV, M = (4, 4, 2, 2), (2, 2, 2, 2), 4, 0.1


def test_coarse_correction_is_exact_on_the_prolongator_span():
    U = synth.su3_links(DIMS, 0.4, 1)
    W = _W(DIMS, BLOCK, NV)
    nc = W.shape[0] * 2 * NV
    rng = np.random.default_rng(5)
    cv = rng.standard_normal((2, nc)) + 1j * rng.standard_normal((2, nc))
    Pc = pr.prolong(W, cv, DIMS, BLOCK)
    r = core.apply(U, DIMS, M, core.OP_A, Pc)
    x = twogrid.apply(U, DIMS, M, W, BLOCK, r, 0)
    assert np.max(np.abs(x - Pc)) <= 1e-12 * np.max(np.abs(Pc))


def test_coarse_error_propagation_is_a_projector():
    U = synth.su3_links(DIMS, 0.4, 1)
    W = _W(DIMS, BLOCK, NV)
    A = dense.dense_operator(U, DIMS, M)
    P = pr.dense_prolongator(W, DIMS, BLOCK)
    Dc = twogrid.coarse_operator(U, DIMS, M, W, BLOCK)
    assert np.allclose(Dc, P.conj().T @ A @ P, atol=1e-12)
    E = np.eye(A.shape[0]) - P @ np.linalg.solve(Dc, P.conj().T @ A)
    assert np.max(np.abs(E @ E - E)) <= 1e-10
    assert np.max(np.abs(E @ P)) <= 1e-10


def test_unitary_prolongator_gives_the_inverse():
    dims = (2, 2, 2, 2)
    U = synth.su3_links(dims, 0.4, 2)
    W = _W(dims, (1, 1, 1, 1), 6)
    A = dense.dense_operator(U, dims, M)
    rng = np.random.default_rng(6)
    r = rng.standard_normal((2, A.shape[0])) + 0j
    x = twogrid.apply(U, dims, M, W, (1, 1, 1, 1), r, 3)
    ref = np.linalg.solve(A, r.T).T
    assert np.max(np.abs(x - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_minimal_residual_steps():
    U = synth.su3_links(DIMS, 0.4, 1)
    rng = np.random.default_rng(7)
    N = 12 * int(np.prod(DIMS))
    r = rng.standard_normal((1, N)) + 1j * rng.standard_normal((1, N))
    x0 = np.zeros_like(r)
    prev = np.linalg.norm(r)
    for nu in range(1, 5):
        x = twogrid.mr_smooth(U, DIMS, M, r, x0, nu)
        s = r - core.apply(U, DIMS, M, core.OP_A, x)
        assert np.linalg.norm(s) <= prev * (1 + 1e-12)
        prev = np.linalg.norm(s)
    # the last step leaves s orthogonal to A s_prev: one more step from x with nu = 1
    x1 = twogrid.mr_smooth(U, DIMS, M, r, x, 1)
    s0 = r - core.apply(U, DIMS, M, core.OP_A, x)
    p = core.apply(U, DIMS, M, core.OP_A, s0)
    s1 = r - core.apply(U, DIMS, M, core.OP_A, x1)
    assert abs(np.vdot(p[0], s1[0])) <= 1e-10 * np.linalg.norm(p) * np.linalg.norm(s1)
