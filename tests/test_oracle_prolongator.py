"""CPU pins of the oracle prolongator (Algorithm 2 blocking) and its coarse operator."""
import numpy as np

import synth
from oracle import core, dense, estimator, prolongator as pr


def test_table2_dimension_arithmetic():
    """Coarse dimensions of Table 2: nagg * 2 * nv per level (32^3x64, 4^4 blocks)."""
    dims = (32, 32, 32, 64)
    nagg = int(np.prod(dims)) // 4 ** 4
    assert nagg * 2 * 24 == 393216 and nagg * 2 * 48 == 786432
    assert (nagg // 2 ** 4) * 2 * 32 == 32768 and (nagg // 2 ** 4) * 2 * 64 == 65536
    assert 12 * int(np.prod(dims)) == 25165824


def _wil(dims, block, nv, seed=3):
    rng = np.random.default_rng(seed)
    N = 12 * int(np.prod(dims))
    Y = rng.standard_normal((nv, N)) + 1j * rng.standard_normal((nv, N))
    return pr.block_orthonormalize(Y, dims, block)


def test_blocks_orthonormal_and_projector_algebra():
    dims, block, nv = (4, 2, 2, 4), (2, 2, 2, 2), 5
    W = _wil(dims, block, nv)
    for a in range(W.shape[0]):
        for c in range(2):
            assert np.allclose(W[a, c].conj() @ W[a, c].T, np.eye(nv), atol=1e-13)
    P = pr.dense_prolongator(W, dims, block)
    assert np.allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-13)  # R P = I
    PR = P @ P.conj().T
    assert np.allclose(PR @ PR, PR, atol=1e-12)  # P R idempotent
    g5 = estimator.g5_vec(P.shape[0])
    g5c = pr.coarse_g5(W.shape[0], nv)
    assert np.allclose(g5[:, None] * P, P * g5c[None, :], atol=1e-14)  # g5 W = W g5^W
    # restrict / prolong agree with the dense matrix
    rng = np.random.default_rng(0)
    y = rng.standard_normal((3, P.shape[0])) + 1j * rng.standard_normal((3, P.shape[0]))
    assert np.allclose(pr.restrict(W, y, dims, block), (P.conj().T @ y.T).T, atol=1e-12)
    cv = rng.standard_normal((2, P.shape[1])) + 0j
    assert np.allclose(pr.prolong(W, cv, dims, block), (P @ cv.T).T, atol=1e-12)


def test_single_site_aggregates_preserve_the_spectrum():
    """Blocks of one site with nv = 6 make W unitary, so W^+ A W has the spectrum of A."""
    dims, m = (2, 2, 2, 2), 0.1
    U = synth.su3_links(dims, 0.4, 5)
    A = dense.dense_operator(U, dims, m)
    W = _wil(dims, (1, 1, 1, 1), 6)
    P = pr.dense_prolongator(W, dims, (1, 1, 1, 1))
    Ac = P.conj().T @ A @ P
    ev = np.sort_complex(np.linalg.eigvals(A))
    evc = np.sort_complex(np.linalg.eigvals(Ac))
    assert np.allclose(np.sort(ev.real), np.sort(evc.real), atol=1e-10)
    assert np.allclose(np.sort(np.abs(ev)), np.sort(np.abs(evc)), atol=1e-10)


def test_coarse_g5_operator_is_hermitian():
    dims, block, nv, m = (4, 2, 2, 4), (2, 2, 2, 2), 4, -0.2
    U = synth.su3_links(dims, 0.5, 2)
    A = dense.dense_operator(U, dims, m)
    W = _wil(dims, block, nv)
    P = pr.dense_prolongator(W, dims, block)
    Hc = pr.coarse_g5(W.shape[0], nv)[:, None] * (P.conj().T @ A @ P)
    assert np.allclose(Hc, Hc.conj().T, atol=1e-12)


def test_prolongator_deflation_identity():
    """Algorithm 2 with X = W U_bar: t0 + trace(A^{-1}(I - P)) = trace(A^{-1}) exactly, and
    the fine-space quantities equal their coarse counterparts (W^+ W = I)."""
    dims, block, nv, m = (2, 2, 2, 4), (2, 2, 2, 2), 3, 0.1
    U = synth.su3_links(dims, 0.3, 4)
    A = dense.dense_operator(U, dims, m)
    Ai = np.linalg.inv(A)
    W = _wil(dims, block, nv)
    P = pr.dense_prolongator(W, dims, block)
    g5c = pr.coarse_g5(W.shape[0], nv)
    Hc = g5c[:, None] * (P.conj().T @ A @ P)
    w, Ub = np.linalg.eigh(Hc)
    idx = np.argsort(np.abs(w))[:4]
    X = (P @ Ub[:, idx]).T  # fine rows
    Uo, lam, ug5u, t0 = estimator.oblique_setup(X, (A @ X.T).T)
    assert np.allclose(np.sort(np.abs(lam)), np.sort(np.abs(w[idx])), rtol=1e-10)
    Pobl = estimator.oblique_projector_dense(A, Uo, lam)
    N = A.shape[0]
    assert abs(t0 + np.trace(Ai @ (np.eye(N) - Pobl)) - np.trace(Ai)) < 1e-10 * abs(np.trace(Ai))
    # u^+ g5 u computed on the coarse vectors equals the fine value
    uc = Ub[:, idx]
    assert np.allclose(np.sort(np.einsum("ni,n,ni->i", uc.conj(), g5c, uc).real),
                       np.sort(np.einsum("in,n,in->i", X.conj(), estimator.g5_vec(N), X).real), atol=1e-12)


def test_aggregate_geometry_free_field_coarse_stencil():
    """Pins the aggregate map itself (the other prolongator pins hold for any partition of the
    sites).  Unit links and near-null vectors constant over each block make W^+ A W a Wilson
    operator of the coarse lattice, in closed form from the operator's definition: with the
    block extents b_mu, a block couples to itself with (4 + m - sum_mu (b_mu - 1)/b_mu) 1 (the
    internal forward and backward hops cancel their gamma parts), to the next block in +mu
    with -(1 - g_mu)/(2 b_mu) and in -mu with -(1 + g_mu)/(2 b_mu) (the face carries 1/b_mu of
    the block's sites), with the antiperiodic -1 on the time hops that wrap, and to no other
    block.  Extents differ per direction, so a strided or permuted map, swapped directions
    or a wrong face weight fail it."""
    dims, block, m = (6, 9, 3, 6), (2, 3, 1, 2), 0.3
    lx, ly, lz, lt = dims
    nco = [d // b for d, b in zip(dims, block)]  # (3, 3, 3, 3)
    V = lx * ly * lz * lt
    N = 12 * V
    # 6 near-null vectors: for spin s2 in {0, 1} and colour col, 1 on spins s2 and 2 + s2
    Y = np.zeros((6, N), dtype=np.complex128)
    for s2 in range(2):
        for col in range(3):
            for sp in (s2, 2 + s2):
                Y[s2 * 3 + col, np.arange(V) * 12 + 3 * sp + col] = 1.0
    W = pr.block_orthonormalize(Y, dims, block)
    P = pr.dense_prolongator(W, dims, block)
    U = synth.unit_links(dims)
    AP = core.apply(U, dims, m, core.OP_A, P.T.copy()).T
    Ac = P.conj().T @ AP
    nagg = int(np.prod(nco))
    # closed form, coarse index (a, c, v), v = s2 * 3 + colour, spin = 2 c + s2
    G = [core.gamma(mu) for mu in range(4)]
    I4 = np.eye(4)

    def spin_block(S):
        out = np.zeros((12, 12), dtype=np.complex128)
        for c in range(2):
            for s2 in range(2):
                for cp in range(2):
                    for s2p in range(2):
                        for col in range(3):
                            out[c * 6 + s2 * 3 + col, cp * 6 + s2p * 3 + col] = S[2 * c + s2, 2 * cp + s2p]
        return out

    ref = np.zeros((nagg * 12, nagg * 12), dtype=np.complex128)
    diag = (4 + m - sum((b - 1) / b for b in block)) * I4
    for a in range(nagg):
        ac = [a % nco[0], (a // nco[0]) % nco[1], (a // (nco[0] * nco[1])) % nco[2], a // (nco[0] * nco[1] * nco[2])]
        ref[a * 12:(a + 1) * 12, a * 12:(a + 1) * 12] += spin_block(diag)
        for mu in range(4):
            for step, S in ((+1, -(I4 - G[mu]) / (2 * block[mu])), (-1, -(I4 + G[mu]) / (2 * block[mu]))):
                bc = list(ac)
                bc[mu] = (ac[mu] + step) % nco[mu]
                wraps = mu == 3 and (ac[mu] + step) % nco[mu] != ac[mu] + step
                b = bc[0] + nco[0] * (bc[1] + nco[1] * (bc[2] + nco[2] * bc[3]))
                ref[a * 12:(a + 1) * 12, b * 12:(b + 1) * 12] += spin_block(-S if wraps else S)
    assert np.max(np.abs(Ac - ref)) <= 1e-13
    # a strided map (aggregate a = sites with index = a mod nagg) is not that stencil
    site = np.arange(V).reshape(V // nagg, nagg).T
    idx = np.empty((nagg, 2, 6 * site.shape[1]), dtype=np.int64)
    for c in range(2):
        for bs in range(site.shape[1]):
            for s2 in range(2):
                for col in range(3):
                    idx[:, c, bs * 6 + s2 * 3 + col] = 12 * site[:, bs] + 3 * (2 * c + s2) + col
    Ps = np.zeros_like(P)
    for a in range(nagg):
        for c in range(2):
            for v in range(6):
                Ps[idx[a, c], (a * 2 + c) * 6 + v] = W[a, c, v]
    Acs = Ps.conj().T @ core.apply(U, dims, m, core.OP_A, Ps.T.copy()).T
    assert np.max(np.abs(Acs - ref)) > 1e-2


def _two_level(dims, block1, nv1, block2, nv2, m=0.1, seed=4):
    from oracle import core as _core
    U = synth.su3_links(dims, 0.4, seed)
    rng = np.random.default_rng(seed)
    N = 12 * int(np.prod(dims))
    W1 = pr.block_orthonormalize(rng.standard_normal((nv1, N)) + 1j * rng.standard_normal((nv1, N)), dims, block1)
    P1 = pr.dense_prolongator(W1, dims, block1)
    Dc = P1.conj().T @ _core.apply(U, dims, m, _core.OP_A, P1.T.copy()).T
    cdims = tuple(L // b for L, b in zip(dims, block1))
    idx2 = pr.coarse_fine_index(cdims, block2, nv1)
    nc1 = P1.shape[1]
    W2 = pr.block_orthonormalize(rng.standard_normal((nv2, nc1)) + 1j * rng.standard_normal((nv2, nc1)), cdims, block2,
                                 idx=idx2)
    P2 = pr.dense_prolongator(W2, cdims, block2, idx=idx2, N=nc1)
    return U, W1, P1, Dc, cdims, W2, P2


def test_second_level_blocks_orthonormal_and_chirality_split():
    """Level-2 blocks of the coarse lattice: W2^+ W2 = I per block, P2^+ P2 = I, and
    g5^{W1} P2 = P2 g5^{W2} (a block holds one chirality of the level-1 coarse entries)."""
    U, W1, P1, Dc, cdims, W2, P2 = _two_level((8, 4, 4, 4), (2, 2, 2, 2), 4, (2, 2, 2, 2), 3)
    for a in range(W2.shape[0]):
        for c in range(2):
            assert np.allclose(W2[a, c].conj() @ W2[a, c].T, np.eye(3), atol=1e-12)
    assert np.allclose(P2.conj().T @ P2, np.eye(P2.shape[1]), atol=1e-12)
    g1 = pr.coarse_g5(W1.shape[0], 4)
    g2 = pr.coarse_g5(W2.shape[0], 3)
    assert np.allclose(g1[:, None] * P2, P2 * g2[None, :], atol=0)
    # every level-1 coarse entry is covered exactly once by the level-2 index map
    idx2 = pr.coarse_fine_index(cdims, (2, 2, 2, 2), 4)
    assert np.array_equal(np.sort(idx2.ravel()), np.arange(P1.shape[1]))


def test_second_level_operator_is_a_nine_point_g5_hermitian_stencil():
    """D_cc = P2^+ D_c P2: g5^{W2} D_cc is Hermitian, and with 4 level-2 blocks along x the
    blocks two apart do not couple (D_c couples only neighbouring level-1 sites, and level-2
    blocks two apart share no level-1 neighbours); the product P1 P2 is an orthonormal
    chirality-split prolongator of the fine lattice."""
    dims, block1, nv1, block2, nv2 = (16, 4, 4, 4), (2, 2, 2, 2), 4, (2, 2, 2, 2), 3
    U, W1, P1, Dc, cdims, W2, P2 = _two_level(dims, block1, nv1, block2, nv2)
    Dcc = P2.conj().T @ Dc @ P2
    g2 = pr.coarse_g5(W2.shape[0], nv2)
    H = g2[:, None] * Dcc
    assert np.max(np.abs(H - H.conj().T)) <= 1e-12 * np.max(np.abs(H))
    nb = 2 * nv2
    assert W2.shape[0] == 4  # level-2 lattice 4 x 1 x 1 x 1
    blk = lambda a, b: Dcc[a * nb:(a + 1) * nb, b * nb:(b + 1) * nb]
    scale = np.max(np.abs(Dcc))
    for a in range(4):
        assert np.max(np.abs(blk(a, (a + 2) % 4))) <= 1e-13 * scale
        assert np.max(np.abs(blk(a, (a + 1) % 4))) > 1e-3 * scale
    P = P1 @ P2
    assert np.allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-12)
    g5 = np.tile(np.array([1.0] * 6 + [-1.0] * 6), P.shape[0] // 12)
    assert np.allclose(g5[:, None] * P, P * g2[None, :], atol=1e-14)
