"""The trace with the partition basis H (spin-colour dilution and hierarchical probing, Section
1; lqt_trace_probing) against the oracle on 4^4: per-draw samples with and without deflation
(fine basis and prolongator basis, oblique projector; orthogonal projector of Algorithm 1),
t0 and the rank curve, the exact trace from one draw when the probing separates every site,
and the argument checks."""
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
    """Error of one draw's sample from solves to xi: (1/hp) sum_v ||v||^2 kappa xi ||A^-1||
    with sum_v ||v||^2 = hp N."""
    return A.shape[0] * np.linalg.cond(A) * xi * np.linalg.norm(Ai, 2)


def _draw_terms(Ai, seed, s, hp, dilute, Uo=None, lam=None, Qm=None):
    """Oracle per draw: the undeflated sample (1/hp) sum_v v^T B v (B = A^-1, or A^-1 (1 - Q Q^+)
    with Qm) and the oblique per-mode terms (1/hp) sum_v (v^T u_i)(u_i^+ g5 v) / lambda_i."""
    base, terms = [], []
    for j in range(s):
        Vj = probing.partition_vectors(seed, j, DIMS, hp, dilute)
        R = Vj if Qm is None else Vj - (Qm @ (Qm.conj().T @ Vj.T)).T
        base.append(np.einsum("pn,pn->", Vj, R @ Ai.T) / hp)
        if Uo is not None:
            terms.append(estimator.oblique_correction_terms(Vj, Uo, lam).sum(axis=0) / hp)
    return np.array(base), (np.array(terms) if terms else None)


@pytest.mark.parametrize("hp,dilute", [(1, True), (2, False), (2, True), (16, True), (32, False)])
def test_partitioned_samples_match_oracle(gpu, op, hp, dilute):
    lq = gpu
    U, A, Ai = op
    s, seed, xi = 3, 1020, 1e-10
    print(f"partition probes hp={hp} dilute={dilute}", flush=True)
    c = lq.Context(DIMS, M)
    c.set_gauge(U)
    r = c.trace(s, seed, xi, samples=True, hp_vectors=hp, dilute=dilute)
    c.close()
    assert r["nsolves"] == s * hp * (12 if dilute else 1) and r["nfailed"] == 0
    ref = probing.estimator_samples(lambda X: X @ Ai.T, seed, s, DIMS, hp, dilute)
    assert np.max(np.abs(r["samples"].numpy() - ref)) <= _bound(A, Ai, xi)


def test_probing_every_site_with_dilution_gives_the_trace(gpu, op):
    """256 probing vectors on 4^4 separate every site, so with dilution one draw (N = 3072
    solves) returns tr A^{-1} up to the solve tolerance."""
    lq = gpu
    U, A, Ai = op
    c = lq.Context(DIMS, M)
    c.set_gauge(U)
    r = c.trace(1, 1021, 1e-10, hp_vectors=256, dilute=True)
    c.close()
    assert r["nsolves"] == 3072 and r["nfailed"] == 0
    assert abs(complex(r["trace_re"], r["trace_im"]) - np.trace(Ai)) <= _bound(A, Ai, 1e-10)


def _fine_basis(A, k):
    g5 = estimator.g5_vec(A.shape[0])
    w, Q = np.linalg.eigh(A * g5[None, :])
    idx = np.argsort(np.abs(w))[:k]
    return Q[:, idx].T.copy()


def _mg_basis(U, A):
    block, nv = (2, 2, 2, 2), 6
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((nv, A.shape[0])) + 1j * rng.standard_normal((nv, A.shape[0]))
    W = pr.block_orthonormalize(Y, DIMS, block)
    P = pr.dense_prolongator(W, DIMS, block)
    Hc = pr.coarse_g5(W.shape[0], nv)[:, None] * (P.conj().T @ A @ P)
    w, Ub = np.linalg.eigh(Hc)
    Ubar = Ub[:, np.argsort(np.abs(w))[:10]].T.copy()
    return block, nv, W, Ubar, (P @ Ubar.T).T


@pytest.mark.parametrize("kind", ["fine", "prolongator"])
@pytest.mark.parametrize("hp,dilute", [(2, True), (16, False)])
def test_deflated_partitioned_trace_matches_oracle(gpu, op, kind, hp, dilute):
    lq = gpu
    U, A, Ai = op
    s, seed, xi = 3, 1022, 1e-10
    print(f"deflated partition probes basis={kind} hp={hp} dilute={dilute}", flush=True)
    c = lq.Context(DIMS, M)
    c.set_gauge(U)
    if kind == "fine":
        X = _fine_basis(A, 8)
        B = c.basis_from_vectors(torch.as_tensor(X).cuda())
    else:
        block, nv, W, Ubar, X = _mg_basis(U, A)
        B = c.basis_prolongator_from(block, nv, torch.as_tensor(W.reshape(-1)).cuda(), torch.as_tensor(Ubar).cuda())
    r = c.trace(s, seed, xi, basis=B, samples=True, rank_curve=True, hp_vectors=hp, dilute=dilute)
    B.close()
    c.close()
    Uo, lam, ug5u, t0 = estimator.oblique_setup(X, (A @ X.T).T)
    base, terms = _draw_terms(Ai, seed, s, hp, dilute, Uo, lam)
    assert abs(complex(r["t0_re"], r["t0_im"]) - t0) <= 1e-9 * abs(t0)
    ref = base - terms.sum(axis=1)
    assert np.max(np.abs(r["samples"].numpy() - ref)) <= _bound(A, Ai, xi)
    curve = r["rank_curve"].numpy()
    cum = np.concatenate([np.zeros((s, 1)), np.cumsum(terms, axis=1)], axis=1)
    t0k = np.concatenate([[0.0], np.cumsum(ug5u / lam)])
    for kk in range(len(lam) + 1):
        ref_k = estimator.summarize(base - cum[:, kk], t0k[kk])
        assert abs(curve[kk, 0] - ref_k["estimate"].real) <= 1e-6 * abs(ref_k["estimate"]) + _bound(A, Ai, xi)


def test_orthogonal_partitioned_trace_matches_oracle(gpu, op):
    """Algorithm 1 with the partition basis: the solves act on (1 - Q Q^+) v and the sample
    pairs them with the unprojected v; t0 = tr Q^+ A^{-1} Q from k extra solves."""
    lq = gpu
    U, A, Ai = op
    s, seed, xi, hp = 2, 1023, 1e-10, 2
    c = lq.Context(DIMS, M)
    c.set_gauge(U)
    B = c.basis_eig(8, xi=1e-2, require_converged=True)
    g5 = estimator.g5_vec(A.shape[0])
    Qm = (g5[None, :] * B.vectors().cpu().numpy()).T  # N x k, orthonormal columns
    r = c.trace(s, seed, xi, basis=B, projector=lq.ORTH, samples=True, hp_vectors=hp, dilute=True)
    B.close()
    c.close()
    assert np.allclose(Qm.conj().T @ Qm, np.eye(8), atol=1e-10)
    base, _ = _draw_terms(Ai, seed, s, hp, True, Qm=Qm)
    assert np.max(np.abs(r["samples"].numpy() - base)) <= _bound(A, Ai, xi)
    t0 = np.trace(Qm.conj().T @ Ai @ Qm)
    assert abs(complex(r["t0_re"], r["t0_im"]) - t0) <= 8 * np.linalg.cond(A) * xi * np.linalg.norm(Ai, 2)


def test_probing_argument_checks(gpu, op):
    lq = gpu
    U, A, Ai = op
    c = lq.Context(DIMS, M)
    c.set_gauge(U)
    for hp in (0, 3, 12):
        with pytest.raises(lq.LqtError):
            c.trace(1, 1, 1e-8, hp_vectors=hp)
    with pytest.raises(lq.LqtError):
        c.trace(1, 1, 1e-8, hp_vectors=512)  # level 2 needs extents divisible by 8
    c.close()
    c = lq.Context((4, 4, 4, 6), M)
    c.set_gauge(synth.su3_links((4, 4, 4, 6), 0.3, 1))
    with pytest.raises(lq.LqtError):
        c.trace(1, 1, 1e-8, hp_vectors=32)  # level 1 needs extents divisible by 4
    r = c.trace(1, 1, 1e-8, hp_vectors=16, dilute=True)
    assert r["nsolves"] == 192
    c.close()


@pytest.mark.parametrize("dims,hp,dilute,p0,nvec", [((16, 16, 16, 32), 16, True, 190, 5),
                                                     ((16, 16, 16, 32), 256, False, 1000, 3),
                                                     ((32, 32, 32, 64), 32, True, 7, 3)])
def test_partition_probes_bit_exact_at_full_size(gpu, dims, hp, dilute, p0, nvec):
    """The device generator of the partition vectors against the oracle's vectors of the same
    draws, bit for bit, at the benchmark lattices (levels 1 and 2 of the nested colourings, a
    range that straddles two draws)."""
    lq = gpu
    print(f"partition probes dims={dims} hp={hp} dilute={dilute}", flush=True)
    c = lq.Context(dims, 0.1)
    seed = 1050
    got = c.partition_probes(seed, nvec, hp, dilute, p0=p0).cpu().numpy()
    c.close()
    nd = 12 if dilute else 1
    q = hp * nd
    for f in range(nvec):
        j, r = divmod(p0 + f, q)
        m, cc = divmod(r, nd)
        # row r of probing.partition_vectors(seed, j, dims, hp, dilute), built alone
        ref = np.repeat(probing.hp_sign(dims, m), 12) * core.probes(seed, 1, got.shape[1], j0=j)[0]
        if dilute:
            ref = np.where(np.arange(got.shape[1]) % 12 == cc, ref, 0.0)
        assert np.array_equal(got[f].real, ref) and not np.any(got[f].imag)


def test_partitioned_trace_at_the_benchmark_size(gpu):
    """16^3x32 at the headline operator, FP16 s-step GMRES(15): one draw of red-black probing
    with dilution (24 solves).  The draw's sample equals (1/2) sum_v v^T y_v over the library's
    own solutions of the same vectors (same batch, bitwise-identical solves), the oracle
    recomputes every solution's FP64 residual (<= xi) and forms the dot products itself."""
    from paper_1909_12234_amd.workloads import PREC, WORKLOADS

    lq = gpu
    w = WORKLOADS["wilson16x32_mixed"]
    dims, m, xi = w["dims"], w["mass"], w["xi"]
    prec = PREC[w["inner_prec"]]
    print("partition trace at 16^3x32", flush=True)
    U = synth.su3_links(dims, w["eps"], w["seed"])
    c = lq.Context(dims, m)
    c.set_gauge(U)
    c.tune(prec, 24)
    seed, hp = 1070, 2
    r = c.trace(1, seed, xi, samples=True, hp_vectors=hp, dilute=True, prec=prec, restart=w["restart"],
                sstep=w["sstep"])
    V = c.partition_probes(seed, 24, hp, True)
    y, st, _ = c.solve(V, xi, prec=prec, restart=w["restart"], sstep=w["sstep"])
    c.close()
    assert r["nfailed"] == 0 and all(s[0] for s in st)
    Vh, yh = V.cpu().numpy(), y.cpu().numpy()
    res = Vh - core.apply(U, dims, m, core.OP_A, yh)
    assert np.max(np.linalg.norm(res, axis=1) / np.linalg.norm(Vh, axis=1)) <= xi * 1.05
    t = np.sum(Vh.real * yh, axis=1).sum() / hp
    assert abs(r["samples"].numpy()[0] - t) <= 1e-9 * abs(t)
