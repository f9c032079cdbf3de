"""Pins of the CPU oracle against facts the paper and the mathematics fix (no GPU).

Each test targets a plausible mistake: a wrong gamma matrix or sign (Clifford algebra,
free-field Fourier spectrum), a swapped hop direction or missing dagger (gauge
covariance, pure gauge, adjoint), a wrong boundary phase (antiperiodic momenta), a broken
solver (dense LU), a wrong estimator or variance formula (exact dense statistics).
"""
import os

import numpy as np
import pytest

import synth
from oracle import core, dense, estimator

HERE = os.path.dirname(os.path.abspath(__file__))


def g5diag(N):
    return np.tile([1.0] * 6 + [-1.0] * 6, N // 12)


# ---------------------------------------------------------------- gamma matrices
def test_gamma_clifford_algebra():
    g = [core.gamma(mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2 * np.eye(4) * (mu == nu))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    # DeGrand-Rossi: gamma_2, gamma_4 real symmetric; gamma_1, gamma_3 imaginary antisymmetric
    assert np.allclose(g[1], g[1].T) and np.allclose(g[3], g[3].T)
    assert np.allclose(g[0], -g[0].T) and np.allclose(g[2], -g[2].T)


# ---------------------------------------------------------------- free field
@pytest.mark.parametrize("dims,antiperiodic", [((4, 4, 4, 4), True), ((2, 2, 2, 4), True), ((2, 2, 2, 4), False),
                                               ((2, 4, 2, 2), False)])
def test_free_field_trace_closed_form(dims, antiperiodic):
    m = 0.1
    A = dense.dense_operator(synth.unit_links(dims), dims, m, antiperiodic=antiperiodic)
    Ai = np.linalg.inv(A)
    tr, fro = dense.free_field_closed_form(dims, m, antiperiodic)
    assert abs(np.trace(Ai) - tr) < 1e-10 * abs(tr)
    assert abs(np.linalg.norm(Ai) ** 2 - fro) < 1e-10 * fro
    # translation invariance: every diagonal element equals trace / N
    assert np.allclose(np.diag(Ai), tr / A.shape[0], atol=1e-12)


def test_free_field_singular_values():
    dims, m = (2, 2, 2, 4), -0.3
    A = dense.dense_operator(synth.unit_links(dims), dims, m)
    sv = np.sort(np.linalg.svd(A, compute_uv=False))
    lx, ly, lz, lt = dims
    expect = []
    for nx in range(lx):
        for ny in range(ly):
            for nz in range(lz):
                for nt in range(lt):
                    p = [2 * np.pi * nx / lx, 2 * np.pi * ny / ly, 2 * np.pi * nz / lz, (2 * nt + 1) * np.pi / lt]
                    a = m + sum(1 - np.cos(q) for q in p)
                    s2 = sum(np.sin(q) ** 2 for q in p)
                    expect += [np.sqrt(a * a + s2)] * 12
    assert np.allclose(sv, np.sort(expect), atol=1e-12)


def test_plane_wave_action_any_size():
    """A e^{ipx} u = (m + sum(1-cos p) + i sum gamma_mu sin p_mu) e^{ipx} u on 4^3 x 8."""
    dims, m = (4, 4, 4, 8), 0.05
    rng = np.random.default_rng(3)
    n = [1, 3, 2, 5]
    p = [2 * np.pi * n[0] / 4, 2 * np.pi * n[1] / 4, 2 * np.pi * n[2] / 4, (2 * n[3] + 1) * np.pi / 8]
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = synth.plane_wave(dims, p, u).reshape(1, -1)
    out = core.apply(synth.unit_links(dims), dims, m, core.OP_A, psi)
    Ap = (m + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(core.gamma(mu) * np.sin(p[mu]) for mu in range(4))
    expect = synth.plane_wave(dims, p, Ap @ u).reshape(1, -1)
    assert np.max(np.abs(out - expect)) < 1e-13


# ---------------------------------------------------------------- gauge field structure
def test_links_special_unitary():
    U = synth.su3_links((4, 4, 4, 4), 0.5, 1).reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.max(np.abs(np.conj(np.swapaxes(U, 1, 2)) @ U - eye)) < 1e-13
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-13


def test_adjoint_and_g5_hermiticity():
    dims = (2, 2, 2, 4)
    U = synth.su3_links(dims, 0.5, 2)
    A = dense.dense_operator(U, dims, 0.1)
    Ad = dense.dense_operator(U, dims, 0.1, op=core.OP_ADAG)
    g5 = np.diag(g5diag(A.shape[0]))
    assert np.max(np.abs(Ad - A.conj().T)) < 1e-14
    assert np.max(np.abs(g5 @ A @ g5 - A.conj().T)) < 1e-14
    Ag5 = dense.dense_operator(U, dims, 0.1, op=core.OP_AG5)
    assert np.max(np.abs(Ag5 - Ag5.conj().T)) < 1e-14
    g5A = dense.dense_operator(U, dims, 0.1, op=core.OP_G5A)
    assert np.max(np.abs(g5A - g5 @ A)) < 1e-14


def test_gauge_covariance():
    dims = (4, 4, 2, 4)
    U = synth.su3_links(dims, 0.5, 3)
    omega = synth.random_su3((4, 2, 4, 4), seed=11)
    Ug = synth.gauge_transform(U, omega)
    psi = synth.random_spinors(dims, 2, 5)
    lhs = core.apply(Ug, dims, 0.2, core.OP_A, synth.transform_spinor(psi, omega).reshape(2, -1))
    rhs = synth.transform_spinor(core.apply(U, dims, 0.2, core.OP_A, psi.reshape(2, -1)).reshape(psi.shape), omega)
    assert np.max(np.abs(lhs - rhs.reshape(2, -1))) < 1e-12


def test_pure_gauge_reproduces_free_trace():
    dims, m = (2, 2, 2, 4), 0.1
    Upg, _ = synth.pure_gauge_links(dims, seed=4)
    assert np.max(np.abs(Upg - synth.unit_links(dims))) > 0.1
    A = dense.dense_operator(Upg, dims, m)
    tr, fro = dense.free_field_closed_form(dims, m)
    Ai = np.linalg.inv(A)
    assert abs(np.trace(Ai) - tr) < 1e-10 * abs(tr)
    assert abs(np.linalg.norm(Ai) ** 2 - fro) < 1e-10 * fro


# ---------------------------------------------------------------- solver
def test_gmres_matches_dense_lu():
    dims = (4, 4, 4, 4)
    U = synth.su3_links(dims, 0.3, 1)
    A = dense.dense_operator(U, dims, 0.1)
    b = synth.random_spinors(dims, 1, 9).reshape(-1)
    x, conv, its, rel = core.gmres(U, dims, 0.1, b, 1e-10)
    assert conv and rel <= 1e-10
    xe = np.linalg.solve(A, b)
    # kappa of this operator is about 7 (checked by SVD in the free-field and estimator tests)
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) <= 1e-8


def test_gmres_true_residual_and_maxit():
    dims = (2, 2, 2, 4)
    U = synth.su3_links(dims, 0.5, 2)
    b = synth.random_spinors(dims, 1, 1).reshape(-1)
    x, conv, its, rel = core.gmres(U, dims, -0.5, b, 1e-12, m=8, maxit=3)
    assert not conv and its == 3
    r = b - core.apply(U, dims, -0.5, core.OP_A, x)
    assert abs(np.linalg.norm(r) / np.linalg.norm(b) - rel) < 1e-12



def test_gmres_solves_a_plane_wave_in_closed_form():
    """Free field on 8^3 x 16 (N = 98304, beyond dense LU): b = e^{ipx} u has the solution
    e^{ipx} A(p)^{-1} u with A(p) = m + sum(1 - cos p) + i sum gamma_mu sin p_mu, for A and,
    with the transposed-conjugate symbol, for A^+."""
    dims, m = (8, 8, 8, 16), 0.2
    n = [1, 2, 7, 3]
    p = [2 * np.pi * n[0] / 8, 2 * np.pi * n[1] / 8, 2 * np.pi * n[2] / 8, (2 * n[3] + 1) * np.pi / 16]
    u = np.random.default_rng(4).standard_normal((4, 3)) + 1j * np.random.default_rng(5).standard_normal((4, 3))
    Ap = (m + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(core.gamma(mu) * np.sin(p[mu]) for mu in range(4))
    b = synth.plane_wave(dims, p, u).reshape(-1)
    for op, sym in ((core.OP_A, Ap), (core.OP_ADAG, Ap.conj().T)):
        x, conv, its, rel = core.gmres(synth.unit_links(dims), dims, m, b, 1e-11, m=16, op=op)
        assert conv and rel <= 1e-11
        xe = synth.plane_wave(dims, p, np.linalg.solve(sym, u)).reshape(-1)
        assert np.linalg.norm(x - xe) / np.linalg.norm(xe) <= 1e-9


# ---------------------------------------------------------------- probes
def test_splitmix64_known_answers():
    vals = [int(l) for l in open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt")) if l.strip()[:1].isdigit()]
    golden = 0x9E3779B97F4A7C15
    got = [core.splitmix64((1234567 + k * golden) % 2**64) for k in range(5)]
    assert got == vals


def test_probes_are_rademacher():
    Z = core.probes(1001, 8, 12 * 4096)
    assert set(np.unique(Z)) == {-1.0, 1.0}
    assert abs(Z.mean()) < 4 / np.sqrt(Z.size)
    G = Z @ Z.T / Z.shape[1]
    assert np.max(np.abs(G - np.eye(8))) < 5 / np.sqrt(Z.shape[1])
    # probe j, entry i is a pure function of (seed, j, i)
    assert np.array_equal(core.probes(1001, 3, 12 * 4096, j0=5), Z[5:8])


# ---------------------------------------------------------------- estimator
@pytest.fixture(scope="module")
def tiny():
    dims = (2, 2, 2, 2)
    U = synth.su3_links(dims, 0.3, 1)
    A = dense.dense_operator(U, dims, 0.1)
    return dims, U, A, np.linalg.inv(A)


def test_printed_variance_is_bound_and_exact_form_matches_statistics(tiny):
    dims, U, A, Ai = tiny
    v = estimator.exact_variances(Ai)
    assert v["exact"] <= v["printed"] + 1e-12
    Z = core.probes(7, 20000, A.shape[0])
    t = np.einsum("jn,jn->j", Z, (Ai @ Z.T).T)
    assert abs(t.mean() - np.trace(Ai)) < 5 * np.sqrt(v["exact"] / len(t))
    emp = np.mean(np.abs(t - np.trace(Ai)) ** 2)
    # chi-square band for 20000 samples
    assert abs(emp / v["exact"] - 1) < 0.06
    emp_re = np.mean((t.real - np.trace(Ai).real) ** 2)
    assert abs(emp_re / v["re"] - 1) < 0.06


def test_oblique_identity_for_any_basis(tiny):
    """t0 + trace(A^{-1}(I-P)) = trace(A^{-1}) for any X (Section 2.1, K = g5)."""
    dims, U, A, Ai = tiny
    N = A.shape[0]
    rng = np.random.default_rng(5)
    X = rng.standard_normal((10, N)) + 1j * rng.standard_normal((10, N))
    Ub, lam, ug5u, t0 = estimator.oblique_setup(X, (A @ X.T).T)
    P = estimator.oblique_projector_dense(A, Ub, lam)
    assert np.max(np.abs(P @ P - P)) < 1e-10 * np.max(np.abs(P))
    assert abs(t0 + np.trace(Ai @ (np.eye(N) - P)) - np.trace(Ai)) < 1e-10 * abs(np.trace(Ai))
    # deflated operator stays g5-Hermitian: g5 (A^{-1}(I-P)) g5 = (A^{-1}(I-P))^+
    g5 = np.diag(g5diag(N))
    D = Ai @ (np.eye(N) - P)
    assert np.max(np.abs(g5 @ D @ g5 - D.conj().T)) < 1e-10 * np.max(np.abs(D))
    # the per-probe correction is z^T A^{-1} P z
    Z = core.probes(3, 4, N)
    c = estimator.oblique_corrections(Z, Ub, lam)
    assert np.allclose(c, np.einsum("jn,jn->j", Z, (Ai @ P @ Z.T).T), atol=1e-10)


def test_oblique_equals_orthogonal_for_exact_eigenvectors(tiny):
    """With X = g5 Q for exact eigenvectors Q of A g5, the oblique P equals Q Q^+."""
    dims, U, A, Ai = tiny
    N = A.shape[0]
    g5 = g5diag(N)
    w, Q = np.linalg.eigh((A * g5[None, :]))  # A g5 (columns scaled)
    idx = np.argsort(np.abs(w))[:6]
    Qk = Q[:, idx].T  # rows
    Ub, lam, ug5u, t0 = estimator.oblique_setup(g5 * Qk, (A @ (g5 * Qk).T).T)
    P = estimator.oblique_projector_dense(A, Ub, lam)
    assert np.max(np.abs(P - Qk.T @ Qk.conj())) < 1e-10
    assert np.allclose(np.sort(np.abs(lam)), np.sort(np.abs(w[idx])), atol=1e-12)


def test_rank_curve_endpoints(tiny):
    dims, U, A, Ai = tiny
    N = A.shape[0]
    rng = np.random.default_rng(1)
    X = rng.standard_normal((4, N)) + 1j * rng.standard_normal((4, N))
    Ub, lam, ug5u, t0 = estimator.oblique_setup(X, (A @ X.T).T)
    Z = core.probes(11, 16, N)
    Y = (Ai @ Z.T).T
    curve = estimator.rank_curve(Z, Y, Ub, lam, ug5u)
    r0 = estimator.summarize(estimator.hutchinson_samples(Z, Y))
    assert np.isclose(curve[0, 0], r0["estimate"].real) and np.isclose(curve[0, 1], r0["var_sample"])
    rk = estimator.summarize(estimator.hutchinson_samples(Z, Y) - estimator.oblique_corrections(Z, Ub, lam), t0)
    assert np.isclose(curve[-1, 0], rk["estimate"].real)


def test_jackknife_of_mean_equals_standard_error():
    t = np.random.default_rng(0).standard_normal(50) + 0j
    r = estimator.summarize(t)
    assert np.isclose(r["jackknife_err"], np.sqrt(r["var_sample"] / 50))


# ---------------------------------------------------------------- exact statistics by enumeration
def _every_sign_vector(n):
    """All 2^n real +-1 vectors of length n, one per row."""
    bits = (np.arange(2 ** n)[:, None] >> np.arange(n)[None, :]) & 1
    return 1.0 - 2.0 * bits


def test_hutchinson_mean_and_variance_over_every_probe():
    """Eq. (1) is unbiased and its one-probe variance is the symmetrised form of Eq. (2):
    averaging over all 4096 sign vectors of length 12 gives both exactly (no sampling)."""
    rng = np.random.default_rng(21)
    B = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
    Z = _every_sign_vector(12)
    t = estimator.hutchinson_samples(Z, (B @ Z.T).T)
    assert abs(t.mean() - np.trace(B)) < 1e-12 * np.abs(B).sum()
    v = estimator.exact_variances(B)
    assert np.isclose(np.mean(np.abs(t - np.trace(B)) ** 2), v["exact"], rtol=1e-12)
    assert np.isclose(np.mean((t.real - np.trace(B).real) ** 2), v["re"], rtol=1e-12)
    # a non-symmetric B: Eq. (2) as printed overstates the variance of real probes
    assert v["printed"] > 1.05 * v["exact"]
    # for a complex-symmetric B the printed form is exact
    Bs = B + B.T
    vs = estimator.exact_variances(Bs)
    assert np.isclose(vs["printed"], vs["exact"], rtol=1e-12)


def test_deflated_estimator_over_every_probe():
    """Section 2.1 with K = g5 on a g5-Hermitian 12 x 12 operator (one lattice site): over all
    sign vectors the corrected samples average to trace(A^{-1}) - t0, and their variance is the
    exact variance of A^{-1}(I - P).  A sign error or a missing Lambda^{-1} in the per-probe
    correction breaks the first; a wrong projector breaks the second."""
    rng = np.random.default_rng(22)
    g5 = g5diag(12)
    H = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
    H = H + H.conj().T + 0.3 * np.eye(12)
    A = g5[:, None] * H  # g5 A = H is Hermitian
    Ai = np.linalg.inv(A)
    X = rng.standard_normal((3, 12)) + 1j * rng.standard_normal((3, 12))
    Ub, lam, ug5u, t0 = estimator.oblique_setup(X, (A @ X.T).T)
    Z = _every_sign_vector(12)
    t = estimator.hutchinson_samples(Z, (Ai @ Z.T).T) - estimator.oblique_corrections(Z, Ub, lam)
    assert abs(t0 + t.mean() - np.trace(Ai)) < 1e-11 * np.abs(Ai).sum()
    D = Ai @ (np.eye(12) - estimator.oblique_projector_dense(A, Ub, lam))
    assert np.isclose(np.mean(np.abs(t - np.trace(D)) ** 2), estimator.exact_variances(D)["exact"], rtol=1e-10)
    # every prefix of the basis gives an unbiased estimator too (the rank curve of Section 2.2)
    base = estimator.hutchinson_samples(Z, (Ai @ Z.T).T)
    for kk in range(4):
        c = estimator.oblique_corrections(Z, Ub, lam, kk) if kk else 0.0
        assert abs(np.sum(ug5u[:kk] / lam[:kk]) + np.mean(base - c) - np.trace(Ai)) < 1e-11 * np.abs(Ai).sum()


def test_mass_tuner_finds_the_free_field_spectral_edge():
    """Unit links, m = 0, 2^3 x 4 with antiperiodic time: the leftmost eigenvalues of A are
    sum_mu (1 - cos p_mu) +- i |sin p| at p = (0, 0, 0, +-pi/4)."""
    from oracle import tune_mass

    dims = (2, 2, 2, 4)
    w = tune_mass.leftmost_eigenvalues(synth.unit_links(dims), dims, k=6)
    assert np.allclose(w.real, 1 - np.cos(np.pi / 4), atol=1e-6)
    assert np.allclose(np.abs(w.imag), np.sin(np.pi / 4), atol=1e-6)


def test_small_pipeline_estimates_bracket_the_exact_trace(capsys):
    """The 4^4 oracle pipeline (64 probes, k = 16 exact A g5 eigenvectors): both estimates lie
    within 4 jackknife errors of the exact trace, and the exact variance falls with the rank."""
    import json

    from oracle import pipeline_small

    pipeline_small.main([])
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    exact = out["trace_exact"][0]
    for key in ("estimate_undeflated", "estimate_deflated"):
        assert abs(out[key]["trace"] - exact) <= 4 * out[key]["jackknife_err"], key
    v = [out["var_exact_by_rank"][r] for r in ("0", "16", "64", "256", "1024")]
    assert all(a > b for a, b in zip(v, v[1:]))
    assert out["var_exact_by_rank"]["16"] == out["var_exact_deflated"]


def test_free_field_solve_by_fft():
    """The momentum-space solve of the free operator: it matches the oracle's GMRES on 4^3 x 8
    (periodic and antiperiodic), the oracle operator maps it back to the right-hand side at
    8^3 x 16, and the mean of its Rademacher samples is the closed-form trace."""
    for anti in (True, False):
        dims, m = (4, 4, 4, 8), 0.3
        z = synth.random_spinors(dims, 2, 4).reshape(2, -1)
        y = dense.free_field_solve(z, dims, m, antiperiodic=anti)
        for j in range(2):
            x, conv, its, rel = core.gmres(synth.unit_links(dims), dims, m, z[j], 1e-12, antiperiodic=anti)
            assert conv and np.linalg.norm(y[j] - x) <= 1e-10 * np.linalg.norm(x)
    dims, m = (8, 8, 8, 16), 0.1
    z = synth.random_spinors(dims, 1, 5).reshape(-1)
    y = dense.free_field_solve(z, dims, m)
    r = z - core.apply(synth.unit_links(dims), dims, m, core.OP_A, y)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(z)
    # every sample z^T A^{-1} z averages to the trace over all probes; with 12 V entries per
    # probe, 200 probes put the mean within a few standard errors of it
    dims = (4, 4, 4, 8)
    N = 12 * 512
    Z = core.probes(77, 200, N)
    t = estimator.hutchinson_samples(Z, dense.free_field_solve(Z, dims, 0.1))
    tr, _ = dense.free_field_closed_form(dims, 0.1)
    assert abs(t.mean().real - tr) <= 4 * np.sqrt(np.var(t.real) / len(t))
