"""Pins of the oracle's Truncated Solver Method combination (Section 1): the correction removes
the bias of a perturbed solver in expectation, vanishes when both solves agree, and the
reported error is the standard error of the two independent means."""
import numpy as np

import synth
from oracle import core, dense, estimator


def test_equal_solves_leave_the_plain_estimate():
    rng = np.random.default_rng(1)
    t = rng.standard_normal(20) + 1j * rng.standard_normal(20)
    c = rng.standard_normal(5) + 0j
    r = estimator.tsm_combine(t, 2.0, c, c)
    plain = estimator.summarize(t, 2.0)
    assert r["estimate"] == plain["estimate"] and r["corr_mean"] == 0
    assert np.isclose(r["err"], np.sqrt(plain["var_mean"]))


def test_correction_removes_a_solver_bias():
    """A 'loose solver' y = (A^{-1} + E) z with a fixed E of large trace biases the plain
    estimate by tr E; with exact tight solves on independent probes the corrected estimate is
    unbiased: over 200 repetitions its mean is within 4 standard errors of tr A^{-1}, and the
    spread of the repetitions matches the reported error."""
    dims, m = (2, 2, 2, 2), 0.2
    U = synth.su3_links(dims, 0.4, 1)
    A = dense.dense_operator(U, dims, m)
    Ai = np.linalg.inv(A)
    N = A.shape[0]
    rng = np.random.default_rng(2)
    E = 0.05 * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(N) + 0.2 * np.eye(N)
    L = Ai + E
    tr = np.trace(Ai)
    s, nc, reps = 32, 16, 200
    ests, errs, plain = [], [], []
    for r in range(reps):
        Z = core.probes(5000 + r, s, N)
        Zc = core.probes(9000 + r, nc, N)
        t_main = np.einsum("jn,jn->j", Z, Z @ L.T)
        cl = np.einsum("jn,jn->j", Zc, Zc @ L.T)
        ct = np.einsum("jn,jn->j", Zc, Zc @ Ai.T)
        o = estimator.tsm_combine(t_main, 0.0, cl, ct)
        ests.append(o["estimate"])
        errs.append(o["err"])
        plain.append(t_main.mean())
    ests = np.array(ests)
    sem = np.std(ests) / np.sqrt(reps)
    assert abs(ests.mean() - tr) <= 4 * sem
    assert abs(np.mean(plain) - tr - np.trace(E)) <= 4 * np.std(plain) / np.sqrt(reps)
    assert abs(np.mean(plain) - tr) > 20 * sem  # the bias is real
    assert 0.8 <= np.std(ests) / np.sqrt(np.mean(np.square(errs))) <= 1.25
