"""Free field at the benchmark size: every probe sample of the GPU trace estimate on 16^3 x 32
against the oracle's exact momentum-space solve, and the estimate against the closed-form
trace (Eq. 1 on unit links, antiperiodic time)."""
import numpy as np
import pytest

import synth
from oracle import core, dense, estimator

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("path", ["f64_gmres32", "f16_sstep15"])
def test_free_field_trace_16x32_against_momentum_space(gpu, path):
    lq = gpu
    dims, m, s, seed = (16, 16, 16, 32), 0.1, 16, 1005
    N = 12 * 16 * 16 * 16 * 32
    print(f"free field 16^3x32 trace, path={path}", flush=True)
    if path == "f64_gmres32":
        xi, opts = 1e-10, dict(prec=lq.F64, restart=32)
    else:
        xi, opts = 1e-8, dict(prec=lq.F16, restart=15, sstep=1)
    c = lq.Context(dims, m)
    c.set_gauge(synth.unit_links(dims))
    r = c.trace(s, seed, xi, samples=True, maxit=20000, **opts)
    c.close()
    assert r["nfailed"] == 0
    Z = core.probes(seed, s, N)
    t_ref = estimator.hutchinson_samples(Z, dense.free_field_solve(Z, dims, m))
    # |z^T (y - y*)| <= ||z|| ||r|| / sigma_min <= N xi / sigma_min, sigma_min of the free
    # operator at the smallest antiperiodic momentum
    a = m + 1 - np.cos(np.pi / 32)
    smin = np.sqrt(a * a + np.sin(np.pi / 32) ** 2)
    assert np.max(np.abs(r["samples"].numpy() - t_ref)) <= N * xi / smin
    tr, _ = dense.free_field_closed_form(dims, m)
    assert abs(r["trace_re"] - tr) <= 4 * np.sqrt(r["var_mean"])


def _free_sigma_range(dims, m):
    """Smallest and largest singular value of the free Wilson operator with antiperiodic time:
    sigma(p) = sqrt(a(p)^2 + s(p)^2), a = m + sum(1 - cos p), s^2 = sum sin^2 p, over the
    lattice momenta (closed form, each 12-fold)."""
    lx, ly, lz, lt = dims
    ks = [2 * np.pi * np.arange(L) / L for L in (lx, ly, lz)] + [(2 * np.arange(lt) + 1) * np.pi / lt]
    P = np.meshgrid(*ks, indexing="ij")
    a = m + sum(1 - np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    sig = np.sqrt(a * a + s2)
    return sig.min(), sig.max()


@pytest.mark.parametrize("path", ["f64_gmres32", "f16_sstep15"])
def test_free_field_solutions_16x32_against_momentum_space(gpu, path):
    """Solution error at the benchmark size against an exact reference: 2 probes on unit links
    solved to xi, compared with the momentum-space solve; the error must stay within the
    bound kappa(A) xi that the residual criterion implies (kappa of the free operator in
    closed form), and the residual is recomputed with the oracle's operator."""
    lq = gpu
    dims, m, seed = (16, 16, 16, 32), 0.1, 1006
    N = 12 * 16 * 16 * 16 * 32
    print(f"free field 16^3x32 solutions, path={path}", flush=True)
    if path == "f64_gmres32":
        xi, opts = 1e-10, dict(prec=lq.F64, restart=32)
    else:
        xi, opts = 1e-8, dict(prec=lq.F16, restart=15, sstep=1)
    c = lq.Context(dims, m)
    c.set_gauge(synth.unit_links(dims))
    z = c.probes(seed, 2)
    x, st, _ = c.solve(z, xi, maxit=20000, **opts)
    c.close()
    zh, xh = z.cpu().numpy(), x.cpu().numpy()
    ref = dense.free_field_solve(zh, dims, m)
    smin, smax = _free_sigma_range(dims, m)
    err = np.linalg.norm(xh - ref, axis=1) / np.linalg.norm(ref, axis=1)
    res = np.linalg.norm(zh - core.apply(synth.unit_links(dims), dims, m, core.OP_A, xh), axis=1) / np.sqrt(N)
    print(f"kappa {smax / smin:.1f}, solution errors {err}, residuals {res}", flush=True)
    assert np.all(res <= xi * 1.05)
    assert np.all(err <= (smax / smin) * xi * 1.05)
