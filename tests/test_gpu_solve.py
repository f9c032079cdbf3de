"""GPU inexact solves A^{-1}_xi (through the C-ABI) against the oracle.

Parity criteria for a solve (true residual ||b - A x|| <= xi ||b||): the FP64 true residual
of the returned x is recomputed with the oracle's operator; on the 4^4 workload the
solution is compared with dense LU (kappa ~ 7, so rel. err <= kappa * xi); elsewhere with
the oracle's own GMRES solved to 1e-12, within kappa (xi_gpu + xi_oracle).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import core, dense

pytestmark = pytest.mark.gpu


def _true_relres(U, dims, m, b, x):
    r = b - core.apply(U, dims, m, core.OP_A, x)
    return np.linalg.norm(r, axis=-1) / np.linalg.norm(b, axis=-1)


@pytest.fixture(scope="module")
def cfg0():
    dims, m = (4, 4, 4, 4), 0.1
    U = synth.su3_links(dims, 0.3, 1)
    A = dense.dense_operator(U, dims, m)
    return dims, m, U, A


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("nrhs,batch", [(1, 0), (6, 0), (5, 2)])
def test_solve_matches_dense_lu(gpu, cfg0, prec, nrhs, batch):
    lq = gpu
    dims, m, U, A = cfg0
    print(f"solve cfg0 prec={prec} nrhs={nrhs} batch={batch}", flush=True)
    b = synth.random_spinors(dims, nrhs, 21).reshape(nrhs, -1)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    xi = 1e-10
    x, stats, rc = c.solve(torch.as_tensor(b).cuda(), xi, prec=prec, max_batch=batch)
    x = x.cpu().numpy()
    rel = _true_relres(U, dims, m, b, x)
    assert np.all(rel <= xi * 1.0000001), rel
    xe = np.linalg.solve(A, b.T).T
    err = np.linalg.norm(x - xe, axis=1) / np.linalg.norm(xe, axis=1)
    assert np.all(err <= 1e-8), err
    for s, r in zip(stats, rel):
        assert s[0] == 1 and s[1] > 0 and s[2] >= 1 and abs(s[3] - r) <= 1e-3 * r + 1e-15
    c.close()


def test_solve_probes_near_critical_vs_oracle(gpu):
    """8^3 x 16, eps = 0.5, mass close to the spectral edge: GPU FP64 and BF16-inner solves of
    Rademacher probes to 1e-8 against the oracle's GMRES at 1e-12."""
    lq = gpu
    dims, m = (8, 8, 8, 16), -1.85
    U = synth.su3_links(dims, 0.5, 1)
    N = 12 * 8 * 8 * 8 * 16
    b = core.probes(1001, 2, N).astype(np.complex128)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    xo = np.stack([core.gmres(U, dims, m, bj, 1e-12)[0] for bj in b])
    for prec in (0, 1, 3):
        print(f"near-critical solve prec={prec}", flush=True)
        x, stats, rc = c.solve(torch.as_tensor(b).cuda(), 1e-8, prec=prec)
        x = x.cpu().numpy()
        rel = _true_relres(U, dims, m, b, x)
        assert np.all(rel <= 1e-8), rel
        err = np.linalg.norm(x - xo, axis=1) / np.linalg.norm(xo, axis=1)
        # ||x - x*|| / ||x*|| <= kappa * xi; kappa of this operator is below 1e3
        assert np.all(err <= 1e3 * (1e-8 + 1e-12)), err
        # probe samples z^T y agree within ||z||^2 (xi_gpu + xi_orc) / sigma_min
        t_gpu = np.einsum("jn,jn->j", b, x)
        t_orc = np.einsum("jn,jn->j", b, xo)
        assert np.all(np.abs(t_gpu - t_orc) <= N * 1e-8 / 0.01)
    c.close()


def test_solve_error_paths(gpu, cfg0):
    lq = gpu
    dims, m, U, A = cfg0
    c = lq.Context(dims, m)
    c.set_gauge(U)
    b = synth.random_spinors(dims, 2, 1).reshape(2, -1)
    x, stats, rc = c.solve(torch.as_tensor(b).cuda(), 1e-12, raise_on_fail=False, maxit=3, restart=2)
    assert rc == lq.lqtrace.LQT_ENOTCONV
    assert all(s[0] == 0 for s in stats) and all(s[1] >= 3 for s in stats)
    assert all(np.isfinite(s[3]) and s[3] < 1 for s in stats)
    bad = b.copy()
    bad[1, 17] = np.nan
    with pytest.raises(lq.LqtError) as e:
        c.solve(torch.as_tensor(bad).cuda(), 1e-8)
    assert e.value.code == -7
    with pytest.raises(lq.LqtError) as e:
        c.solve(torch.as_tensor(b).cuda(), 1e-8, restart=100)
    assert e.value.code == -1
    # empty input is a no-op
    x, stats, rc = c.solve(torch.zeros((0, 12 * 256), dtype=torch.complex128, device="cuda"), 1e-8)
    assert rc == 0 and stats == []
    # zero right-hand side: x = 0, converged
    x, stats, rc = c.solve(torch.zeros((1, 12 * 256), dtype=torch.complex128, device="cuda"), 1e-8)
    assert rc == 0 and torch.count_nonzero(x) == 0
    c.close()
