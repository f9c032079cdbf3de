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
