"""Edge case of the estimator: a single probe.  Its one-probe variance and jackknife error are
0 (no spread to estimate), and the estimate is the probe's own sample z^T A^{-1} z."""
import numpy as np
import pytest

import synth
from oracle import core, dense

pytestmark = pytest.mark.gpu


def test_single_probe_trace(gpu):
    lq = gpu
    dims, m, xi, seed = (4, 4, 4, 4), 0.1, 1e-10, 1000
    print("single-probe trace on 4^4", flush=True)
    U = synth.su3_links(dims, 0.3, 1)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    r = c.trace(1, seed, xi, samples=True)
    c.close()
    A = dense.dense_operator(U, dims, m)
    z = core.probes(seed, 1, A.shape[0])[0]
    t = z @ np.linalg.solve(A, z)
    assert r["nsolves"] == 1 and r["nfailed"] == 0
    assert r["var_sample"] == 0.0 and r["jackknife_err"] == 0.0 and r["var_mean"] == 0.0
    s = r["samples"].numpy()[0]
    assert r["trace_re"] == s.real
    # |z^T (y - y*)| <= N xi / sigma_min, sigma_min of this operator above 1
    assert abs(s - t) <= A.shape[0] * xi
