"""Stalled solves and the fallback chain on the device.

- A constant spinor on a periodic free field is an eigenvector of A (A c = m c).  An s-step
  cycle from it has a rank-one Gram matrix and can take no step.  Without the fallback the
  solve must end as not converged (not loop); with it, the system continues with ordinary
  GMRES cycles and converges to x = c/m.
- A transport net with all weights zero maps every vector to 0, so FGMRES makes no progress at
  all.  With the fallback the solves drop the net after stall_window flat FP64 residuals and
  still meet the tolerance by the oracle's residual, and the statistics report the level.
- An untrained random net must still give solutions that meet the tolerance, whether or not
  it stalls."""
import numpy as np
import pytest
import torch

import synth
from oracle import core

pytestmark = pytest.mark.gpu


def _relres(U, dims, m, b, x, antiperiodic=True):
    r = b - core.apply(U, dims, m, core.OP_A, x, antiperiodic=antiperiodic)
    return np.linalg.norm(r, axis=1) / np.linalg.norm(b, axis=1)


@pytest.mark.parametrize("prec", [2, 3])
def test_eigenvector_rhs_sstep(gpu, prec):
    lq = gpu
    dims, m, xi = (4, 4, 4, 8), 0.1, 1e-10
    print(f"eigenvector right-hand side, s-step cycles, storage {prec}", flush=True)
    c = lq.Context(dims, m, antiperiodic=False)
    c.set_gauge(synth.unit_links(dims))
    b = torch.ones((2, 12 * int(np.prod(dims))), dtype=torch.complex128, device="cuda")
    b[1] *= 0.5 - 0.25j
    # no fallback: the zero-step cycle ends the solve as not converged
    x, st, rc = c.solve(b, xi, raise_on_fail=False, prec=prec, restart=15, sstep=1)
    assert rc == lq.LQT_ENOTCONV
    assert all(s[0] == 0 and s[4] == 0 for s in st)
    # fallback: ordinary GMRES cycles at the same storage
    x, st, rc = c.solve(b, xi, prec=prec, restart=15, sstep=1, fallback=1)
    assert rc == 0 and all(s[0] == 1 and s[4] == 1 for s in st), st
    xh = x.cpu().numpy()
    ref = b.cpu().numpy() / m
    assert np.max(np.abs(xh - ref)) <= 1e-8 * np.max(np.abs(ref))
    c.close()


def test_zero_net_falls_back(gpu):
    lq = gpu
    dims, m, xi = (8, 8, 8, 8), -0.5, 1e-8
    print("zero-weight net, fallback to plain GMRES", flush=True)
    U = synth.su3_links(dims, 0.4, 2)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    c.precond_set(torch.zeros(lq.WEIGHT_COUNT, dtype=torch.complex64))
    z = c.probes(77, 3)
    x, st, rc = c.solve(z, xi, prec=lq.BF16, use_net=1, restart=16, fallback=1, stall_window=2)
    assert rc == 0
    assert all(s[0] == 1 and s[4] == 1 for s in st), st
    rr = _relres(U, dims, m, z.cpu().numpy(), x.cpu().numpy())
    assert np.all(rr <= xi * 1.05), rr
    r = c.trace(3, 77, xi, prec=lq.BF16, use_net=1, restart=16, fallback=1)
    assert r["nfailed"] == 0 and r["nfallback"] == 3
    c.close()


def test_random_net_meets_tolerance(gpu):
    lq = gpu
    dims, m, xi = (8, 8, 8, 8), -0.5, 1e-8
    print("untrained random net with the fallback", flush=True)
    U = synth.su3_links(dims, 0.4, 2)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    rng = np.random.default_rng(9)
    w = (rng.standard_normal(lq.WEIGHT_COUNT) + 1j * rng.standard_normal(lq.WEIGHT_COUNT)) / 3
    c.precond_set(torch.as_tensor(w.astype(np.complex64)))
    z = c.probes(78, 3)
    x, st, rc = c.solve(z, xi, prec=lq.BF16, use_net=1, restart=16, fallback=1, stall_window=1, maxit=4000)
    print("levels", [s[4] for s in st], "steps", [s[1] for s in st], flush=True)
    assert rc == 0 and all(s[0] == 1 for s in st)
    rr = _relres(U, dims, m, z.cpu().numpy(), x.cpu().numpy())
    assert np.all(rr <= xi * 1.05), rr
    c.close()
