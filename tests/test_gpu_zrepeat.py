"""Repeat runs are bitwise identical: no kernel of the library uses atomics, and every reduction
has a fixed order, so a second solve or trace estimate of the same inputs on the same context
reproduces the first bit for bit (a cheap check for races in the kernels)."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("path", ["f64_gmres32", "f16_sstep8", "bf16_gmres8"])
def test_repeat_runs_are_bitwise_identical(gpu, path):
    lq = gpu
    dims, m, xi = (4, 4, 6, 8), -0.6, 1e-9
    print(f"repeat run, path={path}", flush=True)
    opts = {"f64_gmres32": dict(prec=lq.F64, restart=32),
            "f16_sstep8": dict(prec=lq.F16, restart=8, sstep=1),
            "bf16_gmres8": dict(prec=lq.BF16, restart=8)}[path]
    c = lq.Context(dims, m)
    c.set_gauge(synth.su3_links(dims, 0.5, 3))
    b = torch.as_tensor(synth.random_spinors(dims, 5, 4).reshape(5, -1)).cuda()
    x1, st1, _ = c.solve(b, xi, maxit=20000, **opts)
    x2, st2, _ = c.solve(b, xi, maxit=20000, **opts)
    assert all(q[0] for q in st1)
    assert torch.equal(x1, x2) and list(st1) == list(st2)
    r1 = c.trace(8, 1000, xi, samples=True, maxit=20000, **opts)
    r2 = c.trace(8, 1000, xi, samples=True, maxit=20000, **opts)
    assert torch.equal(r1["samples"], r2["samples"])
    assert r1["trace_re"] == r2["trace_re"] and r1["var_sample"] == r2["var_sample"]
    c.close()
