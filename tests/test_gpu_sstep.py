"""s-step cycles (basis of hopping-term powers, Gram pass and FP64 Cholesky) against the oracle
and against ordinary GMRES cycles."""
import numpy as np
import pytest
import torch

import synth
from oracle import core

pytestmark = pytest.mark.gpu


def _relres(U, dims, m, b, x):
    r = b - core.apply(U, dims, m, core.OP_A, x)
    return np.linalg.norm(r, axis=1) / np.linalg.norm(b, axis=1)


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("s", [4, 8])
def test_sstep_solves_match_oracle(gpu, prec, s):
    lq = gpu
    dims, m, xi = (4, 4, 6, 8), -0.6, 1e-9
    print(f"s-step s={s} prec={prec}", flush=True)
    U = synth.su3_links(dims, 0.5, 3)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    b = synth.random_spinors(dims, 5, 4).reshape(5, -1)
    bt = torch.as_tensor(b).cuda()
    x, st, _ = c.solve(bt, xi, prec=prec, restart=s, sstep=1, maxit=20000)
    assert all(q[0] for q in st)
    assert np.all(_relres(U, dims, m, b, x.cpu().numpy()) <= xi * 1.05)
    _, st0, _ = c.solve(bt, xi, prec=prec, restart=s)
    # the same Krylov spaces: whole cycles of s steps against GMRES(s) stopping mid-cycle
    for a, q in zip(st, st0):
        assert a[1] <= 1.15 * q[1] + 2 * s, (a, q)
    c.close()


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("s", [12, 15])
def test_sstep_long_cycles_16bit(gpu, prec, s):
    """Cycles longer than 8 (16-bit storage: the Gram matrix from the matrix cores)."""
    lq = gpu
    dims, m, xi = (4, 4, 6, 8), -0.6, 1e-9
    print(f"s-step s={s} prec={prec}", flush=True)
    U = synth.su3_links(dims, 0.5, 3)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    b = synth.random_spinors(dims, 5, 4).reshape(5, -1)
    bt = torch.as_tensor(b).cuda()
    x, st, _ = c.solve(bt, xi, prec=prec, restart=s, sstep=1, maxit=20000)
    assert all(q[0] for q in st)
    assert np.all(_relres(U, dims, m, b, x.cpu().numpy()) <= xi * 1.05)
    _, st0, _ = c.solve(bt, xi, prec=prec, restart=s)
    for a, q in zip(st, st0):
        assert a[1] <= 1.15 * q[1] + 2 * s, (a, q)
    c.close()


@pytest.mark.parametrize("prec,s", [(0, 8), (1, 8), (2, 15), (3, 15)])
def test_sstep_carry_ragged_lattice(gpu, prec, s):
    """3x5x4x6 (V = 360): the pass that updates x and carries the residual covers a slot in
    16-byte chunks (1080, 2160 and 4320 of them for 16-bit, FP32 and FP64 storage), 256 per
    block, so its last block is partial; the solutions meet xi by the oracle's residual, with
    carried residuals as without them."""
    lq = gpu
    dims, m, xi = (3, 5, 4, 6), -0.6, 1e-9
    print(f"s-step carry on 3x5x4x6 s={s} prec={prec}", flush=True)
    U = synth.su3_links(dims, 0.5, 5)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    b = synth.random_spinors(dims, 7, 6).reshape(7, -1)
    bt = torch.as_tensor(b).cuda()
    for reliable in (0.1, -1.0):  # carried residuals, then an FP64 residual at every cycle
        x, st, _ = c.solve(bt, xi, prec=prec, restart=s, sstep=1, reliable=reliable, maxit=20000)
        assert all(q[0] for q in st)
        assert np.all(_relres(U, dims, m, b, x.cpu().numpy()) <= xi * 1.05)
    c.close()


def test_sstep_near_critical_16x8(gpu):
    """A harder operator (m = -1.4 on 8^3x16): BF16 storage, restart 8, to 1e-8."""
    lq = gpu
    dims, m, xi = (8, 8, 8, 16), -1.4, 1e-8
    U = synth.su3_links(dims, 0.5, 1)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    z = c.probes(77, 8)
    y, st, _ = c.solve(z, xi, prec=3, restart=8, sstep=1, maxit=20000)
    _, st0, _ = c.solve(z, xi, prec=3, restart=8)
    assert all(q[0] for q in st)
    zs, ys = z[:3].cpu().numpy(), y[:3].cpu().numpy()
    assert np.all(_relres(U, dims, m, zs, ys) <= xi * 1.05)
    print("steps s-step", [q[1] for q in st], "GMRES(8)", [q[1] for q in st0], flush=True)
    assert sum(q[1] for q in st) <= 1.15 * sum(q[1] for q in st0) + 8 * len(st)
    c.close()


def test_sstep_graph_bit_identical_and_several_lattices(gpu):
    lq = gpu
    lats, masses = [(4, 4, 4, 4), (2, 4, 6, 4)], [-0.3, 0.05]
    links = [synth.su3_links(d, 0.5, 7 + k) for k, d in enumerate(lats)]
    c = lq.Context(lats, masses)
    c.set_gauge(np.concatenate([u.ravel() for u in links]))
    b = np.concatenate([synth.random_spinors(d, 3, 9 + k).reshape(3, -1) for k, d in enumerate(lats)], axis=1)
    bt = torch.as_tensor(b).cuda()
    x0, st0, _ = c.solve(bt, 1e-9, prec=3, restart=8, sstep=1)
    x1, st1, _ = c.solve(bt, 1e-9, prec=3, restart=8, sstep=1, graph=1)
    assert torch.equal(x0, x1)
    assert [q[:3] for q in st0] == [q[:3] for q in st1]
    x0 = x0.cpu().numpy()
    o = 0
    for k, d in enumerate(lats):
        n = 12 * d[0] * d[1] * d[2] * d[3]
        assert np.all(_relres(links[k], d, masses[k], b[:, o:o + n], x0[:, o:o + n]) <= 1.05e-9)
        o += n
    c.close()


def test_sstep_option_limits(gpu):
    lq = gpu
    dims = (4, 4, 4, 4)
    c = lq.Context(dims, -0.3)
    c.set_gauge(synth.su3_links(dims, 0.5, 1))
    b = torch.as_tensor(synth.random_spinors(dims, 1, 1).reshape(1, -1)).cuda()
    with pytest.raises(lq.LqtError) as ei:
        c.solve(b, 1e-6, restart=9, sstep=1)  # FP64 storage: at most 8
    assert ei.value.code == lq.LQT_EINVAL
    c.close()


@pytest.mark.parametrize("prec,s", [(0, 8), (1, 8), (3, 15), (2, 12)])
@pytest.mark.parametrize("graph", [0, 1])
def test_carried_residual_cycles(gpu, prec, s, graph):
    """Reliable updates: cycles start from the residual carried in the basis and the FP64
    residual is formed only when it fell tenfold, or to verify convergence.  Same solutions
    (oracle residuals below xi), about the same steps, far fewer FP64 residuals."""
    lq = gpu
    dims, m, xi = (6, 6, 6, 8), -1.7, 1e-9  # about 20 cycles: residuals fall slowly per cycle
    print(f"carried residual prec={prec} s={s} graph={graph}", flush=True)
    U = synth.su3_links(dims, 0.5, 5)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    b = synth.random_spinors(dims, 6, 8).reshape(6, -1)
    bt = torch.as_tensor(b).cuda()
    runs = {}
    for rel in (-1.0, 0.1):
        c.kernel_times(mode=2)
        x, st, _ = c.solve(bt, xi, prec=prec, restart=s, sstep=1, graph=graph, reliable=rel, maxit=40000)
        kt = c.kernel_times(mode=3)
        assert all(q[0] for q in st)
        assert np.all(_relres(U, dims, m, b, x.cpu().numpy()) <= xi * 1.05)
        runs[rel] = (sum(q[1] for q in st), kt["residual_fp64"][1], max(q[2] for q in st))
    (it_every, nres_every, cyc), (it_carry, nres_carry, _) = runs[-1.0], runs[0.1]
    print("steps every/carried", it_every, it_carry, "FP64 residuals", nres_every, nres_carry, flush=True)
    assert it_carry <= 1.1 * it_every + 6 * s
    assert nres_every == cyc and nres_carry <= 0.75 * nres_every
    c.close()


def test_reliable_option_limits(gpu):
    lq = gpu
    c = lq.Context((4, 4, 4, 4), 0.1)
    c.set_gauge(synth.su3_links((4, 4, 4, 4), 0.3, 1))
    z = c.probes(1, 1)
    with pytest.raises(lq.LqtError) as e:
        c.solve(z, 1e-8, prec=3, restart=8, sstep=1, reliable=1.5)
    assert e.value.code == -1
    c.close()
