"""GPU parity of the parallel-transport network preconditioner and of FGMRES with it."""
import numpy as np
import pytest
import torch

import synth
from oracle import core, ptc

pytestmark = pytest.mark.gpu

FWD_TOL = 2e-5  # FP32 arithmetic over four layers, max |gpu - oracle| / max |oracle|


def _bf16(w):
    """Round complex64 weights to BF16 (nearest, ties to even), returned as complex128."""
    f = np.ascontiguousarray(np.asarray(w, dtype=np.complex64)).view(np.float32).copy()
    u = f.view(np.uint32)
    fin = (u & 0x7F800000) != 0x7F800000
    u[fin] = (u[fin] + 0x7FFF + ((u[fin] >> 16) & 1)) & 0xFFFF0000
    return f.view(np.complex64).astype(np.complex128)


def _random_weights(seed):
    rng = np.random.default_rng(seed)
    n = ptc.weight_count()
    return ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / 6.0).astype(np.complex64)


def _ctx(lq, dims, mass, eps=0.5, seed=1):
    U = synth.su3_links(dims, eps, seed)
    c = lq.Context(dims, mass)
    c.set_gauge(U)
    return c, U


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 5, 4, 6), (8, 6, 4, 10), (8, 8, 4, 6)])
def test_forward_matches_oracle(gpu, dims):
    lq = gpu
    print(f"net forward dims={dims}", flush=True)
    c, U = _ctx(lq, dims, -0.4)
    w = _random_weights(5)
    c.precond_set(torch.as_tensor(w))
    assert np.array_equal(c.precond_get().numpy(), w)
    nrhs = 3
    psi = synth.random_spinors(dims, nrhs, 2).reshape(nrhs, -1)
    out = c.precond_apply(torch.as_tensor(psi).cuda()).cpu().numpy()
    ref = ptc.forward(U, dims, _bf16(w), psi)
    assert np.max(np.abs(out - ref)) <= FWD_TOL * np.max(np.abs(ref))
    c.close()


def test_forward_full_size_256_fields(gpu):
    """16^3x32 with 256 fields in one application (the grid of the learned-preconditioner
    workload: 64 groups of 4 fields, 8192 site chunks); the first and last fields are checked
    in full against the oracle forward pass."""
    lq = gpu
    dims = (16, 16, 16, 32)
    print("net forward 16^3x32, 256 fields", flush=True)
    c, U = _ctx(lq, dims, -1.9, eps=0.5, seed=1)
    w = _random_weights(5)
    c.precond_set(torch.as_tensor(w))
    z = c.probes(1003, 256)
    out = c.precond_apply(z)
    pick = [0, 255]
    got = out[pick].cpu().numpy()
    zs = z[pick].cpu().numpy()
    del out, z
    ref = ptc.forward(U, dims, _bf16(w), zs)
    assert np.max(np.abs(got - ref)) <= FWD_TOL * np.max(np.abs(ref))
    c.close()


def test_network_with_gamma_weights_is_the_wilson_operator(gpu):
    """First layer = the Wilson operator on features 0..3, then identities: M = A exactly in
    BF16 weights (4+m = 3.5, 1/2 and the gamma entries are BF16 numbers)."""
    lq = gpu
    dims, m = (4, 6, 4, 8), -0.5
    c, U = _ctx(lq, dims, m)
    layers = []
    for li, (fi, fo) in enumerate(zip(ptc.FEATURES[:-1], ptc.FEATURES[1:])):
        W = np.zeros((9, fo, fi), dtype=np.complex128)
        if li == 0:
            W[0, :4, :4] = (4 + m) * np.eye(4)
            for mu in range(4):
                W[1 + 2 * mu, :4, :4] = -0.5 * (np.eye(4) - core.gamma(mu))
                W[2 + 2 * mu, :4, :4] = -0.5 * (np.eye(4) + core.gamma(mu))
        else:
            W[0] = np.eye(fo, fi)
        layers.append(W.ravel())
    c.precond_set(torch.as_tensor(np.concatenate(layers).astype(np.complex64)))
    psi = synth.random_spinors(dims, 2, 3).reshape(2, -1)
    out = c.precond_apply(torch.as_tensor(psi).cuda()).cpu().numpy()
    ref = core.apply(U, dims, m, core.OP_A, psi)
    assert np.max(np.abs(out - ref)) <= 1e-5 * np.max(np.abs(ref))
    c.close()


def test_loss_and_gradient_match_oracle(gpu):
    lq = gpu
    dims, m = (4, 4, 2, 4), -0.3
    c, U = _ctx(lq, dims, m, seed=3)
    w = _random_weights(7)
    c.precond_set(torch.as_tensor(w))
    e = synth.random_spinors(dims, 3, 4).reshape(3, -1)
    loss, grad = c.precond_loss_grad(torch.as_tensor(e).cuda())
    w64 = w.astype(np.complex128)  # the loss uses the FP32 master weights
    ref_loss = ptc.loss(U, dims, m, w64, e)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    # every layer and path: a spread of indices through the weight vector
    rng = np.random.default_rng(0)
    idx = sorted(set(rng.choice(ptc.weight_count(), 40, replace=False).tolist()) | {0, 287, 288, 1727})
    fd = ptc.loss_grad_fd(U, dims, m, w64, e, idx)
    g = grad.numpy()[idx]
    assert np.max(np.abs(g - fd)) <= 1e-4 * np.max(np.abs(grad.numpy())), (g[:4], fd[:4])
    c.close()


def _init_loss(U, dims, m, e):
    """Loss of the point-Jacobi start M = 1/(4+m)."""
    r = core.apply(U, dims, m, core.OP_A, e)
    return float(np.mean(np.sum(np.abs(r / (4 + m) - e) ** 2, axis=1) / np.sum(np.abs(e) ** 2, axis=1)))


@pytest.mark.parametrize("pair_xi", [0.0, 0.1])
def test_training_lowers_the_held_out_loss(gpu, pair_xi):
    lq = gpu
    dims, m = (4, 4, 4, 4), -0.5
    print(f"net training pair_xi={pair_xi}", flush=True)
    c, U = _ctx(lq, dims, m, seed=2)
    last = c.precond_train(16, seed=11, epochs=25, lr=3e-3, batch=4, pair_xi=pair_xi)
    assert np.isfinite(last)
    w = c.precond_get().numpy()
    # held-out errors of the same kind as the training ones
    g = synth.random_spinors(dims, 4, 21).reshape(4, -1)
    if pair_xi > 0:
        e = np.stack([core.gmres(U, dims, m, gi, pair_xi)[0] for gi in g])
    else:
        e = g
    before = _init_loss(U, dims, m, e)
    after = ptc.loss(U, dims, m, _bf16(w), e)
    print(f"held-out loss {before:.4f} -> {after:.4f} (train {last:.4f})", flush=True)
    assert after < 0.8 * before
    c.close()


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_fgmres_with_trained_net_meets_tolerance(gpu, prec):
    lq = gpu
    dims, m, xi = (4, 4, 4, 8), -0.6, 1e-8
    c, U = _ctx(lq, dims, m, seed=5)
    c.precond_train(16, seed=3, epochs=15, lr=3e-3, batch=4, pair_xi=0.1)
    b = synth.random_spinors(dims, 3, 8).reshape(3, -1)
    x, st, _ = c.solve(torch.as_tensor(b).cuda(), xi, prec=prec, use_net=1)
    x = x.cpu().numpy()
    res = b - core.apply(U, dims, m, core.OP_A, x)
    rel = np.linalg.norm(res, axis=1) / np.linalg.norm(b, axis=1)
    assert np.all(rel <= xi * 1.05), rel
    xref = np.stack([core.gmres(U, dims, m, bi, 1e-12)[0] for bi in b])
    # both meet their tolerance: the solutions differ by at most kappa-scaled residuals
    assert np.max(np.abs(x - xref)) / np.max(np.abs(xref)) < 1e-5
    _, st0, _ = c.solve(torch.as_tensor(b).cuda(), xi, prec=prec)
    print(f"prec {prec}: FGMRES+net iters {[s[1] for s in st]}, GMRES iters {[s[1] for s in st0]}", flush=True)
    c.close()


def test_error_paths(gpu):
    lq = gpu
    dims = (4, 4, 4, 4)
    c, U = _ctx(lq, dims, -0.4)
    b = torch.as_tensor(synth.random_spinors(dims, 1, 1).reshape(1, -1)).cuda()
    with pytest.raises(lq.LqtError) as ei:
        c.solve(b, 1e-6, use_net=1)
    assert ei.value.code == lq.LQT_ESTATE
    with pytest.raises(lq.LqtError) as ei:
        c.precond_apply(b)
    assert ei.value.code == lq.LQT_ESTATE
    with pytest.raises(lq.LqtError) as ei:
        c.precond_set(torch.zeros(100, dtype=torch.complex64))
    assert ei.value.code == lq.LQT_EINVAL
    w = _random_weights(1)
    w[17] = np.nan
    with pytest.raises(lq.LqtError) as ei:
        c.precond_set(torch.as_tensor(w))
    assert ei.value.code == lq.LQT_ENAN
    with pytest.raises(lq.LqtError) as ei:
        c.precond_train(0, seed=1)
    assert ei.value.code == lq.LQT_EINVAL
    c.close()
