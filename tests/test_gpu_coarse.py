"""The explicit coarse operator W^+ A W of a prolongator basis (9-point block stencil built from
W and the links) against the oracle's P^+ A P, P the dense prolongator of the same W and A the
oracle operator applied column by column.

Geometries cover coarse extents of 1 (every +-mu hop wraps back into the same aggregate), 2
(+mu and -mu reach the same aggregate) and 3 or more, non-cubic blocks, the antiperiodic time
boundary, nv = 6, 12 and 24 (the workload's), and more right-hand sides than one workgroup
takes."""
import numpy as np
import pytest
import torch

import synth
from oracle import core, prolongator as pr

pytestmark = pytest.mark.gpu


def _W(dims, block, nv, seed):
    rng = np.random.default_rng(seed)
    N = 12 * int(np.prod(dims))
    Y = rng.standard_normal((nv, N)) + 1j * rng.standard_normal((nv, N))
    return pr.block_orthonormalize(Y, dims, block)


CASES = [
    ((4, 4, 4, 4), (2, 2, 2, 2), 6, 0.1),     # coarse 2^4
    ((4, 4, 4, 8), (4, 4, 4, 2), 6, -0.3),    # coarse 1 x 1 x 1 x 4
    ((6, 4, 2, 6), (2, 2, 2, 2), 12, 0.2),    # coarse 3 x 2 x 1 x 3
    ((8, 8, 8, 8), (4, 4, 4, 4), 24, -0.5),   # the workload's blocks and nv, coarse 2^4
    ((12, 6, 4, 8), (3, 2, 2, 4), 5, 0.0),    # non-cubic blocks, coarse 4 x 3 x 2 x 2
]


@pytest.mark.parametrize("dims,block,nv,m", CASES)
def test_explicit_coarse_operator_matches_oracle(gpu, dims, block, nv, m):
    lq = gpu
    print(f"coarse operator dims={dims} block={block} nv={nv}", flush=True)
    U = synth.su3_links(dims, 0.4, 3)
    W = _W(dims, block, nv, 5)
    P = pr.dense_prolongator(W, dims, block)
    AP = core.apply(U, dims, m, core.OP_A, P.T.copy()).T
    Dc = P.conj().T @ AP
    nc = Dc.shape[0]
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator_from(block, nv, torch.as_tensor(W.reshape(-1)).cuda())
    rng = np.random.default_rng(9)
    x = rng.standard_normal((70, nc)) + 1j * rng.standard_normal((70, nc))
    y = B.coarse_apply(torch.as_tensor(x).cuda()).cpu().numpy()
    ref = (Dc @ x.T).T
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
    g5c = pr.coarse_g5(W.shape[0], nv)
    yh = B.coarse_apply(torch.as_tensor(x[:3]).cuda(), herm=True).cpu().numpy()
    assert np.max(np.abs(yh - g5c[None, :] * ref[:3])) <= 1e-12 * np.max(np.abs(ref))
    # g5^W W^+ A W is Hermitian for the gamma5-Hermitian A (g5 W = W g5^W)
    Hc = g5c[:, None] * Dc
    assert np.max(np.abs(Hc - Hc.conj().T)) <= 1e-12 * np.max(np.abs(Hc))
    B.close()
    c.close()
