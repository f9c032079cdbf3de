"""Graph-captured inner cycles give bit-identical solves to the eagerly launched ones."""
import numpy as np
import pytest
import torch

import synth
from oracle import core

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_graph_cycles_bit_identical(gpu, prec):
    lq = gpu
    dims, m = (4, 4, 6, 8), -0.3
    print(f"graph cycles prec={prec}", flush=True)
    U = synth.su3_links(dims, 0.5, 3)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    b = synth.random_spinors(dims, 5, 4).reshape(5, -1)
    b[1] *= 1e-3  # different scales and a zero right-hand side: the active set shrinks
    b[3] = 0
    bt = torch.as_tensor(b).cuda()
    x0, st0, _ = c.solve(bt, 1e-10, prec=prec, restart=8)
    c.kernel_times(mode=2)
    x1, st1, _ = c.solve(bt, 1e-10, prec=prec, restart=8, graph=1)
    kt = c.kernel_times(mode=3)
    assert kt["graph_cycles"][1] >= 3  # several replays
    assert torch.equal(x0, x1)
    assert [s[:3] for s in st0] == [s[:3] for s in st1]
    # and the answer is right
    r = b - core.apply(U, dims, m, core.OP_A, x1.cpu().numpy())
    nb = np.linalg.norm(b, axis=1)
    ok = nb > 0
    assert np.all(np.linalg.norm(r, axis=1)[ok] <= 1.05e-10 * nb[ok])
    c.close()


def test_graph_cycles_several_lattices(gpu):
    lq = gpu
    lats, masses = [(4, 4, 4, 4), (2, 4, 6, 4)], [-0.3, 0.05]
    links = [synth.su3_links(d, 0.5, 7 + k) for k, d in enumerate(lats)]
    c = lq.Context(lats, masses)
    c.set_gauge(np.concatenate([u.ravel() for u in links]))
    b = np.concatenate([synth.random_spinors(d, 3, 9 + k).reshape(3, -1) for k, d in enumerate(lats)], axis=1)
    bt = torch.as_tensor(b).cuda()
    x0, st0, _ = c.solve(bt, 1e-9, prec=3, restart=8)
    x1, st1, _ = c.solve(bt, 1e-9, prec=3, restart=8, graph=1)
    assert torch.equal(x0, x1)
    assert [s[:3] for s in st0] == [s[:3] for s in st1]
    c.close()
