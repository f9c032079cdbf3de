"""The matrix-core Wilson operator (FP16/BF16 storage) against the oracle, for every tiling.

The oracle applies the FP64 operator to the inputs and links as the library stores them (each
real rounded to nearest-even at FP16 or BF16; tests/storage16.py).  The kernel forms exact
products and FP32 sums, then rounds each output real once to the storage format, so every
output real is within u |ref| of the oracle (u = 2^-8 for BF16, 2^-11 for FP16) plus the FP32
summation error, bounded here by 1e-5 max |ref|."""
import numpy as np
import pytest
import torch

import synth
from oracle import core
from storage16 import stored

pytestmark = pytest.mark.gpu

SHAPES = [((4, 4, 4, 4), 0.3), ((3, 5, 4, 6), 0.5), ((8, 6, 4, 10), 0.5)]  # 360 sites: a ragged wave
U16 = {2: 2.0 ** -11, 3: 2.0 ** -8}
# (groups of 4 right-hand sides per lane, block, chunk, kind 1 = matrix cores)
TILES = [(1, 64, 0, 1), (2, 256, 16, 1), (1, 128, 64, 1), (2, 64, 0, 1)]


def _check(out, ref, prec):
    m = np.max(np.abs(ref))
    u = U16[prec]
    for part in (np.real, np.imag):
        d = np.abs(part(out) - part(ref))
        assert np.all(d <= u * np.abs(part(ref)) + 1e-5 * m), float(np.max(d / m))


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("dims,eps", SHAPES)
@pytest.mark.parametrize("op", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", [2, 3])
def test_mfma_dslash_matches_oracle(gpu, dims, eps, op, prec, tile):
    lq = gpu
    nrhs = 9 if tile[0] == 2 else 5  # a partial group of 4 right-hand sides
    print(f"matrix-core dslash dims={dims} op={op} prec={prec} tile={tile} nrhs={nrhs}", flush=True)
    U = synth.su3_links(dims, eps, 1)
    c = lq.Context(dims, -0.4)
    c.set_gauge(U)
    c.set_tile(prec, nrhs, tile)
    psi = synth.random_spinors(dims, nrhs, 2).reshape(nrhs, -1)
    out = c.apply(torch.as_tensor(psi).to(torch.complex64).cuda(), op=op, prec=prec).cpu().numpy()
    ref = core.apply(stored(U, prec, links=True), dims, -0.4, op, stored(psi, prec))
    _check(out.astype(np.complex128), ref, prec)
    c.close()


@pytest.mark.parametrize("prec", [2, 3])
def test_mfma_and_vector_kernels_agree(gpu, prec):
    """same inputs through both kernels: both within the storage rounding of each other"""
    lq = gpu
    dims = (8, 8, 4, 6)
    U = synth.su3_links(dims, 0.5, 3)
    c = lq.Context(dims, -0.7)
    c.set_gauge(U)
    x = torch.as_tensor(synth.random_spinors(dims, 12, 4).reshape(12, -1)).to(torch.complex64).cuda()
    c.set_tile(prec, 12, (2, 128, 0, 1))
    a = c.apply(x, op=0, prec=prec).cpu().numpy().astype(np.complex128)
    c.set_tile(prec, 12, (4, 256, 0, 0))
    b = c.apply(x, op=0, prec=prec).cpu().numpy().astype(np.complex128)
    u = U16[prec]
    assert np.max(np.abs(a - b)) <= 2 * u * np.max(np.abs(b))
    c.close()


def test_mfma_dslash_several_lattices(gpu):
    """three lattices in one context (one launch), each checked against the oracle"""
    lq = gpu
    lats, masses = [(4, 4, 4, 4), (2, 4, 6, 4), (6, 4, 4, 8)], [-0.4, 0.1, -0.2]
    links = [synth.su3_links(d, 0.5, 1 + k) for k, d in enumerate(lats)]
    c = lq.Context(lats, masses)
    c.set_gauge(np.concatenate([u.ravel() for u in links]))
    nrhs = 6
    psi = np.concatenate([synth.random_spinors(d, nrhs, 7 + k).reshape(nrhs, -1) for k, d in enumerate(lats)], axis=1)
    for op in range(4):
        c.set_tile(3, nrhs, (2, 256, 0, 1))
        out = c.apply(torch.as_tensor(psi).to(torch.complex64).cuda(), op=op, prec=3).cpu().numpy()
        o = 0
        for k, d in enumerate(lats):
            n = 12 * int(np.prod(d))
            ref = core.apply(stored(links[k], 3, links=True), d, masses[k], op, stored(psi[:, o:o + n], 3))
            _check(out[:, o:o + n].astype(np.complex128), ref, 3)
            o += n
    c.close()


def test_mfma_solve_converges(gpu):
    """BF16 inner GMRES cycles on the matrix-core operator, FP64 defect correction to 1e-8"""
    lq = gpu
    dims, m = (6, 6, 6, 8), -0.6
    U = synth.su3_links(dims, 0.5, 2)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    z = c.probes(77, 8)
    c.set_tile(3, 8, (2, 256, 0, 1))
    y, st, _ = c.solve(z, 1e-8, prec=3, restart=15, sstep=1)
    assert all(s[0] for s in st)
    zs, ys = z.cpu().numpy(), y.cpu().numpy()
    r = zs - core.apply(U, dims, m, core.OP_A, ys)
    assert np.all(np.linalg.norm(r, axis=1) <= 1.05e-8 * np.linalg.norm(zs, axis=1))
    c.close()


def test_tile_checks(gpu):
    lq = gpu
    c = lq.Context((4, 4, 4, 4), 0.1)
    for prec, tile in [(0, (1, 256, 0, 1)), (1, (1, 256, 0, 1)), (3, (4, 256, 0, 1)), (3, (1, 96, 0, 1)),
                       (0, (4, 256, 0, 0)), (3, (1, 256, -1, 0))]:
        with pytest.raises(lq.LqtError) as e:
            c.set_tile(prec, 8, tile)
        assert e.value.code == -1
    c.set_gauge(synth.su3_links((4, 4, 4, 4), 0.3, 1))
    ms, tile = c.tune(3, 8, return_tile=True)
    assert ms > 0 and len(tile) == 4 and tile[3] in (0, 1)
    c.close()
