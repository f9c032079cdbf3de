"""The FP16 Wilson operator with packed half-precision arithmetic (tuner kinds 2, 3 and 4; kind 3
stages each 256-site block's links in LDS for 8 right-hand-side groups, kind 4 streams each
block through the time slices) against the oracle.

Inputs and links as the library stores them (tests/storage16.py).  The kernel rounds each
half spinor h = p_a + c p_b (c = +-1, +-i) to FP16 (|dh| <= u |h|, u = 2^-11 per real), then
forms link products exactly and sums them in FP32, and rounds the output once to FP16.  A link
row has unit norm, so a rounded half spinor moves U h by at most u |h|_2 <= 2 sqrt(3) u m_psi
per colour (m_psi = the largest |component| of the input); each output real receives 1/2 U h
from each of the 8 hops, so it is within u |ref| + 8 sqrt(3) u m_psi + 1e-5 max |ref| of the
oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import core
from storage16 import stored

pytestmark = pytest.mark.gpu

SHAPES = [((4, 4, 4, 4), 0.3), ((3, 5, 4, 6), 0.5), ((8, 6, 4, 10), 0.5)]
TILES = [(1, 64, 0, 2), (2, 256, 16, 2), (4, 128, 64, 2), (2, 256, 1024, 2),
         (1, 256, 0, 3), (2, 256, 16, 3), (4, 256, 64, 3)]
U = 2.0 ** -11


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("dims,eps", SHAPES)
@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_packed_half_dslash_matches_oracle(gpu, dims, eps, op, tile):
    lq = gpu
    nrhs = 5
    print(f"packed FP16 dslash dims={dims} op={op} tile={tile}", flush=True)
    links = synth.su3_links(dims, eps, 1)
    c = lq.Context(dims, -0.4)
    c.set_gauge(links)
    c.set_tile(2, nrhs, tile)
    psi = synth.random_spinors(dims, nrhs, 2).reshape(nrhs, -1)
    out = c.apply(torch.as_tensor(psi).to(torch.complex64).cuda(), op=op, prec=2).cpu().numpy().astype(np.complex128)
    ps = stored(psi, 2)
    ref = core.apply(stored(links, 2, links=True), dims, -0.4, op, ps)
    m, mpsi = np.max(np.abs(ref)), np.max(np.abs(ps))
    for part in (np.real, np.imag):
        d = np.abs(part(out) - part(ref))
        assert np.all(d <= U * np.abs(part(ref)) + 8 * np.sqrt(3) * U * mpsi + 1e-5 * m), float(np.max(d / m))
    c.close()


# the streaming kernel (kind 4): slices of a multiple of 256 sites; odd Lt (the three-slice
# register rotation ends mid-cycle) and Lt = 2 (the t-1 and t+1 neighbours coincide)
@pytest.mark.parametrize("dims", [(8, 8, 4, 6), (16, 4, 8, 5), (4, 8, 8, 2)])
@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_streaming_dslash_matches_oracle(gpu, dims, op):
    lq = gpu
    nrhs = 3
    print(f"streaming FP16 dslash dims={dims} op={op}", flush=True)
    links = synth.su3_links(dims, 0.5, 1)
    c = lq.Context(dims, -0.4)
    c.set_gauge(links)
    c.set_tile(2, nrhs, (1, 256, 0, 4))
    psi = synth.random_spinors(dims, nrhs, 2).reshape(nrhs, -1)
    out = c.apply(torch.as_tensor(psi).to(torch.complex64).cuda(), op=op, prec=2).cpu().numpy().astype(np.complex128)
    ps = stored(psi, 2)
    ref = core.apply(stored(links, 2, links=True), dims, -0.4, op, ps)
    _check(out, ref, ps)
    c.close()


def _check(out, ref, ps):
    m, mpsi = np.max(np.abs(ref)), np.max(np.abs(ps))
    for part in (np.real, np.imag):
        d = np.abs(part(out) - part(ref))
        assert np.all(d <= U * np.abs(part(ref)) + 8 * np.sqrt(3) * U * mpsi + 1e-5 * m), float(np.max(d / m))


@pytest.mark.parametrize("tile", [(2, 256, 256, 2), (2, 256, 1024, 2), (2, 256, 0, 3), (2, 256, 64, 3), (1, 256, 0, 4)])
def test_packed_half_full_size(gpu, tile):
    """16^3x32 with 128 right-hand sides in the benchmark's launch shapes; sampled right-hand
    sides against the oracle"""
    lq = gpu
    dims, nrhs = (16, 16, 16, 32), 128
    print(f"packed FP16 dslash 16^3x32 tile={tile}", flush=True)
    links = synth.su3_links(dims, 0.5, 1)
    c = lq.Context(dims, -1.9)
    c.set_gauge(links)
    c.set_tile(2, nrhs, tile)
    psi = synth.random_spinors(dims, nrhs, 3).reshape(nrhs, -1)
    out = c.apply(torch.as_tensor(psi).to(torch.complex64).cuda(), op=0, prec=2).cpu().numpy().astype(np.complex128)
    pick = [0, 17, 64, 127]
    ps = stored(psi[pick], 2)
    ref = core.apply(stored(links, 2, links=True), dims, -1.9, 0, ps)
    _check(out[pick], ref, ps)
    c.close()


@pytest.mark.parametrize("nrhs,tile", [(20, (2, 256, 0, 3)), (37, (1, 256, 16, 3)), (9, (4, 256, 0, 3))])
def test_staged_links_several_group_blocks(gpu, nrhs, tile):
    """kind 3 with more right-hand-side groups than one block loops over (8), a partial last
    block of groups and a partial last group; every right-hand side against the oracle"""
    lq = gpu
    dims = (8, 6, 4, 10)
    print(f"staged-link FP16 dslash nrhs={nrhs} tile={tile}", flush=True)
    links = synth.su3_links(dims, 0.5, 4)
    c = lq.Context(dims, -0.4)
    c.set_gauge(links)
    c.set_tile(2, nrhs, tile)
    psi = synth.random_spinors(dims, nrhs, 6).reshape(nrhs, -1)
    for op in (0, 2):
        out = c.apply(torch.as_tensor(psi).to(torch.complex64).cuda(), op=op, prec=2).cpu().numpy()
        ps = stored(psi, 2)
        ref = core.apply(stored(links, 2, links=True), dims, -0.4, op, ps)
        _check(out.astype(np.complex128), ref, ps)
    c.close()


def test_staged_links_several_lattices(gpu):
    """kind 3 over three lattices in one launch, each against the oracle"""
    lq = gpu
    lats, masses = [(4, 4, 4, 4), (2, 4, 6, 4), (6, 4, 4, 8)], [-0.4, 0.1, -0.2]
    links = [synth.su3_links(d, 0.5, 1 + k) for k, d in enumerate(lats)]
    c = lq.Context(lats, masses)
    c.set_gauge(np.concatenate([u.ravel() for u in links]))
    nrhs = 19
    psi = np.concatenate([synth.random_spinors(d, nrhs, 7 + k).reshape(nrhs, -1) for k, d in enumerate(lats)], axis=1)
    c.set_tile(2, nrhs, (2, 256, 0, 3))
    out = c.apply(torch.as_tensor(psi).to(torch.complex64).cuda(), op=0, prec=2).cpu().numpy().astype(np.complex128)
    o = 0
    for k, d in enumerate(lats):
        n = 12 * int(np.prod(d))
        ps = stored(psi[:, o:o + n], 2)
        _check(out[:, o:o + n], core.apply(stored(links[k], 2, links=True), d, masses[k], 0, ps), ps)
        o += n
    c.close()


def test_packed_half_solves(gpu):
    """s-step cycles with the packed FP16 operator: solutions to 1e-8 against the oracle"""
    lq = gpu
    dims, m = (6, 6, 6, 8), -0.6
    links = synth.su3_links(dims, 0.5, 2)
    c = lq.Context(dims, m)
    c.set_gauge(links)
    z = c.probes(91, 8)
    c.set_tile(2, 8, (2, 256, 0, 2))
    y, st, _ = c.solve(z, 1e-8, prec=2, restart=15, sstep=1)
    assert all(s[0] for s in st)
    zs, ys = z.cpu().numpy(), y.cpu().numpy()
    r = zs - core.apply(links, dims, m, core.OP_A, ys)
    assert np.all(np.linalg.norm(r, axis=1) <= 1.05e-8 * np.linalg.norm(zs, axis=1))
    c.close()


def test_packed_half_rejects_other_storage(gpu):
    lq = gpu
    c = lq.Context((4, 4, 4, 4), 0.1)
    for prec in (0, 1, 3):
        for kind in (2, 3):
            with pytest.raises(lq.LqtError) as e:
                c.set_tile(prec, 8, (1, 256, 0, kind))
            assert e.value.code == -1
    for bs in (64, 128):  # the staged-link kernel takes 256-thread blocks only
        with pytest.raises(lq.LqtError) as e:
            c.set_tile(2, 8, (1, bs, 0, 3))
        assert e.value.code == -1
    c.close()
