"""GPU parity of the Wilson operator and the probes against the CPU oracle (through the C-ABI)."""
import numpy as np
import pytest
import torch

import synth
from oracle import core
from storage16 import stored

pytestmark = pytest.mark.gpu

# (dims, eps): several site tiles with a ragged tail, odd extents, and the benchmark lattice
SHAPES = [((4, 4, 4, 4), 0.3), ((3, 5, 4, 6), 0.5), ((8, 6, 4, 10), 0.5)]
TOL = {0: 1e-12, 1: 1e-5}  # max |gpu - oracle| / max |oracle|
# 16-bit storage with FP32 arithmetic (tile kind 0): the oracle applies the FP64 operator to the
# inputs and links as stored (tests/storage16.py); the kernel's FP32 sums of exact-ish
# products are rounded once to the storage format, so every output real is within u |ref|
# (u = 2^-11 FP16, 2^-8 BF16) plus the FP32 summation error, bounded by 1e-5 max |ref|
U16 = {2: 2.0 ** -11, 3: 2.0 ** -8}
KIND0_TILES = [(1, 256, 0, 0), (2, 128, 16, 0), (4, 64, 0, 0)]


def _check16(out, ref, prec):
    m = np.max(np.abs(ref))
    for part in (np.real, np.imag):
        d = np.abs(part(out) - part(ref))
        assert np.all(d <= U16[prec] * np.abs(part(ref)) + 1e-5 * m), float(np.max(d / m))


def _ctx(lq, dims, mass, eps, seed=1, antiperiodic=True):
    U = synth.su3_links(dims, eps, seed)
    c = lq.Context(dims, mass, antiperiodic=antiperiodic)
    c.set_gauge(U)
    return c, U


@pytest.mark.parametrize("dims,eps", SHAPES)
@pytest.mark.parametrize("op", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_dslash_matches_oracle(gpu, dims, eps, op, prec):
    lq = gpu
    print(f"dslash parity dims={dims} op={op} prec={prec}", flush=True)
    c, U = _ctx(lq, dims, -0.4, eps)
    nrhs = 5  # not a multiple of the rhs tile: exercises the ragged rhs group
    psi = synth.random_spinors(dims, nrhs, 2).reshape(nrhs, -1)
    ref = core.apply(U, dims, -0.4, op, psi)
    dt = torch.complex128 if prec == 0 else torch.complex64
    x = torch.as_tensor(psi).to(dt).cuda()
    if prec >= 2:
        c.set_tile(prec, nrhs, KIND0_TILES[0])
    out = c.apply(x, op=op, prec=prec).cpu().numpy().astype(np.complex128)
    if prec >= 2:
        _check16(out, core.apply(stored(U, prec, links=True), dims, -0.4, op, stored(psi, prec)), prec)
    else:
        err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
        assert err <= TOL[prec], err
    c.close()


@pytest.mark.parametrize("tile", KIND0_TILES[1:])
@pytest.mark.parametrize("dims,eps", SHAPES)
@pytest.mark.parametrize("prec", [2, 3])
def test_kind0_16bit_tiles_within_derived_bounds(gpu, dims, eps, prec, tile):
    lq = gpu
    nrhs = 9  # ragged against 2 and 4 right-hand sides per thread
    print(f"kind-0 dslash dims={dims} prec={prec} tile={tile}", flush=True)
    c, U = _ctx(lq, dims, -0.4, eps)
    c.set_tile(prec, nrhs, tile)
    psi = synth.random_spinors(dims, nrhs, 4).reshape(nrhs, -1)
    for op in (0, 2):
        out = c.apply(torch.as_tensor(psi).to(torch.complex64).cuda(), op=op, prec=prec).cpu().numpy()
        _check16(out.astype(np.complex128), core.apply(stored(U, prec, links=True), dims, -0.4, op, stored(psi, prec)),
                 prec)
    c.close()


def test_dslash_benchmark_lattice_fp64_and_fp32(gpu):
    lq = gpu
    dims = (16, 16, 16, 32)
    print("dslash parity 16^3x32", flush=True)
    c, U = _ctx(lq, dims, -0.9, 0.5)
    psi = synth.random_spinors(dims, 2, 3).reshape(2, -1)
    ref = core.apply(U, dims, -0.9, 0, psi)
    out = c.apply(torch.as_tensor(psi).cuda(), op=0, prec=0).cpu().numpy()
    assert np.max(np.abs(out - ref)) / np.max(np.abs(ref)) <= 1e-12
    out32 = c.apply(torch.as_tensor(psi).to(torch.complex64).cuda(), op=0, prec=1).cpu().numpy()
    assert np.max(np.abs(out32 - ref)) / np.max(np.abs(ref)) <= 1e-5
    c.close()


def test_plane_wave_32c64_free_field(gpu):
    """At 32^3 x 64 the free-field plane wave fixes every output: A e^{ipx}u = A(p) e^{ipx}u."""
    lq = gpu
    dims, m = (32, 32, 32, 64), 0.05
    print("plane wave 32^3x64", flush=True)
    c = lq.Context(dims, m)
    c.set_gauge(synth.unit_links(dims))
    rng = np.random.default_rng(4)
    n = [3, 7, 30, 11]
    p = [2 * np.pi * n[0] / 32, 2 * np.pi * n[1] / 32, 2 * np.pi * n[2] / 32, (2 * n[3] + 1) * np.pi / 64]
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = synth.plane_wave(dims, p, u).reshape(1, -1)
    Ap = (m + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(core.gamma(mu) * np.sin(p[mu]) for mu in range(4))
    expect = synth.plane_wave(dims, p, Ap @ u).reshape(1, -1)
    out = c.apply(torch.as_tensor(psi).cuda(), op=0, prec=0).cpu().numpy()
    assert np.max(np.abs(out - expect)) < 1e-12 * np.max(np.abs(expect)) * 10
    c.close()


def test_g5_hermiticity_on_gpu(gpu):
    lq = gpu
    dims = (4, 4, 6, 8)
    c, U = _ctx(lq, dims, 0.1, 0.5)
    phi = torch.as_tensor(synth.random_spinors(dims, 1, 5).reshape(1, -1)).cuda()
    psi = torch.as_tensor(synth.random_spinors(dims, 1, 6).reshape(1, -1)).cuda()
    lhs = torch.vdot(phi.flatten(), c.apply(psi, op=1).flatten())
    rhs = torch.vdot(c.apply(phi, op=0).flatten(), psi.flatten())
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    c.close()


def test_probes_bit_exact(gpu):
    lq = gpu
    dims = (3, 5, 4, 6)
    c = lq.Context(dims, 0.1)
    z = c.probes(1001, 7, j0=3).cpu().numpy()
    ref = core.probes(1001, 7, 12 * 360, j0=3)
    assert np.array_equal(z.real, ref) and np.all(z.imag == 0)
    c.close()


def test_gauge_errors(gpu):
    lq = gpu
    dims = (2, 2, 2, 4)
    c = lq.Context(dims, 0.1)
    U = synth.su3_links(dims, 0.5, 1)
    bad = U.copy()
    bad[0, 0, 0, 0, 2] *= 1.001
    with pytest.raises(lq.LqtError) as e:
        c.set_gauge(bad)
    assert e.value.code == -5
    bad = U.copy()
    bad[1, 0, 1, 0, 0, 1, 1] = np.nan
    with pytest.raises(lq.LqtError) as e:
        c.set_gauge(bad)
    assert e.value.code == -7
    with pytest.raises(lq.LqtError) as e:  # no valid field held
        c.apply(torch.zeros((1, 12 * 32), dtype=torch.complex128, device="cuda"))
    assert e.value.code == -6
    c.close()


def test_autotuner_choice_keeps_results(gpu):
    lq = gpu
    dims = (8, 8, 8, 8)
    c, U = _ctx(lq, dims, -0.5, 0.5)
    psi = torch.as_tensor(synth.random_spinors(dims, 8, 1).reshape(8, -1)).to(torch.complex64).cuda()
    before = c.apply(psi, prec=1)
    ms = c.tune(1, 8)
    after = c.apply(psi, prec=1)
    assert ms > 0
    assert torch.max(torch.abs(before - after)) < 1e-6 * torch.max(torch.abs(before))
    c.close()
