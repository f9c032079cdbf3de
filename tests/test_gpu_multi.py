"""Several lattices in one context: one launch per kernel over all of them, checked per
lattice against the oracle and against single-lattice contexts."""
import numpy as np
import pytest
import torch

import synth
from oracle import core

pytestmark = pytest.mark.gpu

LATS = [(4, 4, 4, 4), (2, 4, 6, 4), (6, 4, 4, 8)]  # volumes 256, 192 (ragged: not a block), 768
MASSES = [-0.4, 0.1, -0.2]
TOL = {0: 1e-12, 1: 1e-5, 3: 4e-2}


def _setup(lq, lats=LATS, masses=MASSES, seed=1):
    links = [synth.su3_links(d, 0.5, seed + k) for k, d in enumerate(lats)]
    c = lq.Context(lats, masses)
    c.set_gauge(np.concatenate([u.ravel() for u in links]))
    return c, links


def _split(x, lats):
    out, o = [], 0
    for d in lats:
        n = 12 * d[0] * d[1] * d[2] * d[3]
        out.append(x[..., o:o + n])
        o += n
    return out


def _fields(lats, nrhs, seed):
    return np.concatenate([synth.random_spinors(d, nrhs, seed + k).reshape(nrhs, -1) for k, d in enumerate(lats)],
                          axis=1)


@pytest.mark.parametrize("op", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", [0, 1, 3])
def test_dslash_per_lattice_matches_oracle(gpu, op, prec):
    lq = gpu
    print(f"multi-lattice dslash op={op} prec={prec}", flush=True)
    c, links = _setup(lq)
    psi = _fields(LATS, 3, 7)
    dt = torch.complex128 if prec == 0 else torch.complex64
    out = c.apply(torch.as_tensor(psi).to(dt).cuda(), op=op, prec=prec).cpu().numpy().astype(np.complex128)
    for k, (d, o, p) in enumerate(zip(LATS, _split(out, LATS), _split(psi, LATS))):
        ref = core.apply(links[k], d, MASSES[k], op, p)
        assert np.max(np.abs(o - ref)) <= TOL[prec] * np.max(np.abs(ref)), (k, d)
    c.close()


def test_probes_restrict_to_single_lattice_probes(gpu):
    lq = gpu
    c, _ = _setup(lq)
    z = c.probes(4321, 5, j0=3).cpu().numpy()
    for k, (d, zk) in enumerate(zip(LATS, _split(z, LATS))):
        ref = core.probes(4321, 5, 12 * d[0] * d[1] * d[2] * d[3], j0=3)
        assert np.array_equal(zk.real, ref) and not np.any(zk.imag)
    c.close()


@pytest.mark.parametrize("prec", [0, 3])
def test_solve_meets_xi_on_every_lattice(gpu, prec):
    lq = gpu
    c, links = _setup(lq)
    xi = 1e-9
    b = _fields(LATS, 4, 11)
    b[2, 12 * 256:12 * (256 + 192)] = 0  # one right-hand side without a source on lattice 1
    x, st, _ = c.solve(torch.as_tensor(b).cuda(), xi, prec=prec, restart=16)
    x = x.cpu().numpy()
    assert all(s[0] for s in st)
    for k, (d, xk, bk) in enumerate(zip(LATS, _split(x, LATS), _split(b, LATS))):
        r = bk - core.apply(links[k], d, MASSES[k], core.OP_A, xk)
        for q in range(4):
            nb = np.linalg.norm(bk[q])
            if nb == 0:
                assert np.linalg.norm(xk[q]) == 0
            else:
                assert np.linalg.norm(r[q]) <= xi * nb * 1.05, (k, q)
    c.close()


def test_trace_lattices_matches_single_lattice_contexts(gpu):
    lq = gpu
    c, links = _setup(lq)
    nprobes, seed, xi = 6, 99, 1e-10
    res = c.trace_lattices(nprobes, seed, xi, samples=True, prec=0)
    assert len(res) == len(LATS)
    for k, d in enumerate(LATS):
        ck = lq.Context(d, MASSES[k])
        ck.set_gauge(links[k])
        rk = ck.trace(nprobes, seed, xi, samples=True, prec=0)
        # the same probes, solved to xi: the samples agree to the solve accuracy
        s_multi, s_single = res[k]["samples"].numpy(), rk["samples"].numpy()
        assert np.max(np.abs(s_multi - s_single)) <= 1e-6 * np.max(np.abs(s_single)), k
        assert abs(res[k]["trace_re"] - rk["trace_re"]) <= 1e-6 * abs(rk["trace_re"])
        # and the oracle's samples from its own solves
        N = 12 * d[0] * d[1] * d[2] * d[3]
        z = core.probes(seed, nprobes, N)
        y = np.stack([core.gmres(links[k], d, MASSES[k], zj.astype(np.complex128), 1e-12)[0] for zj in z])
        t_or = np.sum(z * y, axis=1)
        assert np.max(np.abs(s_multi - t_or)) <= 1e-6 * np.max(np.abs(t_or)), k
        ck.close()
    c.close()


def test_single_lattice_only_calls_reject_several_lattices(gpu):
    lq = gpu
    c, _ = _setup(lq)
    with pytest.raises(lq.LqtError) as ei:
        c.trace(4, 1, 1e-6)
    assert ei.value.code == lq.LQT_EINVAL
    with pytest.raises(lq.LqtError) as ei:
        c.basis_eig(4, xi=1e-2)
    assert ei.value.code == lq.LQT_EINVAL
    c.close()
