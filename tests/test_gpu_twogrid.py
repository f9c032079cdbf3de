"""Two-grid preconditioner from the prolongator (Section 2; lqt_precond_twogrid) against the
oracle: one application with a tightly solved coarse system equals the oracle's exact coarse
grid correction followed by the same minimal-residual smoothing; with a unitary W it is
A^{-1}; inside FGMRES it meets the FP64 true residual (recomputed by the oracle) in fewer
Arnoldi steps than plain GMRES; and the trace accepts it."""
import numpy as np
import pytest
import torch

import synth
from oracle import core, prolongator as pr, twogrid

pytestmark = pytest.mark.gpu


def _W(dims, block, nv, seed=3):
    rng = np.random.default_rng(seed)
    N = 12 * int(np.prod(dims))
    Y = rng.standard_normal((nv, N)) + 1j * rng.standard_normal((nv, N))
    return pr.block_orthonormalize(Y, dims, block)


@pytest.mark.parametrize("dims,block,nv,nu", [((4, 4, 4, 4), (2, 2, 2, 2), 6, 0), ((4, 4, 4, 4), (2, 2, 2, 2), 6, 3),
                                              ((4, 4, 2, 8), (2, 2, 2, 4), 5, 2)])
def test_twogrid_apply_matches_oracle(gpu, dims, block, nv, nu):
    lq = gpu
    m = 0.1
    print(f"two-grid apply dims={dims} block={block} nv={nv} smoothing={nu}", flush=True)
    U = synth.su3_links(dims, 0.4, 1)
    W = _W(dims, block, nv)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator_from(block, nv, torch.as_tensor(W.reshape(-1)).cuda())
    c.precond_twogrid(B)
    rng = np.random.default_rng(8)
    N = 12 * int(np.prod(dims))
    r = rng.standard_normal((5, N)) + 1j * rng.standard_normal((5, N))
    x = c.precond_twogrid_apply(torch.as_tensor(r).cuda(), tg_smooth=nu if nu else -1, tg_coarse_tol=1e-13,
                                tg_coarse_maxit=2000).cpu().numpy()
    ref = twogrid.apply(U, dims, m, W, block, r, nu)
    assert np.max(np.abs(x - ref)) <= 1e-9 * np.max(np.abs(ref))
    B.close()
    with pytest.raises(lq.LqtError):  # freeing the basis cleared the preconditioner
        c.precond_twogrid_apply(torch.as_tensor(r).cuda())
    c.close()


def test_unitary_prolongator_gives_the_inverse(gpu):
    lq = gpu
    dims, m = (4, 4, 4, 4), 0.2
    U = synth.su3_links(dims, 0.4, 2)
    W = _W(dims, (1, 1, 1, 1), 6)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator_from((1, 1, 1, 1), 6, torch.as_tensor(W.reshape(-1)).cuda())
    c.precond_twogrid(B)
    rng = np.random.default_rng(9)
    r = rng.standard_normal((2, 3072)) + 0j
    x = c.precond_twogrid_apply(torch.as_tensor(r).cuda(), tg_smooth=-1, tg_coarse_tol=1e-12,
                                tg_coarse_maxit=4000).cpu().numpy()
    res = r - core.apply(U, dims, m, core.OP_A, x)
    assert np.max(np.linalg.norm(res, axis=1) / np.linalg.norm(r, axis=1)) <= 1e-10
    B.close()
    c.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_fgmres_with_twogrid_meets_the_true_residual(gpu, prec):
    """8^4 near the spectral edge: near-null vectors from the library's own solves, 2^4
    aggregates with 12 vectors per chirality; FGMRES(16) with the two-grid preconditioner in
    FP32 or FP16 storage against plain GMRES(16), the oracle recomputing every residual."""
    lq = gpu
    dims, m = (8, 8, 8, 8), -0.6
    U = synth.su3_links(dims, 0.4, 4)
    c = lq.Context(dims, m)
    c.set_gauge(U)
    B = c.basis_prolongator((2, 2, 2, 2), 12, 0, null_xi=1e-2, null_maxit=200, prec=1)
    c.precond_twogrid(B)
    rng = np.random.default_rng(10)
    N = 12 * 4096
    b = rng.standard_normal((6, N)) + 1j * rng.standard_normal((6, N))
    x_tg, st_tg = c.solve(torch.as_tensor(b).cuda(), 1e-8, prec=prec, restart=16, twogrid=1, tg_smooth=4,
                          tg_coarse_tol=0.05, tg_coarse_maxit=64)[:2]
    x_pl, st_pl = c.solve(torch.as_tensor(b).cuda(), 1e-8, prec=prec, restart=16)[:2]
    it_tg = sum(s[1] for s in st_tg)
    it_pl = sum(s[1] for s in st_pl)
    print(f"prec {prec}: Arnoldi steps two-grid {it_tg}, plain {it_pl}", flush=True)
    for x in (x_tg, x_pl):
        xh = x.cpu().numpy()
        res = b - core.apply(U, dims, m, core.OP_A, xh)
        assert np.max(np.linalg.norm(res, axis=1) / np.linalg.norm(b, axis=1)) <= 1e-8
    assert it_tg * 2 < it_pl
    # the trace takes the option; both runs solve the same probes to 1e-8
    r_tg = c.trace(8, 1040, 1e-8, samples=True, prec=prec, restart=16, twogrid=1, tg_coarse_tol=0.05)
    r_pl = c.trace(8, 1040, 1e-8, samples=True, prec=prec, restart=16)
    assert r_tg["nfailed"] == 0
    d = np.abs(r_tg["samples"].numpy() - r_pl["samples"].numpy())
    assert np.max(d) <= 1e-5 * np.max(np.abs(r_pl["samples"].numpy()))
    with pytest.raises(lq.LqtError):
        c.solve(torch.as_tensor(b[:1]).cuda(), 1e-8, prec=2, restart=8, sstep=1, twogrid=1)
    B.close()
    with pytest.raises(lq.LqtError):  # no preconditioner basis any more
        c.solve(torch.as_tensor(b[:1]).cuda(), 1e-8, prec=prec, restart=16, twogrid=1)
    c.close()
