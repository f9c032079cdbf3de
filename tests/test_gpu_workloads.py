"""The configured workloads at their full sizes, checked on outputs the oracle computes one by
one (sampled probes, sampled aggregates) or through properties that hold at any size."""
import numpy as np
import pytest
import torch

import synth
from oracle import core, prolongator as pr
from paper_1909_12234_amd.workloads import PREC, WORKLOADS

pytestmark = pytest.mark.gpu


def _relres(U, dims, m, b, x):
    r = b - core.apply(U, dims, m, core.OP_A, x)
    return np.linalg.norm(r, axis=1) / np.linalg.norm(b, axis=1)


def test_mixed_16x32_probe_solves(gpu):
    """16^3x32, m = -1.95, the workload's 16-bit inner s-step cycles with FP64 defect correction
    to 1e-8, in the launch configuration of the benchmark (128 probes, autotuned operator
    tiles); 4 sampled solutions are checked with the oracle operator and their samples z^T y
    against the oracle's dot."""
    lq = gpu
    w = WORKLOADS["wilson16x32_mixed"]
    dims, m = w["dims"], w["mass"]
    prec = PREC[w["inner_prec"]]
    print("16^3x32 mixed-precision probe solves", flush=True)
    U = synth.su3_links(dims, w["eps"], w["seed"])
    c = lq.Context(dims, m)
    c.set_gauge(U)
    c.tune(prec, 128)
    z = c.probes(w["probe_seed"], 128)
    y, st, _ = c.solve(z, w["xi"], prec=prec, restart=w["restart"], sstep=w.get("sstep", 0))
    assert all(s[0] for s in st) and max(s[3] for s in st) <= w["xi"]
    pick = [0, 37, 90, 127]
    zs, ys = z[pick].cpu().numpy(), y[pick].cpu().numpy()
    assert np.array_equal(zs.real, core.probes(w["probe_seed"], 128, zs.shape[1])[pick])
    assert np.all(_relres(U, dims, m, zs, ys) <= w["xi"] * 1.05)
    r = c.trace(128, w["probe_seed"], w["xi"], samples=True, prec=prec, restart=w["restart"], sstep=w.get("sstep", 0))
    t = r["samples"].numpy()[pick]
    assert np.max(np.abs(t - np.sum(zs * ys, axis=1))) <= 1e-6 * np.max(np.abs(t))
    c.close()


def test_batched_three_lattices(gpu):
    """8^4, 12^3x24 and 16^3x32 (eps 0.4, seeds 1-3), 64 probes on each lattice solved in
    one batch (every kernel one launch over the three lattices), FP32 storage, FP64 outer
    to 1e-8, graph-captured cycles; sampled solutions checked with the oracle, samples
    against single-lattice contexts."""
    lq = gpu
    w = WORKLOADS["wilson_batched3"]
    lats = [d for d, _ in w["lattices"]]
    links = [synth.su3_links(d, w["eps"], s) for d, s in w["lattices"]]
    print("three lattices in one batch", flush=True)
    c = lq.Context(lats, [w["mass"]] * 3)
    c.set_gauge(np.concatenate([u.ravel() for u in links]))
    per = w["nprobes"] // 3
    res = c.trace_lattices(per, w["probe_seed"], w["xi"], samples=True, prec=lq.F32, restart=16, graph=1)
    assert all(r["nfailed"] == 0 for r in res)
    z = c.probes(w["probe_seed"], 2)
    y, st, _ = c.solve(z, w["xi"], prec=lq.F32, restart=16, graph=1)
    z, y = z.cpu().numpy(), y.cpu().numpy()
    o = 0
    for k, d in enumerate(lats):
        n = 12 * d[0] * d[1] * d[2] * d[3]
        assert np.all(_relres(links[k], d, w["mass"], z[:, o:o + n], y[:, o:o + n]) <= w["xi"] * 1.05)
        t = np.sum(z[:, o:o + n] * y[:, o:o + n], axis=1)
        assert np.max(np.abs(res[k]["samples"].numpy()[:2] - t)) <= 1e-6 * np.max(np.abs(t))
        o += n
    c.close()


def test_net_preconditioned_16x32(gpu):
    """16^3x32 with the transport net as FGMRES right preconditioner: short training, then
    4 probes to 1e-8 with BF16 inner cycles; residuals from the oracle operator and fewer
    Arnoldi steps than plain GMRES on the same probes."""
    lq = gpu
    w = WORKLOADS["wilson16x32_net"]
    dims, m = w["dims"], w["mass"]
    print("16^3x32 FGMRES with the transport net", flush=True)
    U = synth.su3_links(dims, w["eps"], w["seed"])
    c = lq.Context(dims, m)
    c.set_gauge(U)
    c.precond_train(32, seed=5, epochs=4, lr=3e-3, batch=4)
    z = c.probes(w["probe_seed"], 4)
    y, st, _ = c.solve(z, w["xi"], prec=lq.BF16, use_net=1, restart=32)
    _, st0, _ = c.solve(z, w["xi"], prec=lq.BF16, restart=32)
    assert all(s[0] for s in st)
    zs, ys = z.cpu().numpy(), y.cpu().numpy()
    assert np.all(_relres(U, dims, m, zs, ys) <= w["xi"] * 1.05)
    print("steps per probe: net", [s[1] for s in st], "plain", [s[1] for s in st0], flush=True)
    assert sum(s[1] for s in st) < sum(s[1] for s in st0)
    c.close()


def test_prolongator_32x64_sampled_aggregates(gpu):
    """32^3x64, 4^4 aggregates, 24 near-null vectors per chirality: restrict and prolong of
    the full-size prolongator, checked on sampled aggregates against the oracle's sums."""
    lq = gpu
    w = WORKLOADS["wilson32x64_mg"]
    dims, block, nv = w["dims"], w["block"], w["nv"]
    print("32^3x64 prolongator, sampled aggregates", flush=True)
    N = 12 * int(np.prod(dims))
    nagg = int(np.prod([d // b for d, b in zip(dims, block)]))
    d = 6 * int(np.prod(block))
    g = torch.Generator(device="cuda").manual_seed(11)
    W = torch.complex(torch.randn(nagg * 2 * nv * d, generator=g, device="cuda", dtype=torch.float64),
                      torch.randn(nagg * 2 * nv * d, generator=g, device="cuda", dtype=torch.float64))
    c = lq.Context(dims, w["mass"])
    B = c.basis_prolongator_from(block, nv, W)
    y = torch.complex(torch.randn((2, N), generator=g, device="cuda", dtype=torch.float64),
                      torch.randn((2, N), generator=g, device="cuda", dtype=torch.float64))
    cg = B.restrict(y)
    yg = B.prolong(cg)
    idx = pr.fine_index(dims, block)
    Wh = W.view(nagg, 2, nv, d)
    yh = y.cpu().numpy()
    cgh, ygh = cg.cpu().numpy().reshape(2, nagg, 2, nv), yg.cpu().numpy()
    for a in (0, 1, 517, 4096, nagg - 1):
        Wa = Wh[a].cpu().numpy()
        for ch in range(2):
            ref = np.conj(Wa[ch]) @ yh[:, idx[a, ch]].T  # (nv, 2)
            assert np.max(np.abs(cgh[:, a, ch, :].T - ref)) <= 1e-12 * np.max(np.abs(ref))
            back = Wa[ch].T @ cgh[:, a, ch, :].T  # (d, 2)
            assert np.max(np.abs(ygh[:, idx[a, ch]].T - back)) <= 1e-12 * np.max(np.abs(back))
    B.close()
    c.close()
