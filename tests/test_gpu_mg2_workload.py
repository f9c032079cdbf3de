"""Two multigrid levels at the workload's full shape against the oracle: 32^3x64, 4^4
aggregates with 24 near-null vectors per chirality, 2^4 blocks of the 8^3x16 coarse lattice
with 32 near-null vectors of the coarse operator per chirality (the library's own setup).

W and W2 are the library's; the oracle checks what is computed from them with its own code:
W2^+ W2 = I on every level-2 block, and two columns of the level-2 operator (a block on the
last time slice, across the antiperiodic boundary, and an interior one) against
W2^+ W^+ A W W2 e_j formed by the oracle's prolongations, operator and restrictions."""
import numpy as np
import pytest
import torch

import synth
from oracle import core, prolongator as pr
from paper_1909_12234_amd.workloads import PREC, WORKLOADS

pytestmark = pytest.mark.gpu


def test_two_level_workload_full_size_against_oracle(gpu):
    lq = gpu
    w = WORKLOADS["wilson32x64_mg2"]
    dims, m, block, nv, block2, nv2 = w["dims"], w["mass"], w["block"], w["nv"], w["block2"], w["nv2"]
    prec = PREC[w["inner_prec"]]
    print("two-level multigrid 32^3x64: both levels' near-null vectors and operators", flush=True)
    U = synth.su3_links(dims, w["eps"], w["seed"])
    c = lq.Context(dims, m)
    c.set_gauge(U)
    c.tune(prec, nv)
    B = c.basis_prolongator2(block, nv, block2, nv2, 0, null_xi=1e-2, null_maxit=200, prec=prec, restart=w["restart"],
                             sstep=w["sstep"])
    cdims = tuple(L // b for L, b in zip(dims, block))
    nagg1 = int(np.prod(cdims))
    nagg2 = nagg1 // int(np.prod(block2))
    nc2 = 2 * nagg2 * nv2
    W2 = B.prolongator2().cpu().numpy().reshape(nagg2, 2, nv2, -1)
    G = np.matmul(W2.reshape(2 * nagg2, nv2, -1).conj(), W2.reshape(2 * nagg2, nv2, -1).transpose(0, 2, 1))
    assert np.max(np.abs(G - np.eye(nv2)[None])) <= 1e-12
    # columns j of two level-2 blocks: the last one (t = last slice) and one in the middle
    n2 = [L // b for L, b in zip(cdims, block2)]
    A_last = nagg2 - 1
    A_mid = 1 + n2[0] * (2 + n2[1] * (1 + n2[2] * 3))
    cols = [(A_last * 2 + 1) * nv2 + 5, (A_mid * 2 + 0) * nv2 + 17]
    x2 = np.zeros((2, nc2), dtype=np.complex128)
    for r, j in enumerate(cols):
        x2[r, j] = 1.0
    y_gpu = B.coarse2_apply(torch.as_tensor(x2).cuda()).cpu().numpy()
    W1 = B.prolongator().cpu().numpy().reshape(nagg1, 2, nv, -1)
    B.close()
    c.close()
    print("oracle: W W2 e_j, A, W^+, W2^+", flush=True)
    idx2 = pr.coarse_fine_index(cdims, block2, nv)
    nc1 = 2 * nagg1 * nv
    x1 = np.zeros((2, nc1), dtype=np.complex128)
    for r, j in enumerate(cols):
        A2, rem = divmod(j, 2 * nv2)
        ch, v = divmod(rem, nv2)
        x1[r, idx2[A2, ch]] = W2[A2, ch, v]
    xf = pr.prolong(W1, x1, dims, block)
    y1 = pr.restrict(W1, core.apply(U, dims, m, core.OP_A, xf), dims, block)
    del xf
    # y2[A, c, v] = sum_e conj(W2[A, c, v, e]) y1[idx2[A, c, e]]
    y2 = np.einsum("acve,race->racv", W2.conj(), y1[:, idx2]).reshape(2, nc2)
    assert np.max(np.abs(y_gpu - y2)) <= 1e-12 * np.max(np.abs(y2))
