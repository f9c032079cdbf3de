"""Multigrid prolongator of Algorithm 2, written out in numpy (oracle).

TEST INFRASTRUCTURE ONLY: used by tests/ and never by the product library.

Section 2 (blocking): the near-null vectors Y are cut into pieces supported on disjoint
aggregates D_j; for the Wilson operator each piece is also split by chirality (spins {0,1}
and {2,3}) so that g5 W = W g5^W, and each block is orthonormalised.  Here W is stored as
an array of shape (nagg, 2, nv, d), d = 6 * sites per block, with local index
e = bs * 6 + s2 * 3 + colour (bs = site inside the block with x fastest, spin = 2 c + s2),
and the coarse index (a, c, v) flattened in that order.  Fine vectors use the canonical
index 12 * site + 3 * spin + colour.

Second level (Table 2: blocks of the coarse lattice): the level-1 coarse lattice (one site per
aggregate, x fastest) is blocked again; a level-2 block (A, c) gathers the chirality-c entries
(a1, c, v1) of its level-1 sites, local index e = ls * nv1 + v1 (ls = site inside the block,
x fastest), so W2 has shape (nagg2, 2, nv2, bsites2 * nv1) and g5^{W1} W2 = W2 g5^{W2}.
"""
import numpy as np


def aggregates(dims, block):
    """site[a, bs]: lattice site of local site bs of aggregate a (both x-fastest)."""
    lx, ly, lz, lt = dims
    b0, b1, b2, b3 = block
    n0, n1, n2, n3 = lx // b0, ly // b1, lz // b2, lt // b3
    nagg, bsites = n0 * n1 * n2 * n3, b0 * b1 * b2 * b3
    site = np.empty((nagg, bsites), dtype=np.int64)
    for a in range(nagg):
        ax, ay, az, at = a % n0, (a // n0) % n1, (a // (n0 * n1)) % n2, a // (n0 * n1 * n2)
        for bs in range(bsites):
            bx, by, bz, bt = bs % b0, (bs // b0) % b1, (bs // (b0 * b1)) % b2, bs // (b0 * b1 * b2)
            x, y, z, t = ax * b0 + bx, ay * b1 + by, az * b2 + bz, at * b3 + bt
            site[a, bs] = x + lx * (y + ly * (z + lz * t))
    return site


def fine_index(dims, block):
    """idx[a, c, e]: canonical fine index of local dof e of block (a, c)."""
    site = aggregates(dims, block)
    nagg, bsites = site.shape
    idx = np.empty((nagg, 2, 6 * bsites), dtype=np.int64)
    for c in range(2):
        for bs in range(bsites):
            for s2 in range(2):
                for col in range(3):
                    idx[:, c, bs * 6 + s2 * 3 + col] = 12 * site[:, bs] + 3 * (2 * c + s2) + col
    return idx


def coarse_fine_index(cdims, block2, nv1):
    """idx[A, c, e]: level-1 coarse index (a1 * 2 + c) * nv1 + v1 of entry e = ls * nv1 + v1
    of level-2 block (A, c)."""
    site = aggregates(cdims, block2)
    nagg2, bs2 = site.shape
    idx = np.empty((nagg2, 2, bs2 * nv1), dtype=np.int64)
    for c in range(2):
        for ls in range(bs2):
            for v1 in range(nv1):
                idx[:, c, ls * nv1 + v1] = (site[:, ls] * 2 + c) * nv1 + v1
    return idx


def block_orthonormalize(Y, dims, block, idx=None):
    """W from fine vectors Y (nv, N): restrict each vector to every (aggregate, chirality)
    block and run modified Gram-Schmidt twice inside the block (idx: the blocks' index map,
    default the fine lattice's; coarse_fine_index for the second level)."""
    if idx is None:
        idx = fine_index(dims, block)
    nagg, _, d = idx.shape
    nv = Y.shape[0]
    W = np.empty((nagg, 2, nv, d), dtype=np.complex128)
    for a in range(nagg):
        for c in range(2):
            B = Y[:, idx[a, c]].copy()
            for _ in range(2):
                for v in range(nv):
                    for u in range(v):
                        B[v] -= np.vdot(B[u], B[v]) * B[u]
                    nrm = np.linalg.norm(B[v])
                    B[v] = B[v] / nrm if nrm > 1e-300 else 0.0
            W[a, c] = B
    return W


def dense_prolongator(W, dims, block, idx=None, N=None):
    """P as an N x nc matrix (columns = prolongated unit coarse vectors); idx and N for the
    second level (coarse_fine_index, N = nc1)."""
    if idx is None:
        idx = fine_index(dims, block)
    nagg, _, nv, d = W.shape
    if N is None:
        N = 12 * int(np.prod(dims))
    P = np.zeros((N, nagg * 2 * nv), dtype=np.complex128)
    for a in range(nagg):
        for c in range(2):
            for v in range(nv):
                P[idx[a, c], (a * 2 + c) * nv + v] = W[a, c, v]
    return P


def restrict(W, y, dims, block):
    """coarse[r] = W^+ y[r] for y of shape (nrhs, N)."""
    idx = fine_index(dims, block)
    nagg, _, nv, d = W.shape
    out = np.zeros((y.shape[0], nagg, 2, nv), dtype=np.complex128)
    for a in range(nagg):
        for c in range(2):
            out[:, a, c, :] = y[:, idx[a, c]] @ W[a, c].conj().T
    return out.reshape(y.shape[0], -1)


def prolong(W, cvec, dims, block):
    """y[r] = W coarse[r] for coarse of shape (nrhs, nc)."""
    idx = fine_index(dims, block)
    nagg, _, nv, d = W.shape
    N = 12 * int(np.prod(dims))
    cc = cvec.reshape(cvec.shape[0], nagg, 2, nv)
    out = np.zeros((cvec.shape[0], N), dtype=np.complex128)
    for a in range(nagg):
        for c in range(2):
            out[:, idx[a, c]] = cc[:, a, c, :] @ W[a, c]
    return out


def coarse_g5(nagg, nv):
    """Diagonal of g5^W in the coarse index (a, c, v): +1 for c = 0, -1 for c = 1."""
    return np.tile(np.repeat([1.0, -1.0], nv), nagg)
