"""Partition basis H of Algorithms 1 and 2: spin-colour dilution and hierarchical probing
(Section 1, the partitioning paragraph), written out in numpy (oracle).

TEST INFRASTRUCTURE ONLY: used by tests/ and never by the product library.

The paper names hierarchical probing, its nested colourings at growing lattice distance and
its closing colours k = 2^{D i} (D = 4), but prints no construction.  The reading taken here:
probing vector m (0 <= m < k = 2^b) takes at site x the sign

    h_m(x) = prod over the set bits beta of m of (-1)^{f_beta(x)},

with the nested bit functions of level l = beta // 4 on the coordinate bits
x_l = (x >> l) & 1 (likewise y_l, z_l, t_l):

    f_{4l}   = x_l + y_l + z_l + t_l (mod 2)   (the red-black partition of level l)
    f_{4l+1} = x_l,   f_{4l+2} = y_l,   f_{4l+3} = z_l.

The four functions of a level are an invertible map of its four coordinate bits, so the
first 2^{4i} vectors span the indicators of the 2^{4i} classes of sites that agree modulo
2^i in every direction (two sites of one class are at least 2^i apart), and k = 2 is the
red-black partition.  Spin-colour dilution splits each vector into 12, one per spin-colour
component.  A draw j of the estimator takes the Rademacher probe z_j on the vectors

    v_{j,m,c} = z_j (.) h_m (.) e_c    (e_c: component c at every site; all 12 without dilution)

and forms t_j = (1/k) sum_{m < k} sum_c v^T B v: an unbiased estimate of tr B (the paper's
t(B (.) H H^+) with H the k columns h_m / sqrt(k), diluted) whose variance sums
|B_ab + B_ba|^2 over the pairs a < b of one class and, with dilution, one component.
Lattice extents must be multiples of 2^{l+1} for the highest level l in use.
"""
import numpy as np

from . import core


def coords(dims):
    """Site coordinates (x, y, z, t), each of shape (V,), site index x + Lx (y + Ly (z + Lz t))."""
    lx, ly, lz, lt = dims
    s = np.arange(lx * ly * lz * lt)
    return s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)


def check_dims(dims, k):
    """The probing count must be a power of two whose levels divide every extent."""
    if k < 1 or (k & (k - 1)):
        raise ValueError("the number of probing vectors must be a power of two")
    b = k.bit_length() - 1
    if b == 0:
        return
    top = (b - 1) // 4  # highest level in use
    if any(L % (2 << top) for L in dims):
        raise ValueError(f"extents must be multiples of {2 << top} for {k} probing vectors")


def hp_sign(dims, m):
    """h_m at every site, shape (V,), entries +-1."""
    x, y, z, t = coords(dims)
    par = np.zeros(x.shape, dtype=np.int64)
    beta = 0
    while m >> beta:
        if (m >> beta) & 1:
            lvl, which = beta // 4, beta % 4
            xl, yl, zl, tl = (x >> lvl) & 1, (y >> lvl) & 1, (z >> lvl) & 1, (t >> lvl) & 1
            par += (xl + yl + zl + tl, xl, yl, zl)[which]
        beta += 1
    return 1.0 - 2.0 * (par & 1)


def partition_vectors(seed, j, dims, k, dilute):
    """The q = k (12 with dilution) real vectors of draw j, shape (q, N), in the order
    (m, c): row m * nd + c, nd = 12 with dilution, else 1."""
    check_dims(dims, k)
    V = int(np.prod(dims))
    N = 12 * V
    z = core.probes(seed, 1, N, j0=j)[0]
    comp = np.arange(N) % 12
    rows = []
    for m in range(k):
        hv = np.repeat(hp_sign(dims, m), 12) * z
        if dilute:
            for c in range(12):
                rows.append(np.where(comp == c, hv, 0.0))
        else:
            rows.append(hv)
    return np.array(rows)


def draw_samples(per_vector, q, k):
    """t_j = (1/k) sum of the q per-vector values of draw j: (s*q,) -> (s,)."""
    per_vector = np.asarray(per_vector)
    return per_vector.reshape(-1, q).sum(axis=1) / k


def estimator_samples(B_apply, seed, s, dims, k, dilute):
    """The s draws t_j = (1/k) sum_{m,c} v^T B v with B given by its action on rows
    (B_apply: (q, N) -> (q, N))."""
    out = []
    for j in range(s):
        Vj = partition_vectors(seed, j, dims, k, dilute)
        out.append(np.einsum("pn,pn->", Vj, B_apply(Vj)) / k)
    return np.array(out)


def class_mask(dims, k, dilute):
    """Weight of the pair (a, b) in the estimator: (1/k) sum_m h_m(a) h_m(b) (times the
    same-component indicator with dilution), as an N x N array."""
    V = int(np.prod(dims))
    Hs = np.array([np.repeat(hp_sign(dims, m), 12) for m in range(k)])
    M = Hs.T @ Hs / k
    if dilute:
        comp = np.arange(12 * V) % 12
        M = M * (comp[:, None] == comp[None, :])
    return M


def exact_variance(B, mask):
    """Variance E|t - tr B|^2 of one draw: sum over a < b of mask_ab |B_ab + B_ba|^2 (real
    +-1 probes: t - tr B = sum_{a<b} z_a z_b mask_ab (B_ab + B_ba), the products z_a z_b of
    distinct pairs being uncorrelated with unit variance)."""
    S = B + B.T
    iu = np.triu_indices(B.shape[0], 1)
    return float(np.sum(mask[iu] * np.abs(S[iu]) ** 2))
