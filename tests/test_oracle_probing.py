"""Pins of the oracle's partition basis (spin-colour dilution and hierarchical probing,
Section 1) against what the construction must satisfy: the red-black signs written out site by
site, the closing colours as congruence classes modulo 2^i at least 2^i apart, exactness of
dilution for matrices that couple only the components of one site, exactness of red-black
probing with dilution for the nearest-neighbour Wilson operator, the one-draw variance formula
against enumeration of every sign vector, and the empirical variance of many draws."""
import itertools

import numpy as np
import pytest

import synth
from oracle import core, dense, probing


def _torus_dist(a, b, dims):
    d = 0
    for u, v, L in zip(a, b, dims):
        du = abs(u - v)
        d += min(du, L - du)
    return d


def test_first_two_signs_are_one_and_red_black():
    dims = (4, 2, 2, 6)
    assert np.all(probing.hp_sign(dims, 0) == 1.0)
    h1 = probing.hp_sign(dims, 1)
    s = 0
    for t in range(dims[3]):
        for z in range(dims[2]):
            for y in range(dims[1]):
                for x in range(dims[0]):
                    assert h1[s] == (-1.0) ** (x + y + z + t)
                    s += 1


@pytest.mark.parametrize("dims,k,i", [((4, 4, 4, 4), 16, 1), ((2, 4, 2, 6), 16, 1), ((8, 4, 4, 8), 256, 2)])
def test_closing_colours_are_congruence_classes(dims, k, i):
    """(1/k) sum_m h_m(a) h_m(b) at k = 2^{4i} is 1 where a and b agree modulo 2^i in every
    direction and 0 elsewhere; distinct sites of one class are at least 2^i apart."""
    Hs = np.array([probing.hp_sign(dims, m) for m in range(k)])
    M = Hs.T @ Hs / k
    c = np.stack(probing.coords(dims), axis=1)
    same = np.all((c[:, None, :] % (1 << i)) == (c[None, :, :] % (1 << i)), axis=2)
    assert np.array_equal(M, same.astype(float))
    # distinct sites of one class are at least 2^i apart on the torus
    a_idx, b_idx = np.nonzero(np.triu(same, 1))
    dmin = min(_torus_dist(c[a], c[b], dims) for a, b in zip(a_idx[:5000], b_idx[:5000]))
    assert dmin >= (1 << i)


def test_red_black_weight_is_same_parity():
    dims = (4, 4, 2, 2)
    Hs = np.array([probing.hp_sign(dims, m) for m in range(2)])
    c = np.stack(probing.coords(dims), axis=1)
    par = c.sum(axis=1) % 2
    assert np.array_equal(Hs.T @ Hs / 2, (par[:, None] == par[None, :]).astype(float))


def test_probing_vectors_are_orthogonal_characters():
    dims = (4, 4, 4, 8)
    Hs = np.array([probing.hp_sign(dims, m) for m in range(32)])
    assert np.array_equal(Hs @ Hs.T, Hs.shape[1] * np.eye(32))


def test_check_dims():
    with pytest.raises(ValueError):
        probing.check_dims((4, 4, 4, 4), 3)
    with pytest.raises(ValueError):
        probing.check_dims((4, 4, 4, 6), 32)  # level 1 needs extents divisible by 4
    probing.check_dims((4, 4, 4, 6), 16)


def test_dilution_is_exact_for_site_local_matrices():
    """A matrix that couples only the 12 components of one site: with dilution every pair of
    one component sits on two different sites, where B vanishes."""
    dims = (2, 2, 2, 2)
    V = 16
    rng = np.random.default_rng(3)
    blocks = rng.standard_normal((V, 12, 12)) + 1j * rng.standard_normal((V, 12, 12))
    B = np.zeros((12 * V, 12 * V), dtype=complex)
    for s in range(V):
        B[12 * s:12 * s + 12, 12 * s:12 * s + 12] = blocks[s]
    tr = np.trace(B)
    t = probing.estimator_samples(lambda X: X @ B.T, 7, 3, dims, 1, True)
    assert np.max(np.abs(t - tr)) <= 1e-12 * abs(tr)
    t_plain = probing.estimator_samples(lambda X: X @ B.T, 7, 3, dims, 1, False)
    assert np.max(np.abs(t_plain - tr)) > 1e-3 * abs(tr)


@pytest.mark.parametrize("k", [2, 16])
def test_red_black_with_dilution_is_exact_for_the_wilson_operator(k):
    """A couples a site only to itself and its nearest neighbours, which have the other
    parity: red-black probing with dilution gives tr A = 12 V (4 + m) in every draw (and
    so does every later closing of the nested colourings)."""
    dims, m = (4, 4, 4, 4), 0.3
    U = synth.su3_links(dims, 0.5, 2)
    tr = 12 * 256 * (4 + m)
    t = probing.estimator_samples(lambda X: core.apply(U, dims, m, core.OP_A, X), 11, 2, dims, k, True)
    assert np.max(np.abs(t - tr)) <= 1e-12 * tr
    t1 = probing.estimator_samples(lambda X: core.apply(U, dims, m, core.OP_A, X), 11, 2, dims, 1, True)
    assert np.max(np.abs(t1 - tr)) > 1e-3 * tr


def test_variance_formula_against_enumeration():
    """All 2^12 sign vectors on 12 unknowns: the mean of |z^T B z - tr B|^2 equals the
    formula (no probing, no dilution: every pair weighs 1)."""
    rng = np.random.default_rng(5)
    B = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
    tr = np.trace(B)
    acc = 0.0
    for bits in itertools.product((1.0, -1.0), repeat=12):
        z = np.array(bits)
        acc += abs(z @ B @ z - tr) ** 2
    assert abs(acc / 4096 - probing.exact_variance(B, np.ones((12, 12)))) <= 1e-10 * acc / 4096


def test_partitioned_estimator_statistics():
    """Draws on 2^4 (N = 192) of tr A^{-1} with red-black probing and dilution: the mean is
    within 4 standard errors of the exact trace and the sample variance within a chi^2 band
    of the formula; the formula's variances fall as the partition refines."""
    dims, m = (2, 2, 2, 2), 0.2
    U = synth.su3_links(dims, 0.4, 1)
    Ai = np.linalg.inv(dense.dense_operator(U, dims, m))
    tr = np.trace(Ai)
    s = 3000
    t = probing.estimator_samples(lambda X: X @ Ai.T, 21, s, dims, 2, True)
    v_exact = probing.exact_variance(Ai, probing.class_mask(dims, 2, True))
    assert abs(t.mean() - tr) <= 4 * np.sqrt(v_exact / s)
    v_emp = np.sum(np.abs(t - t.mean()) ** 2) / (s - 1)
    assert 0.8 * v_exact <= v_emp <= 1.2 * v_exact
    v_plain = probing.exact_variance(Ai, probing.class_mask(dims, 1, False))
    v_dil = probing.exact_variance(Ai, probing.class_mask(dims, 1, True))
    assert v_exact < v_dil < v_plain
    # 2^4 at 16 probing vectors: every site its own class, the diluted estimate is exact
    assert probing.exact_variance(Ai, probing.class_mask(dims, 16, True)) == 0.0
