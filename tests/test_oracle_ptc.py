"""Pins of the parallel-transport network oracle (CPU only)."""
import numpy as np

import synth
from oracle import core, ptc


def _wilson_weights(mass):
    """One 4 -> 4 layer that is the Wilson-Dirac operator: (4+m) on the identity path and
    -(1 -/+ gamma_mu)/2 on the +/-mu hops."""
    W = np.zeros((9, 4, 4), dtype=np.complex128)
    W[0] = (4 + mass) * np.eye(4)
    for mu in range(4):
        g = core.gamma(mu)
        W[1 + 2 * mu] = -0.5 * (np.eye(4) - g)
        W[2 + 2 * mu] = -0.5 * (np.eye(4) + g)
    return W


def _random_weights(feats, seed):
    rng = np.random.default_rng(seed)
    n = ptc.weight_count(feats)
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / 6.0


def test_one_layer_with_gamma_weights_is_the_wilson_operator():
    for dims, antiperiodic in (((4, 2, 4, 6), True), ((2, 4, 4, 4), False)):
        U = synth.su3_links(dims, 0.5, 2)
        psi = synth.random_spinors(dims, 2, 3).reshape(2, -1)
        m = -0.3
        out = ptc.forward(U, dims, _wilson_weights(m).ravel(), psi, feats=(4, 4), antiperiodic=antiperiodic)
        ref = core.apply(U, dims, m, core.OP_A, psi, antiperiodic)
        assert np.max(np.abs(out - ref)) < 1e-12 * np.max(np.abs(ref))


def test_identity_network():
    dims = (4, 4, 2, 4)
    U = synth.su3_links(dims, 0.5, 4)
    w = []
    for fi, fo in zip(ptc.FEATURES[:-1], ptc.FEATURES[1:]):
        W = np.zeros((9, fo, fi), dtype=np.complex128)
        W[0] = np.eye(fo, fi)
        w.append(W.ravel())
    psi = synth.random_spinors(dims, 1, 5).reshape(1, -1)
    out = ptc.forward(U, dims, np.concatenate(w), psi)
    assert np.max(np.abs(out - psi)) < 1e-14


def test_gauge_equivariance():
    dims = (4, 4, 2, 4)
    U = synth.su3_links(dims, 0.5, 3)
    omega = synth.random_su3((4, 2, 4, 4), seed=11)
    Ug = synth.gauge_transform(U, omega)
    w = _random_weights(ptc.FEATURES, 1)
    psi = synth.random_spinors(dims, 1, 5)
    lhs = ptc.forward(Ug, dims, w, synth.transform_spinor(psi, omega).reshape(1, -1))
    rhs = synth.transform_spinor(ptc.forward(U, dims, w, psi.reshape(1, -1)).reshape(psi.shape), omega)
    assert np.max(np.abs(lhs - rhs.reshape(1, -1))) < 1e-12 * np.max(np.abs(lhs))
    # and a hop path does depend on the links (the test is not vacuous)
    assert np.max(np.abs(ptc.forward(Ug, dims, w, psi.reshape(1, -1)) - ptc.forward(U, dims, w, psi.reshape(1, -1)))) > 1e-3


def test_layer_composition_is_linear():
    dims = (2, 2, 4, 4)
    U = synth.su3_links(dims, 0.5, 6)
    w = _random_weights(ptc.FEATURES, 2)
    a = synth.random_spinors(dims, 2, 7).reshape(2, -1)
    out = ptc.forward(U, dims, w, np.stack([a[0], a[1], 2.0 * a[0] - 1j * a[1]]))
    assert np.max(np.abs(out[2] - (2.0 * out[0] - 1j * out[1]))) < 1e-12 * np.max(np.abs(out))


def test_fd_gradient_matches_the_closed_form_of_a_site_local_layer():
    """For one 4 -> 4 layer with only identity-path weights W0, M r = W0 r per site and
    L = (1/Q) sum_q ||W0 R_q - E_q||^2 / ||e_q||^2, whose gradient is
    dL/dconj(W0) = (1/Q) sum_q (W0 R_q - E_q) R_q^H / ||e_q||^2 (R_q, E_q as 4 x 3V)."""
    dims, m = (2, 2, 2, 4), 0.2
    U = synth.su3_links(dims, 0.5, 8)
    V = core.volume(dims)
    rng = np.random.default_rng(3)
    W = np.zeros((9, 4, 4), dtype=np.complex128)
    W[0] = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    e = synth.random_spinors(dims, 2, 9).reshape(2, -1)
    r = core.apply(U, dims, m, core.OP_A, e)
    G = np.zeros((4, 4), dtype=np.complex128)
    for q in range(2):
        R = r[q].reshape(V, 4, 3).transpose(1, 0, 2).reshape(4, -1)
        E = e[q].reshape(V, 4, 3).transpose(1, 0, 2).reshape(4, -1)
        G += (W[0] @ R - E) @ R.conj().T / np.sum(np.abs(e[q]) ** 2)
    G /= 2
    fd = ptc.loss_grad_fd(U, dims, m, W.ravel(), e, list(range(16)), feats=(4, 4))
    assert np.max(np.abs(fd - G.ravel())) < 1e-8 * np.max(np.abs(G))
    # a hop weight's gradient is not the site-local one: nonzero and finite
    fd_hop = ptc.loss_grad_fd(U, dims, m, W.ravel(), e, [16, 40], feats=(4, 4))
    assert np.all(np.isfinite(fd_hop)) and np.max(np.abs(fd_hop)) > 0


def _identity_weights():
    w = []
    for fi, fo in zip(ptc.FEATURES[:-1], ptc.FEATURES[1:]):
        W = np.zeros((9, fo, fi), dtype=np.complex128)
        W[0] = np.eye(fo, fi)
        w.append(W.ravel())
    return np.concatenate(w)


def test_loss_of_the_zero_network_is_one():
    """M = 0 maps every residual to 0: each pair contributes ||e||^2 / ||e||^2 = 1"""
    dims = (2, 4, 2, 4)
    U = synth.su3_links(dims, 0.5, 6)
    e = synth.random_spinors(dims, 3, 7).reshape(3, -1)
    assert abs(ptc.loss(U, dims, -0.2, np.zeros(ptc.weight_count(), dtype=np.complex128), e) - 1.0) < 1e-14


def test_loss_of_the_identity_network():
    """M = 1: the loss is the mean over the pairs of ||A e - e||^2 / ||e||^2, the mean taken
    pair by pair (two fields of very different norms)"""
    dims = (2, 4, 2, 4)
    U = synth.su3_links(dims, 0.5, 8)
    m = -0.2
    e = synth.random_spinors(dims, 2, 9).reshape(2, -1)
    e[1] *= 1e3
    ae = core.apply(U, dims, m, core.OP_A, e)
    per = [np.sum(np.abs(ae[q] - e[q]) ** 2) / np.sum(np.abs(e[q]) ** 2) for q in range(2)]
    assert abs(ptc.loss(U, dims, m, _identity_weights(), e) - 0.5 * (per[0] + per[1])) <= 1e-12 * max(per)
