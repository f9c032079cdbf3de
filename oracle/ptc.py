"""Oracle of the gauge-equivariant parallel-transport network preconditioner (test
infrastructure only: imported by the tests, the smoke check and the CPU baseline).

The network is a chain of linear layers over colour-vector features; one layer maps
    out_f(x) = sum_p sum_g W[p][f][g] (T_p v_g)(x)
over the nine paths p = 0 (identity), 1+2mu (hop +mu with U_mu(x)) and 2+2mu (hop -mu with
U_mu(x-mu)^+), the links carrying the antiperiodic time boundary sign of the fermion
operator.  The forward pass is the C oracle (orc_ptc_forward, FP64).  The training loss of
a weight vector W on error fields e_q is
    L(W) = (1/Q) sum_q ||M_W (A e_q) - e_q||^2 / ||e_q||^2 .
Its gradient is taken by central differences: M_W is linear in every single weight, so L is
a quadratic polynomial along every real coordinate of W and the central difference is its
exact derivative (up to rounding), whatever the step.

Pins (tests/test_oracle_ptc.py): a one-layer network with weights (4+m) at p = 0 and
-(1 -/+ gamma_mu)/2 on the +/-mu hops is the Wilson-Dirac operator; gauge equivariance;
the identity network; the closed-form gradient of a site-local layer.
"""
import numpy as np

from . import core

FEATURES = (4, 8, 8, 8, 4)


def weight_count(feats=FEATURES):
    return sum(9 * a * b for a, b in zip(feats[:-1], feats[1:]))


def split_weights(w, feats=FEATURES):
    """Flat complex vector (layer by layer, [p][f][g]) -> list of (9, F_out, F_in) arrays."""
    w = np.asarray(w, dtype=np.complex128).ravel()
    out, off = [], 0
    for fi, fo in zip(feats[:-1], feats[1:]):
        out.append(w[off:off + 9 * fo * fi].reshape(9, fo, fi))
        off += 9 * fo * fi
    assert off == w.size
    return out


def forward(links, dims, w, v, feats=FEATURES, antiperiodic=True):
    """M_W v for spinor fields v (nrhs, 12V) or (12V,); features = spins for a spinor."""
    V = core.volume(dims)
    x = np.asarray(v, dtype=np.complex128).reshape(-1, V * feats[0] * 3)
    ws = split_weights(w, feats)
    out = np.stack([core.ptc_forward(links, dims, feats, ws, xi, antiperiodic).ravel() for xi in x])
    return out


def loss(links, dims, mass, w, e, feats=FEATURES, antiperiodic=True):
    """Mean over the fields e of ||M_W (A e) - e||^2 / ||e||^2: the training objective of the
    learned preconditioner (an addition to the paper's method), which maps residuals to
    errors."""
    e = np.asarray(e, dtype=np.complex128).reshape(-1, 12 * core.volume(dims))
    r = core.apply(links, dims, mass, core.OP_A, e, antiperiodic)
    m = forward(links, dims, w, r, feats, antiperiodic)
    return float(np.mean(np.sum(np.abs(m - e) ** 2, axis=1) / np.sum(np.abs(e) ** 2, axis=1)))


def loss_grad_fd(links, dims, mass, w, e, indices, h=1e-2, feats=FEATURES, antiperiodic=True):
    """dL/dconj(W_i) = (dL/dRe W_i + i dL/dIm W_i) / 2 for the weight indices given, by
    central differences (exact for the quadratic dependence on each coordinate)."""
    w = np.asarray(w, dtype=np.complex128).ravel().copy()
    out = np.zeros(len(indices), dtype=np.complex128)
    for k, i in enumerate(indices):
        d = []
        for step in (h, 1j * h):
            w0 = w[i]
            w[i] = w0 + step
            lp = loss(links, dims, mass, w, e, feats, antiperiodic)
            w[i] = w0 - step
            lm = loss(links, dims, mass, w, e, feats, antiperiodic)
            w[i] = w0
            d.append((lp - lm) / (2 * h))
        out[k] = 0.5 * (d[0] + 1j * d[1])
    return out
