"""Dense FP64 pins on tiny lattices (N <= 3072): the operator assembled column by column
through the C oracle, then LAPACK (numpy.linalg) for the exact trace, the Eq. (2)
variances, singular values and the eigen-decomposition of A g5.

TEST INFRASTRUCTURE ONLY.
"""
import numpy as np

from . import core


def dense_operator(links, dims, mass, op=core.OP_A, antiperiodic=True):
    """The N x N matrix of op, column c = op(e_c)."""
    N = 12 * core.volume(dims)
    E = np.eye(N, dtype=np.complex128)
    return core.apply(links, dims, mass, op, E, antiperiodic).T.copy()


def free_field_closed_form(dims, mass, antiperiodic=True):
    """trace A^{-1} and ||A^{-1}||_F^2 of the free Wilson operator from its Fourier form:
    A(p) = m + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu, whose 4x4 blocks have
    eigenvalues a(p) +- i s(p) (each twice, times 3 colours), a = m + sum(1 - cos p),
    s^2 = sum sin^2 p; momenta p_mu = 2 pi n / L_mu, with p_t = (2n+1) pi / L_t when the
    time direction is antiperiodic."""
    lx, ly, lz, lt = dims
    ps = [2 * np.pi * np.arange(l) / l for l in (lx, ly, lz)]
    pt = (2 * np.arange(lt) + (1 if antiperiodic else 0)) * np.pi / lt
    P = np.meshgrid(ps[0], ps[1], ps[2], pt, indexing="ij")
    a = mass + sum(1 - np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    tr = np.sum(12 * a / (a * a + s2))
    fro = np.sum(12 / (a * a + s2))
    return float(tr), float(fro)
