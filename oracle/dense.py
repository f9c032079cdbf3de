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


def free_field_solve(z, dims, mass, antiperiodic=True):
    """y = A^{-1} z for unit links at any lattice size, in momentum space.

    A plane wave e^{ipx} u is mapped to e^{ipx} A(p) u with A(p) = m + sum(1 - cos p_mu)
    + i sum gamma_mu sin p_mu, so y is the sum over momenta of e^{ipx} A(p)^{-1} z(p).  The
    antiperiodic time momenta (2n+1) pi / L_t are reached from the periodic ones of the FFT
    by the phase e^{i pi t / L_t}.  z has shape (12 V,) or (nrhs, 12 V), index
    12 * site + 3 * spin + colour with x fastest."""
    lx, ly, lz, lt = (int(d) for d in dims)
    z = np.asarray(z, dtype=np.complex128)
    single = z.ndim == 1
    zz = z.reshape(-1, lt, lz, ly, lx, 4, 3)
    shift = np.pi / lt if antiperiodic else 0.0
    tw = np.exp(1j * shift * np.arange(lt)).reshape(1, lt, 1, 1, 1, 1, 1)
    zk = np.fft.fftn(zz / tw, axes=(1, 2, 3, 4))
    kt, kz, ky, kx = (2 * np.pi * np.fft.fftfreq(L) for L in (lt, lz, ly, lx))
    T, Z, Y, X = np.meshgrid(kt + shift, kz, ky, kx, indexing="ij")
    P = (X, Y, Z, T)  # mu = 0..3 <-> x, y, z, t
    a = mass + sum(1 - np.cos(p) for p in P)
    Ap = a[..., None, None] * np.eye(4) + 1j * sum(np.sin(P[mu])[..., None, None] * core.gamma(mu)
                                                   for mu in range(4))
    yk = np.linalg.solve(Ap[None], zk)
    y = np.fft.ifftn(yk, axes=(1, 2, 3, 4)) * tw
    y = y.reshape(z.shape[0] if not single else 1, -1)
    return y[0] if single else y
