"""Seeded gauge and spinor fields in the canonical host layout.

Canonical layouts (x runs fastest):
  links   complex128, shape (Lt, Lz, Ly, Lx, 4, 3, 3)  -> U_mu(x)[a][b], mu = 0..3 <-> x, y, z, t
  spinors complex128, shape (nrhs, Lt, Lz, Ly, Lx, 4, 3) -> psi(x)[spin][colour]
`dims` is always (Lx, Ly, Lz, Lt).

Random links follow the recipe U = exp(i*eps*H) with H = sum_a w_a * lambda_a, where the
w_a are independent standard normals and lambda_a the eight Gell-Mann matrices, so H is a
traceless Hermitian 3x3 matrix with E[tr H^2] = 16. The exponential is taken through the
eigen-decomposition of H, which gives an exactly special-unitary matrix up to rounding.
All randomness comes from numpy's counter-based Philox generator keyed by the seed.
"""
import numpy as np

_s3 = 1.0 / np.sqrt(3.0)
GELL_MANN = np.array(
    [
        [[0, 1, 0], [1, 0, 0], [0, 0, 0]],
        [[0, -1j, 0], [1j, 0, 0], [0, 0, 0]],
        [[1, 0, 0], [0, -1, 0], [0, 0, 0]],
        [[0, 0, 1], [0, 0, 0], [1, 0, 0]],
        [[0, 0, -1j], [0, 0, 0], [1j, 0, 0]],
        [[0, 0, 0], [0, 0, 1], [0, 1, 0]],
        [[0, 0, 0], [0, 0, -1j], [0, 1j, 0]],
        [[_s3, 0, 0], [0, _s3, 0], [0, 0, -2 * _s3]],
    ],
    dtype=np.complex128,
)


def lattice_volume(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def _rng(seed, stream=0):
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


def su3_links(dims, eps, seed, norm=1.0):
    """Random near-identity SU(3) links exp(i*eps*norm*sum_a w_a lambda_a).

    `norm` = 1 gives E[tr H^2] = 16; norm = 0.5 gives the lambda_a/2 convention.
    Generated one time-slice at a time so that 32^3x64 stays within a few GB.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    out = np.empty((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    for t in range(lt):
        w = _rng(seed, t).standard_normal((lz, ly, lx, 4, 8))
        h = np.einsum("...a,aij->...ij", w * norm, GELL_MANN)
        d, q = np.linalg.eigh(h)
        ph = np.exp(1j * eps * d)
        out[t] = np.einsum("...ik,...k,...jk->...ij", q, ph, q.conj())
    return out


def unit_links(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    u = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def random_su3(shape, seed, stream=0):
    """Haar-distributed SU(3) matrices (QR of a complex Gaussian, phases fixed)."""
    rng = _rng(seed, 1_000_000 + stream)
    g = rng.standard_normal(tuple(shape) + (3, 3)) + 1j * rng.standard_normal(tuple(shape) + (3, 3))
    q, r = np.linalg.qr(g)
    dg = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (dg / np.abs(dg))[..., None, :]
    det = np.linalg.det(q)
    q[..., :, 0] /= det[..., None]
    return q


def _shift(field, mu, step):
    """field(x + step*mu_hat) for arrays whose leading axes are (Lt, Lz, Ly, Lx)."""
    axis = 3 - mu
    return np.roll(field, -step, axis=axis)


def gauge_transform(links, omega):
    """U_mu(x) -> Omega(x) U_mu(x) Omega(x+mu)^dagger ; omega shape (Lt, Lz, Ly, Lx, 3, 3)."""
    out = np.empty_like(links)
    for mu in range(4):
        om_fwd = _shift(omega, mu, 1)
        out[..., mu, :, :] = omega @ links[..., mu, :, :] @ np.conj(np.swapaxes(om_fwd, -1, -2))
    return out


def transform_spinor(psi, omega):
    """psi(x) -> Omega(x) psi(x) for spinors of shape (nrhs, Lt, Lz, Ly, Lx, 4, 3)."""
    return np.einsum("tzyxab,rtzyxsb->rtzyxsa", omega, psi)


def pure_gauge_links(dims, seed):
    """U_mu(x) = Omega(x) Omega(x+mu)^dagger: a gauge transform of the unit field."""
    lx, ly, lz, lt = (int(d) for d in dims)
    omega = random_su3((lt, lz, ly, lx), seed)
    return gauge_transform(unit_links(dims), omega), omega


def random_spinors(dims, nrhs, seed, stream=7):
    """Complex Gaussian spinor fields, shape (nrhs, Lt, Lz, Ly, Lx, 4, 3)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = _rng(seed, stream)
    shape = (nrhs, lt, lz, ly, lx, 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def plane_wave(dims, p, u):
    """exp(i p.x) u for a single spin-colour vector u (4x3) and momentum p (4 reals)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return (phase[..., None, None] * np.asarray(u)[None, None, None, None])[None]
