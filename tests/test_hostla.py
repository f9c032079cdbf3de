"""The library's host FP64 linear algebra (Jacobi Hermitian eigensolver, Gram orthonormaliser,
Cholesky inverse), compiled on its own with g++ and checked against LAPACK (no GPU).  These
are the small k x k problems of Rayleigh-Ritz, the deflation basis orthonormalisation and the
s-step Gram factorisation."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_12234_amd", "csrc")

WRAPPER = r"""
#include <complex>
#include <vector>
#include "hostla.h"
using lqt::zd;
static std::vector<zd> in(int n, const double* a) {
    std::vector<zd> v((size_t)n * n);
    for (size_t i = 0; i < v.size(); i++) v[i] = zd(a[2 * i], a[2 * i + 1]);
    return v;
}
static void out(const std::vector<zd>& v, double* a) {
    for (size_t i = 0; i < v.size(); i++) { a[2 * i] = v[i].real(); a[2 * i + 1] = v[i].imag(); }
}
extern "C" void t_heev(int n, const double* A, double* w, double* V, int by_abs) {
    std::vector<double> ww; std::vector<zd> VV;
    lqt::heev(n, in(n, A), ww, VV, by_abs != 0);
    for (int i = 0; i < n; i++) w[i] = ww[i];
    out(VV, V);
}
extern "C" int t_orth(int n, const double* G, double* T, double rtol) {
    std::vector<zd> TT;
    int r = lqt::orthonormalizer(n, in(n, G), TT, rtol);
    out(TT, T);
    return r;
}
extern "C" int t_chol(int n, const double* G, double* T) {
    std::vector<zd> TT;
    bool ok = lqt::chol_inverse(n, in(n, G), TT);
    if (ok) out(TT, T);
    return ok ? 1 : 0;
}
"""


@pytest.fixture(scope="module")
def hostla(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("hostla")
    (d / "wrap.cpp").write_text(WRAPPER)
    so = d / "libhostla.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", CSRC, "-x", "c++",
                           os.path.join(CSRC, "hostla.hip"), "-x", "c++", str(d / "wrap.cpp"), "-o", str(so)])
    L = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    L.t_heev.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int]
    L.t_orth.argtypes = [ctypes.c_int, P, P, ctypes.c_double]
    L.t_orth.restype = ctypes.c_int
    L.t_chol.argtypes = [ctypes.c_int, P, P]
    L.t_chol.restype = ctypes.c_int
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _heev(L, A, by_abs):
    n = A.shape[0]
    A = np.ascontiguousarray(A, dtype=np.complex128)
    w = np.zeros(n)
    V = np.zeros((n, n), dtype=np.complex128)
    L.t_heev(n, _p(A), _p(w), _p(V), int(by_abs))
    return w, V


def _herm(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (B + B.conj().T)


@pytest.mark.parametrize("n", [1, 2, 7, 64])
@pytest.mark.parametrize("by_abs", [False, True])
def test_jacobi_eigensolver_matches_lapack(hostla, n, by_abs):
    A = _herm(n, n)
    w, V = _heev(hostla, A, by_abs)
    ref = np.linalg.eigvalsh(A)
    ref = ref[np.argsort(np.abs(ref), kind="stable")] if by_abs else ref
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(w - ref)) <= 1e-13 * scale
    assert np.max(np.abs(V.conj().T @ V - np.eye(n))) <= 1e-13
    assert np.max(np.abs(A @ V - V * w[None, :])) <= 1e-12 * scale


def test_jacobi_eigensolver_degenerate_and_diagonal(hostla):
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)))
    lam = np.array([-2.0] * 4 + [0.5] * 5 + [3.0] * 3)
    A = (Q * lam[None, :]) @ Q.conj().T
    w, V = _heev(hostla, A, False)
    assert np.max(np.abs(w - np.sort(lam))) <= 1e-13 * 3
    assert np.max(np.abs(A @ V - V * w[None, :])) <= 1e-12 * 3
    D = np.diag([3.0, -1.0, 2.0]).astype(np.complex128)
    w, V = _heev(hostla, D, True)
    assert np.allclose(w, [-1.0, 2.0, 3.0]) and np.allclose(np.abs(V), np.eye(3)[:, [1, 2, 0]])


def test_gram_orthonormaliser_drops_dependent_directions(hostla):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((200, 7)) + 1j * rng.standard_normal((200, 7))
    X = np.hstack([X, X[:, :3] @ (rng.standard_normal((3, 3)) + 0j)])  # rank 7 of 10 columns
    G = np.ascontiguousarray(X.conj().T @ X)
    T = np.zeros((10, 10), dtype=np.complex128)
    r = hostla.t_orth(10, _p(G), _p(T), 1e-10)
    assert r == 7
    Tr = T.reshape(-1)[: 10 * r].reshape(10, r)
    Y = X @ Tr
    assert np.max(np.abs(Y.conj().T @ Y - np.eye(r))) <= 1e-10
    # the kept span is the column span of X
    Qx, _ = np.linalg.qr(X[:, :7])
    assert np.max(np.abs(Y - Qx @ (Qx.conj().T @ Y))) <= 1e-10


def test_cholesky_inverse_and_singular_gram(hostla):
    rng = np.random.default_rng(6)
    X = rng.standard_normal((100, 16)) + 1j * rng.standard_normal((100, 16))
    G = np.ascontiguousarray(X.conj().T @ X)
    T = np.zeros((16, 16), dtype=np.complex128)
    assert hostla.t_chol(16, _p(G), _p(T)) == 1
    assert np.allclose(np.tril(T, -1), 0)  # R^{-1} is upper triangular
    Y = X @ T
    assert np.max(np.abs(Y.conj().T @ Y - np.eye(16))) <= 1e-12
    R = np.linalg.cholesky(G).conj().T  # G = R^+ R, R upper with a positive diagonal
    assert np.max(np.abs(T @ R - np.eye(16))) <= 1e-12
    Xs = np.hstack([X[:, :15], X[:, :1]])
    Gs = np.ascontiguousarray(Xs.conj().T @ Xs)
    assert hostla.t_chol(16, _p(Gs), _p(T)) == 0
