"""Host logic of the solver, compiled on its own with g++ (no GPU):
- the stall watch that ends a restarted solve (or hands it to the fallback chain) when its
  FP64 residuals stop decreasing or a cycle can take no step, and the fallback chain's order;
- the small FP64 solve of an s-step cycle: on a healthy basis its coefficients are the
  least-squares minimiser of |r - A K beta| (numpy lstsq on the same vectors), and on a
  rank-one Gram matrix (the start vector is an eigenvector of A) or a non-finite one it
  takes no step, which the solver must not repeat forever."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_12234_amd", "csrc")

WRAPPER = r"""
#include <cmath>
// host stand-ins for the two HIP vector types the header uses
struct double2 { double x, y; };
static inline double2 make_double2(double a, double b) { return double2{a, b}; }
#define __host__
#define __device__
#include "sstep_small.h"
#include "stall.h"

extern "C" int t_sstep(int s, const double* G, double nr, double theta, double sigma, double sqrtN,
                       double* beta, double* est) {
    constexpr int NV = 16;
    double2 g[NV][NV];
    for (int i = 0; i < NV; i++)
        for (int j = 0; j < NV; j++) g[i][j] = make_double2(0, 0);
    for (int i = 0; i <= s; i++)
        for (int j = 0; j <= s; j++) g[i][j] = make_double2(G[2 * (i * (s + 1) + j)], G[2 * (i * (s + 1) + j) + 1]);
    // columns beyond the cycle are left zero: the Cholesky truncates there
    double2 b[NV];
    int k = lqt::sstep_small_solve<NV>(g, nr, theta, sigma, sqrtN, NV - 1, b, est);
    for (int i = 0; i < NV; i++) { beta[2 * i] = b[i].x; beta[2 * i + 1] = b[i].y; }
    return k;
}

extern "C" int t_watch(int window, int n, const double* rr, const int* steps) {
    // feed (cycle steps, formed residual) pairs; return the index of the residual at which the
    // system is declared stalled, or -1
    lqt::StallWatch w;
    w.window = window;
    for (int i = 0; i < n; i++) {
        if (steps[i] >= 0) w.cycle(steps[i]);
        if (w.formed(rr[i])) return i;
    }
    return -1;
}

extern "C" int t_chain(int prec, int net, int sstep, int* out) {
    lqt::ChainCfg c{prec, net, sstep}, n;
    int k = 0;
    while (lqt::chain_next(c, n)) {
        out[3 * k] = n.prec; out[3 * k + 1] = n.net; out[3 * k + 2] = n.sstep;
        c = n;
        k++;
    }
    return k;
}
"""


@pytest.fixture(scope="module")
def L(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("stall")
    (d / "wrap.cpp").write_text(WRAPPER)
    so = d / "libstall.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", CSRC, str(d / "wrap.cpp"),
                           "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    lib.t_sstep.argtypes = [ctypes.c_int, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P]
    lib.t_sstep.restype = ctypes.c_int
    lib.t_watch.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
    lib.t_watch.restype = ctypes.c_int
    lib.t_chain.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
    lib.t_chain.restype = ctypes.c_int
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _watch(L, window, rr, steps=None):
    rr = np.asarray(rr, dtype=np.float64)
    steps = np.asarray(steps if steps is not None else [-1] * len(rr), dtype=np.int32)
    return L.t_watch(window, len(rr), _p(rr), _p(steps))


def test_watch_decreasing_never_stalls(L):
    assert _watch(L, 2, 10.0 ** -np.arange(12)) == -1
    # slow but steady: 1 % per restart
    assert _watch(L, 2, 0.99 ** np.arange(50)) == -1


def test_watch_flat_stalls_after_window(L):
    rr = [1.0, 0.5, 0.5, 0.4999999, 0.6]
    assert _watch(L, 2, rr) == 3  # the 2nd residual in a row without a 0.1 % decrease
    assert _watch(L, 3, rr) == 4
    # a rise counts as no decrease
    assert _watch(L, 1, [1.0, 2.0]) == 1
    # window 0 never stalls on flat residuals
    assert _watch(L, 0, [1.0] * 10) == -1


def test_watch_zero_step_cycle_and_nan(L):
    # the residual formed after a cycle that took no step ends the system at once
    assert _watch(L, 0, [1.0, 0.5, 0.5], steps=[-1, 15, 0]) == 2
    assert _watch(L, 2, [1.0, 0.5, 0.1], steps=[-1, 15, 0]) == 2
    assert _watch(L, 0, [1.0, float("nan")]) == 1


def test_chain_order(L):
    out = np.zeros(30, dtype=np.int32)
    k = L.t_chain(3, 1, 0, _p(out))  # BF16 storage with the net
    assert [tuple(out[3 * i:3 * i + 3]) for i in range(k)] == [(3, 0, 0), (1, 0, 0), (0, 0, 0)]
    k = L.t_chain(2, 0, 1, _p(out))  # FP16 s-step cycles
    assert [tuple(out[3 * i:3 * i + 3]) for i in range(k)] == [(2, 0, 0), (1, 0, 0), (0, 0, 0)]
    assert L.t_chain(0, 0, 0, _p(out)) == 0


def _cycle(A, r, s, theta, sigma):
    """Stored s-step vectors: k_0 = r sqrt(N)/|r|, k_{i+1} = sigma (A - theta) k_i."""
    N = r.size
    K = [r * np.sqrt(N) / np.linalg.norm(r)]
    for _ in range(s):
        K.append(sigma * (A @ K[-1] - theta * K[-1]))
    return np.array(K).T  # (N, s+1)


def test_sstep_small_solve_is_least_squares(L):
    rng = np.random.default_rng(3)
    N, s, theta, sigma = 60, 6, 2.0, 0.5
    A = theta * np.eye(N) + 0.3 * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(N)
    r = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    K = _cycle(A, r, s, theta, sigma)
    G = K.conj().T @ K
    beta = np.zeros(32)
    est = np.zeros(1)
    k = L.t_sstep(s, _p(np.ascontiguousarray(G).view(np.float64)), np.linalg.norm(r), theta, sigma,
                  np.sqrt(N), _p(beta), _p(est))
    assert k == s
    b = beta.view(np.complex128)[:s]
    # reference: min_beta |r - A K_s beta| by LAPACK least squares on the same vectors
    ref, *_ = np.linalg.lstsq(A @ K[:, :s], r, rcond=None)
    assert np.max(np.abs(b - ref)) <= 1e-9 * np.max(np.abs(ref))
    assert abs(est[0] - np.linalg.norm(r - A @ K[:, :s] @ ref)) <= 1e-9 * np.linalg.norm(r)
    assert np.all(beta.view(np.complex128)[s:] == 0)


def test_sstep_small_solve_rank_one_gram_takes_no_step(L):
    # r an eigenvector of A: k_1 is parallel to k_0 and the Gram matrix has rank one
    N, s, theta, sigma = 48, 4, 2.0, 0.5
    lam = 1.3 + 0.2j
    A = np.diag(np.full(N, lam))
    r = np.ones(N, dtype=np.complex128)
    K = _cycle(A, r, s, theta, sigma)
    G = K.conj().T @ K
    beta = np.full(32, 7.0)
    est = np.zeros(1)
    k = L.t_sstep(s, _p(np.ascontiguousarray(G).view(np.float64)), np.linalg.norm(r), theta, sigma,
                  np.sqrt(N), _p(beta), _p(est))
    assert k == 0
    assert np.all(beta == 0)
    assert est[0] == pytest.approx(np.linalg.norm(r))


def test_sstep_small_solve_nonfinite_gram_takes_no_step(L):
    s = 3
    G = np.eye(s + 1, dtype=np.complex128) * 48.0
    G[1, 1] = np.inf
    beta = np.zeros(32)
    est = np.zeros(1)
    assert L.t_sstep(s, _p(np.ascontiguousarray(G).view(np.float64)), 1.0, 2.0, 0.5, np.sqrt(48.0), _p(beta),
                     _p(est)) == 0
    G[1, 1] = np.nan
    assert L.t_sstep(s, _p(np.ascontiguousarray(G).view(np.float64)), 1.0, 2.0, 0.5, np.sqrt(48.0), _p(beta),
                     _p(est)) == 0
