"""ctypes binding of the C oracle (wilson_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the benchmark's
CPU-baseline leg, never by the product library.

Arrays are numpy complex128 in the canonical layouts of the `synth` package:
links (Lt, Lz, Ly, Lx, 4, 3, 3) and spinors (nrhs, 12*V) or (nrhs, Lt, Lz, Ly, Lx, 4, 3).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "wilson_oracle.c")

OP_A, OP_ADAG, OP_AG5, OP_G5A = 0, 1, 2, 3


def build(force=False):
    """Compile the oracle with gcc (plain -O3, OpenMP; no target-specific flags)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, SRC_PATH, "-lm"]
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.orc_apply.argtypes = [P, ctypes.c_double, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int]
        L.orc_apply.restype = ctypes.c_int
        L.orc_gmres.argtypes = [P, ctypes.c_double, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int,
                                ctypes.c_double, ctypes.c_int, P, P]
        L.orc_gmres.restype = ctypes.c_int
        L.orc_splitmix64.argtypes = [ctypes.c_uint64]
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_probes.argtypes = [ctypes.c_uint64, ctypes.c_long, ctypes.c_int, ctypes.c_long, P]
        L.orc_probes.restype = None
        L.orc_gamma.argtypes = [ctypes.c_int, P]
        L.orc_gamma.restype = None
        L.orc_ptc_forward.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P, P, P, P]
        L.orc_ptc_forward.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def volume(dims):
    return int(np.prod(dims))


def gamma(mu):
    out = np.zeros((4, 4), dtype=np.complex128)
    lib().orc_gamma(mu, _ptr(out))
    return out


def apply(links, dims, mass, op, psi, antiperiodic=True):
    """op(psi) for op in {OP_A, OP_ADAG, OP_AG5, OP_G5A}; psi (nrhs, 12V) or (12V,)."""
    N = 12 * volume(dims)
    x = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128).reshape(-1, N))
    out = np.empty_like(x)
    U = np.ascontiguousarray(links, dtype=np.complex128)
    d = _dims(dims)
    rc = lib().orc_apply(_ptr(d), float(mass), int(antiperiodic), _ptr(U), int(op), _ptr(x), _ptr(out), x.shape[0])
    if rc != 0:
        raise MemoryError("orc_apply failed")
    return out.reshape(np.asarray(psi).shape)


def gmres(links, dims, mass, b, xi, m=32, maxit=100000, op=OP_A, antiperiodic=True):
    """x ~ op^{-1} b from restarted GMRES(m), x0 = 0, true residual <= xi*||b||.

    Returns (x, converged, iterations, relative true residual)."""
    N = 12 * volume(dims)
    bb = np.ascontiguousarray(np.asarray(b, dtype=np.complex128).reshape(N))
    x = np.zeros(N, dtype=np.complex128)
    U = np.ascontiguousarray(links, dtype=np.complex128)
    d = _dims(dims)
    its = ctypes.c_int(0)
    rel = ctypes.c_double(0)
    rc = lib().orc_gmres(_ptr(d), float(mass), int(antiperiodic), _ptr(U), int(op), _ptr(bb), _ptr(x),
                         int(m), float(xi), int(maxit), ctypes.byref(its), ctypes.byref(rel))
    if rc < 0:
        raise MemoryError("orc_gmres failed")
    return x, rc == 0, its.value, rel.value


def splitmix64(x):
    return int(lib().orc_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def probes(seed, nprobes, N, j0=0):
    """Real Rademacher probes, shape (nprobes, N), entries +-1 from the SplitMix64 hash."""
    out = np.empty((nprobes, N), dtype=np.float64)
    lib().orc_probes(ctypes.c_uint64(seed), int(j0), int(nprobes), int(N), _ptr(out))
    return out


def ptc_forward(links, dims, feats, weights, v, antiperiodic=True):
    """Linear parallel-transport network forward; v (V, F0, 3) complex, weights list of
    (9, F_out, F_in) complex arrays. Returns (V, F_last, 3)."""
    V = volume(dims)
    feats = np.ascontiguousarray(np.asarray(feats, dtype=np.int32))
    W = np.ascontiguousarray(np.concatenate([np.asarray(w, dtype=np.complex128).ravel() for w in weights]))
    x = np.ascontiguousarray(np.asarray(v, dtype=np.complex128).reshape(V, feats[0], 3))
    out = np.empty((V, int(feats[-1]), 3), dtype=np.complex128)
    U = np.ascontiguousarray(links, dtype=np.complex128)
    rc = lib().orc_ptc_forward(_ptr(_dims(dims)), int(antiperiodic), _ptr(U), len(feats) - 1, _ptr(feats),
                               _ptr(W), _ptr(x), _ptr(out))
    if rc != 0:
        raise MemoryError("orc_ptc_forward failed")
    return out
