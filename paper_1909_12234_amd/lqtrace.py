"""Thin ctypes binding of liblqtrace (include/lqtrace.h).

Argument marshalling only: every numerical step runs in the HIP library.  Torch tensors
provide device memory and the HIP stream; fields are complex128 tensors in the canonical
layout (nrhs, Lt, Lz, Ly, Lx, 4, 3) or flattened (nrhs, 12*V).  The library must have been
built (python -m paper_1909_12234_amd.build); importing this module raises if it has not.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblqtrace.so")

LQT_OK, LQT_EINVAL, LQT_ENOMEM, LQT_EHIP, LQT_ENOTCONV, LQT_ENOTUNITARY, LQT_ESTATE, LQT_ENAN = 0, -1, -2, -3, -4, -5, -6, -7
A, A_DAG, A_G5, G5_A = 0, 1, 2, 3
F64, F32, F16, BF16 = 0, 1, 2, 3
OBLIQUE_G5, ORTH = 0, 1
NET_FEATURES = (4, 8, 8, 8, 4)  # parallel-transport network: features per layer boundary
WEIGHT_COUNT = sum(9 * a * b for a, b in zip(NET_FEATURES[:-1], NET_FEATURES[1:]))  # complex weights

ERROR_NAMES = {0: "LQT_OK", -1: "LQT_EINVAL", -2: "LQT_ENOMEM", -3: "LQT_EHIP", -4: "LQT_ENOTCONV",
               -5: "LQT_ENOTUNITARY", -6: "LQT_ESTATE", -7: "LQT_ENAN"}


class SolverOpts(ctypes.Structure):
    _fields_ = [("inner_prec", ctypes.c_int), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("use_net", ctypes.c_int), ("max_batch", ctypes.c_int), ("cgs2", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("verbose", ctypes.c_int), ("outer_maxit", ctypes.c_int),
                ("graph", ctypes.c_int), ("sstep", ctypes.c_int), ("reliable", ctypes.c_double),
                ("fallback", ctypes.c_int), ("stall_window", ctypes.c_int), ("eig_degree", ctypes.c_int),
                ("eig_xi", ctypes.c_double), ("twogrid", ctypes.c_int), ("tg_smooth", ctypes.c_int),
                ("tg_coarse_tol", ctypes.c_double), ("tg_coarse_maxit", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int), ("iters", ctypes.c_int), ("cycles", ctypes.c_int),
                ("relres", ctypes.c_double), ("fallback", ctypes.c_int)]


class TraceResult(ctypes.Structure):
    _fields_ = [("trace_re", ctypes.c_double), ("trace_im", ctypes.c_double), ("t0_re", ctypes.c_double),
                ("t0_im", ctypes.c_double), ("var_sample", ctypes.c_double), ("var_mean", ctypes.c_double),
                ("jackknife_err", ctypes.c_double), ("var_re_only", ctypes.c_double), ("nsolves", ctypes.c_int),
                ("nfailed", ctypes.c_int), ("iters_total", ctypes.c_longlong), ("seconds_solve", ctypes.c_double),
                ("seconds_setup", ctypes.c_double), ("nfallback", ctypes.c_int)]


class TsmResult(ctypes.Structure):
    _fields_ = [("trace_re", ctypes.c_double), ("trace_im", ctypes.c_double), ("err", ctypes.c_double),
                ("corr_re", ctypes.c_double), ("corr_im", ctypes.c_double), ("corr_var_sample", ctypes.c_double),
                ("corr_jackknife_err", ctypes.c_double), ("nsolves_loose", ctypes.c_longlong),
                ("nsolves_tight", ctypes.c_longlong), ("iters_loose", ctypes.c_longlong),
                ("iters_tight", ctypes.c_longlong), ("nfailed", ctypes.c_int)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("lr", ctypes.c_double), ("batch", ctypes.c_int),
                ("pair_xi", ctypes.c_double), ("verbose", ctypes.c_int)]


class LqtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "lqt_create": ([ctypes.POINTER(_P), _P, _D, _I, _P], _I),
    "lqt_create_multi": ([ctypes.POINTER(_P), _I, _P, _P, _I, _P], _I),
    "lqt_trace_lattices": ([_P, _I, ctypes.c_uint64, _D, _P, _P, _P], _I),
    "lqt_set_gauge": ([_P, _P, _I], _I),
    "lqt_set_mass": ([_P, _D], _I),
    "lqt_apply": ([_P, _I, _I, _P, _P, _I], _I),
    "lqt_solve": ([_P, _P, _P, _I, _D, _P, _P], _I),
    "lqt_basis_eig": ([_P, _I, _D, _D, _P, ctypes.POINTER(_P)], _I),
    "lqt_basis_prolongator": ([_P, _P, _I, _I, _D, _I, _P, ctypes.POINTER(_P)], _I),
    "lqt_basis_from_vectors": ([_P, _P, _I, ctypes.POINTER(_P)], _I),
    "lqt_basis_eigenvalues": ([_P, _P, ctypes.POINTER(_I)], _I),
    "lqt_sigma_max": ([_P, ctypes.POINTER(_D)], _I),
    "lqt_basis_vectors": ([_P, _P], _I),
    "lqt_basis_free": ([_P], None),
    "lqt_precond_set": ([_P, _P, ctypes.c_size_t], _I),
    "lqt_precond_get": ([_P, _P, ctypes.c_size_t], _I),
    "lqt_precond_apply": ([_P, _P, _P, _I], _I),
    "lqt_precond_train": ([_P, _I, ctypes.c_uint64, _P, _P], _I),
    "lqt_precond_loss_grad": ([_P, _P, _I, _P, _P], _I),
    "lqt_trace": ([_P, _P, _I, _I, ctypes.c_uint64, _D, _P, _P, _P, _P], _I),
    "lqt_precond_twogrid": ([_P, _P], _I),
    "lqt_precond_twogrid_apply": ([_P, _P, _P, _I, _P], _I),
    "lqt_trace_probing": ([_P, _P, _I, _I, ctypes.c_uint64, _D, _I, _I, _P, _P, _P, _P], _I),
    "lqt_trace_tsm": ([_P, _P, _I, _I, ctypes.c_uint64, _D, _I, ctypes.c_uint64, _D, _I, _I, _P, _P, _P, _P], _I),
    "lqt_probes": ([_P, ctypes.c_uint64, ctypes.c_longlong, _I, _P], _I),
    "lqt_partition_probes": ([_P, ctypes.c_uint64, ctypes.c_longlong, _I, _I, _I, _P], _I),
    "lqt_gram": ([_P, _P, _I, _P, _I, _P], _I),
    "lqt_gram_noalloc": ([_P, _P, _I, _P, _I, _P], _I),
    "lqt_project_probes": ([_P, _P, _I, ctypes.c_uint64, ctypes.c_longlong, _I, _P, _P], _I),
    "lqt_combine": ([_P, _P, _I, _P, _I, _D, _D, _P], _I),
    "lqt_restrict": ([_P, _P, _P, _P, _I], _I),
    "lqt_prolong": ([_P, _P, _P, _P, _I], _I),
    "lqt_prolongator_get": ([_P, _P, ctypes.POINTER(ctypes.c_longlong)], _I),
    "lqt_coarse_apply": ([_P, _P, _P, _P, _I, _I], _I),
    "lqt_basis_prolongator2": ([_P, _P, _I, _P, _I, _I, _D, _I, _P, ctypes.POINTER(_P)], _I),
    "lqt_basis_prolongator2_from": ([_P, _P, _I, _P, _P, _I, _P, _P, _I, ctypes.POINTER(_P)], _I),
    "lqt_coarse2_apply": ([_P, _P, _P, _P, _I, _I], _I),
    "lqt_prolongator2_get": ([_P, _P, ctypes.POINTER(ctypes.c_longlong)], _I),
    "lqt_basis_prolongator_from": ([_P, _P, _I, _P, _P, _I, ctypes.POINTER(_P)], _I),
    "lqt_tune": ([_P, _I, _I, ctypes.POINTER(_D), _P], _I),
    "lqt_set_tile": ([_P, _I, _I, _P], _I),
    "lqt_kernel_times": ([_P, _P, _P, _P, _I], _I),
    "lqt_last_error": ([_P], ctypes.c_char_p),
    "lqt_destroy": ([_P], None),
}


def lib():
    """Load liblqtrace.so; raises when it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1909_12234_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, per, what):
    """Contiguous device tensor check before its pointer reaches a kernel: a CUDA (HIP)
    tensor of `dtype` whose element count is a multiple of `per` (zero fields is the
    library's no-op).  Raises TypeError or ValueError; nothing is passed to the library
    otherwise."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise TypeError(f"{what}: expected a device tensor, got one on {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if per and t.numel() % per:
        raise ValueError(f"{what}: {t.numel()} elements is not a multiple of {per}")
    return t.contiguous()


def _host(t, dtype, numel, what):
    """Host tensor check for buffers the library writes or reads on the CPU side."""
    if t.is_cuda or t.dtype != dtype or t.numel() != numel:
        raise TypeError(f"{what}: expected a host {dtype} tensor of {numel} elements")
    return t.contiguous()


# complex dtype of the canonical fields lqt_apply takes for each precision
_APPLY_DTYPE = {0: torch.complex128, 1: torch.complex64, 2: torch.complex64, 3: torch.complex64}


def _opts(prec=F64, restart=32, maxit=100000, use_net=0, max_batch=0, cgs2=0, inner_tol=0.0, verbose=0,
          outer_maxit=0, graph=0, sstep=0, reliable=0.0, fallback=0, stall_window=0, eig_degree=0, eig_xi=0.0,
          twogrid=0, tg_smooth=0, tg_coarse_tol=0.0, tg_coarse_maxit=0):
    return SolverOpts(prec, restart, maxit, use_net, max_batch, cgs2, inner_tol, verbose, outer_maxit, graph, sstep,
                      reliable, fallback, stall_window, eig_degree, eig_xi, twogrid, tg_smooth, tg_coarse_tol,
                      tg_coarse_maxit)


class Context:
    """A lattice, its gauge field and the mass, bound to the current torch HIP stream."""

    def __init__(self, dims, mass, antiperiodic=True, stream=None):
        """dims (Lx, Ly, Lz, Lt) and a mass; or a list of such dims and a list of masses for a
        context of several lattices solved together (fields: the lattices one after another)."""
        multi = isinstance(dims[0], (tuple, list))
        self.lattices = [tuple(int(d) for d in x) for x in dims] if multi else [tuple(int(d) for d in dims)]
        self.dims = self.lattices[0]
        self.nlat = len(self.lattices)
        self.V = sum(x[0] * x[1] * x[2] * x[3] for x in self.lattices)
        self.N = 12 * self.V
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = ctypes.c_void_p()
        if multi:
            masses = [float(m) for m in mass] if isinstance(mass, (tuple, list)) else [float(mass)] * self.nlat
            d = (ctypes.c_int * (4 * self.nlat))(*[v for x in self.lattices for v in x])
            m = (ctypes.c_double * self.nlat)(*masses)
            rc = lib().lqt_create_multi(ctypes.byref(self._h), self.nlat, d, m, int(antiperiodic),
                                        ctypes.c_void_p(self.stream.cuda_stream))
        else:
            d = (ctypes.c_int * 4)(*self.dims)
            rc = lib().lqt_create(ctypes.byref(self._h), d, float(mass), int(antiperiodic),
                                  ctypes.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise LqtError(rc, "context creation failed")

    # -- plumbing
    def _check(self, rc, allow=()):
        if rc != 0 and rc not in allow:
            raise LqtError(rc, lib().lqt_last_error(self._h).decode())
        return rc

    def close(self):
        if self._h:
            lib().lqt_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field(self, nrhs, dtype=torch.complex128):
        return torch.zeros((nrhs, self.N), dtype=dtype, device="cuda")

    # -- operator
    def set_gauge(self, links):
        """links: complex128 array/tensor (Lt, Lz, Ly, Lx, 4, 3, 3) on host or device."""
        t = torch.as_tensor(links)
        if t.dtype != torch.complex128:
            raise TypeError("links must be complex128")
        t = t.contiguous()
        on_dev = 1 if t.is_cuda else 0
        return self._check(lib().lqt_set_gauge(self._h, _ptr(t), on_dev))

    def set_mass(self, mass):
        return self._check(lib().lqt_set_mass(self._h, float(mass)))

    def apply(self, x, op=A, prec=F64):
        if int(prec) not in _APPLY_DTYPE:
            raise ValueError(f"unknown precision {prec}")
        x = _dev(x, _APPLY_DTYPE[int(prec)], self.N, "apply input")
        out = torch.empty_like(x)
        nrhs = x.numel() // self.N
        self._check(lib().lqt_apply(self._h, int(op), int(prec), _ptr(x), _ptr(out), nrhs))
        return out

    def solve(self, b, xi, raise_on_fail=True, **opts):
        b = _dev(b, torch.complex128, self.N, "solve right-hand sides")
        x = torch.empty_like(b)
        nrhs = b.numel() // self.N
        st = (SolveStats * max(nrhs, 1))()
        o = _opts(**opts)
        rc = lib().lqt_solve(self._h, _ptr(b), _ptr(x), nrhs, float(xi), ctypes.byref(o), st)
        self._check(rc, allow=() if raise_on_fail else (LQT_ENOTCONV,))
        return x, [(s.converged, s.iters, s.cycles, s.relres, s.fallback) for s in st[:nrhs]], rc

    def probes(self, seed, nprobes, j0=0):
        out = torch.empty((nprobes, self.N), dtype=torch.complex128, device="cuda")
        self._check(lib().lqt_probes(self._h, ctypes.c_uint64(seed), int(j0), int(nprobes), _ptr(out)))
        return out

    def partition_probes(self, seed, nvec, hp_vectors, dilute, p0=0):
        """Partition probe vectors p0 .. p0+nvec-1 of trace(..., hp_vectors, dilute)."""
        out = torch.empty((nvec, self.N), dtype=torch.complex128, device="cuda")
        self._check(lib().lqt_partition_probes(self._h, ctypes.c_uint64(seed), int(p0), int(nvec), int(hp_vectors),
                                               int(bool(dilute)), _ptr(out)))
        return out

    def tune(self, prec, nrhs, return_tile=False):
        """Autotune the dslash tiling for (prec, nrhs); the best time in ms (and the tile
        (rhs per thread or groups per lane, block, chunk, kind) with return_tile)."""
        ms = ctypes.c_double(0)
        tile = (ctypes.c_int * 4)()
        self._check(lib().lqt_tune(self._h, int(prec), int(nrhs), ctypes.byref(ms), tile))
        return (ms.value, tuple(tile)) if return_tile else ms.value

    def set_tile(self, prec, nrhs, tile):
        """Use tile = (rhs per thread or groups per lane, block, chunk, kind) for (prec, nrhs)."""
        t = (ctypes.c_int * 4)(*[int(v) for v in tile])
        self._check(lib().lqt_set_tile(self._h, int(prec), int(nrhs), t))

    KERNEL_FAMILIES = ["dslash", "cgs_dots", "cgs_update", "residual_fp64", "krylov_other", "projections",
                       "prolongator", "net", "graph_cycles"]

    def kernel_times(self, mode=0):
        """{family: (ms, launches, algorithmic bytes)}; mode 2 starts timing, 3 stops it."""
        nf = len(self.KERNEL_FAMILIES)
        ms = (ctypes.c_double * nf)()
        calls = (ctypes.c_longlong * nf)()
        byt = (ctypes.c_double * nf)()
        self._check(lib().lqt_kernel_times(self._h, ms, calls, byt, int(mode)))
        return {f: (ms[i], calls[i], byt[i]) for i, f in enumerate(self.KERNEL_FAMILIES)}

    def sigma_max(self):
        """Largest singular value of A (Lanczos on A A^+)."""
        v = ctypes.c_double(0)
        self._check(lib().lqt_sigma_max(self._h, ctypes.byref(v)))
        return v.value

    # -- dense building blocks
    def gram(self, X, Y):
        X = _dev(X, torch.complex128, self.N, "gram X")
        Y = _dev(Y, torch.complex128, self.N, "gram Y")
        ka, kb = X.numel() // self.N, Y.numel() // self.N
        out = torch.empty((ka, kb), dtype=torch.complex128)
        self._check(lib().lqt_gram(self._h, _ptr(X), ka, _ptr(Y), kb, _ptr(out)))
        return out

    def gram_noalloc(self, X, Y, out=None):
        """C = X^+ Y through the allocation-free entry point (static device workspace);
        `out` (host complex128, ka x kb) may be given to avoid allocating the result too."""
        X = _dev(X, torch.complex128, self.N, "gram X")
        Y = _dev(Y, torch.complex128, self.N, "gram Y")
        ka, kb = X.numel() // self.N, Y.numel() // self.N
        if out is None:
            out = torch.empty((ka, kb), dtype=torch.complex128)
        out = _host(out, torch.complex128, ka * kb, "gram output")
        self._check(lib().lqt_gram_noalloc(self._h, _ptr(X), ka, _ptr(Y), kb, _ptr(out)))
        return out

    def project_probes(self, X, seed, j0, s):
        X = _dev(X, torch.complex128, self.N, "project_probes X")
        ka = X.numel() // self.N
        cup = torch.empty((ka, s), dtype=torch.complex128)
        cdn = torch.empty((ka, s), dtype=torch.complex128)
        self._check(lib().lqt_project_probes(self._h, _ptr(X), ka, ctypes.c_uint64(seed), int(j0), int(s),
                                             _ptr(cup), _ptr(cdn)))
        return cup, cdn

    def combine(self, X, C, Y=None, beta=0.0, alpha=1.0):
        ka, kb = C.shape
        X = _dev(X, torch.complex128, self.N, "combine X")
        if X.numel() // self.N != ka:
            raise ValueError("combine: X must hold as many fields as C has rows")
        C = torch.as_tensor(C, dtype=torch.complex128).contiguous().cpu()
        if Y is None:
            Y = torch.zeros((kb, self.N), dtype=torch.complex128, device="cuda")
        elif not (Y.is_cuda and Y.dtype == torch.complex128 and Y.is_contiguous() and Y.numel() == kb * self.N):
            raise TypeError("combine: Y must be a contiguous complex128 device tensor of kb fields")
        self._check(lib().lqt_combine(self._h, _ptr(X), ka, _ptr(C), kb, float(beta), float(alpha), _ptr(Y)))
        return Y

    # -- deflation bases
    def basis_eig(self, k, xi=1e-2, tau=0.0, require_converged=False, **opts):
        """k smallest-|lambda| eigenpairs of A g5.  A basis whose pairs did not all meet the
        residual criterion is still returned (basis.converged = False) unless required."""
        h = ctypes.c_void_p()
        o = _opts(**opts)
        rc = lib().lqt_basis_eig(self._h, int(k), float(xi), float(tau), ctypes.byref(o), ctypes.byref(h))
        self._check(rc, allow=() if require_converged else (LQT_ENOTCONV,))
        if not h:
            raise LqtError(rc, lib().lqt_last_error(self._h).decode())
        b = Basis(self, h)
        b.converged = rc == 0
        return b

    def basis_prolongator(self, block, nv, k, null_xi=1e-2, null_maxit=200, require_converged=False, **opts):
        """Algorithm 2's basis: W from nv near-null vectors per chirality on the aggregates of
        `block`, then the k smallest-|lambda| coarse eigenvectors.  A basis whose coarse pairs
        did not all meet the residual criterion is still returned (basis.converged = False)
        unless required."""
        h = ctypes.c_void_p()
        o = _opts(**opts)
        b = (ctypes.c_int * 4)(*block)
        rc = lib().lqt_basis_prolongator(self._h, b, int(nv), int(k), float(null_xi), int(null_maxit),
                                         ctypes.byref(o), ctypes.byref(h))
        self._check(rc, allow=() if require_converged else (LQT_ENOTCONV,))
        if not h:
            raise LqtError(rc, lib().lqt_last_error(self._h).decode())
        bas = Basis(self, h, nv=nv)
        bas.converged = rc == 0
        return bas

    def basis_prolongator_from(self, block, nv, W, coarse=None):
        h = ctypes.c_void_p()
        b = (ctypes.c_int * 4)(*block)
        W = _dev(W, torch.complex128, self.N * int(nv), "prolongator W")
        if W.numel() != self.N * int(nv):
            raise ValueError("prolongator W must hold nv * N entries")
        k = 0 if coarse is None else coarse.shape[0]
        cv = None if coarse is None else _dev(coarse, torch.complex128, 0, "coarse vectors")
        self._check(lib().lqt_basis_prolongator_from(self._h, b, int(nv), _ptr(W), _ptr(cv), int(k),
                                                     ctypes.byref(h)))
        return Basis(self, h, nv=nv)

    def basis_prolongator2(self, block, nv, block2, nv2, k, null_xi=1e-2, null_maxit=200, require_converged=False,
                           **opts):
        """Algorithm 2 with two multigrid levels (lqt_basis_prolongator2)."""
        h = ctypes.c_void_p()
        o = _opts(**opts)
        b1 = (ctypes.c_int * 4)(*block)
        b2 = (ctypes.c_int * 4)(*block2)
        rc = lib().lqt_basis_prolongator2(self._h, b1, int(nv), b2, int(nv2), int(k), float(null_xi), int(null_maxit),
                                          ctypes.byref(o), ctypes.byref(h))
        self._check(rc, allow=() if require_converged else (LQT_ENOTCONV,))
        if not h:
            raise LqtError(rc, lib().lqt_last_error(self._h).decode())
        bas = Basis(self, h, nv=nv, nv2=nv2)
        bas.converged = rc == 0
        return bas

    def basis_prolongator2_from(self, block, nv, W, block2, nv2, W2, coarse2=None):
        h = ctypes.c_void_p()
        b1 = (ctypes.c_int * 4)(*block)
        b2 = (ctypes.c_int * 4)(*block2)
        W = _dev(W, torch.complex128, self.N * int(nv), "prolongator W")
        if W.numel() != self.N * int(nv):
            raise ValueError("prolongator W must hold nv * N entries")
        W2 = _dev(W2, torch.complex128, 0, "level-2 prolongator W2")
        k = 0 if coarse2 is None else coarse2.shape[0]
        cv = None if coarse2 is None else _dev(coarse2, torch.complex128, 0, "level-2 coarse vectors")
        self._check(lib().lqt_basis_prolongator2_from(self._h, b1, int(nv), _ptr(W), b2, int(nv2), _ptr(W2), _ptr(cv),
                                                      int(k), ctypes.byref(h)))
        return Basis(self, h, nv=nv, nv2=nv2)

    def basis_from_vectors(self, X):
        h = ctypes.c_void_p()
        X = _dev(X, torch.complex128, self.N, "basis vectors")
        self._check(lib().lqt_basis_from_vectors(self._h, _ptr(X), X.numel() // self.N, ctypes.byref(h)))
        return Basis(self, h)

    # -- learned preconditioner
    def precond_twogrid(self, basis):
        """Use the prolongator of `basis` (None clears) for the two-grid preconditioner."""
        self._check(lib().lqt_precond_twogrid(self._h, basis._h if basis is not None else None))
        self._tg_basis = basis

    def precond_twogrid_apply(self, x, **opts):
        """One two-grid application to canonical complex128 device fields."""
        x = _dev(x, torch.complex128, self.N, "two-grid input")
        out = torch.empty_like(x)
        o = _opts(**opts)
        self._check(lib().lqt_precond_twogrid_apply(self._h, _ptr(x), _ptr(out), x.numel() // self.N, ctypes.byref(o)))
        return out

    def precond_set(self, weights):
        w = torch.as_tensor(weights, dtype=torch.complex64).contiguous().cpu()
        return self._check(lib().lqt_precond_set(self._h, _ptr(w), w.numel() * 8))

    def precond_get(self):
        w = torch.empty(WEIGHT_COUNT, dtype=torch.complex64)
        self._check(lib().lqt_precond_get(self._h, _ptr(w), w.numel() * 8))
        return w

    def precond_apply(self, x):
        x = _dev(x, torch.complex128, self.N, "precond_apply input")
        out = torch.empty_like(x)
        self._check(lib().lqt_precond_apply(self._h, _ptr(x), _ptr(out), x.numel() // self.N))
        return out

    def precond_loss_grad(self, e):
        """Mean loss ||M A e - e||^2/||e||^2 over the fields e and its gradient dL/dconj(W)
        (complex128 array of the 1728 weights) at the current FP32 master weights."""
        e = _dev(e, torch.complex128, self.N, "precond_loss_grad errors")
        npairs = e.numel() // self.N
        g = torch.empty(2 * WEIGHT_COUNT, dtype=torch.float64)
        loss = ctypes.c_double(0)
        self._check(lib().lqt_precond_loss_grad(self._h, _ptr(e), npairs, ctypes.byref(loss), _ptr(g)))
        return loss.value, torch.view_as_complex(g.view(-1, 2))

    def precond_train(self, npairs, seed, epochs=4, lr=1e-3, batch=4, pair_xi=0.0, verbose=0):
        """Adam training on npairs pairs (r = A e, e); returns the last epoch's mean loss."""
        o = TrainOpts(int(epochs), float(lr), int(batch), float(pair_xi), int(verbose))
        loss = ctypes.c_double(0)
        self._check(lib().lqt_precond_train(self._h, int(npairs), ctypes.c_uint64(seed), ctypes.byref(o),
                                            ctypes.byref(loss)))
        return loss.value

    # -- trace
    def trace_lattices(self, nprobes, seed, xi, raise_on_fail=True, samples=False, **opts):
        """One undeflated estimate per lattice (list of dicts)."""
        res = (TraceResult * self.nlat)()
        o = _opts(**opts)
        samp = torch.zeros((self.nlat, nprobes), dtype=torch.complex128) if samples else None
        rc = lib().lqt_trace_lattices(self._h, int(nprobes), ctypes.c_uint64(seed), float(xi), ctypes.byref(o), res,
                                      _ptr(samp))
        self._check(rc, allow=() if raise_on_fail else (LQT_ENOTCONV,))
        out = []
        for k in range(self.nlat):
            d = {f: getattr(res[k], f) for f, _ in TraceResult._fields_}
            d["rc"] = rc
            if samples:
                d["samples"] = samp[k]
            out.append(d)
        return out

    def trace(self, nprobes, seed, xi, basis=None, projector=OBLIQUE_G5, rank_curve=False, samples=False,
              raise_on_fail=True, hp_vectors=1, dilute=False, **opts):
        """Deflated Hutchinson estimate over nprobes draws; hp_vectors > 1 or dilute use the
        partition basis (lqt_trace_probing: each draw solves hp_vectors * (12 if dilute else
        1) vectors)."""
        res = TraceResult()
        o = _opts(**opts)
        k = basis.k if basis is not None else 0
        curve = torch.zeros((k + 1, 3), dtype=torch.float64) if rank_curve else None
        samp = torch.zeros(nprobes, dtype=torch.complex128) if samples else None
        bh = basis._h if basis is not None else None
        if hp_vectors == 1 and not dilute:
            rc = lib().lqt_trace(self._h, bh, int(projector), int(nprobes), ctypes.c_uint64(seed), float(xi),
                                 ctypes.byref(o), ctypes.byref(res), _ptr(curve), _ptr(samp))
        else:
            rc = lib().lqt_trace_probing(self._h, bh, int(projector), int(nprobes), ctypes.c_uint64(seed), float(xi),
                                         int(hp_vectors), int(bool(dilute)), ctypes.byref(o), ctypes.byref(res),
                                         _ptr(curve), _ptr(samp))
        self._check(rc, allow=() if raise_on_fail else (LQT_ENOTCONV,))
        out = {f: getattr(res, f) for f, _ in TraceResult._fields_}
        out["rc"] = rc
        if rank_curve:
            out["rank_curve"] = curve
        if samples:
            out["samples"] = samp
        return out


    def trace_tsm(self, nprobes, seed, xi_loose, ncorr, seed_corr, xi_tight, basis=None, projector=OBLIQUE_G5,
                  hp_vectors=1, dilute=False, raise_on_fail=True, **opts):
        """Truncated Solver Method (lqt_trace_tsm): returns (main trace result, TSM result
        with the correction samples)."""
        main, out = TraceResult(), TsmResult()
        o = _opts(**opts)
        corr = torch.zeros(ncorr, dtype=torch.complex128)
        rc = lib().lqt_trace_tsm(self._h, basis._h if basis is not None else None, int(projector), int(nprobes),
                                 ctypes.c_uint64(seed), float(xi_loose), int(ncorr), ctypes.c_uint64(seed_corr),
                                 float(xi_tight), int(hp_vectors), int(bool(dilute)), ctypes.byref(o),
                                 ctypes.byref(main), ctypes.byref(out), _ptr(corr))
        self._check(rc, allow=() if raise_on_fail else (LQT_ENOTCONV,))
        m = {f: getattr(main, f) for f, _ in TraceResult._fields_}
        t = {f: getattr(out, f) for f, _ in TsmResult._fields_}
        t["corr_samples"] = corr
        t["rc"] = rc
        return m, t


class Basis:
    def __init__(self, ctx, handle, nv=0, nv2=0):
        self.ctx = ctx
        self._h = handle
        self.nv = nv
        self.nv2 = nv2
        k = ctypes.c_int(0)
        ctx._check(lib().lqt_basis_eigenvalues(self._h, None, ctypes.byref(k)))
        self.k = k.value

    def eigenvalues(self):
        lam = torch.empty(self.k, dtype=torch.complex128)
        k = ctypes.c_int(0)
        self.ctx._check(lib().lqt_basis_eigenvalues(self._h, _ptr(lam), ctypes.byref(k)))
        return lam

    def vectors(self):
        out = torch.empty((self.k, self.ctx.N), dtype=torch.complex128, device="cuda")
        self.ctx._check(lib().lqt_basis_vectors(self._h, _ptr(out)))
        return out

    def restrict(self, fine):
        fine = _dev(fine, torch.complex128, self.ctx.N, "restrict input")
        nrhs = fine.numel() // self.ctx.N
        nc = ctypes.c_longlong(0)
        self.ctx._check(lib().lqt_prolongator_get(self._h, None, ctypes.byref(nc)))
        out = torch.empty((nrhs, nc.value), dtype=torch.complex128, device="cuda")
        self.ctx._check(lib().lqt_restrict(self.ctx._h, self._h, _ptr(fine), _ptr(out), nrhs))
        return out

    def prolong(self, coarse):
        nc = ctypes.c_longlong(0)
        self.ctx._check(lib().lqt_prolongator_get(self._h, None, ctypes.byref(nc)))
        coarse = _dev(coarse, torch.complex128, nc.value, "prolong input")
        nrhs = coarse.numel() // nc.value
        out = torch.empty((nrhs, self.ctx.N), dtype=torch.complex128, device="cuda")
        self.ctx._check(lib().lqt_prolong(self.ctx._h, self._h, _ptr(coarse), _ptr(out), nrhs))
        return out

    def coarse_apply(self, coarse, herm=False):
        """W^+ A W (g5^W W^+ A W with herm) applied to coarse vectors by the explicit stencil."""
        nc = ctypes.c_longlong(0)
        self.ctx._check(lib().lqt_prolongator_get(self._h, None, ctypes.byref(nc)))
        coarse = _dev(coarse, torch.complex128, nc.value, "coarse input")
        out = torch.empty_like(coarse)
        self.ctx._check(lib().lqt_coarse_apply(self.ctx._h, self._h, _ptr(coarse), _ptr(out),
                                               coarse.numel() // nc.value, int(bool(herm))))
        return out

    def coarse2_apply(self, x, herm=False):
        """The level-2 operator W2^+ W^+ A W W2 (g5^{W2} times it with herm) on level-2 vectors."""
        nc2 = ctypes.c_longlong(0)
        self.ctx._check(lib().lqt_prolongator2_get(self._h, None, ctypes.byref(nc2)))
        x = _dev(x, torch.complex128, nc2.value, "level-2 input")
        out = torch.empty_like(x)
        self.ctx._check(lib().lqt_coarse2_apply(self.ctx._h, self._h, _ptr(x), _ptr(out), x.numel() // nc2.value,
                                                int(bool(herm))))
        return out

    def prolongator2(self):
        """W2 as a flat complex128 device tensor (layout in the header)."""
        nc2 = ctypes.c_longlong(0)
        self.ctx._check(lib().lqt_prolongator2_get(self._h, None, ctypes.byref(nc2)))
        nc = ctypes.c_longlong(0)
        self.ctx._check(lib().lqt_prolongator_get(self._h, None, ctypes.byref(nc)))
        # every level-1 coarse entry belongs to one level-2 block and chirality: nv2 * nc1 entries
        W2 = torch.empty(self.nv2 * nc.value, dtype=torch.complex128, device="cuda")
        self.ctx._check(lib().lqt_prolongator2_get(self._h, _ptr(W2), ctypes.byref(nc2)))
        return W2

    def prolongator(self):
        """W as a flat complex128 device tensor of nv*N entries (layout in the header)."""
        nc = ctypes.c_longlong(0)
        W = torch.empty(self.nv * self.ctx.N, dtype=torch.complex128, device="cuda")
        self.ctx._check(lib().lqt_prolongator_get(self._h, _ptr(W), ctypes.byref(nc)))
        return W

    def close(self):
        if self._h:
            lib().lqt_basis_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
