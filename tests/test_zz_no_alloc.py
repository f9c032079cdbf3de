"""The allocation-free Gram entry point (lqt_gram_noalloc, static device workspace) against
lqt_gram, through the C-ABI: two calls in a row on the same device, the second with a smaller
input, at FP64 rounding (the two differ only in the order of the sums); a multi-lattice
context; the size limit of the workspace."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _crand(shape, seed):
    r = np.random.default_rng(seed)
    return torch.as_tensor(r.standard_normal(shape) + 1j * r.standard_normal(shape)).cuda()


def _check(c, X, Y):
    ref = c.gram(X, Y).numpy()
    got = c.gram_noalloc(X, Y).numpy()
    n = X.shape[1]
    tol = 1e-13 * np.sqrt(n) * np.max(np.abs(ref))
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= tol, (np.max(np.abs(got - ref)), tol)


def test_noalloc_gram_two_calls_then_smaller(gpu):
    lq = gpu
    dims = (16, 16, 16, 32)
    print("no-alloc gram 16^3x32: 64 x 48, then 5 x 3", flush=True)
    c = lq.Context(dims, -1.9)
    N = c.N
    X, Y = _crand((64, N), 1), _crand((48, N), 2)
    _check(c, X, Y)
    _check(c, X[:5].contiguous(), Y[:3].contiguous())
    c.close()


def test_noalloc_gram_ragged_and_multi_lattice(gpu):
    lq = gpu
    print("no-alloc gram: ragged lattice, then three lattices", flush=True)
    c = lq.Context((3, 5, 4, 6), 0.1)
    _check(c, _crand((19, c.N), 3), _crand((37, c.N), 4))
    _check(c, _crand((1, c.N), 5), _crand((1, c.N), 6))
    c.close()
    # canonical multi-lattice fields are the lattices' arrays one after the other
    c = lq.Context([(8, 8, 8, 8), (4, 4, 4, 4), (3, 5, 4, 6)], [0.1] * 3)
    _check(c, _crand((7, c.N), 7), _crand((9, c.N), 8))
    c.close()


def test_noalloc_gram_rejects_oversize(gpu):
    lq = gpu
    c = lq.Context((2, 2, 2, 2), 0.1)
    X = _crand((1100, c.N), 9)
    with pytest.raises(lq.LqtError) as e:
        c.gram_noalloc(X, X)
    assert e.value.code == lq.LQT_EINVAL and "static workspace" in str(e.value)
    # the largest accepted product still works and matches
    _check(c, X[:1024].contiguous(), X[:1024].contiguous())
    c.close()
