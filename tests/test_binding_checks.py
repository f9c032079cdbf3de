"""The Python binding refuses tensors whose pointer would make a kernel read out of bounds or
dereference host memory (wrong dtype for the precision, a host tensor, a size that is not a
whole number of fields) before it calls into the library.  No GPU: the library entry points
are replaced by a function that fails the test if it is ever reached."""
import pytest
import torch

import paper_1909_12234_amd.lqtrace as L


class _FakeDev(torch.Tensor):
    """A host tensor that reports itself as device-resident (the checks only read
    is_cuda, dtype and numel)."""

    @property
    def is_cuda(self):
        return True


def _dev(n, dtype):
    return torch.zeros(n, dtype=dtype).as_subclass(_FakeDev)


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError(f"library entry point {name} reached despite an invalid argument")


@pytest.fixture
def ctx(monkeypatch):
    monkeypatch.setattr(L, "lib", lambda: _NoLib())
    c = object.__new__(L.Context)
    c.N = 12 * 16
    c._h = None
    return c


def test_apply_rejects_host_tensor(ctx):
    with pytest.raises(TypeError, match="device tensor"):
        ctx.apply(torch.zeros(ctx.N, dtype=torch.complex128))


def test_apply_rejects_dtype_of_other_precision(ctx):
    # complex64 with the default FP64 precision would make the kernel read 2x past the end
    with pytest.raises(TypeError, match="complex128"):
        ctx.apply(_dev(ctx.N, torch.complex64))
    with pytest.raises(TypeError, match="complex64"):
        ctx.apply(_dev(ctx.N, torch.complex128), prec=L.F32)
    with pytest.raises(ValueError):
        ctx.apply(_dev(ctx.N, torch.complex128), prec=7)


def test_apply_rejects_partial_field(ctx):
    with pytest.raises(ValueError, match="multiple"):
        ctx.apply(_dev(ctx.N + 3, torch.complex128))
    # zero fields pass the check (the library treats them as a no-op)
    assert L._dev(_dev(0, torch.complex128), torch.complex128, ctx.N, "x").numel() == 0


@pytest.mark.parametrize("call", ["solve", "precond_apply", "precond_loss_grad", "basis_from_vectors", "gram_x",
                                  "project_probes"])
def test_field_inputs_checked(ctx, call):
    bad = [torch.zeros(ctx.N, dtype=torch.complex128), _dev(ctx.N, torch.complex64),
           _dev(ctx.N - 1, torch.complex128)]
    for t in bad:
        with pytest.raises((TypeError, ValueError)):
            if call == "solve":
                ctx.solve(t, 1e-8)
            elif call == "precond_apply":
                ctx.precond_apply(t)
            elif call == "precond_loss_grad":
                ctx.precond_loss_grad(t)
            elif call == "basis_from_vectors":
                ctx.basis_from_vectors(t)
            elif call == "gram_x":
                ctx.gram(t, t)
            else:
                ctx.project_probes(t, 1, 0, 4)


def test_combine_checks_shapes(ctx):
    C = torch.zeros((2, 3), dtype=torch.complex128)
    with pytest.raises(ValueError, match="rows"):
        ctx.combine(_dev(3 * ctx.N, torch.complex128), C)
    with pytest.raises(TypeError):
        ctx.combine(_dev(2 * ctx.N, torch.complex128), C, Y=torch.zeros(3 * ctx.N, dtype=torch.complex128))
