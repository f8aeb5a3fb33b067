"""Argument checks of the Python binding, run without a GPU.

The library sizes every device read and write from the precision and the
node count it was given, so the binding must reject a tensor of the wrong
dtype, length or aliasing before any call reaches it.  These tests build an
Operator shell without a handle (no library call is made) and check that
every entry point raises ValueError on such input."""
import pytest
import torch

from paper_2109_05072_amd.operator import Operator


def _shell(n_nodes=27, n_elem=8, q=4, ncomp=1):
    op = Operator.__new__(Operator)
    op.n_nodes, op.n_elem, op.q, op.ncomp = n_nodes, n_elem, q, ncomp
    op.handle = None
    op._cg_work = None
    op.device = torch.device("cpu")
    return op


def test_apply_rejects_mismatched_output_dtype():
    op = _shell()
    x = torch.zeros(27, dtype=torch.float64)
    with pytest.raises(ValueError, match="y must be torch.float64"):
        op.apply(x, torch.zeros(27, dtype=torch.float32))
    with pytest.raises(ValueError, match="y must be torch.float64"):
        op.apply_add(x, torch.zeros(27, dtype=torch.float32))
    with pytest.raises(ValueError, match="y must be torch.float32"):
        op.apply_adjoint(x.float(), torch.zeros(27, dtype=torch.float64))


def test_apply_rejects_unsupported_dtype_and_length():
    op = _shell()
    with pytest.raises(ValueError, match="float64 or float32"):
        op.apply(torch.zeros(27, dtype=torch.float16))
    with pytest.raises(ValueError, match="multiple of n_nodes"):
        op.apply(torch.zeros(28, dtype=torch.float64))
    with pytest.raises(ValueError, match="y has 54 entries"):
        op.apply(torch.zeros(27, dtype=torch.float64), torch.zeros(54, dtype=torch.float64))


def test_apply_rejects_aliasing_and_host_tensors():
    op = _shell()
    x = torch.zeros(27, dtype=torch.float64)
    with pytest.raises(ValueError, match="device tensor"):
        op.apply(x, torch.zeros(27, dtype=torch.float64))
    with pytest.raises(ValueError):
        op.apply(x, x)


def test_solver_and_gradient_entry_points_require_float64():
    op = _shell()
    b64 = torch.zeros(27, dtype=torch.float64)
    f32 = torch.zeros(27, dtype=torch.float32)
    with pytest.raises(ValueError, match="b must be torch.float64"):
        op.cg(f32)
    with pytest.raises(ValueError, match="x must be torch.float64"):
        op.cg(b64, x=f32)
    with pytest.raises(ValueError, match="x has 26 entries"):
        op.cg(b64, x=torch.zeros(26, dtype=torch.float64))
    with pytest.raises(ValueError, match="u must be torch.float64"):
        op.kappa_grad(f32, b64)
    with pytest.raises(ValueError, match="r must be torch.float64"):
        op.kappa_grad(b64, f32)
    with pytest.raises(ValueError, match="r must be torch.float64"):
        op.mg_apply(f32)
    with pytest.raises(ValueError, match="z must be torch.float64"):
        op.mg_apply(b64, torch.zeros(27, dtype=torch.float32))


def test_per_point_inputs_are_sized_by_elements_and_points():
    op = _shell(n_elem=8, q=4)
    with pytest.raises(ValueError, match="f_q has 511 entries, expected 512"):
        op.rhs(torch.zeros(511, dtype=torch.float64))
    with pytest.raises(ValueError, match="f_q must be torch.float64"):
        op.rhs(torch.zeros(512, dtype=torch.float32))
    with pytest.raises(ValueError, match="kappa must be torch.float64"):
        op.set_kappa(torch.zeros(512, dtype=torch.float32))
    with pytest.raises(ValueError, match="kappa has 500 entries"):
        op.set_kappa(torch.zeros(500, dtype=torch.float64))
