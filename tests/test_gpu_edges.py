"""Edge cases through the C ABI: no right-hand sides, zero vectors, padded leading dimensions and
the smallest mesh (fewer nodes than one workgroup), checked against the oracle or exactly."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2608_17615_amd as lsg
from oracle import vdim
from oracle.operator import Operator as OOp
from tests.gpu_cases import relmax
from workloads import problems as P

pytestmark = pytest.mark.gpu


def _op(prob, **kw):
    return lsg.Operator(lsg.Scatterer.from_mesh(prob.mesh, prob.m, prob.k), **kw)


def test_no_right_hand_sides_is_a_no_op():
    prob = P.disk_problem(2, 6.0, 2.0)
    op = _op(prob)
    L = lsg.lib()
    x = torch.full((1, prob.n_nodes), 3.0 + 1.0j, dtype=torch.complex128, device="cuda")
    y = x.clone()
    st = lsg._stream()
    assert L.ls_apply(op._h, x.data_ptr(), y.data_ptr(), 0, prob.n_nodes, lsg.FP64, st) == lsg.LS_OK
    assert L.ls_apply_adjoint(op._h, x.data_ptr(), y.data_ptr(), 0, prob.n_nodes, lsg.MIXED, st) == lsg.LS_OK
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    o = lsg._SolveOpts(1e-8, 10, 0, lsg.FP64, 0, 0, 0, 0.0)
    assert L.ls_solve_gmres(op._h, x.data_ptr(), y.data_ptr(), 0, prob.n_nodes, ctypes.byref(o), None, st) == lsg.LS_OK
    assert torch.equal(x, y)


@pytest.mark.parametrize("precision,B", [("fp64", 1), ("fp64", 16), ("mixed", 3)])
def test_zero_vectors(precision, B):
    """L 0 = 0 exactly on every path, and L x = 0 is solved by x = 0 without a step."""
    prob = P.disk_problem(2, 6.0, 2.0)
    op = _op(prob)
    z = torch.zeros((B, prob.n_nodes), dtype=torch.complex128, device="cuda")
    assert op.apply(z, precision=precision).abs().max().item() == 0.0
    assert op.apply(z, precision=precision, adjoint=True).abs().max().item() == 0.0
    x, info = op.solve(z, tol=1e-10, maxit=50, precision=precision)
    assert info["converged"] and x.abs().max().item() == 0.0 and int(info["iters"].max()) == 0


@pytest.mark.parametrize("precision,B", [("fp64", 1), ("fp64", 20), ("mixed", 5)])
def test_padded_leading_dimension(precision, B):
    """Columns with ld > N (padding left untouched) give the contiguous result bit for bit."""
    prob = P.graded_two_material(2, 8.0)
    op = _op(prob)
    n, ld = prob.n_nodes, prob.n_nodes + 37
    rng = np.random.default_rng(7)
    x = torch.tensor(rng.standard_normal((B, n)) + 1j * rng.standard_normal((B, n)), device="cuda")
    ref = op.apply(x, precision=precision)
    xp = torch.full((B, ld), 5.0 - 2.0j, dtype=torch.complex128, device="cuda")
    xp[:, :n] = x
    yp = torch.full((B, ld), -7.0 + 0.5j, dtype=torch.complex128, device="cuda")
    L = lsg.lib()
    assert L.ls_apply(op._h, xp.data_ptr(), yp.data_ptr(), B, ld, lsg._PREC[precision], lsg._stream()) == lsg.LS_OK
    torch.cuda.synchronize()
    assert torch.equal(yp[:, :n], ref)
    assert torch.all(yp[:, n:] == -7.0 + 0.5j)
    # a leading dimension below N is rejected before anything is enqueued
    assert L.ls_apply(op._h, xp.data_ptr(), yp.data_ptr(), B, n - 1, lsg.FP64, lsg._stream()) == -1


def test_smallest_mesh_matches_oracle():
    """N = 100 (ten elements): fewer nodes than one workgroup of the far sum and one tile of 16."""
    prob = P.disk_problem(1, 4.0, 2.0)
    assert prob.n_nodes == 100
    op = _op(prob)
    C = vdim.correction_matrix(prob.mesh, prob.k)
    ref_op = OOp(prob.mesh, prob.k, prob.m, C)
    rng = np.random.default_rng(8)
    for B in (1, 17):
        x = rng.standard_normal((B, 100)) + 1j * rng.standard_normal((B, 100))
        y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
        e = relmax(y, ref_op.apply(x))
        print(f"N=100, B={B}: {e:.2e}", flush=True)
        assert e <= 1e-12
