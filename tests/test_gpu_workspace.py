"""The operator application allocates nothing once its workspace is reserved (the boundary's
rule that ls_apply never allocates), refuses to run on a workspace that is too small, and gives
the same result as an application that reserved for itself."""
import numpy as np
import pytest
import torch

import paper_2608_17615_amd as lsg
from workloads import problems as P

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nrhs,precision", [(1, "fp64"), (3, "fp64"), (16, "fp64"), (16, "mixed")])
def test_apply_after_reserve_allocates_nothing(nrhs, precision):
    p = P.graded_two_material(2, 8.0)
    op = lsg.Operator(lsg.Scatterer.from_mesh(p.mesh, p.m, p.k))
    x = torch.tensor(P.random_vectors(op.n, nrhs, 3), device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(lsg.LSError):        # nothing reserved yet
        op.apply_raw(x, y, precision)
    op.reserve(nrhs, precision)
    torch.cuda.synchronize()
    before = lsg.device_allocations()
    for _ in range(3):
        op.apply_raw(x, y, precision)
        op.apply_raw(x, y, precision, adjoint=True)
    torch.cuda.synchronize()
    assert lsg.device_allocations() == before
    ref = op.apply(x, precision=precision)
    op.apply_raw(x, y, precision)
    assert torch.equal(y, ref)


def test_batched_scatterers_reserve_tables():
    a, b = P.disk_problem(3, 9.0, 2.0), P.graded_two_material(2, 8.0)
    op = lsg.Operator([lsg.Scatterer.from_mesh(q.mesh, q.m, q.k) for q in (a, b)])
    x = torch.tensor(P.random_vectors(op.n, 16, 4), device="cuda")
    y = torch.empty_like(x)
    op.reserve(16, "mixed")
    torch.cuda.synchronize()
    before = lsg.device_allocations()
    op.apply_raw(x, y, "mixed")
    op.apply_raw(x, y, "mixed")
    torch.cuda.synchronize()
    assert lsg.device_allocations() == before
    assert torch.equal(y, op.apply(x, precision="mixed"))
