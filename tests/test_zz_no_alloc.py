"""The allocation-free application ls_apply_noalloc (its workspace is a static per-GPU device array
of the library) against ls_apply on the same inputs, to the FP64 parity bar (and the FP32-tile bar
for the mixed precision), on two calls in a row, the second with a smaller input; it allocates
nothing, and sizes beyond its workspace are refused."""
import numpy as np
import pytest
import torch

import paper_2608_17615_amd as lsg
from workloads import problems as P

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def _pair(op, nrhs, seed, precision):
    x = torch.tensor(P.random_vectors(op.n, nrhs, seed), device="cuda")
    ref = op.apply(x, precision=precision)
    y = torch.full_like(x, complex(np.nan, np.nan))
    torch.cuda.synchronize()
    before = lsg.device_allocations()
    op.apply_noalloc(x, y, precision)
    torch.cuda.synchronize()
    assert lsg.device_allocations() == before
    return _rel(y, ref)


@pytest.mark.parametrize("precision,first,second,bar", [("fp64", 3, 1, 1e-13), ("fp64", 16, 4, 1e-13),
                                                         ("mixed", 16, 2, 1e-5)])
def test_matches_apply_on_two_calls(precision, first, second, bar):
    p = P.graded_two_material(3, 12.0)                      # N = 2 340
    op = lsg.Operator(lsg.Scatterer.from_mesh(p.mesh, p.m, p.k))
    e1 = _pair(op, first, 1, precision)
    e2 = _pair(op, second, 2, precision)                    # smaller input, the same workspace
    print(f"{precision}: {first} columns {e1:.1e}, then {second} columns {e2:.1e}", flush=True)
    assert e1 <= bar and e2 <= bar


def test_full_size_single_wave_and_several_scatterers():
    """N = 58 500, one wave: fewer source splits than ls_apply fit the workspace; and a handle with
    two scatterers (one launch each)."""
    p = P.config2()
    op = lsg.Operator(lsg.Scatterer.from_mesh(p.mesh, p.m, p.k))
    e = _pair(op, 1, 5, "fp64")
    print(f"N={op.n}: {e:.1e}", flush=True)
    assert e <= 1e-13
    op.close()
    a, b = P.disk_problem(3, 9.0, 2.0), P.graded_two_material(2, 8.0)
    two = lsg.Operator([lsg.Scatterer.from_mesh(q.mesh, q.m, q.k) for q in (a, b)])
    assert _pair(two, 16, 6, "fp64") <= 1e-13
    assert _pair(two, 2, 7, "fp64") <= 1e-13


def test_too_large_is_refused_before_anything_runs():
    p = P.config2()
    op = lsg.Operator(lsg.Scatterer.from_mesh(p.mesh, p.m, p.k))
    x = torch.zeros((64, op.n), dtype=torch.complex128, device="cuda")
    y = torch.full_like(x, 7.0)
    with pytest.raises(lsg.LSError, match="64 MiB"):
        op.apply_noalloc(x, y)
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
