"""Property-based checks of the operator on tiny meshes (hypothesis draws seeds and scalars):
linearity, the adjoint identity and invariance under the caller's node order."""
import numpy as np
import pytest
import torch
from hypothesis import given, settings, strategies as st

import paper_2608_17615_amd as lsg
from workloads import problems as P

pytestmark = pytest.mark.gpu

_PROB = {}


def _problem():
    if "p" not in _PROB:
        p = P.graded_two_material(2, 8.0)
        _PROB["p"] = p
        _PROB["op"] = lsg.Operator(lsg.Scatterer.from_mesh(p.mesh, p.m, p.k))
    return _PROB["p"], _PROB["op"]


def _vec(rng, B, n):
    return torch.tensor(rng.standard_normal((B, n)) + 1j * rng.standard_normal((B, n)), device="cuda")


cplx = st.complex_numbers(min_magnitude=0.1, max_magnitude=10.0, allow_nan=False, allow_infinity=False)


@settings(max_examples=15, deadline=None)
@given(seed=st.integers(0, 2**31 - 1), a=cplx, b=cplx, B=st.integers(1, 20),
       precision=st.sampled_from(["fp64", "mixed"]))
def test_linearity(seed, a, b, B, precision):
    p, op = _problem()
    rng = np.random.default_rng(seed)
    x, y = _vec(rng, B, p.n_nodes), _vec(rng, B, p.n_nodes)
    lhs = op.apply(a * x + b * y, precision=precision)
    rhs = a * op.apply(x, precision=precision) + b * op.apply(y, precision=precision)
    scale = (abs(a) * op.apply(x, precision=precision).abs().max() +
             abs(b) * op.apply(y, precision=precision).abs().max()).item()
    tol = 1e-13 if precision == "fp64" else 3e-6
    assert (lhs - rhs).abs().max().item() <= tol * scale


@settings(max_examples=15, deadline=None)
@given(seed=st.integers(0, 2**31 - 1), B=st.integers(1, 20))
def test_adjoint_identity(seed, B):
    p, op = _problem()
    rng = np.random.default_rng(seed)
    x, y = _vec(rng, B, p.n_nodes), _vec(rng, B, p.n_nodes)
    lhs = (op.apply(x) * y.conj()).sum(dim=1)
    rhs = (x * op.apply(y, adjoint=True).conj()).sum(dim=1)
    scale = (x.norm(dim=1) * y.norm(dim=1) * (1 + op.apply(x).norm(dim=1) / x.norm(dim=1)))
    assert ((lhs - rhs).abs() / scale).max().item() <= 1e-14


@settings(max_examples=6, deadline=None)
@given(seed=st.integers(0, 2**31 - 1))
def test_node_order_does_not_matter(seed):
    """Shuffling the elements and the nodes inside each element changes the results only by
    rounding (the library sorts nodes internally and returns the caller's order).  Each element is
    first moved by ~1e-6: the symmetric mesh has elements at exactly equal distances from some
    targets, where the nearest-centroid choice of the correction falls to the caller's element
    index (a reading of the method, not rounding).  The bound allows for the correction rows'
    Vandermonde solves, whose rounding a reordering of an element's nodes changes (condition
    ~1e4: about 4e-12 was measured)."""
    p, _ = _problem()
    rng = np.random.default_rng(seed)
    msh = p.mesh
    ne = p.n_nodes // 10
    jx, jy = np.repeat(1e-6 * rng.standard_normal(ne), 10), np.repeat(1e-6 * rng.standard_normal(ne), 10)
    x0, y0 = msh.x + jx, msh.y + jy
    op1 = lsg.Operator(lsg.Scatterer(x0, y0, msh.w, msh.elem_subdomain, p.m, p.k, list(msh.curves)))
    pe = rng.permutation(ne)
    idx = np.concatenate([10 * e + rng.permutation(10) for e in pe])
    op2 = lsg.Operator(lsg.Scatterer(x0[idx], y0[idx], msh.w[idx], msh.elem_subdomain[pe], p.m[idx], p.k,
                                     list(msh.curves)))
    x = _vec(rng, 3, p.n_nodes)
    it = torch.tensor(idx, device="cuda")
    y = op1.apply(x)
    y2 = op2.apply(x[:, it].contiguous())
    e = ((y2 - y[:, it]).abs().max() / y.abs().max()).item()
    op1.close()
    op2.close()
    assert e <= 1e-10
