"""Pins of the synthetic inputs: the quadrature rule and the curved meshes."""
import itertools
from math import factorial

import numpy as np
import pytest

from workloads import mesh as M
from workloads.rule10 import rule10


def _tri_moment(a, b):
    # int over {xi, eta >= 0, xi + eta <= 1} of xi^a eta^b = a! b! / (a+b+2)!
    return factorial(a) * factorial(b) / factorial(a + b + 2)


def test_rule_exact_to_degree_5():
    bary, w = rule10()
    xi, eta = bary[:, 1], bary[:, 2]
    for d in range(6):
        for a in range(d + 1):
            b = d - a
            assert abs(np.sum(w * xi ** a * eta ** b) - _tri_moment(a, b)) < 4e-17 * 21


def test_rule_not_exact_at_degree_6():
    bary, w = rule10()
    xi, eta = bary[:, 1], bary[:, 2]
    errs = [abs(np.sum(w * xi ** a * eta ** (6 - a)) - _tri_moment(a, 6 - a)) for a in range(7)]
    assert max(errs) > 1e-8


def test_rule_interior_positive_unisolvent():
    bary, w = rule10()
    assert w.min() > 0 and bary.min() > 0.07 and np.allclose(bary.sum(1), 1)
    assert len({tuple(np.round(p, 12)) for p in bary}) == 10
    xi, eta = bary[:, 1], bary[:, 2]
    V = np.stack([xi ** a * eta ** (d - a) for d in range(4) for a in range(d + 1)], 1)
    assert np.linalg.cond(V) < 1e4


def test_rule_symmetric():
    bary, w = rule10()
    for perm in itertools.permutations(range(3)):
        q = bary[:, perm]
        for p, wp in zip(q, w):
            i = np.argmin(np.abs(bary - p).sum(1))
            assert np.abs(bary[i] - p).max() < 1e-15 and abs(w[i] - wp) < 1e-17


def test_central_square_elements_exact_area():
    m = M.ogrid_disk(4)
    n_central = 2 * 16          # affine elements come first
    areas = m.w.reshape(-1, 10)[:n_central].sum(1)
    assert np.allclose(areas, (1.0 / 4) ** 2 / 2, rtol=0, atol=1e-16)


@pytest.mark.parametrize("builder,area,second", [
    (lambda n: M.ogrid_disk(n), np.pi, np.pi / 4),
    (lambda n: M.ellipse(n, 1.3, 0.6), np.pi * 1.3 * 0.6, np.pi * 1.3 ** 3 * 0.6 / 4),
    (lambda n: M.two_material_disk(n), np.pi, np.pi / 4),
])
def test_mesh_area_and_second_moment_converge(builder, area, second):
    e_prev = None
    for n in (2, 4, 8):
        m = builder(n)
        e = abs(m.w.sum() - area)
        e2 = abs(np.sum(m.w * m.x ** 2) - second)
        assert e2 < 1e-4 * 8.0 ** -(np.log2(n))
        if e_prev is not None:
            assert e < e_prev / 20          # high order: ~2^-5 or better per halving
        e_prev = e
    assert e_prev < 1e-10


def test_nodes_inside_their_subdomain():
    m = M.two_material_disk(3)
    r = np.hypot(m.x, m.y)
    sub = m.node_subdomain
    assert np.all(r[sub == 0] < 0.5) and np.all((r[sub == 1] > 0.5) & (r[sub == 1] < 1))
    assert m.n_nodes == 260 * 9


def test_mirror_symmetry_even_n():
    from scipy.spatial import cKDTree
    m = M.ogrid_disk(4)
    d, idx = cKDTree(np.stack([m.x, m.y], 1)).query(np.stack([m.x, -m.y], 1))
    assert d.max() < 1e-14 and np.abs(m.w[idx] - m.w).max() < 1e-16
