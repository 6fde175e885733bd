"""Pins of the oracle's field recovery at exterior points (eq. field_recovery)."""
import numpy as np
import pytest

from oracle import farfield as ff
from oracle import field, krylov, mie, vdim
from oracle.operator import Operator
from workloads import problems as P

K, NIN = 2 * np.pi, 2.0


def _targets():
    """Exterior points at radii 1.2 .. 3 (close to and away from the boundary r = 1)."""
    th = np.linspace(0.1, 2 * np.pi, 7, endpoint=False)
    r = np.array([1.2, 1.5, 2.0, 3.0])
    R, T = np.meshgrid(r, th)
    return (R * np.cos(T)).ravel(), (R * np.sin(T)).ravel()


def _exact_scattered(x, y):
    _, (nus, b) = mie.disk(K, NIN, 1.0, np.zeros(1), np.zeros(1))
    return mie.scattered_from_coefficients(K, nus, b, x, y)


def test_exact_interior_field_recovers_the_exterior_field():
    """The representation formula applied to the exact (Fourier-Bessel) interior field at the
    nodes reproduces the exact exterior field, with an error of the quadrature and VDIM
    discretisation that falls at high order under refinement."""
    tx, ty = _targets()
    ref = _exact_scattered(tx, ty)
    hs, errs = [], []
    for n in (3, 4, 6):
        prob = P.disk_problem(n, K, NIN)
        ue, _ = mie.disk(K, NIN, 1.0, prob.mesh.x, prob.mesh.y)
        us = field.scattered_field(prob.mesh, K, prob.m, ue, tx, ty)[0]
        errs.append(np.abs(us - ref).max() / np.abs(ref).max())
        hs.append(prob.mesh.cell_size)
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert order > 5.0, (errs, order)
    assert errs[-1] < 1e-4, errs


def test_discrete_solution_exterior_error_converges():
    """e_ext of the Nystrom solution itself (the paper's exterior error) converges at high order."""
    tx, ty = _targets()
    ref = _exact_scattered(tx, ty)
    errs = []
    for n in (3, 5):
        prob = P.disk_problem(n, K, NIN)
        C = vdim.correction_matrix(prob.mesh, prob.k)
        op = Operator(prob.mesh, prob.k, prob.m, C)
        u = krylov.lu_solve(op.dense(), prob.incident())
        us = field.scattered_field(prob.mesh, K, prob.m, u, tx, ty)[0]
        errs.append(np.abs(us - ref).max() / np.abs(ref).max())
    order = np.log(errs[0] / errs[1]) / np.log(5 / 3)
    assert order > 5.0 and errs[1] < 3e-4, (errs, order)


def test_large_distance_tends_to_the_exact_far_field():
    """u_s(R x^) sqrt(R) e^{-ikR} at R = 1e5 against the exact far-field pattern of the
    Fourier-Bessel solution (the O(1/(kR)) remainder is ~1e-7): the recovered field's error
    falls at high order under refinement, and it agrees with the far-field oracle (plain
    quadrature of the same asymptotic kernel) to the discretisation error."""
    th = np.array([0.0, 1.0, 2.5, 4.0])
    _, (nus, b) = mie.disk(K, NIN, 1.0, np.zeros(1), np.zeros(1))
    exact = mie.farfield_from_coefficients(K, nus, b, th)
    R = 1e5
    hs, errs = [], []
    for n in (3, 4, 6):
        prob = P.disk_problem(n, K, NIN)
        ue, _ = mie.disk(K, NIN, 1.0, prob.mesh.x, prob.mesh.y)
        us = field.scattered_field(prob.mesh, K, prob.m, ue, R * np.cos(th), R * np.sin(th))[0]
        scaled = us * np.sqrt(R) * np.exp(-1j * K * R)
        errs.append(np.abs(scaled - exact).max() / np.abs(exact).max())
        hs.append(prob.mesh.cell_size)
        uinf = ff.farfield(ff.farfield_matrix(prob.mesh, K, th), prob.m, ue[None, :])[0]
        assert np.abs(uinf - exact).max() / np.abs(exact).max() < 3 * errs[-1] + 1e-6
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert order > 5.0 and errs[-1] < 1e-4, (errs, order)


def test_points_inside_are_rejected():
    prob = P.disk_problem(3, K, NIN)
    with pytest.raises(ValueError):
        field.scattered_field(prob.mesh, K, prob.m, np.ones(prob.n_nodes), np.array([0.5]), np.array([0.0]))
