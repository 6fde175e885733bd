"""Pins of the oracle's discrete solution, adjoint and gradient."""
import numpy as np
import pytest
from scipy import special

from oracle import farfield as ff
from oracle import krylov, mie, vdim
from oracle.operator import Operator
from tests import analytic as an
from workloads import problems as P


def _solve(prob):
    C = vdim.correction_matrix(prob.mesh, prob.k)
    op = Operator(prob.mesh, prob.k, prob.m, C)
    return op, krylov.lu_solve(op.dense(), prob.incident())


def test_mie_series_solves_continuous_equation():
    """u + k^2 int_disk G m u = u_inc at interior points for the Fourier-Bessel field."""
    k, n_in, a = 2 * np.pi, 2.0, 1.0
    ki = k * np.sqrt(n_in)
    m = 1 - n_in
    pts = np.array([[0.3, 0.2], [-0.55, 0.6], [0.0, -0.9]])
    u, _ = mie.disk(k, n_in, a, pts[:, 0], pts[:, 1])
    nmax = int(np.ceil(ki * a + 20 + 6 * (ki * a) ** (1 / 3)))
    nus = np.arange(-nmax, nmax + 1)
    Jia, dJia = special.jv(nus, ki * a), special.jvp(nus, ki * a)
    Ha, dHa = special.hankel1(nus, k * a), special.h1vp(nus, k * a)
    coef = (1j ** nus) * (2j / (np.pi * a)) / (k * Jia * dHa - ki * dJia * Ha)
    for (x, y), uu in zip(pts, u):
        r, th = np.hypot(x, y), np.arctan2(y, x)
        vol = sum(c * an.disk_mode_potential_fn(k, a, int(nu), lambda t, nu=nu: special.jv(nu, ki * t), r, th)
                  for nu, c in zip(nus, coef) if abs(c) > 1e-18)
        lhs = uu + k * k * m * vol
        assert abs(lhs - np.exp(1j * k * x)) < 1e-12


def test_mie_disk_high_order_convergence():
    """Nystrom + VDIM solution against the Fourier-Bessel series: observed order >= 5
    (p = 3 interpolation, degree-5 rule; the paper measures 6.1 at p = 3, Section 6.1)."""
    hs, errs = [], []
    for n in (4, 5, 6):
        prob = P.disk_problem(n, 2 * np.pi, 2.0)
        _, u = _solve(prob)
        ue, _ = mie.disk(prob.k, 2.0, 1.0, prob.mesh.x, prob.mesh.y)
        errs.append(np.abs(u[0] - ue).max() / np.abs(ue).max())
        hs.append(prob.mesh.cell_size)
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert order > 5.0, (errs, order)
    assert errs[1] < 5e-4          # the N = 2500 workload


def test_two_layer_disk_convergence():
    """Two constant-index subdomains with non-matching interface nodes (foreign-subdomain
    rows of C) against the two-layer Fourier-Bessel series."""
    errs = []
    for ni in (2, 3):
        prob = P.two_layer_constant(ni, 2 * np.pi, 2.5, 1.6)
        _, u = _solve(prob)
        ue, _ = mie.two_layer(prob.k, 2.5, 1.6, 0.5, 1.0, prob.mesh.x, prob.mesh.y)
        errs.append(np.abs(u[0] - ue).max() / np.abs(ue).max())
    order = np.log(errs[0] / errs[1]) / np.log(3 / 2)
    assert order > 5.0 and errs[1] < 3e-4, (errs, order)


def test_gmres_matches_lu():
    prob = P.disk_problem(3, 2 * np.pi, 2.0)
    op, u = _solve(prob)
    Ld = op.dense()
    x, it, hist = krylov.gmres(lambda v: Ld @ v, prob.incident()[0], tol=1e-13, maxit=400)
    assert hist[-1] <= 1e-13
    assert np.abs(x - u[0]).max() <= 1e-11 * np.abs(u).max()
    res = np.linalg.norm(op.apply(x)[0] - prob.incident()[0]) / np.linalg.norm(prob.incident()[0])
    assert res < 1e-12


def test_reflection_symmetry():
    prob = P.disk_problem(4, 2 * np.pi, 2.0)
    _, u = _solve(prob)
    from scipy.spatial import cKDTree
    msh = prob.mesh
    _, idx = cKDTree(np.stack([msh.x, msh.y], 1)).query(np.stack([msh.x, -msh.y], 1))
    assert np.abs(u[0][idx] - u[0]).max() < 1e-12 * np.abs(u).max()


def test_farfield_and_energy_balance():
    """Far field of the discrete solution vs the Fourier-Bessel far field, and the energy
    balance Im sum w conj(m u) u_inc = (1/k) ||u_inf||^2 for a real index (Section 5)."""
    prob = P.disk_problem(5, 2 * np.pi, 2.0)
    _, u = _solve(prob)
    th = P.receivers(128)
    A = ff.farfield_matrix(prob.mesh, prob.k, th)
    uinf = ff.farfield(A, prob.m, u)[0]
    _, (nus, b) = mie.disk(prob.k, 2.0, 1.0, prob.mesh.x, prob.mesh.y)
    uinf_exact = mie.farfield_from_coefficients(prob.k, nus, b, th)
    assert np.abs(uinf - uinf_exact).max() < 1e-3 * np.abs(uinf_exact).max()
    lhs = np.imag(np.sum(prob.mesh.w * np.conj(prob.m * u[0]) * prob.incident()[0]))
    rhs = (2 * np.pi / th.size) * np.sum(np.abs(uinf) ** 2) / prob.k
    rhs_exact = (2 * np.pi / th.size) * np.sum(np.abs(uinf_exact) ** 2) / prob.k
    assert lhs > 0 and abs(lhs - rhs) < 1e-3 * rhs and abs(rhs - rhs_exact) < 1e-3 * rhs_exact


def test_adjoint_identity():
    prob = P.two_layer_constant(2, 5.0, 2.0, 1.5)
    C = vdim.correction_matrix(prob.mesh, prob.k)
    op = Operator(prob.mesh, prob.k, prob.m + 0.3j, C)       # complex contrast too
    x = P.random_vectors(prob.n_nodes, 1, 1)
    y = P.random_vectors(prob.n_nodes, 1, 2)
    lhs = np.vdot(op.apply(x)[0], y[0])
    rhs = np.vdot(x[0], op.apply_adjoint(y)[0])
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(op.apply(x)) * np.linalg.norm(y)


def test_gradient_finite_differences_and_identity():
    prob = P.disk_problem(3, 5.0, 1.8, directions=[0.0, 2.0])
    C = vdim.correction_matrix(prob.mesh, prob.k)
    A = ff.farfield_matrix(prob.mesh, prob.k, P.receivers(16))
    m0 = prob.m + 0.05 * np.sin(3 * prob.mesh.x)
    b = prob.incident()

    def J_of(m):
        op = Operator(prob.mesh, prob.k, m, C)
        u = krylov.lu_solve(op.dense(), b)
        return op, u

    dm = P.contrast_perturbation(prob.mesh, seed=7)
    op_t, u_t = J_of(m0 + dm)
    data = ff.farfield(A, op_t.m, u_t)
    op, u = J_of(m0)
    J, grad, a, lam = ff.adjoint_gradient(op, A, u, data)
    rng = np.random.default_rng(11)
    eps = 1e-6 * np.abs(m0).max()
    for _ in range(3):
        d = rng.standard_normal(m0.size)
        Jp = ff.misfit(A, m0 + eps * d, J_of(m0 + eps * d)[1], data)[0]
        Jm = ff.misfit(A, m0 - eps * d, J_of(m0 - eps * d)[1], data)[0]
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - grad @ d) <= 1e-6 * abs(fd)
    ident = np.sum(np.real(np.conj(lam / np.conj(m0)[None, :]) * u), axis=0)
    assert np.abs(ident - grad).max() <= 1e-10 * np.abs(grad).max()
