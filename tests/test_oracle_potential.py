"""Pins of the oracle's Green's function, polynomial potentials and correction C."""
import mpmath as mp
import numpy as np
import pytest
from scipy import special

from oracle import bessel, green, vdim
from tests import analytic as an
from workloads import mesh as M


def test_hankel_against_mpmath():
    mp.mp.dps = 40
    z = np.concatenate([np.logspace(-8, np.log10(120), 300), [2.0, 4.0, 8.0, 12.0, 25.0]])
    for n, f in ((0, bessel.h0), (1, bessel.h1)):
        ref = np.array([complex(mp.hankel1(n, mp.mpf(float(t)))) for t in z])
        err = np.abs(f(z) - ref) / np.abs(ref)
        assert err.max() < 1e-15


def _sample_targets(msh, count, seed):
    rng = np.random.default_rng(seed)
    return rng.choice(msh.n_nodes, count, replace=False)


@pytest.mark.parametrize("k", [2 * np.pi, 20.0])
def test_poly_potential_disk_addition_theorem(k):
    msh = M.ogrid_disk(4)
    curves = msh.curves
    rng = np.random.default_rng(1)
    pts = [np.array([0.3, -0.2]), np.array([0.0, 0.999]), np.array([-0.7, 0.69])]
    for x in pts:
        c = x + rng.uniform(-0.05, 0.05, 2)
        s = 0.09
        E = vdim.poly_potential(curves, True, x, c, s, k)
        for ia, (a, b) in enumerate(vdim.ALPHA):
            ref = an.annulus_poly_potential(k, 0.0, 1.0, an.scaled_monomial_coeffs(a, b, c, s), *x)
            scale = np.abs(an.annulus_poly_potential(k, 0.0, 1.0, {(0, 0): 1.0}, *x)) * (2 / s) ** (a + b)
            assert abs(E[ia] - ref) <= 2e-13 * scale, (x, a, b, E[ia], ref)


def test_poly_potential_annulus_inside_hole_and_outside():
    msh = M.two_material_disk(3)
    curves_ann = [cv for cv in msh.curves if cv.subdomain == 1]
    curves_in = [cv for cv in msh.curves if cv.subdomain == 0]
    k = 12.0
    c, s = np.array([0.1, 0.2]), 0.2
    cases = [(curves_ann, 0.5, 1.0, np.array([0.2, 0.1]), False),     # in the hole
             (curves_ann, 0.5, 1.0, np.array([0.0, 0.4995]), False),  # just inside the hole
             (curves_ann, 0.5, 1.0, np.array([0.0, 0.501]), True),    # just inside the annulus
             (curves_ann, 0.5, 1.0, np.array([0.6, -0.3]), True),     # in the annulus
             (curves_ann, 0.5, 1.0, np.array([0.4999, 0.0]), False),
             (curves_in, 0.0, 0.5, np.array([0.0, -0.5003]), False),  # just outside the inclusion
             (curves_in, 0.0, 0.5, np.array([0.3, 0.1]), True)]
    for curves, a_in, a_out, x, inside in cases:
        E = vdim.poly_potential(curves, inside, x, c, s, k)
        base = np.abs(an.annulus_poly_potential(k, a_in, a_out, {(0, 0): 1.0}, *x))
        for ia, (a, b) in enumerate(vdim.ALPHA):
            ref = an.annulus_poly_potential(k, a_in, a_out, an.scaled_monomial_coeffs(a, b, c, s), *x)
            # near-interface targets cancel layer potentials of size ~ Phi ~ 1/k^2
            assert abs(E[ia] - ref) <= 3e-13 * (base + 1 / k ** 2) * (2 / s) ** (a + b), (x, a, b)


def test_poly_potential_ellipse_brute_force():
    msh = M.ellipse(3, 1.3, 0.6)
    k = 9.0
    c, s = np.array([0.2, -0.1]), 0.3
    for x, nphi in ((np.array([0.25, 0.1]), 400), (np.array([-1.0, 0.35]), 1600)):
        E = vdim.poly_potential(msh.curves, True, x, c, s, k)
        ref = an.polar_potential(k, x, an.ellipse_rho_max(x, 1.3, 0.6),
                                 lambda px, py: vdim.monomials(px, py, c, s), n_phi=nphi)
        base = np.abs(ref[0])
        for ia, (a, b) in enumerate(vdim.ALPHA):
            assert abs(E[ia] - ref[ia]) <= 1e-12 * base * (2 / s) ** (a + b), (x, a, b)


def test_constant_density_closed_form_disk():
    """((G~W + C) 1)_j = -1/k^2 + (i pi a / (2k)) H1(k a) J0(k |y_j|) on the disk |y| < a."""
    msh = M.ogrid_disk(3)
    k = 2 * np.pi
    C = vdim.correction_matrix(msh, k)
    F = green.far_matrix(msh.x, msh.y, msh.w, k)
    v = F.sum(1) + C @ np.ones(msh.n_nodes)
    exact = -1 / k ** 2 + 0.5j * np.pi / k * bessel.h1(k) * special.j0(k * np.hypot(msh.x, msh.y))
    assert np.abs(v - exact).max() <= 1e-13 * np.abs(exact).max()


@pytest.mark.parametrize("which", ["disk", "two-material"])
def test_polynomial_exactness_against_addition_theorem(which):
    """For a cubic P, (G~W + C) P at node j equals int_Omega G(y_j, y) P(y) dy (sum over
    subdomains), which the addition theorem evaluates independently."""
    msh = M.ogrid_disk(3) if which == "disk" else M.two_material_disk(2)
    k = 7.0
    coeffs = {(0, 0): 0.3, (1, 0): -0.2, (0, 1): 0.5, (2, 0): 1.0, (1, 1): -2.0, (0, 2): 0.25,
              (3, 0): 1.0, (2, 1): 0.4, (1, 2): -0.7, (0, 3): 0.1}
    P = sum(v * msh.x ** i * msh.y ** j for (i, j), v in coeffs.items())
    rows = _sample_targets(msh, 12, 3)
    C = vdim.correction_matrix(msh, k, rows)
    far = green.far_rows(msh.x, msh.y, msh.w, k, P, rows)[0]
    got = far + C @ P
    ref = np.array([an.annulus_poly_potential(k, 0.0, 1.0, coeffs, msh.x[j], msh.y[j]) for j in rows])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_correction_row_structure():
    msh = M.two_material_disk(2)
    C = vdim.correction_matrix(msh, 5.0, rows=[0, 700])
    assert C.nnz == 2 * 10 * 2
    cols0 = C[0].indices
    assert set(cols0[:10]) == set(range(10))     # own element first
