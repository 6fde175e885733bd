"""Pins of the oracle's sparsifying Cartesian preconditioner (Section 4, subsection
"Sparsifying preconditioner")."""
import numpy as np
from scipy import integrate, special

from oracle import krylov
from oracle import sparsify as spf
from oracle.transfer import Grid


def _disk_grid(k, kh=0.8, radius=1.0, pad=0.02):
    h = kh / k
    nx = int(np.ceil((2 * (radius + pad)) / h)) + 1
    g = Grid(-radius - pad, -radius - pad, h, nx, nx)
    zx, zy = g.nodes()
    m = np.where(np.hypot(zx, zy) < radius, -1.0, 0.0)   # n^2 = 2 inside, m = 1 - n^2
    return g, m


def test_self_term_is_the_disk_integral():
    """The diagonal of V^(C): the integral of (i/4) H0(k|y|) over the disk of area h^2, against
    adaptive quadrature in the radius (real and imaginary parts separately)."""
    for k, h in ((10.0, 0.08), (40.0, 0.02), (3.0, 0.3)):
        a = h / np.sqrt(np.pi)
        opts = dict(limit=200, epsabs=1e-16, epsrel=1e-13)
        re = integrate.quad(lambda r: 2 * np.pi * r * (-0.25) * special.y0(k * r), 0, a, **opts)[0]
        im = integrate.quad(lambda r: 2 * np.pi * r * 0.25 * special.j0(k * r), 0, a, **opts)[0]
        assert abs(spf.self_term(k, h) - (re + 1j * im)) <= 1e-12 * abs(re + 1j * im)


def test_stencil_weights_minimise_the_far_block():
    """eq. sparsifying_min: no unit vector on the 9 neighbours does better than v, and the
    9-point Laplacian stencil (a fixed finite-difference choice) does far worse."""
    k = 10.0
    g, _ = _disk_grid(k)
    V = spf.cartesian_volume(g, k)
    v, offs, ratio = spf.stencil_weights(g, V)
    j0 = (g.ny // 2) * g.nx + g.nx // 2
    nb = spf.neighbours(g, j0)
    B = V[np.ix_(nb, np.setdiff1d(np.arange(g.n), nb))]
    best = np.linalg.norm(v @ B)
    assert abs(np.linalg.norm(v) - 1) < 1e-14
    assert abs(best / np.linalg.norm(B, 2) - ratio) < 1e-12 * ratio + 1e-18
    rng = np.random.default_rng(3)
    U = rng.standard_normal((4000, 9)) + 1j * rng.standard_normal((4000, 9))
    U /= np.linalg.norm(U, axis=1)[:, None]
    assert np.all(np.linalg.norm(U @ B, axis=1) >= best * (1 - 1e-9))
    lap = np.array([1, 4, 1, 4, -20, 4, 1, 4, 1], dtype=float)   # offsets in row-major order
    lap /= np.linalg.norm(lap)
    assert np.linalg.norm(lap @ B) > 10 * best
    assert ratio < 1e-3


def test_unfiltered_product_gives_the_exact_inverse():
    """With no filtering C^(C) = A L^(C), so S^(C) = (L^(C))^-1 whenever A is invertible."""
    k = 10.0
    g, m = _disk_grid(k, kh=1.2)
    S, L, _, _, _ = spf.sparsifying_preconditioner(g, k, m, width=None)
    assert np.abs(S @ L - np.eye(g.n)).max() < 1e-9


def test_exterior_columns_of_S_minus_I_vanish():
    """eq. S_minus_I: A - C^(C) = -k^2 (filtered A V^(C)) M^(C) has zero columns where m = 0,
    hence so has S^(C) - I, with the filter; columns inside the scatterer do not vanish."""
    k = 10.0
    g, m = _disk_grid(k, kh=1.0)
    S, _, _, _, _ = spf.sparsifying_preconditioner(g, k, m, width=1)
    E = S - np.eye(g.n)
    out, inside = m == 0, m != 0
    assert np.abs(E[:, out]).max() < 1e-12 * np.abs(E).max()
    assert np.abs(E[:, inside]).max(axis=0).min() > 1e-6


def test_sparsified_inverse_cuts_gmres_steps():
    """Right-preconditioned GMRES on the Cartesian system: S^(C) with the compact filter takes
    well under half the steps of the plain iteration (k = 10, 27 x 27 grid)."""
    k = 10.0
    g, m = _disk_grid(k)
    S, L, _, _, _ = spf.sparsifying_preconditioner(g, k, m, width=1)
    zx, _ = g.nodes()
    b = np.exp(1j * k * zx)
    _, it0, _ = krylov.gmres(lambda u: L @ u, b, tol=1e-8, maxit=400)
    y, it1, _ = krylov.gmres(lambda u: L @ (S @ u), b, tol=1e-8, maxit=400)
    assert np.linalg.norm(L @ (S @ y) - b) <= 1e-7 * np.linalg.norm(b)
    assert it0 > 60 and it1 < it0 / 2, (it0, it1)
