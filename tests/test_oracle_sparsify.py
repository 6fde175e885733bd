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
    # an edge row (6 neighbours) and a corner row (4) minimise over their own neighbourhoods, and
    # beat the central weights truncated to them
    A = spf.stencil_matrix(g, V)
    for j in (g.nx // 2, 0):
        nb = spf.neighbours(g, j)
        Bj = V[np.ix_(nb, np.setdiff1d(np.arange(g.n), nb))]
        w = A[j, nb]
        own = np.linalg.norm(w @ Bj)
        assert abs(np.linalg.norm(w) - 1) < 1e-14 and abs(own - np.linalg.svd(Bj, compute_uv=False)[-1]) < 1e-12 * own
        Uj = rng.standard_normal((2000, nb.size)) + 1j * rng.standard_normal((2000, nb.size))
        Uj /= np.linalg.norm(Uj, axis=1)[:, None]
        assert np.all(np.linalg.norm(Uj @ Bj, axis=1) >= own * (1 - 1e-9))
        iy, ix = divmod(j, g.nx)
        trunc = np.array([v[o] for o, (dx, dy) in enumerate(offs)
                          if 0 <= ix + dx < g.nx and 0 <= iy + dy < g.ny])
        assert np.linalg.norm(trunc @ Bj) / np.linalg.norm(trunc) > 10 * own


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


def test_sparsified_S_preconditions_the_nystrom_system():
    """P = I + T_C^Q (S - I) T_Q^C with S = S^(C) on the Nystrom system of a small disk (k = 8,
    N = 1 600, dense oracle matrices): about as few GMRES steps as with the exact inverse of the
    same Cartesian system and a third of the plain count; the central weights truncated at the
    grid's edge instead of each edge row's own take many more."""
    from oracle import green, vdim
    from oracle import transfer as tr
    from workloads import problems as P
    prob = P.disk_problem(4, 8.0, 2.0)
    k = prob.k
    V = green.far_matrix(prob.mesh.x, prob.mesh.y, prob.mesh.w, k) + vdim.correction_matrix(prob.mesh, k).toarray()
    L = np.eye(prob.n_nodes) + k * k * V * prob.m[None, :]
    b = prob.incident()
    b = b[0] if b.ndim == 2 else b
    h, pad = 0.8 / k, 0.02
    x0, y0 = prob.mesh.x.min() - pad, prob.mesh.y.min() - pad
    nx = int(np.ceil((prob.mesh.x.max() + pad - x0) / h)) + 1
    ny = int(np.ceil((prob.mesh.y.max() + pad - y0) / h)) + 1
    g = Grid(x0, y0, h, nx, ny)
    T = tr.cart_to_quad(g, prob.mesh.x, prob.mesh.y)
    zx, zy = g.nodes()
    m = np.asarray(prob.m_at(zx, zy), dtype=np.complex128)
    S, Lc, v, offs, _ = spf.sparsifying_preconditioner(g, k, m, width=1)

    def steps(Smat):
        return krylov.gmres(lambda u: L @ tr.precondition(T, u[None, :], lambda c: c @ Smat.T)[0], b,
                            tol=1e-8, maxit=600)[1]

    it_plain = krylov.gmres(lambda u: L @ u, b, tol=1e-8, maxit=600)[1]
    it_s, it_inv = steps(S), steps(np.linalg.inv(Lc))
    # the central weights truncated at the edge
    At = np.zeros((g.n, g.n), dtype=np.complex128)
    for j in range(g.n):
        iy, ix = divmod(j, g.nx)
        for (dx, dy), w in zip(offs, v):
            if 0 <= ix + dx < g.nx and 0 <= iy + dy < g.ny:
                At[j, (iy + dy) * g.nx + ix + dx] = w
    it_t = steps(np.linalg.solve(spf.filtered_product(g, At, Lc, 1), At))
    print(f"plain {it_plain}, S^(C) {it_s}, exact inverse {it_inv}, truncated edge weights {it_t}")
    assert it_s <= it_inv + 3 and 3 * it_s <= it_plain and it_t >= it_s + 10
