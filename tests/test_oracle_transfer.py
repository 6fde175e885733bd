"""Pins of the oracle's transfer operators and preconditioner wrapper (Section 4)."""
import numpy as np
import pytest

from oracle import transfer as tr
from workloads import problems as P


def _setup(n=4, hk=0.4):
    prob = P.disk_problem(n, 2 * np.pi, 2.0)
    x, y = prob.mesh.x, prob.mesh.y
    g = tr.Grid(-1.1, -1.05, hk, int(np.ceil(2.2 / hk)) + 1, int(np.ceil(2.1 / hk)) + 2)
    return x, y, g, tr.cart_to_quad(g, x, y)


def test_rows_are_the_global_hat_functions():
    """Each entry equals the tensor-product hat max(0, 1-|dx|/h) max(0, 1-|dy|/h) evaluated at
    every grid node (a formula that does not look for the containing cell)."""
    x, y, g, T = _setup()
    zx, zy = g.nodes()
    hat = np.maximum(0, 1 - np.abs(x[:, None] - zx[None, :]) / g.h) * \
        np.maximum(0, 1 - np.abs(y[:, None] - zy[None, :]) / g.h)
    assert np.abs(T - hat).max() < 1e-14
    assert np.all((T != 0).sum(axis=1) <= 4)


def test_constants_and_bilinear_fields_are_reproduced():
    """T_C^Q is exact on bilinear fields: its rows sum to one and reproduce a + bx + cy + dxy."""
    x, y, g, T = _setup()
    assert np.abs(T.sum(axis=1) - 1).max() < 1e-14
    zx, zy = g.nodes()
    f = lambda u, v: 0.3 - 1.7 * u + 2.2 * v + 0.9 * u * v
    assert np.abs(T @ f(zx, zy) - f(x, y)).max() < 1e-13
    # a quadratic is not reproduced: the pin has teeth
    assert np.abs(T @ (zx * zx) - x * x).max() > 1e-3


def test_renormalized_transpose_and_round_trip_keep_constants():
    """eq. roundtrip_constants_int: T_Q^C 1 = 1 and R = T_Q^C T_C^Q keeps constants on the
    pixelation nodes; the other rows are zero."""
    x, y, g, T = _setup()
    Tq = tr.quad_to_cart(T)
    pix = tr.pixelation(T)
    one = Tq @ np.ones(len(x))
    assert np.abs(one[pix] - 1).max() < 1e-14
    rest = np.setdiff1d(np.arange(g.n), pix)
    assert np.all(one[rest] == 0)
    R = Tq @ T
    r1 = R @ np.ones(g.n)
    assert np.abs(r1[pix] - 1).max() < 1e-14
    # the column sums D are positive exactly at the pixelation nodes
    assert np.all(T.sum(axis=0)[rest] == 0)


def test_embedding_is_singular():
    """Proposition non_invertible: with N_Q > N_pix the embedding T S T_Q^C has rank <= N_pix."""
    x, y, g, T = _setup(n=3, hk=0.3)
    pix = tr.pixelation(T)
    assert len(x) > len(pix)
    rng = np.random.default_rng(1)
    S = rng.standard_normal((g.n, g.n))
    E = T @ S @ tr.quad_to_cart(T)
    assert np.linalg.matrix_rank(E) <= len(pix) < len(x)


def test_preconditioner_forms_agree():
    """eq. preconditioner_split equals eq. preconditioner_factored, and S = I gives P = I."""
    x, y, g, T = _setup()
    rng = np.random.default_rng(2)
    Sm = np.eye(g.n) + 0.1 * rng.standard_normal((g.n, g.n))
    v = rng.standard_normal((3, len(x))) + 1j * rng.standard_normal((3, len(x)))
    Tq = tr.quad_to_cart(T)
    split = (T @ Sm @ Tq + np.eye(len(x)) - T @ Tq) @ v.T
    got = tr.precondition(T, v, lambda c: c @ Sm.T)
    assert np.abs(got - split.T).max() < 1e-12
    assert np.abs(tr.precondition(T, v, lambda c: c) - v).max() < 1e-14


def test_adjoint_preconditioner_is_the_adjoint():
    """<P x, y> = <x, P^H y> for the factored form of P^H (and D is the column sums of T_C^Q)."""
    x, y, g, T = _setup()
    rng = np.random.default_rng(4)
    Sm = np.eye(g.n) + 0.1 * (rng.standard_normal((g.n, g.n)) + 1j * rng.standard_normal((g.n, g.n)))
    u = rng.standard_normal(len(x)) + 1j * rng.standard_normal(len(x))
    v = rng.standard_normal(len(x)) + 1j * rng.standard_normal(len(x))
    Pu = tr.precondition(T, u, lambda c: c @ Sm.T)
    PHv = tr.precondition_adjoint(T, v, lambda c: c @ Sm.conj())
    assert abs(np.vdot(v, Pu) - np.vdot(PHv, u)) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(v) * 10
    P = np.stack([tr.precondition(T, e, lambda c: c @ Sm.T) for e in np.eye(len(x))], axis=1)
    PH = np.stack([tr.precondition_adjoint(T, e, lambda c: c @ Sm.conj()) for e in np.eye(len(x))], axis=1)
    assert np.abs(PH - P.conj().T).max() < 1e-12
    assert np.array_equal(tr.column_sums(T)[tr.pixelation(T)], T.sum(axis=0)[tr.pixelation(T)])


def test_nodes_outside_the_grid_are_rejected():
    x, y, g, _ = _setup()
    with pytest.raises(ValueError):
        tr.cart_to_quad(tr.Grid(0.0, 0.0, 0.1, 5, 5), x, y)
