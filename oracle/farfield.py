"""Far-field pattern, misfit and its gradient with respect to the nodal contrast.

With the asymptotics of G (Section 2) the scattered part of the representation formula
(eq. representation_formula) behaves like e^{ik|x|}/sqrt|x| u_inf(x^) with
    u_inf(x^) = -k^2 gamma int e^{-i k x^.y} m(y) u(y) dy,  gamma = e^{i pi/4}/sqrt(8 pi k),
the normalisation under which the paper's energy balance (Section 5, eq.
dissipativity_identity) reads Im int conj(m u) u_inc = int Im n |u|^2 + ||u_inf||^2 / k.
Discretised with the node quadrature: u_inf = A (m * u), A_rq = -k^2 gamma w_q e^{-ik x^_r.y_q}.

Misfit J = 1/2 sum_{d,r} |u_inf - data|^2.  For a real perturbation dm of the contrast,
L du = -k^2 V (dm u), so with a_d = A^H r_d and the adjoint state L^H lambda_d = conj(m) a_d,
    dJ/dm_j = sum_d Re[ conj(a_jd - k^2 (V^H lambda_d)_j) u_jd ].
"""
import numpy as np


def farfield_matrix(mesh, k, thetas):
    th = np.atleast_1d(thetas)
    gamma = np.exp(0.25j * np.pi) / np.sqrt(8 * np.pi * k)
    ph = k * (np.cos(th)[:, None] * mesh.x[None, :] + np.sin(th)[:, None] * mesh.y[None, :])
    return -k * k * gamma * mesh.w[None, :] * np.exp(-1j * ph)


def farfield(A, m, u):
    """u_inf for each column set: u shape (B, N) -> (B, R)."""
    return (A @ (m[None, :] * np.atleast_2d(u)).T).T


def misfit(A, m, u, data):
    r = farfield(A, m, u) - data
    return 0.5 * float(np.sum(np.abs(r) ** 2)), r


def adjoint_gradient(op, A, u, data):
    """Gradient of J with respect to real nodal contrast values by the dense adjoint."""
    from .krylov import lu_solve
    J, r = misfit(A, op.m, u, data)
    a = (A.conj().T @ r.T).T                       # A^H r, shape (B, N)
    LH = op.dense().conj().T
    lam = lu_solve(LH, np.conj(op.m)[None, :] * a)
    VHl = op.potential_adjoint(lam)
    grad = np.sum(np.real(np.conj(a - op.k ** 2 * VHl) * u), axis=0)
    return J, grad, a, lam
