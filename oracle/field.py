"""Field recovery at points outside the scatterer (test infrastructure, not product code).

Section 3, eq. field_recovery (the discrete form of eq. representation_formula): once the
nodal values u of the Nystrom solution are known, the scattered field at any point x is

    u_s(x) = u(x) - u_inc(x) = -k^2 V~_Omega[M u](x),

one more application of the VDIM map, now at a target that is not a node.  For a target
outside every subdomain there is no self term to drop and no own element; in each subdomain
l the interpolation element is the one whose centroid (node mean) is nearest to x, ties to
the smaller element index, as for the nodes of the other subdomains (see vdim.py), and the
exact polynomial potential is taken with x outside Omega_l.

Only tests/, the smoke check and the bench's CPU baseline use this package.
"""
import numpy as np

from .bessel import h0
from .vdim import NQ, Geometry, monomials, poly_potential


def outside(mesh, x, y):
    """True where (x, y) lies outside every curve that encloses a subdomain."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    out = np.ones(x.shape, dtype=bool)
    for cv in mesh.curves:
        if cv.orientation != 1:
            continue
        r = ((x - cv.cx) / cv.a) ** 2 + ((y - cv.cy) / cv.b) ** 2
        out &= r > 1.0
    return out


def correction_row_at(geom, k, x):
    """Columns and values of the correction row for an exterior point x (10 per subdomain)."""
    msh = geom.mesh
    x = np.asarray(x, dtype=np.float64)
    cols, vals = [], []
    for l in range(msh.n_subdomains):
        cand = np.nonzero(msh.elem_subdomain == l)[0]
        d = np.hypot(geom.centroids[cand, 0] - x[0], geom.centroids[cand, 1] - x[1])
        e = int(cand[np.argmin(d)])
        c, s = geom.centroids[e], geom.scale[e]
        E = poly_potential(geom.curves_of[l], False, x, c, s, k)
        q = np.nonzero(geom.node_sub == l)[0]
        rho = np.hypot(msh.x[q] - x[0], msh.y[q] - x[1])
        S = (0.25j * h0(k * rho) * msh.w[q]) @ monomials(msh.x[q], msh.y[q], c, s)
        cols.append(np.arange(NQ * e, NQ * e + NQ))
        vals.append(np.linalg.solve(geom.vandermonde(e).T, E - S))
    return np.concatenate(cols), np.concatenate(vals)


def scattered_field(mesh, k, m, u, tx, ty):
    """u_s at the exterior points (tx, ty) for nodal fields u of shape (B, N) or (N,).

    Returns shape (B, T).  Raises if a point is not outside the scatterer.
    """
    u = np.atleast_2d(np.asarray(u, dtype=np.complex128))
    tx = np.atleast_1d(np.asarray(tx, dtype=np.float64))
    ty = np.atleast_1d(np.asarray(ty, dtype=np.float64))
    if not np.all(outside(mesh, tx, ty)):
        raise ValueError("field recovery here is for points outside the scatterer")
    f = u * m[None, :]
    wf = f * mesh.w[None, :]
    geom = Geometry(mesh)
    out = np.zeros((u.shape[0], tx.size), dtype=np.complex128)
    for i in range(tx.size):
        rho = np.hypot(mesh.x - tx[i], mesh.y - ty[i])
        far = wf @ (0.25j * h0(k * rho))
        cols, vals = correction_row_at(geom, k, (tx[i], ty[i]))
        out[:, i] = -k * k * (far + f[:, cols] @ vals)
    return out
