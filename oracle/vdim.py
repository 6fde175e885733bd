"""Volume density interpolation (VDIM) correction of the Nystrom far sum.

Section 3, eq. DIM_decomp: for a target x in the element tau of subdomain l, the density
f is replaced near x by its degree-p interpolant F on tau and

    V_l[f](x) = V_l[f - F](x) + B_l[F](x),

where the first term is integrated by the node quadrature (its integrand vanishes at
x) and B_l[F](x) = E_l[F](x) := int_{Omega_l} G(x, y) F(y) dy is evaluated exactly
through Green's third identity with a polynomial particular solution Phi,
(Delta + k^2) Phi = F (same passage), as boundary single- and double-layer potentials plus
the local value of Phi.  Each subdomain of eq. vol_pot_decomp is treated this way, so the
discrete potential at node j is

    sum_{n != j} G w f_n  +  sum_l [ E_l[F_l](y_j) - sum_{q in l, q != j} G w F_l(y_q) ].

Writing F_l = sum_n f_n L_n with the Lagrange basis L_n of one element of Omega_l makes the
bracket a sparse row of a matrix C (10 entries per subdomain and row):

    C_jn = E_l[L_n](y_j) - sum_{q in l, q != j} G(y_j, y_q) w_q L_n(y_q).

Readings of the paper (its VDIM internals are in a cited work): the interpolation element
for the target's own subdomain is the target's element; for every other subdomain it is
that subdomain's element whose centroid (node mean) is nearest to the target, ties broken
by the smaller element index.  Boundary integrals use adaptive Gauss-Legendre panels on
the exact curve instead of the density-interpolation method the paper uses for near
targets.
"""
import numpy as np
from numpy.polynomial.legendre import leggauss

from .bessel import h0, h1

NQ = 10
# exponents (a, b) of the scaled monomials u^a v^b, total degree <= 3
ALPHA = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]
_GL_N = 20
_GL_T, _GL_W = leggauss(_GL_N)


def _mono(u, v, a, b):
    if a < 0 or b < 0:
        return np.zeros(np.broadcast(u, v).shape)
    return u ** a * v ** b


def element_frame(xe, ye):
    """Centre (node mean) and scale (largest node-to-node distance) of one element."""
    c = np.array([xe.mean(), ye.mean()])
    s = np.hypot(xe[:, None] - xe[None, :], ye[:, None] - ye[None, :]).max()
    return c, s


def monomials(px, py, c, s):
    """P_alpha((p - c)/s) for all 10 alpha; shape (..., 10)."""
    u = (np.asarray(px) - c[0]) / s
    v = (np.asarray(py) - c[1]) / s
    return np.stack([_mono(u, v, a, b) for a, b in ALPHA], axis=-1)


def particular(px, py, c, s, k):
    """Phi_alpha = P/k^2 - Delta P / k^4 (exact for degree <= 3, so (Delta + k^2) Phi = P)
    and its physical gradient; each of shape (..., 10)."""
    u = (np.asarray(px) - c[0]) / s
    v = (np.asarray(py) - c[1]) / s
    k2, k4 = k * k, k ** 4
    phi, gx, gy = [], [], []
    for a, b in ALPHA:
        P = _mono(u, v, a, b)
        Pu = a * _mono(u, v, a - 1, b)
        Pv = b * _mono(u, v, a, b - 1)
        L = a * (a - 1) * _mono(u, v, a - 2, b) + b * (b - 1) * _mono(u, v, a, b - 2)
        Lu = a * (a - 1) * (a - 2) * _mono(u, v, a - 3, b) + b * (b - 1) * a * _mono(u, v, a - 1, b - 2)
        Lv = a * (a - 1) * b * _mono(u, v, a - 2, b - 1) + b * (b - 1) * (b - 2) * _mono(u, v, a, b - 3)
        phi.append(P / k2 - L / (s * s * k4))
        gx.append(Pu / (s * k2) - Lu / (s ** 3 * k4))
        gy.append(Pv / (s * k2) - Lv / (s ** 3 * k4))
    return np.stack(phi, -1), np.stack(gx, -1), np.stack(gy, -1)


def _curve_eval(cv, t):
    """Point, speed and unit normal (outward of the curve's subdomain) at parameter t."""
    ct, st = np.cos(t), np.sin(t)
    px = cv.cx + cv.a * ct
    py = cv.cy + cv.b * st
    tx, ty = -cv.a * st, cv.b * ct
    sp = np.hypot(tx, ty)
    nx, ny = ty / sp, -tx / sp          # right of the counter-clockwise tangent
    return px, py, sp, cv.orientation * nx, cv.orientation * ny


def boundary_rule(cv, x, k, rel_far=1.5, max_depth=60):
    """Adaptive Gauss-Legendre rule on the closed curve for a smooth or near-singular
    integrand with its singularity at the target x.

    Start from uniform panels with k * (arc length) <= 4, then bisect every panel whose
    distance bound |x - midpoint| - len/2 is below len (i.e. |x - mid| < 1.5 len).
    Returns points, ds weights and unit normals.
    """
    vmax = max(cv.a, cv.b)
    L = 2 * np.pi * vmax
    m0 = int(max(16, np.ceil(k * L / 4.0)))
    stack = [(2 * np.pi * i / m0, 2 * np.pi * (i + 1) / m0, 0) for i in range(m0)]
    done = []
    while stack:
        t0, t1, d = stack.pop()
        tm = 0.5 * (t0 + t1)
        mx, my, _, _, _ = _curve_eval(cv, tm)
        ln = vmax * (t1 - t0)          # upper bound of the panel's arc length
        if d < max_depth and np.hypot(x[0] - mx, x[1] - my) < rel_far * ln:
            stack.append((t0, tm, d + 1))
            stack.append((tm, t1, d + 1))
        else:
            done.append((t0, t1))
    done = np.array(done)
    h = 0.5 * (done[:, 1] - done[:, 0])
    t = (0.5 * (done[:, 0] + done[:, 1]))[:, None] + h[:, None] * _GL_T[None, :]
    px, py, sp, nx, ny = _curve_eval(cv, t)
    ds = sp * h[:, None] * _GL_W[None, :]
    return px.ravel(), py.ravel(), ds.ravel(), nx.ravel(), ny.ravel()


def poly_potential(curves, inside, x, c, s, k):
    """E[P_alpha](x) = int_{Omega_l} G(x, y) P_alpha(y) dy for the 10 scaled monomials.

    Green's third identity with (Delta + k^2) Phi = P and (Delta_y + k^2) G = -delta_x:
        E[P](x) = -Phi(x) [x in Omega_l] + oint_{dOmega_l} (G d_nu Phi - Phi d_nu_y G) ds_y,
    nu the outward normal of Omega_l and d_nu_y G = -(i k / 4) H1(k rho) (y - x).nu / rho.
    """
    x = np.asarray(x, dtype=np.float64)
    acc = np.zeros(NQ, dtype=np.complex128)
    for cv in curves:
        px, py, ds, nx, ny = boundary_rule(cv, x, k)
        rx, ry = px - x[0], py - x[1]
        rho = np.hypot(rx, ry)
        G = 0.25j * h0(k * rho)
        dG = -0.25j * k * h1(k * rho) * (rx * nx + ry * ny) / rho
        phi, gx, gy = particular(px, py, c, s, k)
        dphi = gx * nx[:, None] + gy * ny[:, None]
        acc += ((G * ds)[:, None] * dphi - (dG * ds)[:, None] * phi).sum(0)
    if inside:
        phi_x, _, _ = particular(x[0], x[1], c, s, k)
        acc -= phi_x
    return acc


class Geometry:
    """Per-element data derived from the node arrays (frames, Vandermonde matrices)."""

    def __init__(self, mesh):
        self.mesh = mesh
        X = mesh.x.reshape(-1, NQ)
        Y = mesh.y.reshape(-1, NQ)
        self.centroids = np.stack([X.mean(1), Y.mean(1)], 1)
        self.scale = np.hypot(X[:, :, None] - X[:, None, :], Y[:, :, None] - Y[:, None, :]).max((1, 2))
        self.node_sub = mesh.node_subdomain
        self.curves_of = {l: [cv for cv in mesh.curves if cv.subdomain == l]
                          for l in range(mesh.n_subdomains)}

    def element_for(self, j, l):
        """Interpolation element of subdomain l for target node j."""
        e_own = j // NQ
        if self.mesh.elem_subdomain[e_own] == l:
            return e_own
        cand = np.nonzero(self.mesh.elem_subdomain == l)[0]
        d = np.hypot(self.centroids[cand, 0] - self.mesh.x[j], self.centroids[cand, 1] - self.mesh.y[j])
        return int(cand[np.argmin(d)])

    def vandermonde(self, e):
        sl = slice(NQ * e, NQ * e + NQ)
        return monomials(self.mesh.x[sl], self.mesh.y[sl], self.centroids[e], self.scale[e])


def correction_row(geom, k, j):
    """Columns and values of row j of C (10 entries per subdomain)."""
    msh = geom.mesh
    cols, vals = [], []
    yj = np.array([msh.x[j], msh.y[j]])
    for l in range(msh.n_subdomains):
        e = geom.element_for(j, l)
        c, s = geom.centroids[e], geom.scale[e]
        E = poly_potential(geom.curves_of[l], geom.node_sub[j] == l, yj, c, s, k)
        q = np.nonzero(geom.node_sub == l)[0]
        q = q[q != j]
        rho = np.hypot(msh.x[q] - yj[0], msh.y[q] - yj[1])
        g = 0.25j * h0(k * rho) * msh.w[q]
        S = g @ monomials(msh.x[q], msh.y[q], c, s)
        D = E - S
        V = geom.vandermonde(e)              # V[i, alpha] = P_alpha(node i)
        # C_j,node_i = sum_alpha (V^-1)[alpha, i] D_alpha  =>  V^T r = D
        cols.append(np.arange(NQ * e, NQ * e + NQ))
        vals.append(np.linalg.solve(V.T, D))
    return np.concatenate(cols), np.concatenate(vals)


def correction_matrix(mesh, k, rows=None):
    """C (or the listed rows of it) as a scipy.sparse CSR matrix of shape (len(rows), N)."""
    import scipy.sparse as sp
    geom = Geometry(mesh)
    rows = np.arange(mesh.n_nodes) if rows is None else np.asarray(rows)
    indptr = [0]
    cols, vals = [], []
    for j in rows:
        c, v = correction_row(geom, k, int(j))
        cols.append(c)
        vals.append(v)
        indptr.append(indptr[-1] + c.size)
    return sp.csr_matrix((np.concatenate(vals), np.concatenate(cols), np.array(indptr)),
                         shape=(rows.size, mesh.n_nodes))
