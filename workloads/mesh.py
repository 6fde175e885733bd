"""Curved, conforming triangular meshes with 10 quadrature nodes per element.

Geometry only: every element is the image of the reference triangle under an exact
map (a transfinite blend onto circular arcs, an exact polar map, or an affine
stretch of those), so the boundary curves are represented exactly.  The nodes of
element e are the consecutive indices 10 e ... 10 e + 9, and the weight of a node is
the rule weight times the Jacobian determinant of the element map at that node.
"""
from dataclasses import dataclass, field

import numpy as np

from .rule10 import rule10

NQ = 10


@dataclass
class Curve:
    """An analytic closed boundary curve of one subdomain.

    kind: 'circle' (radius a) or 'ellipse' (semi-axes a along x, b along y), centred at
    (cx, cy), parametrised by angle t in [0, 2 pi).  orientation = +1 when the
    subdomain lies inside the curve (normal (outward of the subdomain) points away from
    the centre), -1 when it lies outside (e.g. the inner circle of an annulus).
    """
    kind: str
    cx: float
    cy: float
    a: float
    b: float
    orientation: int
    subdomain: int


@dataclass
class Mesh:
    x: np.ndarray
    y: np.ndarray
    w: np.ndarray
    elem_subdomain: np.ndarray
    curves: list = field(default_factory=list)
    cell_size: float = 0.0

    @property
    def n_nodes(self):
        return self.x.size

    @property
    def n_elems(self):
        return self.elem_subdomain.size

    @property
    def n_subdomains(self):
        return int(self.elem_subdomain.max()) + 1 if self.n_elems else 0

    @property
    def node_subdomain(self):
        return np.repeat(self.elem_subdomain, NQ)

    def max_diameter(self):
        """Largest distance between two nodes of one element (a lower bound on h)."""
        X = self.x.reshape(-1, NQ)
        Y = self.y.reshape(-1, NQ)
        d = np.hypot(X[:, :, None] - X[:, None, :], Y[:, :, None] - Y[:, None, :])
        return float(d.max())


def _cell_triangles(i, j, flip):
    """Two triangles (as 3 vertex (s,t) index pairs) splitting cell (i, j).

    flip=False uses the diagonal (i,j)-(i+1,j+1); flip=True uses (i+1,j)-(i,j+1).
    """
    if not flip:
        return [((i, j), (i + 1, j), (i + 1, j + 1)), ((i, j), (i + 1, j + 1), (i, j + 1))]
    return [((i, j), (i + 1, j), (i, j + 1)), ((i + 1, j), (i + 1, j + 1), (i, j + 1))]


def _patch_nodes(tris, n_s, n_t, X, DX):
    """Map the rule onto triangles given in (s, t) index space of an n_s x n_t patch.

    X(s, t) -> (x, y) and DX(s, t) -> det of the patch Jacobian (both vectorised).
    """
    bary, wq = rule10()
    V = np.array(tris, dtype=np.float64)            # [E, 3, 2] in index units
    V[:, :, 0] /= n_s
    V[:, :, 1] /= n_t
    P = np.einsum('qv,evc->eqc', bary, V)           # [E, 10, 2] parameter points
    e1 = V[:, 1] - V[:, 0]
    e2 = V[:, 2] - V[:, 0]
    detA = np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    s, t = P[..., 0], P[..., 1]
    x, y = X(s, t)
    w = wq[None, :] * detA[:, None] * np.abs(DX(s, t))
    return x.ravel(), y.ravel(), w.ravel()


def _ogrid(n, R, sub):
    """Five-patch O-grid of the disk |x| < R: central square of half-side R/2 plus four
    patches blended linearly from a square edge onto its quarter arc (exact on the circle).

    Cell diagonals are mirror-symmetric about the x-axis when n is even.
    """
    S = 0.5 * R
    xs, ys, ws = [], [], []
    # central square [-S, S]^2, s along x, t along y
    tris = []
    for i in range(n):
        for j in range(n):
            tris += _cell_triangles(i, j, flip=(2 * j >= n))
    x, y, w = _patch_nodes(tris, n, n,
                           lambda s, t: (-S + 2 * S * s, -S + 2 * S * t),
                           lambda s, t: np.full_like(s, 4 * S * S))
    xs.append(x); ys.append(y); ws.append(w)
    # four blended patches, arc angle phi0 + s*pi/2, t = 0 on the square edge, 1 on the arc
    for phi0, flip_rule in ((-np.pi / 4, 'half'), (np.pi / 4, 'never'),
                            (3 * np.pi / 4, 'half'), (5 * np.pi / 4, 'always')):
        c0 = np.sqrt(2.0) * S * np.array([np.cos(phi0), np.sin(phi0)])
        c1 = np.sqrt(2.0) * S * np.array([np.cos(phi0 + np.pi / 2), np.sin(phi0 + np.pi / 2)])

        def X(s, t, phi0=phi0, c0=c0, c1=c1):
            ph = phi0 + s * np.pi / 2
            ex = (1 - s) * c0[0] + s * c1[0]
            ey = (1 - s) * c0[1] + s * c1[1]
            return (1 - t) * ex + t * R * np.cos(ph), (1 - t) * ey + t * R * np.sin(ph)

        def DX(s, t, phi0=phi0, c0=c0, c1=c1):
            ph = phi0 + s * np.pi / 2
            xs_ = (1 - t) * (c1[0] - c0[0]) - t * R * (np.pi / 2) * np.sin(ph)
            ys_ = (1 - t) * (c1[1] - c0[1]) + t * R * (np.pi / 2) * np.cos(ph)
            ex = (1 - s) * c0[0] + s * c1[0]
            ey = (1 - s) * c0[1] + s * c1[1]
            xt = R * np.cos(ph) - ex
            yt = R * np.sin(ph) - ey
            return xs_ * yt - ys_ * xt

        tris = []
        for i in range(n):
            for j in range(n):
                flip = {'half': 2 * i >= n, 'never': False, 'always': True}[flip_rule]
                tris += _cell_triangles(i, j, flip)
        x, y, w = _patch_nodes(tris, n, n, X, DX)
        xs.append(x); ys.append(y); ws.append(w)
    x = np.concatenate(xs); y = np.concatenate(ys); w = np.concatenate(ws)
    sub_arr = np.full(x.size // NQ, sub, dtype=np.int32)
    return x, y, w, sub_arr


def ogrid_disk(n, R=1.0):
    """Disk of radius R as one subdomain; N = 100 n^2 nodes, cell size R/n."""
    x, y, w, sub = _ogrid(n, R, 0)
    return Mesh(x, y, w, sub, [Curve('circle', 0.0, 0.0, R, R, +1, 0)], cell_size=R / n)


def _annulus(n_theta, n_r, r0, r1, sub):
    """Exact polar mesh of r0 < |x| < r1 (angle from 0, cell diagonals mirror-symmetric)."""
    tris = []
    for i in range(n_theta):
        for j in range(n_r):
            tris += _cell_triangles(i, j, flip=(2 * i >= n_theta))

    def X(s, t):
        r = r0 + t * (r1 - r0)
        return r * np.cos(2 * np.pi * s), r * np.sin(2 * np.pi * s)

    def DX(s, t):
        return (r0 + t * (r1 - r0)) * (r1 - r0) * 2 * np.pi

    x, y, w = _patch_nodes(tris, n_theta, n_r, X, DX)
    return x, y, w, np.full(x.size // NQ, sub, dtype=np.int32)


def two_material_disk(n_i, r_in=0.5, R=1.0):
    """Inclusion |x| < r_in (subdomain 0, O-grid with n_i cells) and annulus
    r_in < |x| < R (subdomain 1, 8 n_i angular x n_i radial cells); N = 260 n_i^2.
    The two meshes conform to both circles; their interface nodes need not match."""
    x0, y0, w0, s0 = _ogrid(n_i, r_in, 0)
    x1, y1, w1, s1 = _annulus(8 * n_i, n_i, r_in, R, 1)
    curves = [Curve('circle', 0.0, 0.0, r_in, r_in, +1, 0),
              Curve('circle', 0.0, 0.0, R, R, +1, 1),
              Curve('circle', 0.0, 0.0, r_in, r_in, -1, 1)]
    return Mesh(np.concatenate([x0, x1]), np.concatenate([y0, y1]), np.concatenate([w0, w1]),
                np.concatenate([s0, s1]), curves, cell_size=r_in / n_i)


def ellipse(n, a, b):
    """Ellipse x^2/a^2 + y^2/b^2 < 1: the unit O-grid disk stretched by diag(a, b)."""
    x, y, w, sub = _ogrid(n, 1.0, 0)
    return Mesh(a * x, b * y, a * b * w, sub, [Curve('ellipse', 0.0, 0.0, a, b, +1, 0)],
                cell_size=max(a, b) / n)
