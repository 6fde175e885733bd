"""Seeded synthetic scattering problems: meshes, wavenumbers, contrast, incident fields.

Conventions follow the paper's problem statement (Section 2): the refractive index n
enters Delta u + k^2 n u = 0, and the contrast handed to the solver is m = 1 - n
evaluated at the quadrature nodes with the formula of the subdomain that owns each
element (nodes are strictly interior, so no node sits on an interface).
"""
from dataclasses import dataclass, field

import numpy as np

from . import mesh as _mesh


@dataclass
class Problem:
    mesh: _mesh.Mesh
    k: float
    m: np.ndarray                   # contrast 1 - n at the nodes (complex128 or float64)
    name: str = ''
    directions: np.ndarray = field(default_factory=lambda: np.zeros(1))   # incidence angles
    m_at: object = None             # contrast at arbitrary points (x, y) -> m, 0 outside; None if unknown

    @property
    def n_nodes(self):
        return self.mesh.n_nodes

    def incident(self, thetas=None):
        """Plane waves exp(i k x.d), d = (cos th, sin th); shape (B, N) complex128."""
        th = self.directions if thetas is None else np.atleast_1d(thetas)
        x, y = self.mesh.x, self.mesh.y
        ph = self.k * (np.cos(th)[:, None] * x[None] + np.sin(th)[:, None] * y[None])
        return np.exp(1j * ph)


def contrast_from_index(mesh, index_funcs):
    """m = 1 - n(y_j) with n given per subdomain as a callable (x, y) -> n."""
    sub = mesh.node_subdomain
    n = np.empty(mesh.n_nodes, dtype=np.complex128)
    for s, f in enumerate(index_funcs):
        sel = sub == s
        n[sel] = f(mesh.x[sel], mesh.y[sel])
    m = 1.0 - n
    return m.real.copy() if np.all(m.imag == 0) else m


def const(v):
    return lambda x, y: np.full(x.shape, v, dtype=np.float64)


def disk_problem(n, k, index=2.0, R=1.0, directions=(0.0,), name='disk'):
    msh = _mesh.ogrid_disk(n, R)
    m_at = lambda x, y: np.where(np.hypot(x, y) < R, 1.0 - index, 0.0)
    return Problem(msh, k, contrast_from_index(msh, [const(index)]), name,
                   np.asarray(directions, dtype=np.float64), m_at)


def two_layer_constant(n_i, k, n_in, n_out, directions=(0.0,)):
    """Two-material disk with constant indices (inclusion n_in, annulus n_out)."""
    msh = _mesh.two_material_disk(n_i)
    return Problem(msh, k, contrast_from_index(msh, [const(n_in), const(n_out)]),
                   'two-layer-const', np.asarray(directions, dtype=np.float64))


def graded_two_material(n_i, k, directions=(0.0,)):
    """Inclusion |x| < 0.5 with n = 3; annulus 0.5 < |x| < 1 with n = 1 + 0.5 exp(-|x|^2)."""
    msh = _mesh.two_material_disk(n_i)
    graded = lambda x, y: 1.0 + 0.5 * np.exp(-(x * x + y * y))
    m = contrast_from_index(msh, [const(3.0), graded])

    def m_at(x, y):
        r = np.hypot(x, y)
        return np.where(r < 0.5, 1.0 - 3.0, np.where(r < 1.0, 1.0 - graded(x, y), 0.0))
    return Problem(msh, k, m, 'two-material', np.asarray(directions, dtype=np.float64), m_at)


def even_directions(B):
    return 2 * np.pi * np.arange(B) / B


# ---- the five workloads -------------------------------------------------------------

def config1():
    """Unit disk, n = 2, k = 2 pi, O-grid n = 5 (cell 0.2), N = 2500, one wave along +x."""
    return disk_problem(5, 2 * np.pi, 2.0, name='disk-N2500-k2pi')


def config2(n_i=15):
    """Two-material disk, k = 20, n_i = 15 (cell 1/30), N = 58500, one wave along +x."""
    p = graded_two_material(n_i, 20.0)
    p.name = f'two-material-N{p.n_nodes}-k20'
    return p


def config3(n=35, B=64):
    """Unit disk, n = 2, k = 40, O-grid n = 35, N = 122500, 64 evenly spaced directions."""
    return disk_problem(n, 40.0, 2.0, directions=even_directions(B), name=f'disk-N{100*n*n}-k40-B{B}')


def config4(seed=4, count=16, B=8, n_min=5e3, n_max=8e4, resolve=0.5):
    """16 seeded scatterers (disk or ellipse, semi-axes U[0.5,1.5], one constant index
    U[0.5,3], k U[5,40], node count log-uniform in [5e3, 8e4]), 8 directions each.  With
    resolve, a draw whose mesh would not resolve its interior wave (k sqrt(n) times the node
    spacing sqrt(area / N) above resolve) gets the smallest mesh that does, within n_max nodes;
    the random draws are the same either way."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        is_disk = rng.random() < 0.5
        a = rng.uniform(0.5, 1.5)
        b = a if is_disk else rng.uniform(0.5, 1.5)
        idx = rng.uniform(0.5, 3.0)
        k = rng.uniform(5.0, 40.0)
        n_target = np.exp(rng.uniform(np.log(n_min), np.log(n_max)))
        n = max(1, int(round(np.sqrt(n_target / 100.0))))
        if resolve:
            # N = 100 n^2 nodes over the area pi a b
            need = int(np.ceil(k * np.sqrt(idx) * np.sqrt(np.pi * a * b / 100.0) / resolve))
            n = max(n, min(need, int(np.sqrt(n_max / 100.0))))
        msh = _mesh.ogrid_disk(n, a) if is_disk else _mesh.ellipse(n, a, b)
        m_at = lambda x, y, a=a, b=b, idx=idx: np.where((x / a) ** 2 + (y / b) ** 2 < 1.0, 1.0 - idx, 0.0)
        out.append(Problem(msh, k, contrast_from_index(msh, [const(idx)]),
                           f'{"disk" if is_disk else "ellipse"}-{s}', even_directions(B), m_at))
    return out


def config5(n_i=21, B=16):
    """Two-material disk at k = 40 with n_i = 21 (N = 114660) and 16 directions."""
    p = graded_two_material(n_i, 40.0, directions=even_directions(B))
    p.name = f'two-material-N{p.n_nodes}-k40-B{B}'
    return p


def contrast_perturbation(mesh, seed=5, count=3):
    """Seeded smooth perturbation dm = sum_b A_b exp(-|y - c_b|^2 / (2 s_b^2)),
    A_b ~ U[-0.1, 0.1], c_b uniform in the disk of radius 0.8, s_b ~ U[0.1, 0.3]."""
    rng = np.random.default_rng(seed)
    dm = np.zeros(mesh.n_nodes)
    for _ in range(count):
        A = rng.uniform(-0.1, 0.1)
        r = 0.8 * np.sqrt(rng.random())
        ph = rng.uniform(0, 2 * np.pi)
        s = rng.uniform(0.1, 0.3)
        dm += A * np.exp(-((mesh.x - r * np.cos(ph)) ** 2 + (mesh.y - r * np.sin(ph)) ** 2) / (2 * s * s))
    return dm


def random_vectors(N, B=1, seed=0):
    """Standard complex normal vectors, shape (B, N)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((B, N)) + 1j * rng.standard_normal((B, N))) / np.sqrt(2.0)


def receivers(R=128):
    return 2 * np.pi * np.arange(R) / R


def cartesian_grid(prob, kh, pad=0.02):
    """A uniform Cartesian grid of spacing kh / k covering the scatterer's nodes with a margin pad:
    (x0, y0, h, nx, ny), node (ix, iy) at (x0 + ix h, y0 + iy h)."""
    h = kh / prob.k
    x, y = prob.mesh.x, prob.mesh.y
    x0, y0 = x.min() - pad, y.min() - pad
    nx = int(np.ceil((x.max() + pad - x0) / h)) + 1
    ny = int(np.ceil((y.max() + pad - y0) / h)) + 1
    return float(x0), float(y0), float(h), nx, ny


def grid_contrast(prob, grid):
    """The contrast m = 1 - n at the nodes of grid (x0, y0, h, nx, ny), in grid order (0 outside)."""
    x0, y0, h, nx, ny = grid
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    return np.asarray(prob.m_at(x0 + ix * h, y0 + iy * h), dtype=np.complex128)
