"""Transfer operators between the quadrature nodes and a Cartesian grid, and the preconditioner
wrapper built from them (test infrastructure, not product code).

Section 4 of the paper.  The Cartesian grid has nodes z_(ix, iy) = (x0 + ix h, y0 + iy h),
0 <= ix < nx, 0 <= iy < ny, numbered j = iy nx + ix.

  T_C^Q (grid -> nodes, eq. psi_def): row q holds the bilinear hat functions
      psi_j(y_q) = (1 - |y_q1 - z_j1| / h)(1 - |y_q2 - z_j2| / h)
  of the four vertices of the cell containing y_q.
  T_Q^C (nodes -> grid, Approach II, eqs. T_H^C_def and D_def): D^-1 (T_C^Q)^T, D = diag of the
      column sums of T_C^Q, and 1 where a column sums to zero.
  P (eq. preconditioner_factored): P = I + T_C^Q (S - I) T_Q^C for a Cartesian approximate
      inverse S (here any linear map on grid vectors the caller supplies).

Readings: a node on a grid line belongs to the cell on its upper/right side (floor of the
scaled coordinate), except on the grid's last line, where it takes the cell below/left; the
off-line vertices then get weight zero, as the paper notes.  A column whose entries are all
zero weights gets D_jj = 1, like the columns no node reaches.

Only tests/, the smoke check and the bench's CPU baseline use this package.
"""
import numpy as np


class Grid:
    """Uniform Cartesian grid: origin (x0, y0), spacing h, nx by ny nodes."""

    def __init__(self, x0, y0, h, nx, ny):
        self.x0, self.y0, self.h = float(x0), float(y0), float(h)
        self.nx, self.ny = int(nx), int(ny)

    @property
    def n(self):
        return self.nx * self.ny

    def nodes(self):
        ix, iy = np.meshgrid(np.arange(self.nx), np.arange(self.ny))
        return self.x0 + ix.ravel() * self.h, self.y0 + iy.ravel() * self.h


def containing_cell(grid, x, y):
    """Lower-left vertex (ix, iy) of the cell containing each point (the reading above)."""
    sx = (np.asarray(x) - grid.x0) / grid.h
    sy = (np.asarray(y) - grid.y0) / grid.h
    if np.any(sx < 0) or np.any(sy < 0) or np.any(sx > grid.nx - 1) or np.any(sy > grid.ny - 1):
        raise ValueError("a node lies outside the grid")
    ix = np.floor(sx).astype(np.int64)
    iy = np.floor(sy).astype(np.int64)
    return np.minimum(ix, grid.nx - 2), np.minimum(iy, grid.ny - 2)


def cart_to_quad(grid, x, y):
    """T_C^Q as a dense (N_Q, N_C) array, from the hat functions of eq. psi_def."""
    zx, zy = grid.nodes()
    ix, iy = containing_cell(grid, x, y)
    T = np.zeros((len(x), grid.n))
    for q in range(len(x)):
        for dx in (0, 1):
            for dy in (0, 1):
                j = (iy[q] + dy) * grid.nx + ix[q] + dx
                a = abs(x[q] - zx[j]) / grid.h
                b = abs(y[q] - zy[j]) / grid.h
                T[q, j] = (1.0 - a) * (1.0 - b)
    return T


def quad_to_cart(T):
    """T_Q^C = D^-1 T^T (Approach II)."""
    d = T.sum(axis=0)
    d = np.where(d > 0, d, 1.0)
    return T.T / d[:, None]


def pixelation(T):
    """Indices of the grid nodes some quadrature node reaches with a positive weight."""
    return np.nonzero(T.sum(axis=0) > 0)[0]


def precondition(T, x, S):
    """P x = x + T_C^Q (S - I) T_Q^C x for columns x of shape (N_Q,) or (B, N_Q); S maps grid
    vectors of the same leading shape."""
    c = np.asarray(x) @ quad_to_cart(T).T
    return np.asarray(x) + (S(c) - c) @ T.T


def column_sums(T):
    """D of eq. D_def: column sums of T_C^Q, 1 where a column sums to zero."""
    d = T.sum(axis=0)
    return np.where(d > 0, d, 1.0)


def precondition_adjoint(T, x, SH):
    """P^H x for P of precondition(): since T_C^Q is real and T_Q^C = D^-1 (T_C^Q)^T,
    P^H = I + T_C^Q (D^-1 S^H D - I) T_Q^C, where SH applies S^H to grid vectors."""
    d = column_sums(T)
    return precondition(T, x, lambda c: SH(c * d) / d)
