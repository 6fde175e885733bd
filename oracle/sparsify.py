"""The sparsifying Cartesian preconditioner S^(C) = (C^(C))^-1 A (test infrastructure, not
product code).

Section 4, subsection "Sparsifying preconditioner" (eqs. LS_eq_on_cartesian_points,
cart_neighbors_LS, sparsifying_min, LC_def, S_minus_I).  On a uniform grid (oracle.transfer.Grid)
the Cartesian system is L^(C) = I + k^2 V^(C) M^(C) with M^(C) = diag(m(z_j)).

Readings (the paper's own choices are not available here):
  * V^(C): the paper uses a high-order Cartesian rule (Duan-Rokhlin), whose weights are not
    given.  This oracle uses the first-order rule: V_ij = h^2 G(z_i, z_j) for i != j, and on the
    diagonal the integral of G over the disk of the cell's area centred on the node,
    (-1 + (i pi/2) k a H1(k a)) / k^2 with a = h / sqrt(pi).
  * Stencil: the 3 x 3 neighbours of the node within the grid's box (eq. cart_neighbors_LS with D
    the box), so 6 at an edge and 4 at a corner.  Each row's weights solve eq. sparsifying_min for
    its own neighbourhood: the smallest left singular vector of V(N(j), N(j)^c).  Rows with all 9
    neighbours share the weights of the grid's central node (the translation invariance the paper
    invokes); every edge and corner row gets its own (truncating the central weights instead left
    the dropped part of A L^(C) large in those rows and tripled the GMRES steps).
  * Filter: C^(C) keeps the entries of A L^(C) whose row and column nodes are at most `width`
    grid steps apart in each direction (the compact finite-difference pattern for width 1);
    width=None keeps everything (then S^(C) = (L^(C))^-1 exactly).

Only tests/, the smoke check and the bench's CPU baseline use this package.
"""
import numpy as np

from .bessel import green, h1


def self_term(k, h):
    """Integral of G(0, y) over the disk |y| < a of area h^2: (-1 + (i pi / 2) k a H1(k a)) / k^2."""
    a = h / np.sqrt(np.pi)
    return (-1.0 + 0.5j * np.pi * k * a * h1(k * a)) / (k * k)


def cartesian_volume(grid, k):
    """V^(C) of the first-order rule above, dense (N_C, N_C)."""
    zx, zy = grid.nodes()
    r = np.hypot(zx[:, None] - zx[None, :], zy[:, None] - zy[None, :])
    np.fill_diagonal(r, 1.0)
    V = grid.h * grid.h * green(k, r)
    np.fill_diagonal(V, self_term(k, grid.h))
    return V


def cartesian_system(grid, k, m):
    """L^(C) = I + k^2 V^(C) M^(C) (eq. LS_eq_on_cartesian_points); m holds m(z_j) per grid node."""
    return np.eye(grid.n) + k * k * cartesian_volume(grid, k) * np.asarray(m)[None, :]


def neighbours(grid, j):
    """Indices of the grid nodes at most one step from node j in each direction (eq. cart_neighbors_LS)."""
    iy, ix = divmod(int(j), grid.nx)
    out = []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if 0 <= ix + dx < grid.nx and 0 <= iy + dy < grid.ny:
                out.append((iy + dy) * grid.nx + ix + dx)
    return np.array(out)


def row_weights(grid, V, j):
    """Eq. sparsifying_min for row j: the unit vector v on N(j) minimising ||v V(N(j), N(j)^c)||,
    the left singular vector of the smallest singular value.  Returns (N(j), v, smallest /
    largest singular value)."""
    nb = neighbours(grid, j)
    comp = np.setdiff1d(np.arange(grid.n), nb)
    U, s, _ = np.linalg.svd(V[np.ix_(nb, comp)])
    return nb, U[:, -1].conj(), s[-1] / s[0]


def stencil_weights(grid, V):
    """The weights of the grid's central node j0 and their offsets (dx, dy), with the smallest /
    largest singular value."""
    j0 = (grid.ny // 2) * grid.nx + grid.nx // 2
    nb, v, ratio = row_weights(grid, V, j0)
    assert nb.size == 9, "the grid needs at least 3 x 3 nodes"
    iy0, ix0 = divmod(j0, grid.nx)
    offs = [(int(j % grid.nx) - ix0, int(j // grid.nx) - iy0) for j in nb]
    return v, offs, ratio


def stencil_matrix(grid, V):
    """A (dense (N_C, N_C)): the central weights on every row with 9 neighbours, each edge and
    corner row's own weights on its 6 or 4."""
    v, offs, _ = stencil_weights(grid, V)
    A = np.zeros((grid.n, grid.n), dtype=np.complex128)
    for j in range(grid.n):
        iy, ix = divmod(j, grid.nx)
        if 0 < ix < grid.nx - 1 and 0 < iy < grid.ny - 1:
            for (dx, dy), w in zip(offs, v):
                A[j, (iy + dy) * grid.nx + ix + dx] = w
        else:
            nb, w, _ = row_weights(grid, V, j)
            A[j, nb] = w
    return A


def filtered_product(grid, A, L, width=1):
    """C^(C): A L^(C) with the entries farther apart than `width` steps set to zero."""
    AL = A @ L
    if width is None:
        return AL
    iy, ix = np.divmod(np.arange(grid.n), grid.nx)
    near = (np.abs(ix[:, None] - ix[None, :]) <= width) & (np.abs(iy[:, None] - iy[None, :]) <= width)
    return np.where(near, AL, 0.0)


def sparsifying_preconditioner(grid, k, m, width=1):
    """S^(C) = (C^(C))^-1 A (eq. LC_def) as a dense matrix, with L^(C) and the stencil data."""
    V = cartesian_volume(grid, k)
    L = np.eye(grid.n) + k * k * V * np.asarray(m)[None, :]
    v, offs, ratio = stencil_weights(grid, V)
    A = stencil_matrix(grid, V)
    C = filtered_product(grid, A, L, width)
    return np.linalg.solve(C, A), L, v, offs, ratio
