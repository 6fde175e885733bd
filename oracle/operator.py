"""The Nystrom system matrix L = I + k^2 V M with V = G~ W + C.

Section 3, eqs. linear_system, nystrom_linear_system, linear_system_matrix: (V)_jn is the
discrete potential of the n-th unit vector at node j and M = diag(m(y_j)), m = 1 - n.
The adjoint is L^H = I + k^2 conj(M) V^H with V^H = W conj(G~) + C^H (G~ is symmetric).
"""
import numpy as np

from . import green


class Operator:
    """Matrix-free L and L^H from the node arrays, the wavenumber, the contrast and C."""

    def __init__(self, mesh, k, m, C):
        self.mesh, self.k, self.m, self.C = mesh, float(k), np.asarray(m), C.tocsr()
        self.CH = self.C.conj().T.tocsr()

    def potential(self, f, rows=None):
        """V f (rows of it); f shape (B, N)."""
        f = np.atleast_2d(f)
        msh = self.mesh
        rows = np.arange(msh.n_nodes) if rows is None else np.asarray(rows)
        far = green.far_rows(msh.x, msh.y, msh.w, self.k, f, rows)
        return far + (self.C[rows] @ f.T).T

    def potential_adjoint(self, g):
        """V^H g = w * (conj(G~) g) + C^H g; g shape (B, N)."""
        g = np.atleast_2d(g)
        msh = self.mesh
        ones = np.ones_like(msh.w)
        far = green.far_rows(msh.x, msh.y, ones, self.k, g, np.arange(msh.n_nodes), conj=True)
        return msh.w[None, :] * far + (self.CH @ g.T).T

    def apply(self, x, rows=None):
        x = np.atleast_2d(x)
        rows = np.arange(self.mesh.n_nodes) if rows is None else np.asarray(rows)
        return x[:, rows] + self.k ** 2 * self.potential(self.m[None, :] * x, rows)

    def apply_adjoint(self, x):
        x = np.atleast_2d(x)
        return x + self.k ** 2 * np.conj(self.m)[None, :] * self.potential_adjoint(x)

    def dense(self):
        """Dense L (small N only)."""
        msh = self.mesh
        V = green.far_matrix(msh.x, msh.y, msh.w, self.k) + self.C.toarray()
        return np.eye(msh.n_nodes) + self.k ** 2 * V * self.m[None, :]
