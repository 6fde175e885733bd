"""Punctured Nystrom sum of the Green's function over all quadrature nodes.

For density values f at the nodes, the far part of the discrete volume potential at
node j is  sum_{n != j} G(y_j, y_n) w_n f_n  (Section 3: the regularized integrand of
eq. DIM_decomp is integrated with the element quadrature; its value at y = y_j is zero
because the interpolant matches f there, so the j = n term is dropped).
"""
import numpy as np

from .bessel import green


def far_matrix(x, y, w, k):
    """Dense G~ W with G~_jn = G(y_j, y_n) for j != n and 0 on the diagonal."""
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    r = np.hypot(dx, dy)
    np.fill_diagonal(r, 1.0)
    G = green(k, r)
    np.fill_diagonal(G, 0.0)
    return G * w[None, :]


def far_rows(x, y, w, k, f, rows, conj=False, block=256):
    """(G~ W f)_j for the target indices in ``rows``; f has shape (B, N) or (N,).

    conj=True uses conj(G) (the adjoint's kernel) with the weights still on the source side.
    """
    f = np.atleast_2d(f)
    rows = np.asarray(rows)
    out = np.zeros((f.shape[0], rows.size), dtype=np.complex128)
    wf = f * w[None, :]
    for b0 in range(0, rows.size, block):
        rr = rows[b0:b0 + block]
        r = np.hypot(x[rr, None] - x[None, :], y[rr, None] - y[None, :])
        self_mask = rr[:, None] == np.arange(x.size)[None, :]
        r[self_mask] = 1.0
        G = green(k, r)
        G[self_mask] = 0.0
        if conj:
            G = G.conj()
        out[:, b0:b0 + block] = wf @ G.T
    return out
