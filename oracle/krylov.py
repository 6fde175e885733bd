"""Dense LU and GMRES without restart (the paper solves eq. nystrom_linear_system by GMRES
without restart, Section 6 setup; here unpreconditioned, initial guess 0, stopping on the
relative residual ||b - L x||_2 / ||b||_2)."""
import numpy as np


def lu_solve(L, b):
    return np.linalg.solve(L, np.atleast_2d(b).T).T


def gmres(matvec, b, tol=1e-10, maxit=1000):
    """Arnoldi with modified Gram-Schmidt and one re-orthogonalisation pass, Givens
    rotations on the Hessenberg matrix.  Returns (x, iterations, relative residual
    estimate history)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    beta = np.linalg.norm(b)
    if beta == 0:
        return np.zeros_like(b), 0, [0.0]
    V = np.zeros((maxit + 1, n), dtype=np.complex128)
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    cs = np.zeros(maxit, dtype=np.complex128)
    sn = np.zeros(maxit, dtype=np.complex128)
    g = np.zeros(maxit + 1, dtype=np.complex128)
    g[0] = beta
    V[0] = b / beta
    hist = [1.0]
    j = -1
    for j in range(maxit):
        w = matvec(V[j])
        for _ in range(2):
            for i in range(j + 1):
                hij = np.vdot(V[i], w)
                H[i, j] += hij
                w = w - hij * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] != 0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
            H[i, j] = t
        a, bb = H[j, j], H[j + 1, j]
        den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
        # unitary [[c, s], [-conj(s), conj(c)]] with c = conj(a)/rho, s = conj(b)/rho
        cs[j] = np.conj(a) / den if den else 1.0
        sn[j] = np.conj(bb) / den if den else 0.0
        H[j, j] = cs[j] * a + sn[j] * bb
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        hist.append(abs(g[j + 1]) / beta)
        if hist[-1] <= tol:
            break
    m = j + 1
    y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
    return V[:m].T @ y, m, hist
