"""Write tests/golden/gradient_twomat6500.npz: the oracle's far-field misfit gradient on a
two-material disk at N = 6 500 (a realistic size for the dense CPU adjoint), for the GPU gradient
test.

Run: python tests/golden/make_gradient_case.py   (a few minutes on 8 cores)
Calls only workloads/ (inputs) and oracle/ (expected values); nothing here touches the GPU
library.  The case: inclusion |x| < 0.5 with n = 3, annulus with n = 1 + 0.5 exp(-|x|^2), inner
O-grid with 5 cells (N = 6 500), k = 10, 4 plane waves, 32 receivers; data are the far fields of
the contrast perturbed by the seeded Gaussian bumps of the gradient workload, computed by dense LU;
the gradient (Section 5's far-field pattern, the Nystrom system of Section 3 and its exact
adjoint) is taken at the unperturbed contrast.  Stored: C (CSR, caller node order), the
perturbation, the data, J and the gradient.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import farfield, krylov, vdim  # noqa: E402
from oracle.operator import Operator  # noqa: E402
from workloads import problems as P  # noqa: E402

N_I, K, B, R = 5, 10.0, 4, 32


def problem():
    return P.graded_two_material(N_I, K, directions=P.even_directions(B))


def main():
    t0 = time.time()
    p = problem()
    C = vdim.correction_matrix(p.mesh, p.k)
    print(f"N = {p.n_nodes}, C nnz {C.nnz}, {time.time() - t0:.0f} s", flush=True)
    th = P.receivers(R)
    A = farfield.farfield_matrix(p.mesh, p.k, th)
    b = p.incident()
    dm = P.contrast_perturbation(p.mesh, seed=5)
    u_t = krylov.lu_solve(Operator(p.mesh, p.k, p.m + dm, C).dense(), b)
    data = farfield.farfield(A, p.m + dm, u_t)
    op = Operator(p.mesh, p.k, p.m, C)
    u = krylov.lu_solve(op.dense(), b)
    J, grad, _, _ = farfield.adjoint_gradient(op, A, u, data)
    print(f"J = {J:.6e}, |grad| = {np.linalg.norm(grad):.3e}, {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "gradient_twomat6500.npz"),
                        rowptr=C.indptr.astype(np.int64), col=C.indices.astype(np.int32),
                        val=C.data.astype(np.complex128), dm=dm, data=data, J=np.array(J), grad=grad)


if __name__ == "__main__":
    main()
