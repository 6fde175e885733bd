"""Write tests/golden/oracle_cases.npz: oracle-only expected values for the GPU parity tests.

Run: python tests/golden/make_oracle_cases.py
Calls only workloads/ (inputs) and oracle/ (expected values); nothing here touches the GPU
library.  Each case stores its correction C (CSR, caller node order), seeded input vectors
and the oracle's L x, L^H x and, for the smaller cases, the dense-LU solution of L u = b.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import krylov, vdim  # noqa: E402
from oracle.operator import Operator  # noqa: E402
from workloads import mesh as M  # noqa: E402
from workloads import problems as P  # noqa: E402


def cases():
    yield "disk2500", P.config1()
    yield "twomat1040", P.graded_two_material(2, 20.0)
    p = P.disk_problem(3, 5.0, 2.0)
    p.m = p.m + 0.3j                         # absorbing medium: complex contrast
    yield "absorb900", p
    e = M.ellipse(3, 1.3, 0.7)
    yield "ellipse900", P.Problem(e, 9.0, P.contrast_from_index(e, [P.const(1.7)]), "ellipse900")


def main():
    out = {}
    for name, p in cases():
        C = vdim.correction_matrix(p.mesh, p.k)
        op = Operator(p.mesh, p.k, p.m, C)
        x = P.random_vectors(p.n_nodes, 3, seed=0)
        b = p.incident(np.array([0.0, 1.0]))
        X = np.concatenate([x, b])
        out[f"{name}/rowptr"] = C.indptr.astype(np.int64)
        out[f"{name}/col"] = C.indices.astype(np.int32)
        out[f"{name}/val"] = C.data.astype(np.complex128)
        out[f"{name}/x"] = X
        out[f"{name}/Lx"] = op.apply(X)
        out[f"{name}/LHx"] = op.apply_adjoint(X)
        if p.n_nodes <= 2600:
            out[f"{name}/b"] = b
            out[f"{name}/u"] = krylov.lu_solve(op.dense(), b)
        print(name, p.n_nodes, C.nnz, flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_cases.npz"), **out)


if __name__ == "__main__":
    main()
