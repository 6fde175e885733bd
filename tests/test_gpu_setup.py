"""Native ls_setup (Green's-identity potentials on the host, punctured sums on the GPU)
against the oracle's correction C on the golden meshes.

Entry by entry the two constructions differ by rounding amplified by the size of the
extended cubic Lagrange basis over the subdomain (differences of two numbers ~(diam/h)^3
larger than the entry), so entries are compared relative to those magnitudes and the
action of C on smooth densities (cubics, plane waves) is compared at 1e-12."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_2608_17615_amd as lsg
from tests.gpu_cases import golden_problem, load_case, relmax, scatterer

pytestmark = pytest.mark.gpu

CASES = ["disk2500", "twomat1040", "absorb900", "ellipse900"]


def _csr(rowptr, col, val, n):
    return sp.csr_matrix((val, col, rowptr), shape=(n, n))


@pytest.mark.parametrize("name", CASES)
def test_native_correction_matches_oracle(name):
    p = golden_problem(name)
    c = load_case(name)
    n = p.n_nodes
    op = lsg.Operator(scatterer(p))
    rp, col, val = op.export_correction()
    Cn = _csr(rp, col, val, n)
    Co = _csr(c["rowptr"], c["col"], c["val"], n)
    same_cols = np.mean([set(Cn[j].indices) == set(Co[j].indices) for j in range(n)])
    print(f"{name}: nnz native {Cn.nnz} oracle {Co.nnz}, rows with identical columns {same_cols:.4f}", flush=True)
    assert Cn.nnz == Co.nnz and same_cols >= 0.999
    # action on smooth densities
    x, y = p.mesh.x, p.mesh.y
    smooth = [np.ones(n), x, y * x, x ** 3 - 2 * x * y * y + 0.3, np.exp(1j * p.k * x),
              np.exp(1j * p.k * (0.6 * x + 0.8 * y))]
    worst = 0.0
    for f in smooth:
        d = np.abs(Cn @ f - Co @ f).max() / max(np.abs(Co @ f).max(), 1e-300)
        worst = max(worst, d)
    print(f"{name}: C f relative difference on smooth f {worst:.3e}", flush=True)
    assert worst <= 1e-11
    # entries (rows with identical columns), relative to the largest entry of their row
    D = (Cn - Co).tocsr()
    rowmax = np.maximum(np.abs(Co).max(axis=1).toarray().ravel(), 1e-300)
    ent = (np.abs(D).max(axis=1).toarray().ravel() / rowmax)
    print(f"{name}: max entrywise difference / row max {np.max(ent):.3e}, median {np.median(ent):.3e}", flush=True)
    assert np.median(ent) <= 1e-7 and np.max(ent) <= 1e-5


@pytest.mark.parametrize("name", ["disk2500", "twomat1040"])
def test_native_setup_apply_matches_oracle(name):
    p = golden_problem(name)
    c = load_case(name)
    op = lsg.Operator(scatterer(p))
    xb = torch.tensor(c["x"][3:], device="cuda")          # the two plane waves
    y = op.apply(xb).cpu().numpy()
    e = relmax(y, c["Lx"][3:])
    print(f"{name}: native-setup apply on plane waves rel err {e:.3e}", flush=True)
    assert e <= 1e-10
