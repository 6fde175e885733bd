"""GPU apply and adjoint apply against the FP64 oracle (element by element, same seeded
inputs, the oracle's own correction C loaded through ls_setup_from_csr)."""
import numpy as np
import pytest
import torch

import paper_2608_17615_amd as lsg
from oracle import green as ogreen
from tests.gpu_cases import golden_problem, load_case, relmax, scatterer
from workloads import problems as P

pytestmark = pytest.mark.gpu

CASES = ["disk2500", "twomat1040", "absorb900", "ellipse900"]


def _op(name, **opts):
    p = golden_problem(name)
    c = load_case(name)
    op = lsg.Operator(scatterer(p), correction=(c["rowptr"], c["col"], c["val"]), **opts)
    return p, c, op


@pytest.mark.parametrize("name", CASES)
def test_apply_matches_oracle(name):
    p, c, op = _op(name)
    x = torch.tensor(c["x"], device="cuda")
    y = op.apply(x).cpu().numpy()
    e = relmax(y, c["Lx"])
    print(f"{name}: apply rel err {e:.3e}", flush=True)
    assert e <= 1e-12


@pytest.mark.parametrize("name", CASES)
def test_adjoint_apply_matches_oracle(name):
    p, c, op = _op(name)
    x = torch.tensor(c["x"], device="cuda")
    y = op.apply_adjoint(x).cpu().numpy()
    e = relmax(y, c["LHx"])
    print(f"{name}: adjoint rel err {e:.3e}", flush=True)
    assert e <= 1e-12


@pytest.mark.parametrize("opts", [dict(source_split=1), dict(source_split=7, targets_per_lane=1),
                                  dict(source_split=3, rhs_chunk=4), dict(rhs_chunk=16, targets_per_lane=1),
                                  dict(rhs_chunk=8, targets_per_lane=2), dict(source_split=200)])
def test_launch_configurations_agree(opts):
    p, c, op = _op("disk2500", **opts)
    x = torch.tensor(np.concatenate([c["x"]] * 6)[:16], device="cuda")   # 16 columns
    y = op.apply(x).cpu().numpy()
    ref = np.concatenate([c["Lx"]] * 6)[:16]
    assert relmax(y, ref) <= 1e-12
    ya = op.apply_adjoint(x).cpu().numpy()
    assert relmax(ya, np.concatenate([c["LHx"]] * 6)[:16]) <= 1e-12


def test_adjoint_identity_on_device():
    p, c, op = _op("twomat1040")
    x = torch.tensor(P.random_vectors(p.n_nodes, 2, 3), device="cuda")
    y = torch.tensor(P.random_vectors(p.n_nodes, 2, 4), device="cuda")
    Lx = op.apply(x)
    LHy = op.apply_adjoint(y)
    lhs = torch.sum(Lx.conj() * y).item()
    rhs = torch.sum(x.conj() * LHy).item()
    assert abs(lhs - rhs) <= 1e-13 * torch.linalg.norm(Lx).item() * torch.linalg.norm(y).item()


def test_full_size_far_sum_sampled_rows():
    """Two-material disk, k = 20, N = 58500 (the benchmark workload) with a zero correction:
    y = x + k^2 G~ W (m x); sampled rows against the oracle's punctured sum."""
    p = P.config2()
    n = p.n_nodes
    op = lsg.Operator(scatterer(p), correction=(np.zeros(n + 1, np.int64), np.zeros(0, np.int32),
                                                np.zeros(0, np.complex128)))
    x = P.random_vectors(n, 1, 0)
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()[0]
    rows = np.random.default_rng(1).choice(n, 48, replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    far = ogreen.far_rows(p.mesh.x, p.mesh.y, p.mesh.w, p.k, p.m * x[0], rows)[0]
    ref = x[0][rows] + p.k ** 2 * far
    e = float(np.abs(y[rows] - ref).max() / np.abs(ref).max())
    print(f"N={n}: sampled far-sum rel err {e:.3e}", flush=True)
    assert e <= 1e-12
