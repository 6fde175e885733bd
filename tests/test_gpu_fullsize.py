"""Full-size parity at the benchmark workloads, in the launch configurations bench.py times.

The GPU operator is built by the library's own setup (so the sparse correction is the native
one), applied to the workloads' plane waves, and sampled rows are compared with the oracle, which
computes each sampled row one by one: its punctured far sum with SciPy's H0 plus its own
correction row.  The FP64 bar is 1e-12 or five times the oracle's own conditioning floor for the
same rows (tests/oracle_floor.py; the reasoning is in tests/test_gpu_setup.py), whichever is larger.  Properties that hold at any size (the
adjoint identity) are checked on the full vectors."""
import numpy as np
import pytest
import torch

import paper_2608_17615_amd as lsg
from oracle import green as ogreen
from oracle import vdim
from tests import oracle_floor as of
from tests.gpu_cases import relmax
from workloads import problems as P

pytestmark = pytest.mark.gpu


def oracle_rows(prob, x, rows):
    """Rows of L x = x + k^2 (G~ W + C)(m x) for x of shape (B, N)."""
    msh, k = prob.mesh, prob.k
    f = prob.m[None, :] * x
    far = ogreen.far_rows(msh.x, msh.y, msh.w, k, f, rows)
    geom = vdim.Geometry(msh)
    corr = np.zeros_like(far)
    for i, j in enumerate(rows):
        cols, vals = vdim.correction_row(geom, k, int(j))
        corr[:, i] = f[:, cols] @ vals
    return x[:, rows] + k * k * (far + corr)


def sample(n, count, seed):
    rows = np.random.default_rng(seed).choice(n, count, replace=False)
    return np.unique(np.concatenate([rows, [0, n - 1]]))


def test_c3_batched_tiles_sampled_rows():
    """Unit disk, k = 40, N = 122 500, 64 plane waves: FP64 and FP32 matrix-core tiles."""
    prob = P.config3()
    op = lsg.Operator(lsg.Scatterer.from_mesh(prob.mesh, prob.m, prob.k))
    x = prob.incident()
    xt = torch.tensor(x, device="cuda")
    y64 = op.apply(xt).cpu().numpy()
    ym = op.apply(xt, precision="mixed").cpu().numpy()
    rows = sample(prob.n_nodes, 16, 11)
    fl, ref = of.floor(lambda: oracle_rows(prob, x, rows))
    e64, em = relmax(y64[:, rows], ref), relmax(ym[:, rows], ref)
    bar = max(1e-12, 5 * fl)
    print(f"C3 N={prob.n_nodes} B=64: FP64 tiles {e64:.2e} (oracle floor {fl:.2e}, bar {bar:.1e}), "
          f"FP32 tiles {em:.2e} ({rows.size} rows)", flush=True)
    assert e64 <= bar
    assert em <= 3e-5


def test_c4_persistent_batch_sampled_rows():
    """16 scatterers of uneven size in one persistent launch (FP64 and FP32 tiles), 8 plane
    waves each: every scatterer's sampled rows against the oracle."""
    probs = P.config4()
    scats = [lsg.Scatterer.from_mesh(p.mesh, p.m, p.k) for p in probs]
    op64 = lsg.Operator(scats, fp64_matrix=2)
    x = np.concatenate([p.incident() for p in probs], axis=1)
    xt = torch.tensor(x, device="cuda")
    y64 = op64.apply(xt).cpu().numpy()
    ym = op64.apply(xt, precision="mixed").cpu().numpy()
    worst64 = worstm = 0.0
    for s, p in enumerate(probs):
        o = op64.offsets[s]
        rows = sample(p.n_nodes, 3, 20 + s)
        fl, ref = of.floor(lambda: oracle_rows(p, x[:, o:o + p.n_nodes], rows))
        e64 = relmax(y64[:, o + rows], ref)
        worst64 = max(worst64, e64 / max(1e-12, 5 * fl))
        worstm = max(worstm, relmax(ym[:, o + rows], ref))
    print(f"C4 16 scatterers, N = {op64.n}: FP64 tiles at most {worst64:.2f} of the bar max(1e-12, 5 x oracle "
          f"floor), FP32 tiles {worstm:.2e}", flush=True)
    assert worst64 <= 1.0
    assert worstm <= 3e-5


def test_c5_forward_rows_and_adjoint_identity():
    """Two-material disk, k = 40, N = 114 660, 16 plane waves: sampled forward rows against the
    oracle and <L x, y> = <x, L^H y> on the full vectors (FP64 tiles)."""
    prob = P.config5()
    op = lsg.Operator(lsg.Scatterer.from_mesh(prob.mesh, prob.m, prob.k))
    x = prob.incident()
    xt = torch.tensor(x, device="cuda")
    y = op.apply(xt).cpu().numpy()
    rows = sample(prob.n_nodes, 16, 12)
    fl, ref = of.floor(lambda: oracle_rows(prob, x, rows))
    e = relmax(y[:, rows], ref)
    yv = torch.tensor(P.random_vectors(prob.n_nodes, 16, 13), device="cuda")
    Lx = op.apply(xt)
    LHy = op.apply_adjoint(yv)
    lhs = torch.sum(Lx.conj() * yv).item()
    rhs = torch.sum(xt.conj() * LHy).item()
    ident = abs(lhs - rhs) / (torch.linalg.norm(Lx).item() * torch.linalg.norm(yv).item())
    print(f"C5 N={prob.n_nodes} B=16: forward rows {e:.2e} (oracle floor {fl:.2e}), adjoint identity {ident:.1e}",
          flush=True)
    assert e <= max(1e-12, 5 * fl)
    assert ident <= 1e-13
