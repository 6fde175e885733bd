"""Host-side logic of bench.py: the flop model by argument range, the z-distribution sampler and
the one-GPU contract (no GPU needed)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from workloads import problems as P  # noqa: E402


def test_z_fractions_match_brute_force():
    """The sampled range fractions equal a brute-force count over every pair of a small mesh."""
    p = P.disk_problem(3, 9.0, 2.0)
    x, y, k, n = p.mesh.x, p.mesh.y, p.k, p.n_nodes
    z = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :]) * k
    z = z[~np.eye(n, dtype=bool)]
    want = np.histogram(z, bins=[0.0, *bench.Z_BOUNDS, np.inf])[0] / z.size
    got = bench.z_fractions([(p.mesh, k)], rows=n)     # every row: exact
    assert np.allclose([got[r] for r in ("small", "mid1", "mid2", "far")], want, atol=1e-15)
    assert abs(sum(got.values()) - 1.0) < 1e-14


def test_flops_per_pair_is_a_weighted_mean_of_the_ranges():
    f = bench.FLOPS_RANGE
    for r in f:
        frac = {q: float(q == r) for q in f}
        assert bench.flops_per_pair(frac, 1) == f[r] + bench.FLOPS_PER_RHS
    frac = {"small": 0.1, "mid1": 0.2, "mid2": 0.3, "far": 0.4}
    want = 0.1 * f["small"] + 0.2 * f["mid1"] + 0.3 * f["mid2"] + 0.4 * f["far"] + 3 * bench.FLOPS_PER_RHS
    assert abs(bench.flops_per_pair(frac, 3) - want) < 1e-12


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_sparsifying_preconditioner_matches_the_oracle():
    """The bench's host construction of S^(C) = (C^(C))^-1 A (library host Green's values, 25
    offsets) equals the oracle's dense construction (SciPy Hankel values, the full product A L^(C)
    and its 3 x 3 filter) on 21 x 21 and 23 x 17 grids over a disk; S does not depend on the
    phase of each row's singular vector, so the two are compared entry by entry."""
    from oracle import sparsify as spf
    from oracle.transfer import Grid
    k, h = 8.0, 0.11
    for nx, ny in ((21, 21), (23, 17)):   # a non-square grid catches swapped indices
        g = Grid(-1.1, -0.9, h, nx, ny)
        zx, zy = g.nodes()
        m = np.where(np.hypot(zx, zy) < 0.85, -1.0, 0.0)
        S, ratio = bench.sparsifying_S(g.x0, g.y0, g.h, g.nx, g.ny, k, m)
        So, _, _, _, ratio_o = spf.sparsifying_preconditioner(g, k, m, width=1)
        assert abs(ratio - ratio_o) <= 1e-9 * ratio_o
        assert np.abs(S - So).max() <= 1e-12 * np.abs(So).max()


def test_block_lu_applier_matches_the_dense_sparsifying_S():
    """BlockSparsifier (block LU of C^(C) by grid rows, 9-point stencil for A) applies S^(C) and
    S^(C)^H as the dense (C^(C))^-1 A does, run with torch on the CPU; edge and corner rows carry
    their own weights, so a non-square grid checks the block bookkeeping."""
    import torch
    k, h = 8.0, 0.11
    rng = np.random.default_rng(11)
    for nx, ny in ((21, 21), (23, 17)):
        zx = -1.1 + h * np.tile(np.arange(nx), ny)
        zy = -0.9 + h * np.repeat(np.arange(ny), nx)
        m = np.where(np.hypot(zx, zy) < 0.85, -1.0 + 0.3j, 0.0)
        W, E, _ = bench.sparsifying_stencil(-1.1, -0.9, h, nx, ny, k, m)
        S = np.linalg.solve(bench.stencil_to_dense(E, nx, ny), bench.stencil_to_dense(W, nx, ny))
        v = rng.standard_normal((3, nx * ny)) + 1j * rng.standard_normal((3, nx * ny))
        fwd = bench.BlockSparsifier(W, E, nx, ny, "cpu")(torch.tensor(v)).numpy()
        adj = bench.BlockSparsifier(W, E, nx, ny, "cpu", adjoint=True)(torch.tensor(v)).numpy()
        ref, refh = v @ S.T, v @ S.conj()
        assert np.abs(fwd - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.abs(adj - refh).max() <= 1e-12 * np.abs(refh).max()
