"""Host-side logic of bench.py: the flop model by argument range, the z-distribution sampler and
the one-GPU contract (no GPU needed).  The preconditioner the bench uses is the library's (its
host construction is checked against the oracle in test_sparsify_host.py)."""
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
