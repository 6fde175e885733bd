"""Uneven batch of scatterers in one persistent matrix-core launch: each scatterer's block of the
result equals the single-scatterer computation; results are independent of the schedule; the
autotuner returns a supported shape whose results agree."""
import os

import numpy as np
import pytest
import torch

import paper_2608_17615_amd as lsg
from tests.gpu_cases import relmax
from workloads import mesh as M
from workloads import problems as P

pytestmark = pytest.mark.gpu


def _batch():
    out = [P.disk_problem(3, 9.0, 2.0), P.graded_two_material(2, 14.0)]
    e = M.ellipse(4, 1.3, 0.6)
    out.append(P.Problem(e, 22.0, P.contrast_from_index(e, [P.const(0.7)]), "ellipse"))
    out.append(P.disk_problem(2, 5.0, 2.6))
    return out


def _scats(probs):
    return [lsg.Scatterer.from_mesh(p.mesh, p.m, p.k) for p in probs]


@pytest.mark.parametrize("precision,fp64_matrix,B,tol", [("fp64", 2, 5, 1e-13), ("fp64", 2, 8, 1e-13),
                                                         ("fp64", 2, 16, 1e-13), ("fp64", 2, 24, 1e-13),
                                                         ("mixed", 0, 8, 3e-5), ("mixed", 0, 33, 3e-5)])
def test_batch_equals_separate(precision, fp64_matrix, B, tol):
    """Each scatterer's block of the batched persistent launch against that scatterer alone through
    the FP64 VALU sum (no matrix cores), forward and adjoint; B <= 8 takes the split-column tiles."""
    probs = _batch()
    big = lsg.Operator(_scats(probs), fp64_matrix=fp64_matrix)
    ntot = sum(p.n_nodes for p in probs)
    x = torch.tensor(P.random_vectors(ntot, B, 2), device="cuda")
    for adj in (False, True):
        y = big.apply(x, precision=precision, adjoint=adj).cpu().numpy()
        off = 0
        for p, s in zip(probs, _scats(probs)):
            single = lsg.Operator(s, fp64_matrix=1)
            xs = x[:, off:off + p.n_nodes].contiguous()
            ref = single.apply(xs, precision="fp64", adjoint=adj).cpu().numpy()
            e = relmax(y[:, off:off + p.n_nodes], ref)
            print(f"{precision} B={B} adjoint={adj} {p.name or 'scatterer'} N={p.n_nodes}: {e:.2e}", flush=True)
            assert e <= tol
            off += p.n_nodes
    y1 = big.apply(x, precision=precision).cpu().numpy()
    y2 = big.apply(x, precision=precision).cpu().numpy()
    assert np.array_equal(y1, y2)


def test_autotune_and_cache(tmp_path):
    probs = _batch()
    big = lsg.Operator(_scats(probs))
    ntot = sum(p.n_nodes for p in probs)
    x = torch.tensor(P.random_vectors(ntot, 8, 5), device="cuda")
    y0 = big.apply(x, precision="mixed").cpu().numpy()
    cache = os.path.join(str(tmp_path), "tiles.json")
    mt, sl, ms = big.autotune(8, "mixed", cache=cache)
    print(f"autotune: mt={mt} split_len={sl} far {ms:.3f} ms", flush=True)
    assert mt in (2, 4) and sl in (1024, 2048, 4096, 8192) and ms > 0
    mt2, sl2, ms2 = big.autotune(8, "mixed", cache=cache)
    assert (mt2, sl2, ms2) == (mt, sl, None)
    y1 = big.apply(x, precision="mixed").cpu().numpy()
    assert relmax(y1, y0) <= 3e-5


def test_batch_solve_mixed_and_fp64():
    probs = _batch()
    big = lsg.Operator(_scats(probs))
    b = np.concatenate([p.incident(np.array([0.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0])) for p in probs], axis=1)
    bt = torch.tensor(b, device="cuda")
    x64, i64 = big.solve(bt, tol=1e-10, maxit=1500)
    xm, im = big.solve(bt, tol=1e-10, maxit=1500, precision="mixed")
    print(f"batch solve: fp64 iters {i64['iters'].max()} mixed iters {im['iters'].max()} "
          f"mixed applies {im['n_apply_mixed'] // 8} fp64 applies {im['n_apply_fp64'] // 8}", flush=True)
    assert i64["converged"] and im["converged"]
    assert relmax(xm.cpu().numpy(), x64.cpu().numpy()) <= 1e-7


def test_scatterers_are_independent_systems():
    """In a multi-scatterer handle every (scatterer, column) pair is its own GMRES system: each
    block of the solution equals the separate single-scatterer solve (same tiles, same order of
    the sums), and a column takes as many steps as its hardest scatterer."""
    probs = _batch()
    big = lsg.Operator(_scats(probs))
    th = np.array([0.0, 2.0])
    b = np.concatenate([p.incident(th) for p in probs], axis=1)
    x, info = big.solve(torch.tensor(b, device="cuda"), tol=1e-10, maxit=1500)
    assert info["converged"]
    x = x.cpu().numpy()
    its = np.zeros(2, dtype=int)
    for s, p in enumerate(probs):
        one = lsg.Operator(_scats([p]))
        xs, i1 = one.solve(torch.tensor(p.incident(th), device="cuda"), tol=1e-10, maxit=1500)
        assert i1["converged"]
        its = np.maximum(its, i1["iters"])
        blk = x[:, big.offsets[s]:big.offsets[s] + p.n_nodes]
        e = relmax(blk, xs.cpu().numpy())
        print(f"scatterer {s}: iters {i1['iters']}, block vs separate {e:.1e}", flush=True)
        assert e <= 1e-13
    assert np.array_equal(info["iters"], its)
