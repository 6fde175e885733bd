"""Batched right-hand sides: FP64 matrix-core tiles (exact variant) and FP32 mixed tiles
against the oracle, including padded (ragged) RHS counts."""
import numpy as np
import pytest
import torch

import paper_2608_17615_amd as lsg
from tests.gpu_cases import golden_problem, load_case, relmax, scatterer

pytestmark = pytest.mark.gpu


def _op(name, **kw):
    p = golden_problem(name)
    c = load_case(name)
    return p, c, lsg.Operator(scatterer(p), correction=(c["rowptr"], c["col"], c["val"]), **kw)


def _cols(c, key, B):
    reps = (B + c[key].shape[0] - 1) // c[key].shape[0]
    return np.concatenate([c[key]] * reps)[:B]


@pytest.mark.parametrize("name", ["disk2500", "twomat1040", "absorb900"])
@pytest.mark.parametrize("B", [1, 5, 8, 16, 20, 64])
def test_fp64_tiles_match_oracle(name, B):
    """FP64 tiles forced onto the matrix cores; up to 8 right-hand sides take the split-column form
    (Re X and Im X in the two halves of one 16-column tile)."""
    p, c, op = _op(name, fp64_matrix=2)
    x = torch.tensor(_cols(c, "x", B), device="cuda")
    e = relmax(op.apply(x).cpu().numpy(), _cols(c, "Lx", B))
    ea = relmax(op.apply_adjoint(x).cpu().numpy(), _cols(c, "LHx", B))
    print(f"{name} B={B}: FP64 tiles apply {e:.2e} adjoint {ea:.2e}", flush=True)
    assert e <= 1e-12 and ea <= 1e-12


@pytest.mark.parametrize("name", ["disk2500", "twomat1040", "ellipse900"])
@pytest.mark.parametrize("B", [1, 5, 8, 16, 48])
def test_mixed_tiles_error(name, B):
    """FP32 Green's tiles (phase reduced in FP64) with FP32 accumulation per source split: the
    error of L x stays at the FP32 level (observed 1e-9 to 1e-7 of the largest entry)."""
    p, c, op = _op(name)
    x = torch.tensor(_cols(c, "x", B), device="cuda")
    y = op.apply(x, precision="mixed").cpu().numpy()
    ref = _cols(c, "Lx", B)
    e = relmax(y, ref)
    ya = op.apply_adjoint(x, precision="mixed").cpu().numpy()
    ea = relmax(ya, _cols(c, "LHx", B))
    print(f"{name} B={B}: mixed apply {e:.2e} adjoint {ea:.2e}", flush=True)
    assert e <= 1e-6 and ea <= 1e-6


@pytest.mark.parametrize("name", ["disk2500", "twomat1040", "ellipse900"])
@pytest.mark.parametrize("B", [5, 16, 20, 48, 64, 100])
def test_split_fp16_tiles_error(name, B):
    """Split-FP16 matrix-core tiles (each operand a sum of two FP16 numbers, three FP16 products with
    FP32 accumulation): forward and adjoint within the FP32 tiles' bar of the oracle's L x, for
    every tile shape (one, two and four 16-column tiles per wave, ragged column counts)."""
    p, c, op = _op(name, mixed_fp16=1)
    x = torch.tensor(_cols(c, "x", B), device="cuda")
    y = op.apply(x, precision="mixed").cpu().numpy()
    e = relmax(y, _cols(c, "Lx", B))
    ea = relmax(op.apply_adjoint(x, precision="mixed").cpu().numpy(), _cols(c, "LHx", B))
    print(f"{name} B={B}: split-FP16 apply {e:.2e} adjoint {ea:.2e}", flush=True)
    assert e <= 1e-6 and ea <= 1e-6


def test_split_fp16_is_the_default_at_64_columns():
    """A single-scatterer handle takes the split-FP16 tiles by default at 64 columns and the FP32
    tiles at 16: the default equals the forced variant bit for bit."""
    p, c, op = _op("disk2500")
    _, _, h16 = _op("disk2500", mixed_fp16=1)
    _, _, f32 = _op("disk2500", mixed_fp16=2)
    for B, same in ((64, h16), (16, f32)):
        x = torch.tensor(_cols(c, "x", B), device="cuda")
        assert torch.equal(op.apply(x, precision="mixed"), same.apply(x, precision="mixed"))


@pytest.mark.parametrize("fp16", [2, 1])
@pytest.mark.parametrize("name", ["disk2500", "twomat1040", "absorb900"])
def test_near_pairs_taken_in_fp64(name, fp16):
    """Mixed applications leave the far sum's pairs with z = k |y_j - y_n| < 1 (the logarithmic
    part of G) out of the FP32 / split-FP16 tiles and add them with an FP64 near launch: the
    number of such pairs against a count from the node positions, and forward and adjoint against
    the oracle's L x, with the near launch and with the pairs kept in the tiles."""
    p, c, op = _op(name, mixed_fp16=fp16)
    _, _, keep = _op(name, mixed_fp16=fp16, mixed_near=1)
    x, y, k = p.mesh.x, p.mesh.y, p.k
    z2 = k * k * ((x[:, None] - x[None, :]) ** 2 + (y[:, None] - y[None, :]) ** 2)
    count = int((z2 < 1.0).sum()) - x.size
    assert abs(op.near_pairs() - count) <= max(2, count // 10000) and keep.near_pairs() == 0
    B = 20
    xt = torch.tensor(_cols(c, "x", B), device="cuda")
    res = {}
    for tag, o in (("near in FP64", op), ("near in the tiles", keep)):
        e = relmax(o.apply(xt, precision="mixed").cpu().numpy(), _cols(c, "Lx", B))
        ea = relmax(o.apply_adjoint(xt, precision="mixed").cpu().numpy(), _cols(c, "LHx", B))
        res[tag] = (e, ea)
    kind = "split-FP16" if fp16 == 1 else "FP32"
    print(f"{name} {kind}, {count} near pairs: " + ", ".join(f"{t}: apply {e:.2e} adjoint {ea:.2e}"
                                                          for t, (e, ea) in res.items()), flush=True)
    e, ea = res["near in FP64"]
    assert e <= 1e-6 and ea <= 1e-6
