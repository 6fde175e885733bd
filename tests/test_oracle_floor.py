"""The conditioning-floor helper: the Cephes Bessel values it swaps in agree with the oracle's AMOS
values to 1e-14 relative (so the floor it reports is a perturbation within FP64 accuracy), the
swap is undone afterwards, and on a correction row it reports a nonzero change well below 1e-9."""
import numpy as np

from oracle import bessel, vdim
from tests import oracle_floor as of
from workloads import problems as P


def test_swap_is_a_small_perturbation_and_is_undone():
    z = np.concatenate([np.logspace(-6, 2, 400), np.linspace(0.5, 60, 333)])
    a0, a1 = bessel.h0(z), bessel.h1(z)
    with of.cephes_bessel():
        b0, b1 = bessel.h0(z), vdim.h1(z)
    assert np.abs(b0 - a0).max() <= 1e-14 * np.abs(a0).max()
    assert np.all(np.abs(b1 - a1) <= 1e-14 * np.abs(a1))
    assert bessel.h0 is not None and np.array_equal(bessel.h0(z), a0)


def test_floor_of_a_correction_row():
    p = P.config1()
    g = vdim.Geometry(p.mesh)
    f, row = of.floor(lambda: vdim.correction_row(g, p.k, 1234)[1])
    assert 0 < f < 1e-9
