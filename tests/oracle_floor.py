"""The FP64 conditioning floor of an oracle result, for tolerances derived from the arithmetic.

The correction C is a difference of two numbers far larger than C itself: the exact potential
of the element's cubic interpolant, extended over the whole subdomain, minus its Nystrom sum (the
interpolant grows like (diameter / element size)^3 away from its element).  Any FP64 evaluation of
it therefore carries rounding far above the unit roundoff.  `floor(fn)` measures that:
the relative change of the oracle's own result fn() when its Hankel evaluation switches from
SciPy's AMOS routines to SciPy's Cephes J0 + i Y0 and J1 + i Y1.  Both are accurate to about 1e-15
relative on the arguments involved, so the change is what FP64 arithmetic alone leaves
undetermined.  Nothing here touches the GPU library.
"""
import contextlib

import numpy as np
from scipy import special

from oracle import bessel, field, vdim


@contextlib.contextmanager
def cephes_bessel():
    saved = (bessel.h0, bessel.h1, vdim.h0, vdim.h1, field.h0)
    h0 = lambda z: special.j0(np.asarray(z, dtype=np.float64)) + 1j * special.y0(np.asarray(z, dtype=np.float64))
    h1 = lambda z: special.j1(np.asarray(z, dtype=np.float64)) + 1j * special.y1(np.asarray(z, dtype=np.float64))
    bessel.h0 = vdim.h0 = field.h0 = h0
    bessel.h1 = vdim.h1 = h1
    try:
        yield
    finally:
        bessel.h0, bessel.h1, vdim.h0, vdim.h1, field.h0 = saved


def floor(fn):
    """max |fn()_cephes - fn()_amos| / max |fn()_amos| and the AMOS result."""
    a = np.asarray(fn())
    with cephes_bessel():
        b = np.asarray(fn())
    return float(np.abs(b - a).max() / np.abs(a).max()), a
