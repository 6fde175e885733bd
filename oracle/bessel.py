"""Hankel functions of the first kind used by the oracle.

G(x, y) = (i/4) H0^(1)(k |x - y|) is the paper's free-space Green's function (Section 2,
after eq. Lippmann-Schwinger).  H0 and H1 are SciPy's AMOS
Hankel routines (relative error below 1e-15 on (0, 120]); a test pins them against mpmath.
"""
import numpy as np
from scipy import special


def h0(z):
    return special.hankel1(0, np.asarray(z, dtype=np.float64))


def h1(z):
    return special.hankel1(1, np.asarray(z, dtype=np.float64))


def green(k, r):
    """(i/4) H0^(1)(k r) for r > 0."""
    return 0.25j * h0(k * np.asarray(r, dtype=np.float64))
