"""The 10-node, degree-5, fully symmetric rule on the reference triangle (area 1/2).

Constants printed by ``python -m workloads.gen_rule10`` (orbit structure and selection
criterion are described there).  Returned barycentric coordinates are (l1, l2, l3); the
reference point is (xi, eta) = (l2, l3).
"""
import itertools

import numpy as np

W0 = 0.0994826828130151708088378591031
W1 = 0.0301261671531544061428377079157
W2 = 0.0516898026212536017937748361917
A = 0.071094437341974341875366894758
C = 0.313951119736123944213543061725


def rule10():
    """Return (bary[10, 3], weights[10]) in a fixed node order."""
    pts = [(1.0 / 3, 1.0 / 3, 1.0 / 3)]
    wts = [W0]
    for p in sorted(set(itertools.permutations((A, A, 1.0 - 2.0 * A)))):
        pts.append(p)
        wts.append(W1)
    for p in sorted(set(itertools.permutations((A, C, 1.0 - A - C)))):
        pts.append(p)
        wts.append(W2)
    return np.array(pts, dtype=np.float64), np.array(wts, dtype=np.float64)
