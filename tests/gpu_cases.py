"""Helpers shared by the GPU tests (inputs and oracle-written expected values only)."""
import os

import numpy as np

import paper_2608_17615_amd as lsg
from workloads import mesh as M
from workloads import problems as P

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_cases.npz")


def golden_problem(name):
    if name == "disk2500":
        return P.config1()
    if name == "twomat1040":
        return P.graded_two_material(2, 20.0)
    if name == "absorb900":
        p = P.disk_problem(3, 5.0, 2.0)
        p.m = p.m + 0.3j
        return p
    if name == "ellipse900":
        e = M.ellipse(3, 1.3, 0.7)
        return P.Problem(e, 9.0, P.contrast_from_index(e, [P.const(1.7)]), "ellipse900")
    raise KeyError(name)


def load_case(name):
    z = np.load(GOLDEN, allow_pickle=False)
    return {k.split("/", 1)[1]: z[k] for k in z.files if k.startswith(name + "/")}


def scatterer(p):
    return lsg.Scatterer.from_mesh(p.mesh, p.m, p.k)


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())
