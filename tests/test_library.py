"""Host-side checks of the C-ABI library: it loads, exports every declared entry point,
validates arguments without touching a GPU, and its Hankel arithmetic (compiled for the host
from the same source as the kernels) matches mpmath."""
import ctypes
import os
import re

import mpmath as mp
import numpy as np
import pytest

import paper_2608_17615_amd as lsg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "ls.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    # function names followed by their parameter list; "ls_status (*ls_grid_op)(" is a pointer type
    return sorted(set(re.findall(r"\b(ls_[a-z0-9_]+)\s*\((?!\*)", txt)))


def test_every_declared_symbol_is_exported():
    L = lsg.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = lsg.lib()
    for st in (0, 1, -1, -2, -3, -4, -5, -6):
        assert L.ls_status_str(st)


def test_argument_validation_before_any_device_call():
    L = lsg.lib()
    y = ctypes.c_void_p()
    assert L.ls_apply(None, None, None, 1, 1, 0, None) == -1
    assert L.ls_solve_gmres(None, None, None, 1, 1, None, None, None) < 0
    # a scatterer with a wrong node count per element is rejected before any HIP call
    s = lsg._Scatterer(25, 2, 10, None, None, None, None, None, 1.0, 0, 0, None)
    assert L.ls_setup_from_csr(ctypes.byref(s), None, None, None, None, ctypes.byref(y)) == -1
    assert L.ls_eval_green_host(None, None, -1) == -1
    assert L.ls_transfer_setup(None, 0, None) == -1
    assert L.ls_quad_to_cart(None, 0, None, 1, None, 1, 1, None) == -1
    assert L.ls_precond_finish(None, 0, None, 1, None, None, 1, None, 1, None) == -1


def test_host_green_matches_mpmath():
    mp.mp.dps = 40
    z = np.concatenate([np.logspace(-7, np.log10(150), 1500),
                        np.linspace(1.995, 2.005, 11), np.linspace(4.995, 5.005, 11),
                        np.linspace(11.995, 12.005, 11)])
    g = lsg.eval_green_host(z * z)
    ref = np.array([complex(0.25j * mp.hankel1(0, mp.mpf(float(t)))) for t in z])
    err = np.abs(g - ref) / np.abs(ref)
    # the argument arrives as z^2, so the phase inherits ~z eps/2 from rounding z^2 itself
    assert np.all(err <= 4.5e-16 * np.maximum(1.0, z)), err.max()


def test_workspace_and_options_structs_match_header():
    assert ctypes.sizeof(lsg._Curve) == 48
    assert ctypes.sizeof(lsg._Scatterer) == 80
    assert ctypes.sizeof(lsg._SolveOpts) == 40
    assert ctypes.sizeof(lsg._Options) == 24
    assert ctypes.sizeof(lsg._Profile) == 40
    assert ctypes.sizeof(lsg._SolveInfo) == 48
    assert ctypes.sizeof(lsg._Grid) == 32
