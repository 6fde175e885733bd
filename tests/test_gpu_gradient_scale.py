"""The contrast gradient of the far-field misfit (autograd through the forward and adjoint GPU
solves) at a realistic size, N = 6 500 (two-material disk, k = 10, 4 waves, 32 receivers), against
the oracle's dense adjoint gradient stored by tests/golden/make_gradient_case.py (the GPU operator
takes the oracle's correction C, so both differentiate the same discrete system), and against
central finite differences of the GPU misfit along three seeded directions.  Solves that miss their
tolerance raise instead of returning a gradient."""
import os

import numpy as np
import pytest
import torch

import paper_2608_17615_amd as lsg
from tests.gpu_cases import relmax, scatterer
from workloads import problems as P

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gradient_twomat6500.npz")


def _setup():
    z = np.load(GOLDEN, allow_pickle=False)
    p = P.graded_two_material(5, 10.0, directions=P.even_directions(4))
    op = lsg.Operator(scatterer(p), correction=(z["rowptr"], z["col"], z["val"]))
    return p, op, z


def test_gradient_matches_oracle_at_n6500():
    p, op, z = _setup()
    th = P.receivers(32)
    bt = torch.tensor(p.incident(), device="cuda")
    dt = torch.tensor(z["data"], device="cuda")
    m = torch.tensor(np.real(p.m), device="cuda", requires_grad=True)
    J = lsg.farfield_misfit(m, op, bt, dt, th, tol=1e-13, maxit=1500)
    J.backward()
    g = m.grad.cpu().numpy()
    eJ = abs(J.item() - float(z["J"])) / float(z["J"])
    eg = relmax(g, z["grad"])
    print(f"N={p.n_nodes}: J {J.item():.9e} (oracle {float(z['J']):.9e}, {eJ:.1e}), gradient {eg:.2e}", flush=True)
    assert eJ <= 1e-10 and eg <= 1e-10
    # central differences with one Richardson step (error O(eps^4)); the step is large enough that
    # the solves' own tolerance (1e-13) stays far below the difference of the two misfits
    rng = np.random.default_rng(7)
    eps = 1e-4 * float(np.abs(p.m).max())

    def cd(d, h):
        with torch.no_grad():
            Jp = lsg.farfield_misfit(m.detach() + h * d, op, bt, dt, th, tol=1e-13, maxit=1500).item()
            Jm = lsg.farfield_misfit(m.detach() - h * d, op, bt, dt, th, tol=1e-13, maxit=1500).item()
        return (Jp - Jm) / (2 * h)
    for i in range(3):
        d = torch.tensor(rng.standard_normal(p.n_nodes), device="cuda")
        fd = (4 * cd(d, eps / 2) - cd(d, eps)) / 3
        ad = float(torch.dot(m.grad, d))
        print(f"direction {i}: finite difference {fd:.9e}, adjoint {ad:.9e}", flush=True)
        assert abs(fd - ad) <= 1e-6 * abs(fd)


def test_unconverged_solves_raise():
    p, op, z = _setup()
    th = P.receivers(32)
    bt = torch.tensor(p.incident(), device="cuda")
    dt = torch.tensor(z["data"], device="cuda")
    m = torch.tensor(np.real(p.m), device="cuda", requires_grad=True)
    with pytest.raises(lsg.LSError, match="forward solve"):
        lsg.farfield_misfit(m, op, bt, dt, th, tol=1e-13, maxit=3)
    J = lsg.farfield_misfit(m, op, bt, dt, th, tol=1e-13, maxit=1500, adjoint_maxit=3)
    with pytest.raises(lsg.LSError, match="adjoint solve"):
        J.backward()
