"""Device Hankel evaluation against mpmath and against the same code compiled for the host."""
import mpmath as mp
import numpy as np
import pytest
import torch

import paper_2608_17615_amd as lsg

pytestmark = pytest.mark.gpu


def test_device_green_matches_mpmath_and_host():
    mp.mp.dps = 40
    z = np.concatenate([np.logspace(-7, np.log10(150), 3000),
                        np.linspace(1.995, 2.005, 11), np.linspace(4.995, 5.005, 11),
                        np.linspace(11.995, 12.005, 11)])
    z2 = torch.tensor(z * z, dtype=torch.float64, device="cuda")
    g = lsg.eval_green(z2).cpu().numpy()
    ref = np.array([complex(0.25j * mp.hankel1(0, mp.mpf(float(t)))) for t in z])
    err = np.abs(g - ref) / np.abs(ref)
    print("device green max rel err / max(1,z):", (err / np.maximum(1, z)).max(), flush=True)
    assert np.all(err <= 4.5e-16 * np.maximum(1.0, z))
    # host and device start the Halley step from different first approximations of z^(-1/2)
    # (hardware reciprocal square root vs libm), so they may differ by a rounding of that root
    h = lsg.eval_green_host(z * z)
    assert np.all(np.abs(g - h) <= 1e-15 * np.abs(h) * np.maximum(1.0, z))


def test_device_green_single_precision():
    """FP32 evaluation used by the mixed-precision tiles (FP64 below z = 1)."""
    mp.mp.dps = 30
    z = np.concatenate([np.logspace(-5, np.log10(160), 2000), np.linspace(0.99, 1.01, 21), np.linspace(7.99, 8.01, 21)])
    z2 = torch.tensor(z * z, dtype=torch.float64, device="cuda")
    g = lsg.eval_green(z2, single=True).cpu().numpy()
    ref = np.array([complex(0.25j * mp.hankel1(0, mp.mpf(float(t)))) for t in z])
    err = np.abs(g - ref) / np.abs(ref)
    print("single-precision green: max rel err", err.max(), "(z<1)", err[z < 1].max(), flush=True)
    assert np.all(err[z < 1] <= 1e-7)                       # FP64 series, rounded to FP32
    assert np.all(err <= 5e-7)                               # phase reduced in FP64: FP32 level at every z
