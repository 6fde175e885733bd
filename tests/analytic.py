"""Independent analytic and brute-force evaluations used to pin the oracle.

None of this reuses the oracle's Green's-identity machinery: volume potentials of
polynomials on disks and annuli come from Graf's addition theorem
    H0(k|x - y|) = sum_m J_m(k r_<) H_m(k r_>) e^{i m (theta - phi)},
which reduces them to 1-D radial integrals, and on general star-shaped domains from
polar coordinates centred at the target with panels graded geometrically toward it.
"""
from math import comb

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy import special

_T, _W = leggauss(24)


def _gl(a, b, f, panels=None):
    """Composite Gauss-Legendre of a vectorised f on [a, b]."""
    if b <= a:
        return 0.0
    if panels is None:
        panels = max(4, int(np.ceil((b - a) / 0.02)))
    e = np.linspace(a, b, panels + 1)
    h = 0.5 * np.diff(e)
    t = (0.5 * (e[:-1] + e[1:]))[:, None] + h[:, None] * _T[None, :]
    return np.sum(f(t) * (h[:, None] * _W[None, :]))


def _graded(a, b, f, toward='left', levels=40):
    """GL on [a, b] with panels halving toward one end (for a log/derivative singularity)."""
    L = b - a
    edges = [L * 2.0 ** (-i) for i in range(levels)][::-1]
    tot = 0.0
    prev = 0.0
    for e in edges:
        if toward == 'left':
            tot += _gl(a + prev, a + e, f, panels=1)
        else:
            tot += _gl(b - e, b - prev, f, panels=1)
        prev = e
    return tot


def poly_fourier(i, j):
    """Fourier coefficients c_m (m = -3..3) with cos^i(phi) sin^j(phi) = sum c_m e^{i m phi}."""
    M = 16
    ph = 2 * np.pi * np.arange(M) / M
    vals = np.cos(ph) ** i * np.sin(ph) ** j
    c = np.fft.fft(vals) / M
    return {m: c[m % M] for m in range(-3, 4)}


def annulus_mode_potential(k, a_in, a_out, m, power, r, theta):
    """int_{a_in < rho < a_out} G(x, y) rho^power e^{i m phi} dy at x = (r, theta)
    = (i pi / 2) e^{i m theta} int J_m(k r_<) H_m(k r_>) rho^(power+1) d rho."""
    J = lambda z: special.jv(m, z)
    H = lambda z: special.hankel1(m, z)
    f_in = lambda t: J(k * t) * t ** (power + 1)
    f_out = lambda t: H(k * t) * t ** (power + 1)
    lo, hi = a_in, a_out
    if r <= lo:       # target inside the hole (or the disk centre region): r < rho throughout
        val = J(k * r) * _gl(lo, hi, f_out)
    elif r >= hi:     # target outside: rho < r throughout
        val = H(k * r) * _gl(lo, hi, f_in)
    else:
        inner = _graded(lo, r, f_in, toward='right') if lo == 0 else _gl(lo, r, f_in)
        val = H(k * r) * inner + J(k * r) * _graded(r, hi, f_out, toward='left')
    return 0.5j * np.pi * np.exp(1j * m * theta) * val


def annulus_poly_potential(k, a_in, a_out, coeffs, x, y):
    """int over the annulus (a disk when a_in = 0) of G(x, .) P, P = sum coeffs[(i,j)] x^i y^j."""
    r = np.hypot(x, y)
    th = np.arctan2(y, x)
    tot = 0.0
    for (i, j), p in coeffs.items():
        if p == 0:
            continue
        for m, c in poly_fourier(i, j).items():
            if abs(c) < 1e-15:
                continue
            tot += p * c * annulus_mode_potential(k, a_in, a_out, m, i + j, r, th)
    return tot


def scaled_monomial_coeffs(a, b, c, s):
    """((x - c0)/s)^a ((y - c1)/s)^b as a dict of global monomial coefficients."""
    out = {}
    for i in range(a + 1):
        for j in range(b + 1):
            v = comb(a, i) * (-c[0]) ** (a - i) * comb(b, j) * (-c[1]) ** (b - j) / s ** (a + b)
            out[(i, j)] = out.get((i, j), 0.0) + v
    return out


def polar_potential(k, x0, rho_max, P, n_phi=400, levels=45):
    """Brute force int_D G(x0, y) P(y) dy for D star-shaped about x0 with boundary
    distance rho_max(phi): trapezoid in phi (periodic), graded GL in rho toward the target.
    P maps (px, py) arrays to an array with a trailing axis of outputs."""
    ph = 2 * np.pi * np.arange(n_phi) / n_phi
    R = rho_max(ph)                                   # [n_phi]
    tot = 0.0
    prev = np.zeros_like(R)
    for i in range(levels)[::-1]:
        e = R * 2.0 ** (-i)
        h = 0.5 * (e - prev)
        t = (0.5 * (e + prev))[:, None] + h[:, None] * _T[None, :]      # [n_phi, 24]
        px = x0[0] + t * np.cos(ph)[:, None]
        py = x0[1] + t * np.sin(ph)[:, None]
        g = 0.25j * (special.j0(k * t) + 1j * special.y0(k * t)) * t
        wts = h[:, None] * _W[None, :]
        vals = P(px, py)                              # [n_phi, 24, n_out]
        tot = tot + np.sum((g * wts)[..., None] * vals, axis=(0, 1))
        prev = e
    return tot * (2 * np.pi / n_phi)


def ellipse_rho_max(x0, a, b):
    """Distance from x0 (inside) to the ellipse x^2/a^2 + y^2/b^2 = 1 along direction phi."""
    def f(ph):
        dx, dy = np.cos(ph), np.sin(ph)
        A = dx * dx / a ** 2 + dy * dy / b ** 2
        B = 2 * (x0[0] * dx / a ** 2 + x0[1] * dy / b ** 2)
        C = x0[0] ** 2 / a ** 2 + x0[1] ** 2 / b ** 2 - 1
        return (-B + np.sqrt(B * B - 4 * A * C)) / (2 * A)
    return f


def disk_mode_potential_fn(k, a, m, f, r, theta):
    """int_{|y| < a} G(x, y) f(rho) e^{i m phi} dy at x = (r, theta), r < a, for a smooth
    radial profile f (vectorised), by the same addition-theorem reduction."""
    J = lambda z: special.jv(m, z)
    H = lambda z: special.hankel1(m, z)
    inner = _graded(0.0, r, lambda t: J(k * t) * f(t) * t, toward='right')
    outer = _graded(r, a, lambda t: H(k * t) * f(t) * t, toward='left')
    return 0.5j * np.pi * np.exp(1j * m * theta) * (H(k * r) * inner + J(k * r) * outer)
