"""Fourier-Bessel (Mie) series for plane-wave scattering by radially layered disks.

The paper's benchmark reference (Section 6.1) for the constant-index disk.  With
u_inc = exp(i k r cos(theta - theta_d)) = sum_nu i^nu J_nu(k r) e^{i nu (theta - theta_d)},
each angular mode is a solution of Bessel's equation with wavenumber k sqrt(n) in every
layer; continuity of u and du/dr across each circle fixes the coefficients.
"""
import numpy as np
from scipy import special


def _nu_max(kr):
    kr = abs(kr)
    return int(np.ceil(kr + 20 + 6 * kr ** (1 / 3)))


def disk(k, n_in, a, x, y, theta_d=0.0):
    """Total field at points inside the disk r < a of constant index n_in (n = 1 outside).

    a_nu = i^nu (2i/(pi a)) / [k J_nu(k_i a) H_nu'(k a) - k_i J_nu'(k_i a) H_nu(k a)],
    from the two continuity conditions and the Wronskian J H' - J' H = 2i/(pi z).
    Returns (u, b) where b are the exterior scattered coefficients (for the far field).
    """
    ki = k * np.sqrt(complex(n_in))
    r = np.hypot(x, y)
    th = np.arctan2(y, x)
    nmax = _nu_max(ki * a)
    nus = np.arange(-nmax, nmax + 1)
    Jia = special.jv(nus, ki * a)
    dJia = special.jvp(nus, ki * a)
    Ha = special.hankel1(nus, k * a)
    dHa = special.h1vp(nus, k * a)
    coef = (1j ** nus) * (2j / (np.pi * a)) / (k * Jia * dHa - ki * dJia * Ha)
    u = np.zeros(np.shape(x), dtype=np.complex128)
    for nu, c in zip(nus, coef):
        u = u + c * special.jv(nu, ki * r) * np.exp(1j * nu * (th - theta_d))
    bcoef = (coef * Jia - (1j ** nus) * special.jv(nus, k * a)) / Ha
    return u, (nus, bcoef)


def two_layer(k, n_in, n_out, a1, a2, x, y, theta_d=0.0):
    """Total field inside the two-layer disk: index n_in for r < a1, n_out for a1 < r < a2.

    Per mode: A J(k2 r) inside, B J(k1 r) + C H(k1 r) in the shell, i^nu J(k r) + D H(k r)
    outside; 4x4 continuity system at r = a1 and r = a2 (columns scaled for conditioning).
    """
    k2 = k * np.sqrt(complex(n_in))
    k1 = k * np.sqrt(complex(n_out))
    r = np.hypot(x, y)
    th = np.arctan2(y, x)
    nmax = _nu_max(max(abs(k1), abs(k2)) * a2)
    u = np.zeros(np.shape(x), dtype=np.complex128)
    bs = []
    J, H = special.jv, special.hankel1
    dJ, dH = special.jvp, special.h1vp
    inner = r < a1
    for nu in range(-nmax, nmax + 1):
        sA, sB, sC, sD = J(nu, k2 * a1), J(nu, k1 * a2), H(nu, k1 * a1), H(nu, k * a2)
        M = np.array([
            [J(nu, k2 * a1) / sA, -J(nu, k1 * a1) / sB, -H(nu, k1 * a1) / sC, 0],
            [k2 * dJ(nu, k2 * a1) / sA, -k1 * dJ(nu, k1 * a1) / sB, -k1 * dH(nu, k1 * a1) / sC, 0],
            [0, J(nu, k1 * a2) / sB, H(nu, k1 * a2) / sC, -H(nu, k * a2) / sD],
            [0, k1 * dJ(nu, k1 * a2) / sB, k1 * dH(nu, k1 * a2) / sC, -k * dH(nu, k * a2) / sD]],
            dtype=np.complex128)
        rhs = np.array([0, 0, 1j ** nu * J(nu, k * a2), 1j ** nu * k * dJ(nu, k * a2)])
        A, B, C, D = np.linalg.solve(M, rhs) / np.array([sA, sB, sC, sD])
        ph = np.exp(1j * nu * (th - theta_d))
        u = u + np.where(inner, A * J(nu, k2 * r), B * J(nu, k1 * r) + C * H(nu, k1 * r)) * ph
        bs.append(D)
    return u, (np.arange(-nmax, nmax + 1), np.array(bs))


def farfield_from_coefficients(k, nus, bcoef, thetas, theta_d=0.0):
    """Far-field pattern of sum_nu b_nu H_nu(k r) e^{i nu (theta - theta_d)}:
    H_nu(k r) ~ sqrt(2/(pi k r)) e^{i(k r - nu pi/2 - pi/4)}."""
    th = np.atleast_1d(thetas)
    ph = np.exp(1j * np.outer(th - theta_d, nus)) * ((-1j) ** nus)[None, :]
    return np.sqrt(2 / (np.pi * k)) * np.exp(-0.25j * np.pi) * (ph @ bcoef)


def scattered_from_coefficients(k, nus, bcoef, x, y, theta_d=0.0):
    """Exterior scattered field sum_nu b_nu H_nu(k r) e^{i nu (theta - theta_d)} at (x, y)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r = np.hypot(x, y)
    th = np.arctan2(y, x)
    u = np.zeros(np.shape(x), dtype=np.complex128)
    for nu, b in zip(nus, bcoef):
        u = u + b * special.hankel1(nu, k * r) * np.exp(1j * nu * (th - theta_d))
    return u
