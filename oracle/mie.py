"""Lorenz-Mie series for a homogeneous sphere (test infrastructure only).

Used to pin the discrete VIE against the exact physics of the paper's
validation case (a dielectric sphere, Sec. III-A).  Convention of Bohren &
Huffman (e^{-i w t}, incident E0 e^{i k z}): the scattered far field is
E_s = e^{ikr}/(-ikr) [S2 E_par; S1 E_perp], so with F = lim r e^{-ikr} E_s the
amplitude is F = (i/k) (S2 E_par e_par_s + S1 E_perp e_perp).
"""

from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def nmax(x):
    """Series truncation x + 4 x^(1/3) + 2 (Wiscombe's criterion)."""
    return int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0))


def coefficients(x, m):
    """Mie coefficients a_n, b_n (n = 1..nmax) for size parameter x = k a and
    relative refractive index m, from Riccati-Bessel functions
    psi_n(z) = z j_n(z), xi_n(z) = z h_n^(1)(z)."""
    N = nmax(abs(m) * x if abs(m) > 1 else x)
    n = np.arange(1, N + 1)
    mx = m * x

    def psi(z, deriv=False):
        j = spherical_jn(n, z)
        if not deriv:
            return z * j
        return j + z * spherical_jn(n, z, derivative=True)

    def xi(z, deriv=False):
        hn = spherical_jn(n, z) + 1j * spherical_yn(n, z)
        if not deriv:
            return z * hn
        dh = spherical_jn(n, z, derivative=True) + 1j * spherical_yn(n, z, derivative=True)
        return hn + z * dh

    px, dpx = psi(x), psi(x, True)
    pm, dpm = psi(mx), psi(mx, True)
    xx, dxx = xi(x), xi(x, True)
    a = (m * pm * dpx - px * dpm) / (m * pm * dxx - xx * dpm)
    b = (pm * dpx - m * px * dpm) / (pm * dxx - m * xx * dpm)
    return a, b


def amplitudes(x, m, Theta):
    """Scattering amplitudes S1(Theta), S2(Theta) (Theta = scattering angle)."""
    a, b = coefficients(x, m)
    N = len(a)
    mu = np.cos(np.atleast_1d(np.asarray(Theta, float)))
    S1 = np.zeros(mu.shape, complex)
    S2 = np.zeros(mu.shape, complex)
    pi_prev = np.zeros_like(mu)  # pi_0
    pi_n = np.ones_like(mu)  # pi_1
    for n in range(1, N + 1):
        tau_n = n * mu * pi_n - (n + 1) * pi_prev
        f = (2 * n + 1) / (n * (n + 1))
        S1 += f * (a[n - 1] * pi_n + b[n - 1] * tau_n)
        S2 += f * (a[n - 1] * tau_n + b[n - 1] * pi_n)
        pi_next = ((2 * n + 1) * mu * pi_n - (n + 1) * pi_prev) / n
        pi_prev, pi_n = pi_n, pi_next
    return S1, S2


def efficiencies(x, m):
    """Q_ext and Q_sca (Bohren-Huffman eqs. 4.61-4.62)."""
    a, b = coefficients(x, m)
    n = np.arange(1, len(a) + 1)
    qext = 2.0 / x**2 * np.sum((2 * n + 1) * np.real(a + b))
    qsca = 2.0 / x**2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return float(qext), float(qsca)


def farfield_vec(k0, radius, eps, khat, pol, rhat):
    """Cartesian far-field amplitude F(rhat) of a sphere centred at 0 for the
    plane wave pol exp(i k0 khat . r).  Basis: e_perp = -(khat x r)/|.|,
    e_par_i = khat x e_perp, e_par_s = r x e_perp;
    F = (i/k0) [S2 (pol.e_par_i) e_par_s + S1 (pol.e_perp) e_perp].
    Forward/backward directions use any perpendicular basis."""
    m = np.sqrt(complex(eps))
    x = k0 * radius
    khat = np.asarray(khat, float)
    pol = np.asarray(pol, complex)
    rhat = np.atleast_2d(np.asarray(rhat, float))
    ct = np.clip(rhat @ khat, -1.0, 1.0)
    S1, S2 = amplitudes(x, m, np.arccos(ct))
    out = np.zeros((len(rhat), 3), complex)
    for d, r in enumerate(rhat):
        c = np.cross(khat, r)
        nc = np.linalg.norm(c)
        if nc < 1e-12:
            t = np.array([1.0, 0, 0]) if abs(khat[0]) < 0.9 else np.array([0, 1.0, 0])
            c = np.cross(khat, t)
            nc = np.linalg.norm(c)
        e_perp = -c / nc
        e_pi = np.cross(khat, e_perp)
        e_ps = np.cross(r, e_perp)
        out[d] = (1j / k0) * (S2[d] * (pol @ e_pi) * e_ps + S1[d] * (pol @ e_perp) * e_perp)
    return out
