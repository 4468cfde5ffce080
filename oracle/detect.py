"""Finite-aperture detection (test infrastructure only).

The paper defines an aperture-collected field operator (eq. NAfield): the
field weighted by the detector's angular sensitivity W(k) and integrated
over its numerical aperture; the two-photon observables then follow from it
as from a point detector.  Under the narrowband reduction of Sec. II the
collected field of channel j is again a transfer coefficient.  With a
uniform sensitivity over a cone of half-angle alpha about the axis u and a
fixed detection polarisation p it reads

    T_NA = (1 / Omega) * integral over the cone of p . F(r) dOmega(r),
    Omega = 2 pi (1 - cos alpha),

F the Cartesian far field of eq. 25.  alpha = 0 is the point detector on u.

Quadrature: Gauss-Legendre in the cosine of the angle from u on
[cos alpha, 1] times the midpoint rule in azimuth.  The closed form for a
single radiating dipole (`dipole_cone_mean`) pins it.
"""

from __future__ import annotations

import numpy as np

from .vie_dense import direction, farfield_vec


def cone_nodes(theta0, phi0, alpha, n_rad, n_az):
    """Quadrature nodes (D, 3) and weights (D,) for the mean over the cone of
    half-angle ``alpha`` about the direction (theta0, phi0); the weights sum to
    one.  alpha = 0 gives the single node on the axis."""
    u, e1, e2 = (v.reshape(3) for v in direction(theta0, phi0))
    if alpha == 0.0:
        return u[None, :], np.ones(1)
    c0 = np.cos(alpha)
    omega = 2.0 * np.pi * (1.0 - c0)
    x, w = np.polynomial.legendre.leggauss(n_rad)
    mu = 0.5 * (1.0 - c0) * x + 0.5 * (1.0 + c0)  # cosine of the angle from the axis
    wmu = 0.5 * (1.0 - c0) * w
    beta = 2.0 * np.pi * (np.arange(n_az) + 0.5) / n_az
    s = np.sqrt(1.0 - mu * mu)
    dirs = (mu[:, None, None] * u
            + s[:, None, None] * (np.cos(beta)[None, :, None] * e1 + np.sin(beta)[None, :, None] * e2))
    wts = np.broadcast_to(wmu[:, None] * (2.0 * np.pi / n_az) / omega, (n_rad, n_az))
    return dirs.reshape(-1, 3), wts.ravel()


def transfer_na(w, pos, h, k0, theta0, phi0, alpha, pol, n_rad=8, n_az=16):
    """T_NA of the current ``w`` (3, M) for one detector (definition above)."""
    d, wt = cone_nodes(theta0, phi0, alpha, n_rad, n_az)
    F = farfield_vec(w, pos, h, k0, d)
    return complex(np.sum(wt * (F @ np.asarray(pol, complex))))


def dipole_cone_mean(theta0, phi0, alpha):
    """(1 / Omega) * integral over the cone of r r^T dOmega, in closed form.
    About the axis u the mean of cos^2 is b = (1 + c + c^2) / 3 (c = cos alpha)
    and each transverse direction gets a = (1 - b) / 2, so the mean is
    a I + (b - a) u u^T; alpha = 0 gives u u^T."""
    u = direction(theta0, phi0)[0].reshape(3)
    c = np.cos(alpha)
    b = (1.0 + c + c * c) / 3.0
    a = 0.5 * (1.0 - b)
    return a * np.eye(3) + (b - a) * np.outer(u, u)
