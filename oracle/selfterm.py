"""Exact-cube self term of the discrete operator (test infrastructure only).

The paper leaves the singular self-term integral open (it names a rooftop
basis and does not give the diagonal entries).  The default operator uses
the equal-volume sphere.  This module writes out the alternative in which the
source cell is the voxel itself, a cube of edge h centred on the collocation
point, with w constant over it:

    s_cube = k0^2 PV integral over the cube of G(r) dV
           = -1/3 + (2 k0^2 / 3) integral over the cube of e^{i k0 r} / (4 pi r) dV.

Derivation, as for the sphere: split G = [g I + grad grad (g - g0) / k0^2] +
grad grad g0 / k0^2 with g0 = 1 / (4 pi r).  The principal value of the
static part over a cube centred on the point is -(1/3) I / k0^2 by cubic
symmetry (the cube's depolarisation dyadic is I / 3, like the sphere's).  The
rest is integrable, diagonal by symmetry, and its trace is
3 g + (laplacian of (g - g0)) / k0^2 = 2 g.  The same formula with a sphere of
radius a reproduces -1/3 + 2/3 ((1 - i k0 a) e^{i k0 a} - 1), the real part of
the default self term.

Unlike the default, the imaginary part is not the exact radiation reaction
k0^3 h^3 / (6 pi); it agrees only to leading order in k0 h, so the discrete
model with this term is not exactly lossless.
"""

from __future__ import annotations

import numpy as np
import scipy.integrate

FOUR_PI = 4.0 * np.pi
# integral of 1/r over the unit cube centred on the origin (potential at the
# centre of a uniform cube): 3 ln((sqrt3 + 1)/(sqrt3 - 1)) - pi/2
CUBE_INV_R = 3.0 * np.log((np.sqrt(3.0) + 1.0) / (np.sqrt(3.0) - 1.0)) - np.pi / 2.0


def cube_integral(k0, h):
    """I = integral over the cube [-h/2, h/2]^3 of e^{i k0 r} / (4 pi r) dV.

    In spherical coordinates about the centre the radial integral is
    elementary: int_0^R r e^{ikr} dr = (e^{ikR} (1 - ikR) - 1) / k^2.  The solid
    angle is covered face by face; on the face x = h/2 the direction to the
    point (h/2, y, z) has R = sqrt(h^2/4 + y^2 + z^2) and
    dOmega = (h/2) dy dz / R^3.  The six faces are equal by symmetry."""
    k = k0
    c = h / 2.0

    def radial(R):
        if k * R < 1e-4:  # series: R^2/2 + i k R^3 / 3 - k^2 R^4 / 8
            return R * R / 2.0 + 1j * k * R**3 / 3.0 - k * k * R**4 / 8.0
        return (np.exp(1j * k * R) * (1.0 - 1j * k * R) - 1.0) / (k * k)

    def f(z, y, part):
        R = np.sqrt(c * c + y * y + z * z)
        v = radial(R) * c / R**3
        return v.real if part == 0 else v.imag

    # the integrand is even in y and z: integrate over one quarter of the face
    tol = dict(epsabs=1e-15 * c * c, epsrel=1e-12)
    re = 4.0 * scipy.integrate.dblquad(lambda z, y: f(z, y, 0), 0.0, c, 0.0, c, **tol)[0]
    im = 4.0 * scipy.integrate.dblquad(lambda z, y: f(z, y, 1), 0.0, c, 0.0, c, **tol)[0]
    return 6.0 * complex(re, im) / FOUR_PI


def self_term_cube(k0, h):
    """Diagonal coefficient with the exact cube cell (module docstring)."""
    return -1.0 / 3.0 + (2.0 * k0 * k0 / 3.0) * cube_integral(k0, h)
