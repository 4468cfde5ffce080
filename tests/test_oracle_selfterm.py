"""Pins of the exact-cube self term (the cell's own singular integral, a
reading of the self-term integral the paper leaves open).

* static limit: the cube integral of 1/r equals the closed form
  h^2 (3 ln((sqrt3 + 1)/(sqrt3 - 1)) - pi/2) (potential at a uniform cube's
  centre);
* the imaginary part equals a direct volume quadrature of the smooth
  integrand sin(k r) / (4 pi r), and the real part minus the static limit a
  direct quadrature of (cos(k r) - 1) / (4 pi r): a route without the face
  parametrisation;
* the small-cell limits: Im s -> k^3 h^3 / (6 pi) (radiation reaction) and
  s_cube - s_sphere = O((k h)^2).
"""

import numpy as np
import pytest
import scipy.integrate

from oracle import selfterm as st
from oracle import vie_dense as vd

K0 = 2 * np.pi


def test_static_limit_closed_form():
    for h in (1.0, 0.05):
        got = st.cube_integral(1e-9, h) * 4 * np.pi / h**2
        want = 3 * np.log((np.sqrt(3) + 1) / (np.sqrt(3) - 1)) - np.pi / 2
        assert abs(got.real - want) < 1e-11 * want


@pytest.mark.parametrize("kh", [0.2, 0.39, 1.0])
def test_parts_by_volume_quadrature(kh):
    h = kh / K0
    c = h / 2
    I = st.cube_integral(K0, h)

    def vol(fun):
        return 8 * scipy.integrate.tplquad(lambda z, y, x: fun(np.sqrt(x * x + y * y + z * z)),
                                           0, c, 0, c, 0, c, epsabs=1e-14 * h**2, epsrel=1e-10)[0]

    im = vol(lambda r: np.sinc(K0 * r / np.pi) * K0 / (4 * np.pi))  # sin(kr)/(4 pi r)
    re_dyn = vol(lambda r: (np.cos(K0 * r) - 1) / (4 * np.pi * r) if r > 0 else 0.0)
    re_static = h**2 * st.CUBE_INV_R / (4 * np.pi)
    assert abs(I.imag - im) < 1e-9 * abs(im)
    assert abs(I.real - re_static - re_dyn) < 1e-9 * abs(re_dyn)


def test_small_cell_limits():
    r = []
    for kh in (0.02, 0.01):
        h = kh / K0
        s = st.self_term_cube(K0, h)
        assert abs(s.imag / (K0**3 * h**3 / (6 * np.pi)) - 1) < kh**2
        r.append(abs(s - vd.self_term(K0, h)) / kh**2)
    assert abs(r[0] / r[1] - 1) < 0.01  # difference scales as (k h)^2
