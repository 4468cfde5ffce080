"""Pins of the finite-aperture detector oracle (eq. NAfield, uniform cone
sensitivity, narrowband reduction).

* A single radiating voxel: F(r) = C (I - r r) w, so the cone mean of p . F is
  C p^T (I - M) w with M the cone mean of r r^T, known in closed form; the
  quadrature must reproduce it to rounding for every axis and half-angle.
* alpha = 0 is the point detector of eq. Eproj, with c_theta = p . theta-hat
  and c_phi = p . phi-hat on the axis; small apertures approach it as alpha^2.
* The quadrature weights sum to one and every node lies inside the cone.
"""

import numpy as np
import pytest

from oracle import detect as dt
from oracle import vie_dense as vd

K0 = 2 * np.pi


def _rand_c(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("alpha", [0.05, 0.4, 1.2, np.pi / 2, 2.5])
def test_single_dipole_closed_form(alpha):
    rng = np.random.default_rng(int(alpha * 100))
    h = 0.05
    pos = np.zeros((1, 3))
    w = _rand_c(rng, 3)[:, None]
    C = K0 * K0 * h**3 / (4 * np.pi)
    for _ in range(3):
        t0, p0 = rng.uniform(0, np.pi), rng.uniform(-np.pi, np.pi)
        pol = _rand_c(rng, 3)
        got = dt.transfer_na(w, pos, h, K0, t0, p0, alpha, pol, n_rad=3, n_az=4)
        M = dt.dipole_cone_mean(t0, p0, alpha)
        want = C * pol @ (np.eye(3) - M) @ w[:, 0]
        assert abs(got - want) < 1e-13 * abs(want)


def test_point_detector_limit():
    rng = np.random.default_rng(9)
    n = (5, 4, 3)
    h = 0.11
    pos = vd.voxel_centres(n, h, -h * (np.array(n) - 1) / 2)
    w = _rand_c(rng, 3 * pos.shape[0]).reshape(3, -1)
    t0, p0 = 0.7, -2.1
    pol = _rand_c(rng, 3)
    _, th, ph = vd.direction(t0, p0)
    Ft, Fp = vd.farfield(w, pos, h, K0, np.array([t0]), np.array([p0]))
    point = (pol @ th.reshape(3)) * Ft[0] + (pol @ ph.reshape(3)) * Fp[0]
    assert abs(dt.transfer_na(w, pos, h, K0, t0, p0, 0.0, pol) - point) < 1e-13 * abs(point)
    e1 = abs(dt.transfer_na(w, pos, h, K0, t0, p0, 1e-2, pol, 4, 8) - point)
    e2 = abs(dt.transfer_na(w, pos, h, K0, t0, p0, 2e-2, pol, 4, 8) - point)
    assert 3.5 < e2 / e1 < 4.5  # second order in alpha


def test_nodes_and_weights():
    for alpha in (0.1, 1.0, np.pi):
        d, wt = dt.cone_nodes(0.3, 1.1, alpha, 5, 7)
        u = vd.direction(0.3, 1.1)[0].reshape(3)
        assert abs(wt.sum() - 1.0) < 1e-14
        assert np.all(d @ u >= np.cos(alpha) - 1e-14)
        assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
