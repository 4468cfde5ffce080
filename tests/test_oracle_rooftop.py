"""Pins of the rooftop-basis oracle (Sec. II-C, eq. Js_expand; the reading of
entries and surface treatment is in the module docstring of oracle/rooftop.py).

* Lorenz-Mie: the far field of a homogeneous sphere converges to the Mie
  series under refinement, at size parameter pi (r = lambda / 2) and in the
  quasi-static regime (size parameter 0.3, where the depolarisation carried by
  the grad phi term sets the whole answer);
* Born limit of a box: for chi -> 0 the far field is the box's volume integral
  of e^{i q . r}, a closed form; the faces' weights (1/2 on the surface) and
  positions (h/2 off the cell centre) make the discrete sum the trapezoid rule
  along each current's own axis, so the error is second order in h;
* static limit: the operator tends to the grad phi part, which is negative
  semidefinite (the electrostatic energy of the cell charges is positive);
* structure: the full-layout product is the identity on inactive faces, they do
  not couple to active ones, and a body split into two regions of equal chi
  gives the homogeneous body's operator.
"""

import numpy as np
import pytest

from oracle import mie
from oracle import rooftop as rt
from oracle import vie_dense as vd
from synth import Grid, sphere

K0 = 2 * np.pi


def _mie_error(N, k0, radius, eps):
    g = Grid.centred(N, 2 * radius / N)
    chi = sphere(g, radius, eps) - 1
    w = rt.solve_lu(chi, g.h, g.origin, k0, [0, 0, 1], [1, 0, 0])
    th = np.deg2rad(np.arange(0, 181, 5))
    r = np.concatenate([vd.direction(th, 0 * th)[0], vd.direction(th, 0 * th + np.pi / 2)[0]])
    F = rt.farfield_vec(chi, g.h, g.origin, k0, w, r)
    M = mie.farfield_vec(k0, radius, eps, [0, 0, 1], [1, 0, 0], r)
    return np.linalg.norm(F - M) / np.linalg.norm(M)


def test_sphere_against_mie_converges():
    """r = 0.5 lambda, eps 2.25: 8.3 % at 8^3, 5.1 % at 12^3 (4.2 % at 16^3 in
    the slow tier)."""
    e8 = _mie_error(8, K0, 0.5, 2.25)
    e12 = _mie_error(12, K0, 0.5, 2.25)
    assert e12 < e8
    assert e12 < 0.06


@pytest.mark.slow
def test_sphere_16_against_mie():
    assert _mie_error(16, K0, 0.5, 2.25) < 0.045


def test_quasi_static_sphere_against_mie():
    """Size parameter 0.3, eps 4: the induced dipole is Clausius-Mossotti's
    chi / (1 + chi / 3), half the undepolarised chi; dropping the grad phi term
    misses it by a factor of 2, flipping it by more.  14.4 % at 8^3, 7.7 % at
    12^3 (the pulse basis: 6.3 %, 2.2 %): the surface charge sits half a cell
    off the staircase surface, a first-order error."""
    k0 = 0.6
    e8 = _mie_error(8, k0, 0.5, 4.0)
    e12 = _mie_error(12, k0, 0.5, 4.0)
    assert e12 < e8
    assert e12 < 0.09


def _box_born(n_cells, h, k0, rhat, khat, pol):
    """Far field of a weak box (chi = 1e-9) from the oracle's solve, divided by
    chi, and the closed form k0^2/(4 pi) (I - r r) pol prod_a L_a sinc(q_a L_a / 2)
    e^{i q . centre} with q = k0 (khat - r)."""
    chi0 = 1e-9
    n = tuple(n_cells)
    origin = (0.0, 0.0, 0.0)
    chi = np.full(n[::-1], chi0)
    w = rt.solve_lu(chi, h, origin, k0, khat, pol)
    F = rt.farfield_vec(chi, h, origin, k0, w, rhat) / chi0
    q = k0 * (np.asarray(khat, float)[None, :] - rhat)
    L = h * np.asarray(n, float)
    centre = h * (np.asarray(n, float) - 1) / 2
    box = np.prod(L * np.sinc(q * L / (2 * np.pi)), axis=1) * np.exp(1j * q @ centre)
    P = np.asarray(pol, complex)
    S = box[:, None] * P[None, :]
    S = S - rhat * np.einsum("dc,dc->d", rhat, S)[:, None]
    return F, k0 * k0 / (4 * np.pi) * S


def test_born_box_closed_form_second_order():
    th = np.deg2rad(np.array([0.0, 30.0, 60.0, 120.0, 150.0, 180.0]))
    r = vd.direction(th, 0.3 + 0 * th)[0]
    khat, pol = [0.0, 0.0, 1.0], [1.0, 0.5, 0.0]
    errs = []
    for m in (1, 2):  # the same 0.6 x 0.8 x 1.0 box at two resolutions
        F, want = _box_born((3 * m, 4 * m, 5 * m), 0.2 / m, K0, r, khat, pol)
        errs.append(np.max(np.abs(F - want)) / np.max(np.abs(want)))
    assert errs[0] < 0.05
    assert errs[1] < errs[0] / 3.0  # second order (a surface weight of 1 is first order)


def test_static_limit_charge_energy():
    """At k0 -> 0 the operator is -D^T Gc D (grad phi of the charges): real
    symmetric and negative semidefinite, because the electrostatic energy of any
    cell charge distribution, rho^T Gc rho / 2 with the cell potentials of 1/r
    (self term the cube integral), is positive.  A flipped grad phi term or a
    self term too small for Gc to stay positive definite breaks it; the null
    space is the divergence-free currents."""
    rng = np.random.default_rng(3)
    g = Grid.centred((5, 4, 6), 0.15)
    chi = np.where(rng.random(g.n[::-1]) < 0.6, rng.uniform(0.5, 3.0, g.n[::-1]), 0.0)
    K, idx, _, _, _, _ = rt.system(chi, g.h, g.origin, 1e-7)
    assert len(idx) > 50
    scale = np.max(np.abs(K))
    assert np.max(np.abs(K.imag)) < 1e-12 * scale
    assert np.max(np.abs(K - K.T)) < 1e-12 * scale
    ev = np.linalg.eigvalsh(K.real)
    assert ev.max() < 1e-10 * scale
    assert ev.min() < -1e-2 * scale


def test_structure_inactive_faces_and_equal_split():
    rng = np.random.default_rng(5)
    g = Grid.centred((4, 5, 3), 0.2)
    chi = np.zeros(g.n[::-1])
    chi[1:3, 1:4, 1:3] = 1.5
    act, alpha, chif, _ = rt.face_data(chi, g.h, g.origin)
    x = rng.standard_normal(act.shape) + 1j * rng.standard_normal(act.shape)
    y = rt.matvec(chi, g.h, g.origin, K0, x)
    assert np.array_equal(y[~act], x[~act])
    x0 = np.where(act, x, 0)
    y0 = rt.matvec(chi, g.h, g.origin, K0, x0)
    assert np.allclose(y0[act], y[act], rtol=0, atol=1e-13)
    # surface faces weigh 1/2 and carry chi; faces between body cells weigh 1
    assert set(np.unique(alpha[act])) == {0.5, 1.0}
    assert np.allclose(chif[act], 1.5)
    # two regions of equal chi: the interface rule reduces to chi
    K1, i1, c1, _, _, _ = rt.system(chi, g.h, g.origin, K0)
    chi2 = chi.copy()
    chi2[:, :, 2:] = np.where(chi2[:, :, 2:] != 0, 1.5, 0.0)
    K2, i2, c2, _, _, _ = rt.system(chi2, g.h, g.origin, K0)
    assert np.array_equal(i1, i2) and np.allclose(c1, c2) and np.allclose(K1, K2)


def test_matvec_rows_equals_dense():
    rng = np.random.default_rng(9)
    g = Grid.centred((5, 6, 4), 0.12)
    chi = np.where(rng.random(g.n[::-1]) < 0.5, rng.uniform(0.3, 4.0, g.n[::-1]), 0.0)
    act, _, _, _ = rt.face_data(chi, g.h, g.origin)
    x = rng.standard_normal(act.shape) + 1j * rng.standard_normal(act.shape)
    y = rt.matvec(chi, g.h, g.origin, 1.3 * K0, x).ravel()
    rows = rng.choice(np.nonzero(act.ravel())[0], 25, replace=False)
    got = rt.matvec_rows(chi, g.h, g.origin, 1.3 * K0, x, rows)
    assert np.max(np.abs(got - y[rows])) < 1e-12 * np.max(np.abs(y))
