"""Pins of the Mie and two-photon oracles against closed forms and brute force."""

import json
import os

import numpy as np

from oracle import hom, mie
from oracle import vie_dense as vd
from synth import Grid, pb_rotation_step, sphere

K0 = 2 * np.pi
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Mie ------
def test_mie_energy_balance_lossless():
    """Real refractive index: Q_ext = Q_sca."""
    for x, m in [(0.3, 1.5), (3.0, 1.33), (6.28, 2.0)]:
        qe, qs = mie.efficiencies(x, m)
        assert abs(qe - qs) / qe < 1e-10


def test_mie_forward_optical_theorem():
    """Q_ext = 4/x^2 Re S(0), with S1(0) = S2(0)."""
    x, m = 4.0, 1.5
    S1, S2 = mie.amplitudes(x, m, np.array([0.0]))
    assert abs(S1[0] - S2[0]) < 1e-12 * abs(S1[0])
    qe, _ = mie.efficiencies(x, m)
    assert abs(qe - 4 / x**2 * S1[0].real) < 1e-10 * qe


def test_mie_rayleigh_limit():
    """x -> 0: far field of a dipole of polarisability a^3 (eps-1)/(eps+2)."""
    a, eps = 1e-3, 3.0
    pol = np.array([1.0, 0, 0], complex)
    r, _, _ = vd.direction(np.array([0.4, 1.3, 2.8]), np.array([0.2, 1.0, 3.0]))
    F = mie.farfield_vec(K0, a, eps, [0, 0, 1], pol, r)
    ref = K0**2 * a**3 * (eps - 1) / (eps + 2) * (pol[None] - r * (r @ pol)[:, None])
    assert np.abs(F - ref).max() / np.abs(ref).max() < 1e-4


def test_mie_rayleigh_gans_limit():
    """m -> 1 (first Born approximation of a sphere, any size):
    F = k^2 V (m^2 - 1)/(4 pi) 3 (sin u - u cos u)/u^3 (I - rr) e, u = |q| a."""
    a, eps = 0.4, 1.0 + 2e-4
    ki = np.array([0, 0, 1.0])
    pol = np.array([0, 1.0, 0], complex)
    r, _, _ = vd.direction(np.deg2rad([10, 50, 90, 140]), np.deg2rad([0, 30, 120, 250]))
    F = mie.farfield_vec(K0, a, eps, ki, pol, r)
    u = np.linalg.norm(K0 * (ki[None] - r), axis=1) * a
    form = 3 * (np.sin(u) - u * np.cos(u)) / u**3
    V = 4 / 3 * np.pi * a**3
    ref = (K0**2 * V * (eps - 1) / (4 * np.pi) * form)[:, None] * (pol[None] - r * (r @ pol)[:, None])
    assert np.abs(F - ref).max() / np.abs(ref).max() < 5e-4


def test_mie_oblique_incidence_is_rotation_of_axial():
    """Rotating incidence, polarisation and observation together leaves F
    rotated (isotropy of the sphere), exercising the general basis."""
    a, eps = 0.4, 2.25
    th = 0.7
    Rm = np.array([[np.cos(th), 0, np.sin(th)], [0, 1, 0], [-np.sin(th), 0, np.cos(th)]])
    ki = np.array([0, 0, 1.0])
    pol = np.array([1.0, 0.5j, 0])
    pol /= np.linalg.norm(pol)
    r, _, _ = vd.direction(np.array([0.3, 1.0, 2.0, np.pi]), np.array([0.0, 1.0, 2.0, 0.0]))
    F0 = mie.farfield_vec(K0, a, eps, ki, pol, r)
    F1 = mie.farfield_vec(K0, a, eps, Rm @ ki, Rm @ pol, r @ Rm.T)
    assert np.abs(F1 - F0 @ Rm.T).max() < 1e-12 * np.abs(F0).max()


# ---------------------------------------------------------------- HOM ------
def _rand_T(rng):
    return rng.standard_normal(4) + 1j * rng.standard_normal(4)


def test_g2_matches_fock_space_expectation_sum():
    """The compact g2 (eq. 10) equals the normally ordered sum (eq. 11)
    evaluated by brute force with |1_1,1_2> in a truncated Fock space."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        T = _rand_T(rng)
        om = tuple(rng.uniform(0.5, 2.0, 2))
        assert abs(hom.g2(T, om) - hom.g2_fock(T, om)) < 1e-12


def test_g2_beam_splitter_closed_form():
    """Beam splitter (eqs. 15-16): g2 = (T - R)^2, zero when balanced."""
    for Tbs in (0.5, 0.3, 0.9):
        T = hom.beam_splitter_T(Tbs, 1 - Tbs)
        assert abs(hom.g2(T) - (Tbs - (1 - Tbs)) ** 2) < 1e-14
    assert hom.g2(hom.beam_splitter_T(0.5, 0.5)) < 1e-30


def test_g2_bounds_invariances_and_dark_detector():
    rng = np.random.default_rng(4)
    for _ in range(50):
        T = _rand_T(rng)
        g = hom.g2(T)
        assert -1e-15 <= g <= 1 + 1e-12
        da, db = _rand_T(rng)[:2]
        p1, p2 = np.exp(1j * rng.uniform(0, 6.3, 2))
        T2 = (da * T[0] * p1, da * T[1] * p2, db * T[2] * p1, db * T[3] * p2)
        assert abs(hom.g2(T2) - g) < 1e-12
        assert abs(hom.g2((T[1], T[0], T[3], T[2])) - g) < 1e-12  # swap channels
        assert abs(hom.g2((T[2], T[3], T[0], T[1])) - g) < 1e-12  # swap detectors
    assert np.isnan(hom.g2((0, 0, 1, 1j)))
    assert hom.g2((1.0, 0.0, 1.0, 0.0)) == 0.0  # single path: trivially zero


def test_coincidence_closed_form_matches_tau_quadrature():
    rng = np.random.default_rng(5)
    dt = np.linspace(-5, 5, 21)
    for _ in range(5):
        T = _rand_T(rng)
        raw, _ = hom.coincidence(T, 1.2, dt)
        quad = hom.coincidence_quadrature(T, 1.2, dt)
        assert np.abs(raw - quad).max() < 1e-10 * np.abs(raw).max()


def test_coincidence_reduces_to_beam_splitter_hom_dip():
    """eq. G2_scatter with A_dir = T, A_ex = -R reproduces eq. 17; balanced:
    R1 gives 1 - exp(-dtau^2/sigma^2), R2 gives (1 - c)/2 ... here R^2+T^2-2RTc."""
    dt = np.linspace(-4, 4, 17)
    for Tbs in (0.5, 0.7):
        Rbs = 1 - Tbs
        T = hom.beam_splitter_T(Tbs, Rbs)
        raw, r1 = hom.coincidence(T, 1.2, dt, "R1")
        _, r2 = hom.coincidence(T, 1.2, dt, "R2")
        bs = hom.beam_splitter_nc_quadrature(Tbs, Rbs, 1.2, dt)
        assert np.abs(raw - bs).max() < 1e-10 * np.abs(bs).max()
        c = np.exp(-(dt**2) / 1.2**2)
        assert np.allclose(r1, 1 - 2 * Rbs * Tbs * c / (Rbs**2 + Tbs**2), atol=1e-13)
        assert np.allclose(r2, Rbs**2 + Tbs**2 - 2 * Rbs * Tbs * c, atol=1e-13)


def test_coincidence_normalisation_identities():
    rng = np.random.default_rng(6)
    for _ in range(10):
        T = _rand_T(rng)
        _, r2 = hom.coincidence(T, 1.2, [0.0], "R2")
        assert abs(r2[0] - hom.g2(T)) < 1e-12
        _, r1 = hom.coincidence(T, 1.2, [60.0], "R1")
        assert abs(r1[0] - 1.0) < 1e-12
    _, r2 = hom.coincidence((1.0, 0.0, 1.0, 0.0), 1.2, np.linspace(-5, 5, 7), "R2")
    assert np.all(r2 == 0.0)  # single path stays suppressed at every delay


def test_coincidence_channel_weights():
    """Unequal channel weights (the sqrt(omega) factors of eqs. 8-9): the
    R2-normalised dip at zero delay equals the Fock-space g2 computed
    independently with the same weights, R1 does not depend on them, and the
    raw count equals the tau quadrature of the weighted path amplitudes."""
    rng = np.random.default_rng(16)
    dt = np.linspace(-5, 5, 11)
    for _ in range(6):
        T = _rand_T(rng)
        om = tuple(rng.uniform(0.3, 3.0, 2))
        _, r2 = hom.coincidence(T, 1.2, [0.0], "R2", omega=om)
        assert abs(r2[0] - hom.g2_fock(T, om)) < 1e-12
        _, r1w = hom.coincidence(T, 1.2, dt, "R1", omega=om)
        _, r1 = hom.coincidence(T, 1.2, dt, "R1")
        assert np.abs(r1w - r1).max() < 1e-12
        raw, _ = hom.coincidence(T, 1.2, dt, omega=om)
        quad = hom.coincidence_quadrature(T, 1.2, dt, omega=om)
        assert np.abs(raw - quad).max() < 1e-10 * np.abs(raw).max()
        raw1, _ = hom.coincidence(T, 1.2, dt)
        assert np.abs(raw - om[0] * om[1] * raw1).max() < 1e-12 * np.abs(raw).max()


# ------------------------------------------------------- VIE + HOM chain ---
def test_rayleigh_sphere_g2zz_is_sin2_sum_of_azimuths():
    """Small sphere, channels k1 = k x (y-pol), k2 = k y (x-pol), z-detection at
    theta1 = 45, theta2 = 135 deg: in the dipole limit g2_zz = sin^2(phi1+phi2),
    diagonal HOM stripes (Sec. III-A)."""
    g = Grid.centred(5, 0.002)
    chi = (sphere(g, 0.005, 2.1) - 1).ravel()  # k0 a = 0.03: error O((k0 a)^2)
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    w1 = vd.solve_lu(chi, pos, g.h, K0, [1, 0, 0], [0, 1, 0])
    w2 = vd.solve_lu(chi, pos, g.h, K0, [0, 1, 0], [1, 0, 0])
    rng = np.random.default_rng(7)
    for _ in range(10):
        p1, p2 = rng.uniform(0, 2 * np.pi, 2)
        t1, t2 = np.deg2rad(45), np.deg2rad(135)
        Ft1, _ = vd.farfield(w1, pos, g.h, K0, np.array([t1, t2]), np.array([p1, p2]))
        Ft2, _ = vd.farfield(w2, pos, g.h, K0, np.array([t1, t2]), np.array([p1, p2]))
        cz = -np.sin(np.array([t1, t2]))  # z-component of theta-hat
        Ta1, Tb1 = cz * Ft1
        Ta2, Tb2 = cz * Ft2
        assert abs(hom.g2((Ta1, Ta2, Tb1, Tb2)) - np.sin(p1 + p2) ** 2) < 2e-4


# --------------------------------------------------------------- golden ----
def test_paper_printed_numbers():
    """Numbers printed in the paper (Sec. III-B): PB rotation increment of
    eq. 32 and the unknown count of the metasurface run."""
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        gold = json.load(f)
    pb = gold["pb_rotation_step"]
    lam = pb["wavelength_nm"]
    step = pb_rotation_step(2 * np.pi / lam, np.deg2rad(pb["theta_t_deg"]), pb["period_nm"])
    assert abs(np.rad2deg(step) - pb["step_deg"]) < pb["tolerance_deg"]
    u = gold["metasurface_run"]
    assert 3 * u["mesh_elements"] == u["current_unknowns"]
    fr = gold["fraunhofer"]
    assert abs(2 * fr["aperture_wavelengths"] ** 2 - fr["distance_wavelengths"]) < 1e-9
    assert abs(fr["distance_wavelengths"] * fr["wavelength_nm"] * 1e-6 - fr["distance_mm"]) < 0.01


def test_classical_p2_is_intensity_product_of_superposed_response():
    """eq. 27: P2 from the transfer coefficients equals the intensity product of
    the far field of the superposed current w1 + w2 (linearity of eq. 25),
    with z-detection c = (-sin theta, 0); beam splitter: |t + r|^4."""
    rng = np.random.default_rng(27)
    n = (4, 3, 5)
    h = 0.1
    pos = vd.voxel_centres(n, h, -h * (np.array(n) - 1) / 2)
    w1, w2 = (rng.standard_normal((3, pos.shape[0])) + 1j * rng.standard_normal((3, pos.shape[0]))
              for _ in range(2))
    th = np.array([0.6, 2.2])
    ph = np.array([0.3, -1.9])
    T = []
    for w in (w1, w2):
        Ft, _ = vd.farfield(w, pos, h, 2 * np.pi, th, ph)
        T.append(-np.sin(th) * Ft)
    Tv = (T[0][0], T[1][0], T[0][1], T[1][1])
    Fs, _ = vd.farfield(w1 + w2, pos, h, 2 * np.pi, th, ph)
    Es = -np.sin(th) * Fs
    want = abs(Es[0]) ** 2 * abs(Es[1]) ** 2
    assert abs(hom.classical_p2(Tv) - want) < 1e-12 * want
    t, r = 1 / np.sqrt(2), 1j / np.sqrt(2)
    assert abs(hom.classical_p2((t, r, r, t)) - abs(t + r) ** 4) < 1e-15
