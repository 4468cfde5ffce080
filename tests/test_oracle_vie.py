"""Pins of the dense VIE oracle against facts fixed outside it.

Each test checks the oracle against something it does not contain: finite
differences of the scalar Green's function, the static Clausius-Mossotti /
Rayleigh limit, the optical theorem of a lossless body, reciprocity,
translation covariance, the first-order Born closed form of a uniform box,
Mie series, and an independent solver.  A plausible mistake (dropped term,
wrong sign or index, transposed operand) fails at least one of them.
"""

import numpy as np
import pytest

from oracle import mie
from oracle import vie_dense as vd
from synth import Grid, ellipsoid_union, sphere

K0 = 2 * np.pi


def _scalar_g(R, k):
    r = np.linalg.norm(R)
    return np.exp(1j * k * r) / (4 * np.pi * r)


def test_green_dyadic_equals_definition_by_finite_differences():
    """eq. dyadicG: G = (I + grad grad / k^2) g, second derivatives of g by
    4th-order central differences."""
    rng = np.random.default_rng(0)
    for _ in range(5):
        R = rng.uniform(-0.6, 0.6, 3) + np.array([0.3, 0.0, 0.0])
        d = 1e-3
        H = np.zeros((3, 3), complex)
        for a in range(3):
            for b in range(3):
                ea, eb = np.eye(3)[a] * d, np.eye(3)[b] * d

                def f(i, j):
                    return _scalar_g(R + i * ea + j * eb, K0)

                if a == b:
                    H[a, b] = (-f(2, 0) + 16 * f(1, 0) - 30 * f(0, 0) + 16 * f(-1, 0) - f(-2, 0)) / (12 * d * d)
                else:
                    H[a, b] = (f(1, 1) - f(1, -1) - f(-1, 1) + f(-1, -1)) / (4 * d * d)
        ref = np.eye(3) * _scalar_g(R, K0) + H / K0**2
        got = vd.green_dyadic(R, K0)
        assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-5  # O(d^2) stencil error


def test_self_term_imaginary_part_is_radiation_reaction():
    """Im s must equal k0^2 h^3 Im G(R -> 0) = k0^3 h^3 / (6 pi) (the regular
    limit of the Green's function), which is what makes the model lossless."""
    h = 0.05
    tiny = np.array([1e-4, 2e-4, -1.5e-4])
    ImG0 = np.imag(vd.green_dyadic(tiny, K0))
    assert np.allclose(ImG0, np.eye(3) * K0 / (6 * np.pi), rtol=0, atol=1e-5)  # O((k0 R)^2)
    s = vd.self_term(K0, h)
    assert abs(s.imag - K0**3 * h**3 / (6 * np.pi)) < 1e-15


def test_single_voxel_static_limit_is_clausius_mossotti_and_rayleigh():
    """One voxel, k0 h -> 0: w -> 3 (eps-1)/(eps+2) e (field inside a sphere)
    and the far field -> k0^2 a^3 (eps-1)/(eps+2) (I - rr) e for the
    equal-volume sphere (Rayleigh dipole)."""
    eps = 3.7
    h = 1e-3
    g = Grid.centred(1, h)
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    chi = np.array([eps - 1.0])
    pol = np.array([0.3, -0.5j, 0.0])
    pol = pol / np.linalg.norm(pol)
    w = vd.solve_lu(chi, pos, h, K0, [0, 0, 1], pol)
    cm = 3 * (eps - 1) / (eps + 2)
    assert np.allclose(w[:, 0], cm * pol, rtol=1e-4)
    a = h * (3 / (4 * np.pi)) ** (1 / 3)
    th = np.array([0.3, 1.2, 2.5])
    ph = np.array([0.1, 2.0, 4.0])
    r, _, _ = vd.direction(th, ph)
    F = vd.farfield_vec(w, pos, h, K0, r)
    ref = K0**2 * a**3 * (eps - 1) / (eps + 2) * (pol[None, :] - r * (r @ pol)[:, None])
    assert np.abs(F - ref).max() / np.abs(ref).max() < 1e-4


def _small_body():
    g = Grid.centred((5, 4, 6), 0.07)
    ells = [((0.02, -0.03, 0.0), (0.17, 0.12, 0.2), np.eye(3)),
            ((0.1, 0.05, 0.1), (0.1, 0.1, 0.08), np.eye(3))]
    body = ellipsoid_union(g, ells, 4.2)
    body[0, 0, 0] = 2.0  # an extra isolated voxel of another permittivity
    return g, (body - 1).ravel()


def test_operator_is_complex_symmetric():
    """Reciprocity at matrix level: Ghat_mn = Ghat_nm^T (no conjugate)."""
    g, chi = _small_body()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    G = vd.green_matrix(pos[:20], g.h, K0)
    assert np.abs(G - G.T).max() < 1e-14 * np.abs(G).max()


def test_optical_theorem_lossless():
    """Extinction (optical theorem) equals the integrated scattered power for a
    lossless body, exactly for this discrete model."""
    g, chi = _small_body()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    for khat, pol in [([0, 0, 1], [1, 0, 0]), ([0.6, 0, 0.8], [0.8j, 0.3, -0.6j])]:
        k = np.asarray(khat, float)
        p = np.asarray(pol, complex)
        p = p - k * (k @ p)
        p /= np.linalg.norm(p)
        w = vd.solve_lu(chi, pos, g.h, K0, k, p)
        se = vd.extinction_cross_section(w, pos, g.h, K0, k, p)
        ss = vd.scattering_cross_section(w, pos, g.h, K0)
        assert se > 0
        assert abs(se - ss) / se < 1e-10


def test_reciprocity_of_far_field():
    """e_s . F(r_s; k_i, e_i) = e_i . F(-k_i; -r_s, e_s)."""
    g, chi = _small_body()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    ki = np.array([0.0, 0.6, 0.8])
    ei = np.array([1.0, 0, 0], complex)
    rs = np.array([0.48, -0.6, 0.64])
    es = np.cross(rs, [0, 0, 1.0])
    es = (es / np.linalg.norm(es)).astype(complex) * (1 + 0.5j)
    w1 = vd.solve_lu(chi, pos, g.h, K0, ki, ei)
    lhs = es @ vd.farfield_vec(w1, pos, g.h, K0, rs[None])[0]
    w2 = vd.solve_lu(chi, pos, g.h, K0, -rs, es)
    rhs_ = ei @ vd.farfield_vec(w2, pos, g.h, K0, -ki[None])[0]
    assert abs(lhs - rhs_) / abs(lhs) < 1e-11


def test_translation_covariance():
    """Moving the body by d multiplies F by exp(i k0 (k_i - r) . d)."""
    g, chi = _small_body()
    d = np.array([0.21, -0.14, 0.07])
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    ki = np.array([0.0, 0.0, 1.0])
    ei = np.array([1.0, 1j, 0]) / np.sqrt(2)
    r, _, _ = vd.direction(np.array([0.4, 1.9]), np.array([0.3, 5.0]))
    F0 = vd.farfield_vec(vd.solve_lu(chi, pos, g.h, K0, ki, ei), pos, g.h, K0, r)
    F1 = vd.farfield_vec(vd.solve_lu(chi, pos + d, g.h, K0, ki, ei), pos + d, g.h, K0, r)
    ph = np.exp(1j * K0 * ((ki[None] - r) @ d))
    assert np.abs(F1 - F0 * ph[:, None]).max() / np.abs(F0).max() < 1e-11


def test_born_limit_of_uniform_box():
    """chi -> 0 on a full N^3 box: F = k0^2 h^3 chi/(4 pi) (I - rr) e
    prod_a D_N(q_a h) + O(chi^2), D_N(u) = sin(N u/2)/sin(u/2), q = k0 (k - r)."""
    N, h, chi0 = 6, 0.09, 1e-6
    g = Grid.centred(N, h)
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    chi = np.full(N**3, chi0)
    ki = np.array([0, 0, 1.0])
    ei = np.array([1.0, 0, 0], complex)
    w = vd.solve_lu(chi, pos, h, K0, ki, ei)
    r, _, _ = vd.direction(np.array([0.2, 1.0, 2.0, 3.0]), np.array([0.0, 0.7, 2.0, 4.0]))
    F = vd.farfield_vec(w, pos, h, K0, r)
    q = K0 * (ki[None] - r)
    u = q * h
    D = np.prod(np.where(np.abs(u) < 1e-12, N, np.sin(N * u / 2) / np.where(np.abs(u) < 1e-12, 1, np.sin(u / 2))), axis=1)
    ref = (K0**2 * h**3 * chi0 / (4 * np.pi)) * D[:, None] * (ei[None] - r * (r @ ei)[:, None])
    assert np.abs(F - ref).max() <= 10 * chi0 * np.abs(ref).max()


def test_matvec_rows_matches_dense_matrix():
    """The O(M) row-sampled product equals the explicit dense operator."""
    g, chi = _small_body()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, len(chi))) + 1j * rng.standard_normal((3, len(chi)))
    G = vd.green_matrix(pos, g.h, K0)
    y_ref = x.reshape(-1) - np.tile(chi, 3) * (G @ x.reshape(-1))
    y = vd.matvec(chi, pos, g.h, K0, x)
    assert np.abs(y.reshape(-1) - y_ref).max() / np.abs(y_ref).max() < 1e-13
    rows = np.array([0, 7, 33, len(chi) - 1])
    yr = vd.matvec_rows(chi, pos, g.h, K0, x, rows)
    assert np.abs(yr - y_ref.reshape(3, -1)[:, rows]).max() < 1e-12 * np.abs(y_ref).max()


def test_bicgstab_matches_lu():
    g, chi = _small_body()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    ki, ei = np.array([0.0, 0, 1]), np.array([0, 1.0, 0], complex)
    w_lu = vd.solve_lu(chi, pos, g.h, K0, ki, ei)
    b = vd.rhs(chi, pos, K0, ki, ei)
    w, it, hist = vd.bicgstab(lambda v: vd.matvec(chi, pos, g.h, K0, v), b, tol=1e-13)
    assert hist[-1] <= 1e-13 and it > 3
    assert np.linalg.norm(w - w_lu) / np.linalg.norm(w_lu) < 1e-11


def test_sphere_against_mie_converges():
    """Sphere r = 0.5 lambda, eps 2.25, x-polarised +z incidence, far field in
    the phi = 0 and phi = 90 deg planes: relative L2 error against the Mie
    series decreases with refinement and is below 5 % at 12 cells per
    diameter (16^3: 2.8 %, checked in the slow tier)."""
    errs = []
    for N in (8, 12):
        g = Grid.centred(N, 1.0 / N)
        chi = (sphere(g, 0.5, 2.25) - 1).ravel()
        pos = vd.voxel_centres(g.n, g.h, g.origin)
        w = vd.solve_lu(chi, pos, g.h, K0, [0, 0, 1], [1, 0, 0])
        th = np.deg2rad(np.arange(0, 181, 5))
        r = np.concatenate([vd.direction(th, 0 * th)[0], vd.direction(th, 0 * th + np.pi / 2)[0]])
        F = vd.farfield_vec(w, pos, g.h, K0, r)
        M = mie.farfield_vec(K0, 0.5, 2.25, [0, 0, 1], [1, 0, 0], r)
        errs.append(np.linalg.norm(F - M) / np.linalg.norm(M))
    assert errs[1] < errs[0]
    assert errs[1] < 0.05


@pytest.mark.slow
def test_sphere_16_against_mie():
    g = Grid.centred(16, 1.0 / 16)
    chi = (sphere(g, 0.5, 2.25) - 1).ravel()
    assert int((chi != 0).sum()) == 2176
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    w = vd.solve_lu(chi, pos, g.h, K0, [0, 0, 1], [1, 0, 0])
    th = np.deg2rad(np.arange(181))
    r = np.concatenate([vd.direction(th, 0 * th)[0], vd.direction(th, 0 * th + np.pi / 2)[0]])
    F = vd.farfield_vec(w, pos, g.h, K0, r)
    M = mie.farfield_vec(K0, 0.5, 2.25, [0, 0, 1], [1, 0, 0], r)
    assert np.linalg.norm(F - M) / np.linalg.norm(M) < 0.035
