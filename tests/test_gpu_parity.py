"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: FP64 operator product rel-L2 <= 1e-12; FP32 product <= 5e-6;
FP64 far field <= 1e-10; mixed path far field <= 1e-6; g2 / coincidences
absolute <= 1e-12 (the bar is 1e-6).  Solutions are compared at a solver
tolerance tight enough that kappa * tol stays below the bar.
"""

import numpy as np
import pytest

from oracle import hom, mie
from oracle import vie_dense as vd
from synth import Grid, circular_pol_basis, ellipsoid_union, sphere

pytestmark = pytest.mark.gpu
K0 = 2 * np.pi


@pytest.fixture(scope="module")
def V():
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie

    vie.lib()
    return vie


def _random_body(rng, n, h, fill=0.6):
    eps = 1.0 + rng.uniform(0.5, 5.0, size=(n[2], n[1], n[0]))
    eps[rng.random(eps.shape) > fill] = 1.0
    return eps


def _rand_vec(rng, n):
    return rng.standard_normal((3, n[2], n[1], n[0])) + 1j * rng.standard_normal((3, n[2], n[1], n[0]))


def _relerr(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("n", [(5, 4, 3), (13, 11, 9), (20, 17, 24), (1, 1, 1), (2, 9, 1)])
def test_matvec_fp64_and_fp32_match_dense(V, n):
    rng = np.random.default_rng(sum(n))
    h = 0.045
    g = Grid((n[0], n[1], n[2]), h, tuple(-h * (np.array(n) - 1) / 2 + np.array([0.1, -0.2, 0.05])))
    eps = _random_body(rng, n, h)
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    chi = (eps - 1).ravel()
    x = _rand_vec(rng, n)
    ref = vd.matvec(chi, pos, h, K0, x.reshape(3, -1)).reshape(x.shape)
    ctx = V.vie_setup([(eps, h, g.origin)], V.make_options(K0))
    try:
        y64 = V.vie_matvec(ctx, 0, x, V.VIE_FP64)
        y32 = V.vie_matvec(ctx, 0, x, V.VIE_MIXED)
        ys = V.vie_matvec(ctx, 0, np.stack([x, 2j * x]), V.VIE_FP64)  # batched
    finally:
        V.vie_destroy(ctx)
    print(n, "fp64", _relerr(y64, ref), "fp32", _relerr(y32, ref))
    assert _relerr(y64, ref) < 1e-12
    assert _relerr(y32, ref) < 5e-6
    assert _relerr(ys[0], ref) < 1e-12 and _relerr(ys[1], 2j * ref) < 1e-12


def test_solve_and_farfield_match_lu(V):
    g = Grid.centred((7, 6, 8), 0.06)
    ells = [((0.02, -0.03, 0.0), (0.2, 0.14, 0.22), np.eye(3))]
    eps = ellipsoid_union(g, ells, 4.2)
    eps[0, 0, 0] = 2.0
    chi = (eps - 1).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    k, p = np.array([0.6, 0, 0.8]), np.array([0.8, 0.3j, -0.6]) / np.sqrt(1.09)
    chans = [(k, p), ([0, 0, 1.0], [0, 1.0, 0])]
    th = np.deg2rad(np.arange(0, 181, 10.0))
    ph = np.deg2rad(np.arange(0, 361, 20.0))
    ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0, tol=1e-13, max_iter=2000))
    try:
        rc, st = V.vie_solve(ctx, chans, [2])
        F = V.vie_farfield(ctx, 0, th, ph, 2)
        ws = [V.vie_get_current(ctx, 0, q, g.n) for q in range(2)]
    finally:
        V.vie_destroy(ctx)
    for q, (kk, pp) in enumerate(chans):
        assert st[q]["converged"] == 1 and st[q]["rel_res"] <= 1e-13
        w_lu = vd.solve_lu(chi, pos, g.h, K0, kk, pp)
        assert _relerr(ws[q].reshape(3, -1), w_lu) < 1e-10
        Ft, Fp = vd.farfield(ws[q].reshape(3, -1), pos, g.h, K0, th, ph)
        assert _relerr(F[q], np.stack([Ft, Fp], -1)) < 1e-12  # far-field kernel alone
        Ft, Fp = vd.farfield(w_lu, pos, g.h, K0, th, ph)
        assert _relerr(F[q], np.stack([Ft, Fp], -1)) < 1e-10  # whole path


def _c1_sphere():
    g = Grid.centred(16, 1.0 / 16)
    return g, sphere(g, 0.5, 2.25)


@pytest.fixture(scope="module")
def c1_oracle():
    g, eps = _c1_sphere()
    chi = (eps - 1).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    w = vd.solve_lu(chi, pos, g.h, K0, [0, 0, 1], [1, 0, 0])
    th = np.deg2rad(np.arange(181.0))
    Ft, Fp = vd.farfield(w, pos, g.h, K0, th, 0 * th)
    Ft9, Fp9 = vd.farfield(w, pos, g.h, K0, th, 0 * th + np.pi / 2)
    return g, eps, np.stack([Ft, Fp], -1), np.stack([Ft9, Fp9], -1)


@pytest.mark.parametrize("precision,tol,bar", [(0, 1e-12, 1e-10), (1, 1e-10, 1e-6)])
def test_c1_sphere_farfield(V, c1_oracle, precision, tol, bar):
    """Sphere r = 0.5, eps 2.25, 16^3, x-pol +z: far field on 181 theta points
    (phi = 0 and 90 deg) against the oracle's LU solution; Mie within 3.5 %."""
    g, eps, ref0, ref90 = c1_oracle
    th = np.deg2rad(np.arange(181.0))
    ctx = V.vie_setup([(eps, g.h, g.origin)],
                      V.make_options(K0, precision=precision, tol=tol, max_iter=3000, inner_tol=1e-4))
    try:
        rc, st = V.vie_solve(ctx, [([0, 0, 1.0], [1, 0, 0])], [1])
        F0 = V.vie_farfield(ctx, 0, th, 0 * th, 1)[0]
        F90 = V.vie_farfield(ctx, 0, th, 0 * th + np.pi / 2, 1)[0]
    finally:
        V.vie_destroy(ctx)
    err = _relerr(np.concatenate([F0, F90]), np.concatenate([ref0, ref90]))
    print("precision", precision, "iters", st[0]["iters"], "res", st[0]["rel_res"], "ff err", err)
    assert st[0]["rel_res"] <= tol
    assert err < bar
    r = np.concatenate([vd.direction(th, 0 * th)[0], vd.direction(th, 0 * th + np.pi / 2)[0]])
    M = mie.farfield_vec(K0, 0.5, 2.25, [0, 0, 1], [1, 0, 0], r)
    _, tht, php = vd.direction(np.concatenate([th, th]), np.concatenate([0 * th, 0 * th + np.pi / 2]))
    Mtp = np.stack([np.einsum("dc,dc->d", tht, M), np.einsum("dc,dc->d", php, M)], -1)
    assert _relerr(np.concatenate([F0, F90]), Mtp) < 0.035


def test_batched_bodies_and_linearity(V):
    """Two bodies on different grids, several channels each, in one solve:
    each equals its single solve; H/V responses are the L/R combinations."""
    rng = np.random.default_rng(11)
    gA = Grid.centred((9, 8, 7), 0.05)
    gB = Grid.centred((6, 10, 5), 0.05)
    eA = _random_body(rng, gA.n, gA.h, 0.7)
    eB = _random_body(rng, gB.n, gB.h, 0.7)
    k = np.array([0.0, 0.28, 0.96])
    H, Vv, L, R = circular_pol_basis(k)
    chA = [(k, L), (k, R), (k, H)]
    chB = [([1.0, 0, 0], [0, 0, 1.0]), (k, Vv)]
    th = np.deg2rad([10.0, 40, 80, 130])
    ph = np.deg2rad([0.0, 45, 190, 300])
    ctx = V.vie_setup([(eA, gA.h, gA.origin), (eB, gB.h, gB.origin)], V.make_options(K0, tol=1e-12))
    try:
        rc, st = V.vie_solve(ctx, chA + chB, [3, 2])
        FA = V.vie_farfield(ctx, 0, th, ph, 3)
        FB = V.vie_farfield(ctx, 1, th, ph, 2)
    finally:
        V.vie_destroy(ctx)
    assert all(s["converged"] for s in st)
    for eps, g, chans, Fb in ((eA, gA, chA, FA), (eB, gB, chB, FB)):
        chi = (eps - 1).ravel()
        pos = vd.voxel_centres(g.n, g.h, g.origin)
        for q, (kk, pp) in enumerate(chans):
            w = vd.solve_lu(chi, pos, g.h, K0, kk, pp)
            Ft, Fp = vd.farfield(w, pos, g.h, K0, th, ph)
            assert _relerr(Fb[q], np.stack([Ft, Fp], -1)) < 1e-9
    # linearity: H = (L + R)/sqrt2
    assert _relerr(FA[2], (FA[0] + FA[1]) / np.sqrt(2)) < 1e-9


def test_hom_g2_matches_oracle(V):
    rng = np.random.default_rng(12)
    dt = np.linspace(-5, 5, 200)
    for _ in range(20):
        T = rng.standard_normal(4) + 1j * rng.standard_normal(4)
        om = rng.uniform(0.5, 2, 2)
        g, raw, n1 = V.hom_g2(T, 1.2, dt, V.VIE_NORM_R1, omega=om)
        assert abs(g - hom.g2(T, tuple(om))) < 1e-12
        r_raw, r_n1 = hom.coincidence(T, 1.2, dt, "R1", omega=tuple(om))
        assert np.abs(raw - r_raw).max() < 1e-12 * np.abs(r_raw).max()
        assert np.abs(n1 - r_n1).max() < 1e-12
        _, _, n2 = V.hom_g2(T, 1.2, dt, V.VIE_NORM_R2)
        assert np.abs(n2 - hom.coincidence(T, 1.2, dt, "R2")[1]).max() < 1e-12
        # unequal weights: R2 against the oracle, and its zero-delay value is g2
        g, _, n2w = V.hom_g2(T, 1.2, np.r_[0.0, dt], V.VIE_NORM_R2, omega=om)
        assert np.abs(n2w[1:] - hom.coincidence(T, 1.2, dt, "R2", omega=tuple(om))[1]).max() < 1e-12
        assert abs(n2w[0] - g) < 1e-12
    g, _, n = V.hom_g2([0, 0, 1, 1j], 1.2, dt[:3])
    assert np.isnan(g) and np.all(np.isnan(n))
    g, _, _ = V.hom_g2(hom.beam_splitter_T(0.5, 0.5))
    assert abs(g) < 1e-15
    g, _, _ = V.hom_g2(hom.beam_splitter_T(0.5, 0.5), omega=(2.0, 1.0))
    assert abs(g - hom.g2_fock(hom.beam_splitter_T(0.5, 0.5), (2.0, 1.0))) < 1e-12


def test_hom_classical_p2_matches_oracle(V):
    rng = np.random.default_rng(27)
    for _ in range(20):
        T = rng.standard_normal(4) + 1j * rng.standard_normal(4)
        want = hom.classical_p2(T)
        assert abs(V.hom_classical_p2(T) - want) < 1e-13 * want
    with pytest.raises(V.VieError) as e:
        V.hom_classical_p2([np.nan, 0, 1, 1])
    assert e.value.code == V.VIE_EINVAL


def test_error_paths(V):
    g = Grid.centred(4, 0.1)
    eps = np.full((4, 4, 4), 2.0)
    with pytest.raises(V.VieError) as e:
        V.vie_setup([(eps * 0.4, g.h, g.origin)], V.make_options(K0))
    assert e.value.code == V.VIE_EINVAL
    bad = eps.copy()
    bad[1, 1, 1] = np.nan
    with pytest.raises(V.VieError) as e:
        V.vie_setup([(bad, g.h, g.origin)], V.make_options(K0))
    assert e.value.code == V.VIE_EINVAL
    for shape in [(300, 2, 2), (2, 2, 3100), (2, 3100, 2)]:  # N3 > 256, N1 or N2 > 3072
        with pytest.raises(V.VieError) as e:
            V.vie_setup([(np.ones(shape), g.h, g.origin)], V.make_options(K0))
        assert e.value.code == V.VIE_ENOTSUP
    ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0, tol=1e-12, max_iter=1))
    try:
        rc, st = V.vie_solve(ctx, [([0, 0, 1.0], [1, 0, 0])], [1], allow_noconv=True)
        assert rc == V.VIE_ENOCONV and st[0]["converged"] == 0 and st[0]["iters"] == 1
        V.vie_set_options(ctx, V.make_options(K0, tol=1e-12, max_iter=100))
        rc, st = V.vie_solve(ctx, [([0, 0, 1.0], [0, 0, 0])], [1])  # zero right-hand side
        assert st[0]["iters"] == 0 and st[0]["converged"] == 1
        assert np.all(V.vie_get_current(ctx, 0, 0, g.n) == 0)
        with pytest.raises(V.VieError) as e:
            V.vie_solve(ctx, [([0, 0, 2.0], [1, 0, 0])], [1])
        assert e.value.code == V.VIE_EINVAL
    finally:
        V.vie_destroy(ctx)
    # background-only body: w = 0
    ctx = V.vie_setup([(np.ones((3, 3, 3)), g.h, g.origin)], V.make_options(K0))
    try:
        rc, st = V.vie_solve(ctx, [([0, 0, 1.0], [1, 0, 0])], [1])
        assert st[0]["iters"] == 0
        F = V.vie_farfield(ctx, 0, [0.3], [0.2], 1)
        assert np.all(F == 0)
    finally:
        V.vie_destroy(ctx)


@pytest.mark.parametrize("n,rows", [((64, 64, 64), 48), ((128, 128, 128), 24), ((48, 48, 48), 32),
                                    ((96, 96, 96), 24), ((256, 256, 48), 16), ((256, 256, 256), 12),
                                    ((48, 40, 192), 16)])
def test_matvec_sampled_rows_large(V, n, rows):
    """Full-size grids: sampled rows of the FP64/FP32 product against the
    oracle's O(M)-per-row direct sum (x supported on a metasurface-like body).
    FFT lengths: 128, 256 (2^k); 96, 192 (3 x 2^k); 512 x 512 x 96 (the
    256 x 256 x 48 metasurface grid, mixed); 512^3 (the largest grid, every
    axis at its maximum line length); 96 x 96 x 384 (the longest 3 x 2^k
    z line)."""
    rng = np.random.default_rng(n[0])
    h = 1.0 / 32
    g = Grid.centred(n, h)
    eps = np.ones((n[2], n[1], n[0]))
    z0 = n[2] // 2 - 4
    eps[z0:z0 + 3] = 2.1
    eps[z0 + 3:z0 + 9, ::4, ::3] = 5.0
    chi = (eps - 1).ravel()
    x = _rand_vec(rng, n) * (chi.reshape(eps.shape) != 0)[None]
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    body = np.nonzero(chi)[0]
    sel = np.concatenate([rng.choice(body, rows - 4, replace=False), [0, len(chi) - 1, body[0], body[-1]]])
    ref = vd.matvec_rows(chi, pos, h, K0, x.reshape(3, -1), sel)
    ctx = V.vie_setup([(eps, h, g.origin)], V.make_options(K0))
    try:
        y64 = V.vie_matvec(ctx, 0, x, V.VIE_FP64).reshape(3, -1)[:, sel]
        y32 = V.vie_matvec(ctx, 0, x, V.VIE_MIXED).reshape(3, -1)[:, sel]
    finally:
        V.vie_destroy(ctx)
    print(n, _relerr(y64, ref), _relerr(y32, ref))
    assert _relerr(y64, ref) < 1e-12
    assert _relerr(y32, ref) < 5e-6


@pytest.mark.parametrize("zvar", [0, 1, 2])
@pytest.mark.parametrize("n", [(64, 64, 64), (24, 20, 17), (32, 17, 29), (64, 24, 37)])
def test_every_z_pass_shape_matches_oracle(V, zvar, n):
    """Each fused z-pass shape the autotuner may pick (forced through
    VIE_ZVAR), FP64 and FP32, two vectors per call, against the oracle's
    direct sum on sampled rows.  (32, 17, 29) and (64, 24, 37) have N3 below
    half the z line (64 and 96 points) with the blocked layout holding exactly
    half a line: the shift-addressed launches with zero-filled padding rows.
    Shape 2 (the register-lean kernel) runs on the three layouts with N3
    rounded to 16 equal to half the z line (FP64 96-point lines and the
    (24, 20, 17) grid fall back to shape 0)."""
    import os

    rng = np.random.default_rng(7 * zvar + n[0])
    h = 1.0 / 32
    g = Grid.centred(n, h)
    eps = sphere(g, 0.45 * n[0] * h, 4.0)
    chi = (eps - 1).ravel()
    body = np.nonzero(chi)[0]
    xs = np.stack([_rand_vec(rng, n) * (chi.reshape(eps.shape) != 0)[None] for _ in range(2)])
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    sel = np.concatenate([rng.choice(body, 28, replace=False), [0, len(chi) - 1, body[0], body[-1]]])
    refs = [vd.matvec_rows(chi, pos, h, K0, x.reshape(3, -1), sel) for x in xs]
    old = os.environ.get("VIE_ZVAR")
    os.environ["VIE_ZVAR"] = str(zvar)
    try:
        ctx = V.vie_setup([(eps, h, g.origin)], V.make_options(K0))
        try:
            y64 = V.vie_matvec(ctx, 0, xs, V.VIE_FP64)
            y32 = V.vie_matvec(ctx, 0, xs, V.VIE_MIXED)
        finally:
            V.vie_destroy(ctx)
    finally:
        if old is None:
            del os.environ["VIE_ZVAR"]
        else:
            os.environ["VIE_ZVAR"] = old
    for q in range(2):
        e64 = _relerr(y64[q].reshape(3, -1)[:, sel], refs[q])
        e32 = _relerr(y32[q].reshape(3, -1)[:, sel], refs[q])
        print("zvar", zvar, n, q, e64, e32)
        assert e64 < 1e-12
        assert e32 < 5e-6
