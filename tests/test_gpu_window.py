"""GPU parity of the z window (VIE_FLAG_Z_WINDOW): a grid group computed on
the z layers that hold its bodies instead of the whole grid.  Voxels outside the window have chi = 0, so the system of the body's
unknowns is unchanged; the checks are against the oracle on the full grid.

* vie_grid reports the window, its FFT lengths and each body's offset;
* the product on body-supported box vectors equals the oracle on every row
  (FP64 rel. 1e-12, FP32 5e-6); components outside the window pass through;
* BiCGSTAB and block-Jacobi FGMRES solves, currents and far fields equal the
  dense LU solution (rel. 1e-10), for two bodies at different heights sharing
  one window, and equal the solves of a context without the window;
* the block-Jacobi preconditioner applied alone (vie_precond_apply) on box
  vectors of the body's grid equals the oracle's block Jacobi on the full
  grid (rel. 1e-9), and is zero off the body;
* the flag is fixed at setup.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import precond as pc
from oracle import vie_dense as vd
from synth import Grid

pytestmark = pytest.mark.gpu
K0 = 2 * np.pi
N = (14, 12, 40)
H = 0.06
CHANS = [((0.0, 0.6, 0.8), (1.0, 0.0, 0.0)), ((0.0, 0.0, 1.0), (0.3, 1j, 0.0))]


@pytest.fixture(scope="module")
def V():
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie

    vie.lib()
    return vie


def _slab_body(rng, z0, z1):
    """A rough slab with bumps in layers [z0, z1) of the N grid."""
    eps = np.ones(N[::-1])
    eps[z0:z1 - 2, 2:12, 1:13] = 2.2
    mask = rng.random((2, N[1], N[0])) < 0.4
    eps[z1 - 2:z1][mask] = rng.uniform(3.0, 6.0, size=int(mask.sum()))
    return eps


def _relerr(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def test_window_geometry_and_product(V):
    rng = np.random.default_rng(1)
    g = Grid.centred(N, H)
    eps = _slab_body(rng, 15, 23)
    chi = (eps - 1).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    x = (rng.standard_normal((3,) + N[::-1]) + 1j * rng.standard_normal((3,) + N[::-1]))
    xb = x * (eps != 1)[None]  # supported on the body
    ref = vd.matvec(chi, pos, H, K0, xb.reshape(3, -1)).reshape(x.shape)
    ctx = V.vie_setup([(eps, H, g.origin)], V.make_options(K0, flags=V.VIE_FLAG_Z_WINDOW))
    try:
        grid, fft, off = V.vie_grid(ctx, 0)
        assert grid == (14, 12, 8) and off == (0, 0, 15) and fft[2] == 16
        y64 = V.vie_matvec(ctx, 0, xb, V.VIE_FP64)
        y32 = V.vie_matvec(ctx, 0, xb, V.VIE_MIXED)
        # outside the window the input passes through
        xo = x.copy()
        xo[:, 15:23] = 0
        yo = V.vie_matvec(ctx, 0, xo, V.VIE_FP64)
    finally:
        V.vie_destroy(ctx)
    print("window product", _relerr(y64, ref), _relerr(y32, ref))
    assert _relerr(y64, ref) < 1e-12
    assert _relerr(y32, ref) < 5e-6
    assert np.array_equal(yo, xo)


@pytest.mark.parametrize("solver", ["bicgstab", "fgmres"])
def test_window_solves_match_lu(V, solver):
    rng = np.random.default_rng(2)
    g = Grid.centred(N, H)
    bodies = [_slab_body(rng, 15, 23), _slab_body(rng, 4, 10)]
    th = np.deg2rad(np.array([0.0, 35.0, 90.0, 160.0]))
    ph = np.deg2rad(np.array([0.0, 20.0, 250.0, 90.0]))
    res = {}
    for flag in (V.VIE_FLAG_Z_WINDOW, 0):
        opt = V.make_options(K0, precision=V.VIE_FP64, tol=1e-12, max_iter=4000, flags=flag)
        ctx = V.vie_setup([(e, H, g.origin) for e in bodies], opt)
        try:
            if flag:
                (g0, _, o0), (g1, _, o1) = V.vie_grid(ctx, 0), V.vie_grid(ctx, 1)
                assert g0 == g1 and g0[2] < N[2] and o0 != o1  # one window, two offsets
            if solver == "bicgstab":
                rc, st = V.vie_solve(ctx, CHANS * 2, [2, 2])
            else:
                rc, st = V.vie_solve_fgmres(ctx, CHANS * 2, [2, 2],
                                            V.fgmres_options(10, (2, 2), 3, V.VIE_FP64))
            assert rc == 0
            res[flag] = [([V.vie_get_current(ctx, b, q, N) for q in range(2)],
                          V.vie_farfield(ctx, b, th, ph, 2)) for b in range(2)]
        finally:
            V.vie_destroy(ctx)
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    for b, eps in enumerate(bodies):
        chi = (eps - 1).ravel()
        for q, (kh, p) in enumerate(CHANS):
            w = vd.solve_lu(chi, pos, H, K0, kh, p)
            ft, fp = vd.farfield(w, pos, H, K0, th, ph)
            ws, F = res[V.VIE_FLAG_Z_WINDOW][b]
            e_w = _relerr(ws[q].reshape(3, -1), w)
            e_f = _relerr(F[q], np.stack([ft, fp], -1))
            e_full = _relerr(ws[q], res[0][b][0][q])
            print(solver, b, q, e_w, e_f, e_full)
            assert e_w < 1e-10 and e_f < 1e-10 and e_full < 1e-10


def test_window_precond_apply_matches_oracle(V):
    rng = np.random.default_rng(4)
    g = Grid.centred(N, H)
    eps = _slab_body(rng, 15, 23)
    chi = (eps - 1).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    A, body = vd.body_system(chi, pos, H, K0)
    r = rng.standard_normal((2, 3) + N[::-1]) + 1j * rng.standard_normal((2, 3) + N[::-1])
    blocks, k = (3, 2), 3
    bset = pc.block_index_sets(pc.lateral_blocks(g.n, *blocks)[body])
    ctx = V.vie_setup([(eps, H, g.origin)], V.make_options(K0, flags=V.VIE_FLAG_Z_WINDOW))
    try:
        assert V.vie_grid(ctx, 0)[2] == (0, 0, 15)
        z = V.vie_precond_apply(ctx, V.fgmres_options(blocks=blocks, inner_iters=k,
                                                      inner_precision=V.VIE_FP64), r)
    finally:
        V.vie_destroy(ctx)
    off = np.ones(int(np.prod(g.n)), bool)
    off[body] = False
    for q in range(2):
        want = pc.block_jacobi(A, bset, r[q].reshape(3, -1)[:, body].reshape(-1), k=k)
        got = z[q].reshape(3, -1)[:, body].reshape(-1)
        err = _relerr(got, want)
        print("window precond", q, err)
        assert err < 1e-9
        assert np.all(z[q].reshape(3, -1)[:, off] == 0)


def test_window_flag_fixed_at_setup(V):
    rng = np.random.default_rng(3)
    g = Grid.centred(N, H)
    ctx = V.vie_setup([(_slab_body(rng, 15, 23), H, g.origin)],
                      V.make_options(K0, flags=V.VIE_FLAG_Z_WINDOW))
    try:
        with pytest.raises(V.VieError) as e:
            V.vie_set_options(ctx, V.make_options(K0))
        assert e.value.code == V.VIE_EINVAL
    finally:
        V.vie_destroy(ctx)
