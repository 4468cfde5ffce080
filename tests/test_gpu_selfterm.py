"""GPU parity of the exact-cube self term (VIE_FLAG_CUBE_SELF) against the
oracle (oracle/selfterm.py: adaptive face quadrature; the library uses its
own Gauss-Legendre rule with a cancellation-free radial factor).

* vie_self_term equals the oracle's coefficient, both kinds, k0 h from 0.01
  to 2 (rel. 1e-13);
* the FP64 product with the cube term equals the dense oracle operator with
  the cube term, every row (rel. 1e-12), and differs from the default one;
* solve + far field equal the dense LU solution with the cube term
  (rel. 1e-10); the block preconditioner's sub-problems carry the same term
  (vie_precond_apply against the oracle's block Jacobi, rel. 1e-9);
* the flag is fixed at setup.
"""

import numpy as np
import pytest

from oracle import precond as pc
from oracle import selfterm as st
from oracle import vie_dense as vd
from synth import Grid, random_ellipsoid_body

pytestmark = pytest.mark.gpu
K0 = 2 * np.pi


@pytest.fixture(scope="module")
def V():
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie

    vie.lib()
    return vie


def _case(seed, n=(13, 11, 9), h=0.07):
    rng = np.random.default_rng(seed)
    g = Grid.centred(n, h)
    eps = random_ellipsoid_body(rng, g, kmax=3, axis_range=(0.2, 0.5))
    return g, eps, (eps - 1.0).ravel(), vd.voxel_centres(g.n, g.h, g.origin)


def test_self_term_values(V):
    for kh in (0.01, 0.1, 0.39, 1.0, 2.0):
        h = kh / K0
        for kind, ref in ((0, vd.self_term(K0, h)), (1, st.self_term_cube(K0, h))):
            got = V.vie_self_term(kind, K0, h)
            assert abs(got - ref) < 1e-13 * abs(ref), (kind, kh, got, ref)
    for bad in [(2, K0, 0.1), (1, -1.0, 0.1), (0, K0, 0.0), (1, K0, np.nan)]:
        with pytest.raises(V.VieError) as e:
            V.vie_self_term(*bad)
        assert e.value.code == V.VIE_EINVAL


def test_cube_product_matches_oracle(V):
    g, eps, chi, pos = _case(31)
    rng = np.random.default_rng(2)
    x = (rng.standard_normal((3,) + g.n[::-1]) + 1j * rng.standard_normal((3,) + g.n[::-1]))
    x.reshape(3, -1)[:, chi == 0] = 0.0
    s_cube = st.self_term_cube(K0, g.h)
    ys = {}
    for flag in (0, V.VIE_FLAG_CUBE_SELF):
        ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0, flags=flag))
        try:
            ys[flag] = V.vie_matvec(ctx, 0, x, V.VIE_FP64).reshape(3, -1)
        finally:
            V.vie_destroy(ctx)
    want = vd.matvec(chi, pos, g.h, K0, x.reshape(3, -1), s_self=s_cube)
    err = np.linalg.norm(ys[V.VIE_FLAG_CUBE_SELF] - want) / np.linalg.norm(want)
    diff = np.linalg.norm(ys[0] - want) / np.linalg.norm(want)
    print("cube product", err, "default vs cube", diff)
    assert err < 1e-12
    assert diff > 1e-6


def test_cube_solve_and_precond_match_oracle(V):
    g, eps, chi, pos = _case(32, n=(12, 10, 6))
    s_cube = st.self_term_cube(K0, g.h)
    chans = [((0.0, 0.6, 0.8), (1.0, 0.0, 0.0)), ((0.0, 0.0, 1.0), (0.3, 1j, 0.0))]
    th = np.deg2rad(np.array([0.0, 40.0, 90.0, 150.0]))
    ph = np.deg2rad(np.array([0.0, 30.0, 200.0, 90.0]))
    A, body = vd.body_system(chi, pos, g.h, K0, s_self=s_cube)
    bset = pc.block_index_sets(pc.lateral_blocks(g.n, 3, 2)[body])
    rng = np.random.default_rng(4)
    r = rng.standard_normal((3,) + g.n[::-1]) + 1j * rng.standard_normal((3,) + g.n[::-1])
    opt = V.make_options(K0, tol=1e-12, max_iter=2000, flags=V.VIE_FLAG_CUBE_SELF)
    ctx = V.vie_setup([(eps, g.h, g.origin)], opt)
    try:
        rc, st_ = V.vie_solve(ctx, chans, [2])
        assert rc == 0
        F = V.vie_farfield(ctx, 0, th, ph, 2)
        z = V.vie_precond_apply(ctx, V.fgmres_options(blocks=(3, 2), inner_iters=3,
                                                      inner_precision=V.VIE_FP64), r)
        with pytest.raises(V.VieError) as e:  # the self-term kind is fixed at setup
            V.vie_set_options(ctx, V.make_options(K0, tol=1e-12, max_iter=2000))
        assert e.value.code == V.VIE_EINVAL
    finally:
        V.vie_destroy(ctx)
    for q, (kh, p) in enumerate(chans):
        w = vd.solve_lu(chi, pos, g.h, K0, kh, p, s_self=s_cube)
        ft, fp = vd.farfield(w, pos, g.h, K0, th, ph)
        ref = np.stack([ft, fp], -1)
        err = np.linalg.norm(F[q] - ref) / np.linalg.norm(ref)
        print("far field", q, err)
        assert err < 1e-10
    want = pc.block_jacobi(A, bset, r.reshape(3, -1)[:, body].reshape(-1), k=3)
    got = z.reshape(3, -1)[:, body].reshape(-1)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("block Jacobi with the cube term", err)
    assert err < 1e-9
