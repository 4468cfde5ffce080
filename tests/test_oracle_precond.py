"""Pins of the block-Jacobi / flexible-GMRES oracle (block preconditioner of
the full-wave metasurface solve, Sec. III-B; FGMRES after Saad 1993).

Each check compares against something the oracle does not contain:

* the partition: every voxel in exactly one block, parts contiguous and
  within one voxel of equal size, the block of a voxel found by a direct scan
  of the part bounds;
* k-step GMRES is the minimal-residual element of the Krylov space, here
  computed by least squares over the explicit power basis (no Arnoldi), and
  the exact solution once k reaches the dimension;
* FGMRES with the identity is GMRES: its j-step iterate is that Krylov
  minimiser too; with a nonlinear preconditioner its iterate minimises the
  residual over the stored preconditioned vectors;
* exact block Jacobi on an operator without cross-block couplings, or with a
  single block, is the exact inverse: one step;
* the converged FGMRES solution of a VIE body equals the dense LU solution.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import precond as pc
from oracle import vie_dense as vd
from synth import Grid, random_ellipsoid_body

K0 = 2 * np.pi


def _rand_system(rng, n, shift=3.0):
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return A / np.sqrt(n) + shift * np.eye(n)


def _krylov_min(A, r, k):
    """argmin_{x in span(r, A r, ..., A^{k-1} r)} ||r - A x|| via the power basis."""
    K = np.stack([np.linalg.matrix_power(A, i) @ r for i in range(k)], axis=1)
    c = np.linalg.lstsq(A @ K, r, rcond=None)[0]
    return K @ c


def _vie_case(seed, n=(9, 8, 3), h=0.08):
    rng = np.random.default_rng(seed)
    g = Grid.centred(n, h)
    eps = random_ellipsoid_body(rng, g, kmax=3, axis_range=(0.2, 0.5))
    chi = (eps - 1.0).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    A, body = vd.body_system(chi, pos, g.h, K0)
    b = vd.rhs(chi, pos, K0, (0.0, 0.6, 0.8), (1.0, 0.0, 0.0))[:, body].reshape(-1)
    return g, chi, pos, A, body, b


@pytest.mark.parametrize("n,bx,by", [((14, 14, 3), 7, 7), ((10, 23, 2), 3, 7), ((5, 4, 2), 5, 1),
                                     ((3, 3, 1), 1, 1)])
def test_partition(n, bx, by):
    blk = pc.lateral_blocks(n, bx, by)
    n1, n2, n3 = n
    assert blk.shape == (n1 * n2 * n3,)
    ix = np.arange(n1 * n2 * n3) % n1
    iy = (np.arange(n1 * n2 * n3) // n1) % n2
    # direct scan of the bounds floor(p N / parts)
    for i in range(n1 * n2 * n3):
        px = [p for p in range(bx) if (p * n1) // bx <= ix[i] < ((p + 1) * n1) // bx]
        py = [p for p in range(by) if (p * n2) // by <= iy[i] < ((p + 1) * n2) // by]
        assert len(px) == 1 and len(py) == 1 and blk[i] == px[0] + bx * py[0]
    sizes_x = np.bincount(blk[:n1] % bx, minlength=bx)
    assert sizes_x.max() - sizes_x.min() <= 1 and sizes_x.min() >= 1
    assert np.all(np.diff(blk[:n1]) >= 0)  # contiguous along x
    assert set(np.unique(blk)) == set(range(bx * by))


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_gmres_k_is_krylov_minimiser(k):
    rng = np.random.default_rng(40 + k)
    A = _rand_system(rng, 12)
    r = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    x = pc.gmres_k(A, r, k)
    want = _krylov_min(A, r, k)
    assert np.linalg.norm(x - want) < 1e-10 * np.linalg.norm(want)


def test_gmres_k_full_dimension_is_exact():
    rng = np.random.default_rng(7)
    A = _rand_system(rng, 10, shift=1.0)
    r = rng.standard_normal(10) + 1j * rng.standard_normal(10)
    x = pc.gmres_k(A, r, 10)
    assert np.linalg.norm(A @ x - r) < 1e-10 * np.linalg.norm(r)
    assert np.all(pc.gmres_k(A, np.zeros(10, complex), 3) == 0)


@pytest.mark.parametrize("j", [1, 2, 4])
def test_fgmres_identity_is_gmres(j):
    rng = np.random.default_rng(60 + j)
    A = _rand_system(rng, 14, shift=1.5)
    b = rng.standard_normal(14) + 1j * rng.standard_normal(14)
    x, steps, hist = pc.fgmres(lambda v: A @ v, b, None, m=8, tol=1e-15, maxit=j)
    assert steps == j
    want = _krylov_min(A, b, j)
    assert np.linalg.norm(x - want) < 1e-10 * np.linalg.norm(want)
    assert all(hist[i + 1] <= hist[i] + 1e-15 for i in range(len(hist) - 1))


def test_fgmres_nonlinear_preconditioner_minimises_over_z():
    g, chi, pos, A, body, b = _vie_case(3)
    blocks = pc.block_index_sets(pc.lateral_blocks(g.n, 3, 2)[body])
    M = lambda v: pc.block_jacobi(A, blocks, v, k=2)  # noqa: E731  (nonlinear in v)
    x, steps, hist, Z, x0 = pc.fgmres(lambda v: A @ v, b, M, m=6, tol=1e-15, maxit=6,
                                      keep_basis=True)
    assert steps == 6 and Z.shape[1] == 6 and np.all(x0 == 0)
    y = np.linalg.lstsq(A @ Z, b, rcond=None)[0]
    best = np.linalg.norm(b - A @ (Z @ y))
    assert abs(np.linalg.norm(b - A @ x) - best) < 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(x - Z @ y) < 1e-9 * np.linalg.norm(x)
    # k-step GMRES is homogeneous in its input but not additive
    v1, v2 = Z[:, 0], Z[:, 1]
    assert np.linalg.norm(M(v1 + v2) - M(v1) - M(v2)) > 1e-6 * np.linalg.norm(M(v1 + v2))


def test_exact_block_jacobi_without_couplings_is_one_step():
    g, chi, pos, A, body, b = _vie_case(5)
    blocks = pc.block_index_sets(pc.lateral_blocks(g.n, 3, 3)[body])
    Ab = np.zeros_like(A)
    for idx in blocks.values():
        Ab[np.ix_(idx, idx)] = A[np.ix_(idx, idx)]
    x, steps, _ = pc.fgmres(lambda v: Ab @ v, b, lambda v: pc.block_jacobi(Ab, blocks, v),
                            m=5, tol=1e-12)
    assert steps == 1
    assert np.linalg.norm(Ab @ x - b) < 1e-12 * np.linalg.norm(b)


def test_single_block_is_exact_inverse():
    g, chi, pos, A, body, b = _vie_case(6)
    blocks = pc.block_index_sets(pc.lateral_blocks(g.n, 1, 1)[body])
    assert len(blocks) == 1
    x, steps, _ = pc.fgmres(lambda v: A @ v, b, lambda v: pc.block_jacobi(A, blocks, v), m=5,
                            tol=1e-12)
    assert steps == 1
    assert np.linalg.norm(A @ x - b) < 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("k", [None, 3])
def test_fgmres_solution_equals_lu(k):
    g, chi, pos, A, body, b = _vie_case(8)
    blocks = pc.block_index_sets(pc.lateral_blocks(g.n, 3, 2)[body])
    x, steps, hist = pc.fgmres(lambda v: A @ v, b, lambda v: pc.block_jacobi(A, blocks, v, k=k),
                               m=4, tol=1e-11, maxit=400)
    want = scipy.linalg.lu_solve(scipy.linalg.lu_factor(A), b)
    assert hist[-1] <= 1e-11
    assert np.linalg.norm(x - want) < 1e-9 * np.linalg.norm(want)
    # restarts happened (m = 4 is far below what the body needs)
    assert steps > 4
