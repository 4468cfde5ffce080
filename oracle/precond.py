"""Block-Jacobi preconditioner on a lateral partition, and flexible GMRES
(test infrastructure only).

The paper accelerates its largest solve (the full-wave metasurface, Sec. III-B; the method of Sec. II-C)
with a block preconditioner over a 7 x 7 partition of the structure and a
parallel implementation; it gives no further detail of the block solve.  The
reading written out here:

* partition: the grid's x index range is cut into ``bx`` contiguous parts,
  part i = [floor(i N1 / bx), floor((i + 1) N1 / bx)), the y range likewise
  into ``by`` parts; a block is one (x part, y part) pair and spans the whole
  z extent.  Block id = ix + bx * iy;
* preconditioner: block Jacobi.  M = blockdiag(A_bb), where A_bb is the
  discrete system (``vie_dense.body_system``) restricted to the body voxels
  of block b, i.e. the operator with every interaction between two different
  blocks dropped;
* block solve: exact (dense LU of A_bb), or inexact: ``k`` steps of GMRES
  from zero on every block, the element of the k-th Krylov space
  span{r_b, A_bb r_b, ...} with the smallest residual.  The inexact form
  changes with its input nonlinearly, so the outer method must be flexible;
* outer method: FGMRES(m) with right preconditioning (Saad, SIAM J. Sci.
  Comput. 14, 1993): Arnoldi on A M_j^{-1}, the preconditioned vectors
  z_j = M_j^{-1} v_j kept, x = x0 + Z y with y the least-squares solution of
  the small Hessenberg problem, restarted from the true residual.

Vectors are flat over the body unknowns in ``body_system`` order
(component-major: comp * Mb + k).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


def lateral_blocks(n, bx, by):
    """Block id of every voxel of an (N1, N2, N3) grid, x fastest (see the
    module docstring for the partition)."""
    n1, n2, n3 = (int(v) for v in n)

    def part(nn, nparts):
        lo = [(p * nn) // nparts for p in range(nparts)]  # first index of each part
        return np.searchsorted(lo, np.arange(nn), side="right") - 1

    px, py = part(n1, bx), part(n2, by)
    blk = px[None, None, :] + bx * py[None, :, None]
    return np.broadcast_to(blk, (n3, n2, n1)).reshape(-1).copy()


def block_index_sets(blk_of_body_voxel):
    """Unknown indices (component-major over Mb body voxels) of every block,
    as a dict block id -> index array (blocks with no body voxel omitted)."""
    mb = len(blk_of_body_voxel)
    out = {}
    for b in np.unique(blk_of_body_voxel):
        k = np.nonzero(blk_of_body_voxel == b)[0]
        out[int(b)] = np.concatenate([k, k + mb, k + 2 * mb])
    return out


def gmres_k(A, r, k):
    """k steps of GMRES from x = 0 on A x = r: the minimiser of ||r - A x|| over
    the Krylov space K_k(A, r).  Arnoldi with modified Gram-Schmidt, then the
    (k+1) x k least-squares problem; stops early at an invariant subspace."""
    beta = np.linalg.norm(r)
    if beta == 0.0:
        return np.zeros_like(r)
    n = len(r)
    V = np.zeros((n, k + 1), complex)
    H = np.zeros((k + 1, k), complex)
    V[:, 0] = r / beta
    j_used = k
    for j in range(k):
        w = A @ V[:, j]
        for i in range(j + 1):
            H[i, j] = np.vdot(V[:, i], w)
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] <= 1e-14 * beta:
            j_used = j + 1
            break
        V[:, j + 1] = w / H[j + 1, j]
    e1 = np.zeros(j_used + 1, complex)
    e1[0] = beta
    y = np.linalg.lstsq(H[: j_used + 1, :j_used], e1, rcond=None)[0]
    return V[:, :j_used] @ y


def block_jacobi(A, blocks, r, k=None):
    """z = M^{-1} r for the block-diagonal part of A over ``blocks`` (from
    ``block_index_sets``): exact block solves when k is None, else k steps of
    GMRES from zero per block."""
    z = np.zeros_like(r)
    for idx in blocks.values():
        Ab = A[np.ix_(idx, idx)]
        z[idx] = scipy.linalg.solve(Ab, r[idx]) if k is None else gmres_k(Ab, r[idx], k)
    return z


def fgmres(apply_A, b, apply_M=None, m=30, tol=1e-8, maxit=1000, keep_basis=False):
    """Restarted flexible GMRES with right preconditioning (see the module
    docstring).  ``apply_M`` may change from call to call; None means the
    identity (then this is plain restarted GMRES).

    Returns (x, steps, history of the relative residual estimate per step)
    and, with keep_basis, also the preconditioned vectors Z of the last cycle
    and the iterate x0 it started from."""
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    hist = [1.0]
    if bn == 0.0:
        return (x, 0, hist, None, x) if keep_basis else (x, 0, hist)
    n = len(b)
    steps = 0
    Z = None
    x0 = x
    while True:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        hist[-1] = beta / bn  # true residual replaces the estimate at a restart
        if beta <= tol * bn or steps >= maxit:
            break
        x0 = x.copy()
        V = np.zeros((n, m + 1), complex)
        Z = np.zeros((n, m), complex)
        H = np.zeros((m + 1, m), complex)
        V[:, 0] = r / beta
        j_used = 0
        for j in range(m):
            Z[:, j] = V[:, j] if apply_M is None else apply_M(V[:, j])
            w = apply_A(Z[:, j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            j_used = j + 1
            steps += 1
            e1 = np.zeros(j + 2, complex)
            e1[0] = beta
            y = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)[0]
            est = np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y) / bn
            hist.append(est)
            if est <= tol or H[j + 1, j] <= 1e-14 * beta or steps >= maxit:
                break
            V[:, j + 1] = w / H[j + 1, j]
        x = x0 + Z[:, :j_used] @ y
        Z = Z[:, :j_used]
    if keep_basis:
        return x, steps, hist, Z, x0
    return x, steps, hist
