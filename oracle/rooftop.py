"""Dense FP64 oracle of the rooftop-basis discretisation (test infrastructure only).

The paper discretises eq. 24 by the method of moments with rooftop
(piecewise-linear) basis functions along the three Cartesian directions on
the uniform hexahedral grid and pulse testing (Sec. II-C, eq. Js_expand).  It
gives neither the entries nor the treatment at the body surface; this module
writes out the reading taken, in the most direct way (dense matrices over the
active faces, no FFT):

* unknown: the contrast current w = chi E (as in the pulse-basis operator),
  component i expanded in rooftops centred on the faces normal to i.  The
  rooftop of the face between cells c and c + e_i is 1 on the face and falls
  linearly to 0 at the far faces of both cells (pulse across).  A face is
  *active* if at least one of its two cells belongs to the body.  A face
  between two body cells carries a full rooftop; a face on the body surface
  carries the half of the rooftop inside the body, so the normal current
  drops to zero across the surface in a sheet of charge.
* grid: the body grid padded by one cell on every side, so that every active
  face has both of its cells in the grid.  Extended cell c is centred at
  origin + h (c - 1); face i of cell c sits at that centre + (h/2) e_i.
* charge: rho = div w is constant in every cell,
  rho(c) = sum_i (W_i(c) - W_i(c - e_i)) / h.  A surface face's sheet charge is
  carried by the outside cell of the face (the cell the cut-off half of the
  rooftop would have covered), so rho is the divergence of the full rooftops
  and the total charge is zero.
* scattered field: E_sca = k0^2 A + grad phi, A = g * w, phi = g * rho,
  g = e^{i k0 r} / (4 pi r) (eq. dyadicG written as (k0^2 + grad div) g).
  Pulse testing in the collocation manner: A and grad phi are evaluated at
  the face centre.  Off-diagonal couplings use the midpoint rule: a rooftop
  carries h^3 alpha (alpha = 1 full, 1/2 surface) at its face centre, a cell's
  charge h^3 at its centre.  The singular self couplings use the integral of
  g over the cube cell, I = int_cube g dV (a rooftop's own A term, a cell's
  own potential).  grad phi at face i of cell c is (phi(c + e_i) - phi(c)) / h.
* tested equation at an active face: E_i = W / chi_f with
  1/chi_f = (1/chi_a + 1/chi_b) / 2 between body cells a and b (the mean of
  the two one-sided values at the face) and 1/chi_f = 1/chi_body on the
  surface.  So the system is
        W - chi_f (k0^2 A + grad phi) = chi_f e(r_f),
  the same form as the pulse-basis operator I - chi Ghat.
* far field (eq. 25, same normalisation as the pulse basis):
  F(r) = k0^2 h^3 / (4 pi) (I - r r) sum_faces alpha W_i e_i exp(-i k0 r . r_f).

Vectors in the full layout are complex arrays of shape (3, M) over the
extended grid (x fastest), M = (N1 + 2)(N2 + 2)(N3 + 2), with W_i(c) the face
between c and c + e_i; entries of inactive faces are zero.  The product of
the full layout is the identity on inactive entries, which do not couple to
active ones.
"""

from __future__ import annotations

import numpy as np

from .selfterm import cube_integral

FOUR_PI = 4.0 * np.pi


def extended_chi(chi):
    """chi (N3, N2, N1) of the body grid padded by one zero cell per side."""
    return np.pad(np.asarray(chi, float), 1)


def face_data(chi, h, origin):
    """Per-face data of the full layout over the extended grid.

    Returns (active, alpha, chif, pos): active/alpha/chif of shape (3, M),
    pos of shape (3, M, 3) (face centres).  chi: (N3, N2, N1) body contrast."""
    X = extended_chi(chi)
    n3, n2, n1 = X.shape
    M = n1 * n2 * n3
    body = X != 0
    active = np.zeros((3, M), bool)
    alpha = np.zeros((3, M))
    chif = np.zeros((3, M))
    pos = np.zeros((3, M, 3))
    z, y, x = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    cen = np.stack([origin[0] + h * (x - 1), origin[1] + h * (y - 1), origin[2] + h * (z - 1)], -1)
    cen = cen.reshape(M, 3)
    for i in range(3):
        a_body = body
        b_body = np.zeros_like(body)
        # neighbour along axis i (array axis 2 - i)
        sl_src = [slice(None)] * 3
        sl_dst = [slice(None)] * 3
        sl_src[2 - i] = slice(1, None)
        sl_dst[2 - i] = slice(0, -1)
        b_body[tuple(sl_dst)] = body[tuple(sl_src)]
        chib = np.zeros_like(X)
        chib[tuple(sl_dst)] = X[tuple(sl_src)]
        act = a_body | b_body
        both = a_body & b_body
        inv = np.zeros_like(X)
        inv[both] = 0.5 * (1.0 / X[both] + 1.0 / chib[both])
        only_a = a_body & ~b_body
        only_b = b_body & ~a_body
        inv[only_a] = 1.0 / X[only_a]
        inv[only_b] = 1.0 / chib[only_b]
        active[i] = act.ravel()
        alpha[i] = np.where(both, 1.0, np.where(act, 0.5, 0.0)).ravel()
        cf = np.zeros_like(X)
        cf[act] = 1.0 / inv[act]
        chif[i] = cf.ravel()
        p = cen.copy()
        p[:, i] += 0.5 * h
        pos[i] = p
    return active, alpha, chif, pos


def _scalar_green(P, Q, h, k0, I):
    """h^3 g(|p - q|) between point sets, I where they coincide."""
    R = np.linalg.norm(P[:, None, :] - Q[None, :, :], axis=-1)
    zero = R < 1e-9 * h
    Rs = np.where(zero, 1.0, R)
    G = h**3 * np.exp(1j * k0 * Rs) / (FOUR_PI * Rs)
    G[zero] = I
    return G


def system(chi, h, origin, k0):
    """Dense operator over the active faces.

    Returns (K, idx, chif_a, pos_a, alpha_a, comp_a): E_sca at the active faces
    is K @ W_active; idx are the flat full-layout indices (comp * M + cell) of
    the active faces in the order of K."""
    X = extended_chi(chi)
    n3, n2, n1 = X.shape
    M = n1 * n2 * n3
    active, alpha, chif, pos = face_data(chi, h, origin)
    idx = np.nonzero(active.ravel())[0]
    comp = idx // M
    cell = idx % M
    P = pos.reshape(3 * M, 3)[idx]
    al = alpha.ravel()[idx]
    I = cube_integral(k0, h)
    # charge cells: every cell touching an active face
    step = np.array([1, n1, n1 * n2])
    c_lo = cell
    c_hi = cell + step[comp]
    cells = np.unique(np.concatenate([c_lo, c_hi]))
    where = {int(c): k for k, c in enumerate(cells)}
    D = np.zeros((len(cells), len(idx)))
    for f in range(len(idx)):
        D[where[int(c_lo[f])], f] += 1.0 / h  # out of the + face of the lower cell
        D[where[int(c_hi[f])], f] -= 1.0 / h  # into the - face of the upper cell
    z, y, x = np.unravel_index(cells, (n3, n2, n1))
    Pc = np.stack([origin[0] + h * (x - 1), origin[1] + h * (y - 1), origin[2] + h * (z - 1)], -1)
    Gc = _scalar_green(Pc, Pc, h, k0, I)
    Ga = _scalar_green(P, P, h, k0, I) * (comp[:, None] == comp[None, :]) * al[None, :]
    # grad phi at a face = (phi(upper cell) - phi(lower cell)) / h = -(D^T phi)
    K = k0 * k0 * Ga - D.T @ Gc @ D
    return K, idx, chif.ravel()[idx], P, al, comp


def rhs(chi, h, origin, k0, khat, pol):
    """b = chi_f e(r_f) in the full layout, (3, M)."""
    active, alpha, chif, pos = face_data(chi, h, origin)
    ph = np.exp(1j * k0 * (pos @ np.asarray(khat, float)))  # (3, M)
    return chif * np.asarray(pol, complex)[:, None] * ph


def matvec(chi, h, origin, k0, x):
    """y = x - chi_f (K x) on active faces, y = x elsewhere.  x: (3, M)."""
    K, idx, cf, _, _, _ = system(chi, h, origin, k0)
    xf = np.asarray(x, complex).ravel()
    y = xf.copy()
    y[idx] = xf[idx] - cf * (K @ xf[idx])
    return y.reshape(3, -1)


def solve_lu(chi, h, origin, k0, khat, pol):
    """Exact solution of the rooftop system for one plane wave, full layout."""
    K, idx, cf, _, _, _ = system(chi, h, origin, k0)
    b = rhs(chi, h, origin, k0, khat, pol).ravel()
    A = np.eye(len(idx)) - cf[:, None] * K
    w = np.zeros_like(b)
    w[idx] = np.linalg.solve(A, b[idx])
    return w.reshape(3, -1)


def farfield_vec(chi, h, origin, k0, w, rhat):
    """Cartesian far-field amplitude of a full-layout solution (module docstring).
    rhat: (D, 3).  Returns (D, 3)."""
    active, alpha, _, pos = face_data(chi, h, origin)
    rhat = np.atleast_2d(np.asarray(rhat, float))
    S = np.zeros((len(rhat), 3), complex)
    for i in range(3):
        m = active[i]
        ph = np.exp(-1j * k0 * (rhat @ pos[i][m].T))
        S[:, i] = ph @ (alpha[i][m] * w[i][m])
    S = S - rhat * np.einsum("dc,dc->d", rhat, S)[:, None]
    return (k0 * k0 * h**3 / FOUR_PI) * S


def matvec_rows(chi, h, origin, k0, x, rows):
    """Rows of the full-layout product y = x - chi_f (k0^2 A + grad phi),
    summing directly over every active face and every charged cell (O(M) per
    row, for grids too large for the dense matrix).  rows: flat full-layout
    indices (comp * M + cell) of active faces."""
    X = extended_chi(chi)
    n3, n2, n1 = X.shape
    M = n1 * n2 * n3
    active, alpha, chif, pos = face_data(chi, h, origin)
    W = np.where(active, np.asarray(x, complex).reshape(3, M), 0.0)
    I = cube_integral(k0, h)
    # cell charges: + face of the cell minus its - face, per component
    Wg = W.reshape(3, n3, n2, n1)
    rho = np.zeros((n3, n2, n1), complex)
    for i in range(3):
        ax = 2 - i
        lower = np.zeros_like(Wg[i])
        sl_dst = [slice(None)] * 3
        sl_src = [slice(None)] * 3
        sl_dst[ax] = slice(1, None)
        sl_src[ax] = slice(0, -1)
        lower[tuple(sl_dst)] = Wg[i][tuple(sl_src)]
        rho += (Wg[i] - lower) / h
    rho = rho.ravel()
    z, y, xx = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    cen = np.stack([origin[0] + h * (xx - 1), origin[1] + h * (y - 1), origin[2] + h * (z - 1)],
                   -1).reshape(M, 3)
    qc = np.nonzero(rho != 0)[0]
    step = np.array([1, n1, n1 * n2])

    def pot(points, src_pos, src_val):
        return (_scalar_green(points, src_pos, h, k0, I) @ src_val) if len(src_val) else \
            np.zeros(len(points), complex)

    rows = np.asarray(rows, dtype=np.int64)
    out = np.zeros(len(rows), complex)
    xf = np.asarray(x, complex).ravel()
    for k, f in enumerate(rows):
        i, c = int(f // M), int(f % M)
        src = np.nonzero(active[i])[0]
        A = pot(pos[i][c][None, :], pos[i][src], alpha[i][src] * W[i][src])[0]
        lo_hi = np.stack([cen[c], cen[c + step[i]]])
        phi = pot(lo_hi, cen[qc], rho[qc])
        Es = k0 * k0 * A + (phi[1] - phi[0]) / h
        out[k] = xf[f] - chif[i][c] * Es
    return out
