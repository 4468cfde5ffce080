"""Voxelised bodies, plane-wave channels and detector grids (inputs only).

Conventions (shared by every consumer, so both sides read the same input):

* A grid has ``n = (N1, N2, N3)`` voxels of edge ``h``; voxel ``(i, j, l)``
  has its centre at ``origin + h * (i, j, l)``.  The default origin centres
  the grid on 0 (``origin = -h (N - 1) / 2`` per axis).
* Permittivity arrays are real, shape ``(N3, N2, N1)`` (C order, so x is the
  fastest index in memory), background 1 (vacuum).
* A voxel belongs to a region when its centre lies inside it (centre
  inclusion); later regions overwrite earlier ones.
* Lengths are in wavelengths unless a caller says otherwise (k0 = 2 pi).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Grid:
    n: tuple  # (N1, N2, N3)
    h: float
    origin: tuple  # centre of voxel (0, 0, 0)

    @staticmethod
    def centred(n, h):
        n = tuple(int(v) for v in (n if np.ndim(n) else (n, n, n)))
        return Grid(n, float(h), tuple(default_origin(n, h)))

    def axes(self):
        """Voxel-centre coordinates along x, y, z."""
        return [self.origin[a] + self.h * np.arange(self.n[a]) for a in range(3)]

    def mesh(self):
        """Centre coordinates X, Y, Z, each of shape (N3, N2, N1)."""
        x, y, z = self.axes()
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return X, Y, Z


def default_origin(n, h):
    n = np.asarray(n if np.ndim(n) else (n, n, n), dtype=float)
    return -float(h) * (n - 1.0) / 2.0


def sphere(grid: Grid, radius, eps, centre=(0.0, 0.0, 0.0)):
    """Homogeneous sphere by centre inclusion."""
    X, Y, Z = grid.mesh()
    inside = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2 <= radius**2
    out = np.ones(inside.shape)
    out[inside] = eps
    return out


def _rotation(rng):
    """Uniform random rotation matrix (QR of a Gaussian matrix)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def ellipsoid_union(grid: Grid, ellipsoids, eps):
    """Union of ellipsoids, each ``(centre[3], semi_axes[3], rotation[3x3])``."""
    X, Y, Z = grid.mesh()
    P = np.stack([X, Y, Z], axis=-1)
    inside = np.zeros(X.shape, dtype=bool)
    for c, ax, rot in ellipsoids:
        u = (P - np.asarray(c)) @ np.asarray(rot)  # body-frame coordinates
        inside |= ((u / np.asarray(ax)) ** 2).sum(-1) <= 1.0
    out = np.ones(X.shape)
    out[inside] = eps
    return out


def random_ellipsoid_body(rng, grid: Grid, kmax=6, axis_range=(0.2, 1.0), eps_range=(1.5, 6.0)):
    """Union of 1..kmax random ellipsoids with one random permittivity,
    centres uniform in the box (parts outside the box are clipped)."""
    k = int(rng.integers(1, kmax + 1))
    lo = np.asarray(grid.origin)
    hi = lo + grid.h * (np.asarray(grid.n) - 1)
    ells = []
    for _ in range(k):
        c = rng.uniform(lo, hi)
        ax = rng.uniform(axis_range[0], axis_range[1], size=3)
        ells.append((c, ax, _rotation(rng)))
    eps = float(rng.uniform(*eps_range))
    body = ellipsoid_union(grid, ells, eps)
    if (body > 1.0).sum() == 0:  # keep at least one voxel so the body exists
        body.flat[body.size // 2] = eps
    return body


def metasurface_fins(grid: Grid, *, slab_eps, slab_cells, fin_eps, fin_len, fin_wid,
                     fin_cells, period, count, angles, z0_cells=0):
    """Rectangular fins on a slab (Pancharatnam-Berry phase metasurface).

    The slab fills z-cells ``[z0, z0 + slab_cells)`` over the whole lateral
    extent; fin (a, b) of a ``count x count`` array with lattice ``period``
    (length) is centred at ``((a + 1/2) p, (b + 1/2) p)`` from the grid's lower
    corner, occupies z-cells ``[z0 + slab_cells, z0 + slab_cells + fin_cells)``
    and is a ``fin_len x fin_wid`` rectangle rotated by ``angles[b, a]`` about
    z.  ``fin_len``/``fin_wid``/``fin_eps`` may be scalars or per-fin arrays.
    """
    X, Y, Z = grid.mesh()
    out = np.ones(X.shape)
    h = grid.h
    zc = np.arange(grid.n[2])
    slab = (zc >= z0_cells) & (zc < z0_cells + slab_cells)
    out[slab, :, :] = slab_eps
    fz = (zc >= z0_cells + slab_cells) & (zc < z0_cells + slab_cells + fin_cells)
    x_lo = grid.origin[0] - h / 2
    y_lo = grid.origin[1] - h / 2
    L = np.broadcast_to(np.asarray(fin_len, float), (count, count))
    W = np.broadcast_to(np.asarray(fin_wid, float), (count, count))
    E = np.broadcast_to(np.asarray(fin_eps, float), (count, count))
    Xs, Ys = X[fz], Y[fz]
    Os = out[fz]
    for b in range(count):
        for a in range(count):
            cx = x_lo + (a + 0.5) * period
            cy = y_lo + (b + 0.5) * period
            t = angles[b, a]
            u = (Xs - cx) * np.cos(t) + (Ys - cy) * np.sin(t)
            v = -(Xs - cx) * np.sin(t) + (Ys - cy) * np.cos(t)
            m = (np.abs(u) <= L[b, a] / 2) & (np.abs(v) <= W[b, a] / 2)
            Os[m] = E[b, a]
    out[fz] = Os
    return out


def pb_rotation_step(k0, theta_t, period):
    """Rotation increment between adjacent cells of a Pancharatnam-Berry
    phase gradient that deflects normal incidence to ``theta_t``: half the
    transverse phase step k0 sin(theta_t) p (the paper's design rule, eq. 32)."""
    return 0.5 * k0 * np.sin(theta_t) * period


def metasurface_family(rng, n=128, h=1.0 / 32):
    """One body of the learned-warm-start family on an ``n^3`` grid: slab
    (eps 2.1, 6 cells) under an 8x8 fin array (period 16 cells, nominal
    5x13x19 cells, each dimension jittered by up to +-20 %, one fin
    permittivity drawn from U[4, 7] per body), centred in z.  Rotations: with
    probability 1/2 a linear PB gradient (supercell of 4, 6 or 8 columns
    along x or y, random offset), else i.i.d. U[0, pi)."""
    grid = Grid.centred(n, h)
    per_cells = n // 8
    if rng.random() < 0.5:
        sup = int(rng.choice([4, 6, 8]))
        off = rng.uniform(0, np.pi)
        idx = np.arange(8)
        ang1 = (off + np.pi * idx / sup) % np.pi
        ang = np.tile(ang1, (8, 1)) if rng.random() < 0.5 else np.tile(ang1[:, None], (1, 8))
    else:
        ang = rng.uniform(0, np.pi, size=(8, 8))
    jit = lambda nom: nom * h * rng.uniform(0.8, 1.2, size=(8, 8))  # noqa: E731
    wid = jit(5 * n / 128)
    ln = jit(13 * n / 128)
    fin_cells = int(round(19 * n / 128 * rng.uniform(0.8, 1.2)))
    slab_cells = max(1, int(round(6 * n / 128)))
    z0 = (n - slab_cells - fin_cells) // 2
    eps_fin = float(rng.uniform(4.0, 7.0))
    body = metasurface_fins(grid, slab_eps=2.1, slab_cells=slab_cells, fin_eps=eps_fin,
                            fin_len=ln, fin_wid=wid, fin_cells=fin_cells,
                            period=per_cells * h, count=8, angles=ang, z0_cells=z0)
    return grid, body


def pb_metasurface(n=(256, 256, 48), h=1.0 / 60, count=8):
    """The benchmark Pancharatnam-Berry metasurface (lengths in wavelengths):
    a ``count x count`` array of 0.15 x 0.4 x 0.6 fins (eps 5.8) on a lossless
    slab 0.2 thick (eps 2.1), lateral period ``n[0] h / count``, fin rotation
    stepped linearly through [0, pi) across x (angle pi a / count in column
    a), slab and fins centred in z on an ``n`` grid of spacing ``h``.  At the
    defaults (h = lambda/60) the slab is 12 cells, the fins 9 x 24 x 36 cells
    on a 32-cell period, and slab plus fins fill the 48 z cells."""
    grid = Grid.centred(n, h)
    fin_cells = int(round(0.6 / h))
    slab_cells = max(1, int(round(0.2 / h)))
    if slab_cells + fin_cells > n[2]:
        raise ValueError("grid too thin for slab and fins")
    z0 = (n[2] - slab_cells - fin_cells) // 2
    ang = np.tile(np.pi * np.arange(count) / count, (count, 1))
    body = metasurface_fins(grid, slab_eps=2.1, slab_cells=slab_cells, fin_eps=5.8, fin_len=0.4,
                            fin_wid=0.15, fin_cells=fin_cells, period=n[0] * h / count, count=count,
                            angles=ang, z0_cells=z0)
    return grid, body


def paper_metasurface(h=1.0 / 62, n=(2480, 744, 124), substrate_cells=2):
    """The paper's full-wave PB metasurface at its stated size (lengths in
    wavelengths, lambda = 1550 nm): a 40 x 12 x 2 box at 62 cells per
    wavelength (2480 x 744 x 124 voxels).  Unit cell of period 667 nm with a
    silicon nanofin (n = 3.44, eps = 11.83) of 486 x 219 x 830 nm on a glass
    substrate of eps 2.25 (the paper's n_glass = 2.25 read as the
    permittivity).  91 unit cells along x (7 groups of 13) and as many along
    y as fit the 12-wavelength width (27), centred laterally; fin m along x
    is rotated by m times 13.44 deg (eq. 32, deflection 10 deg); the
    substrate is ``substrate_cells`` thick (the paper leaves it open; 2 cells
    puts the element count near the paper's 18,013,710), fins on top, the
    stack centred in z.  Built fin by fin on its own bounding box (the
    lateral fin map is shared by every fin layer)."""
    lam_nm = 1550.0
    p = 667.0 / lam_nm
    fl, fw, fh = 486.0 / lam_nm, 219.0 / lam_nm, 830.0 / lam_nm
    eps_si, eps_glass = 3.44 ** 2, 2.25
    grid = Grid.centred(n, h)
    nx, ny = 91, int(np.floor(n[1] * h / p))
    dth = pb_rotation_step(2 * np.pi, np.deg2rad(10.0), p)
    fin_cells = int(round(fh / h))
    z0 = (n[2] - substrate_cells - fin_cells) // 2
    # lateral fin map (x fastest): eps of the fin covering each column, 1 elsewhere
    fmap = np.ones((n[1], n[0]))
    xs = grid.origin[0] + h * np.arange(n[0])
    ys = grid.origin[1] + h * np.arange(n[1])
    x0 = -0.5 * nx * p  # array centred on the grid centre (0, 0)
    y0 = -0.5 * ny * p
    half = 0.5 * np.hypot(fl, fw) + h
    for a in range(nx):
        t = a * dth
        c, sn = np.cos(t), np.sin(t)
        cx = x0 + (a + 0.5) * p
        i0, i1 = np.searchsorted(xs, cx - half), np.searchsorted(xs, cx + half)
        for b in range(ny):
            cy = y0 + (b + 0.5) * p
            j0, j1 = np.searchsorted(ys, cy - half), np.searchsorted(ys, cy + half)
            X, Y = np.meshgrid(xs[i0:i1] - cx, ys[j0:j1] - cy, indexing="xy")
            u = X * c + Y * sn
            v = -X * sn + Y * c
            m = (np.abs(u) <= fl / 2) & (np.abs(v) <= fw / 2)
            fmap[j0:j1, i0:i1][m] = eps_si
    body = np.ones(n[::-1])
    body[z0:z0 + substrate_cells] = eps_glass
    body[z0 + substrate_cells:z0 + substrate_cells + fin_cells] = fmap[None]
    return grid, body


def uv_directions(values=np.arange(-0.3, 0.41, 0.1)):
    """Incident directions (u, v, sqrt(1 - u^2 - v^2)) on the product grid of
    transverse components ``values`` (default -0.3 ... 0.4 in steps of 0.1:
    64 directions, normal incidence included), u fastest."""
    vals = np.round(np.asarray(values, float), 12)
    U, Vv = np.meshgrid(vals, vals, indexing="xy")
    u, v = U.ravel(), Vv.ravel()
    return np.stack([u, v, np.sqrt(1.0 - u * u - v * v)], axis=1)


def cap_directions(count, cap_deg):
    """``count`` directions spread evenly (Fibonacci spiral in cos theta) over
    the cap of half-angle ``cap_deg`` about +z."""
    cmin = np.cos(np.deg2rad(cap_deg))
    i = np.arange(count) + 0.5
    ct = 1.0 - (1.0 - cmin) * i / count
    ph = np.pi * (3.0 - np.sqrt(5.0)) * i
    st = np.sqrt(1.0 - ct * ct)
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)


def planewave(khat, pol):
    """Normalised plane-wave channel ``(khat[3] real, pol[3] complex)``;
    ``pol`` is projected orthogonal to ``khat`` and normalised."""
    k = np.asarray(khat, float)
    k = k / np.linalg.norm(k)
    p = np.asarray(pol, complex)
    p = p - k * (k @ p)
    return k, p / np.linalg.norm(p)


def _hv_basis(khat):
    """(H, V) = (x, y) carried to khat by the minimal rotation taking z to khat."""
    z = np.array([0.0, 0.0, 1.0])
    k = np.asarray(khat, float) / np.linalg.norm(khat)
    c = float(k @ z)
    if c > 1 - 1e-15:
        return np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    if c < -1 + 1e-15:  # rotation by pi about x
        return np.array([1.0, 0, 0]), np.array([0, -1.0, 0])
    v = np.cross(z, k)
    s = np.linalg.norm(v)
    vx = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
    R = np.eye(3) + vx + vx @ vx * ((1 - c) / s**2)
    return R @ np.array([1.0, 0, 0]), R @ np.array([0, 1.0, 0])


def circular_pol_basis(khat):
    """Linear (H, V) and circular L = (H + iV)/sqrt2, R = (H - iV)/sqrt2
    polarisations for direction khat (the paper's circular convention)."""
    H, V = _hv_basis(khat)
    L = (H + 1j * V) / np.sqrt(2)
    R = (H - 1j * V) / np.sqrt(2)
    return H.astype(complex), V.astype(complex), L, R


def random_planewave(rng, cap_deg=None, elliptical=False):
    """Random channel: direction uniform on the sphere (or in a cap of
    half-angle ``cap_deg`` about +z); linear polarisation with uniform angle,
    or a random elliptical one."""
    if cap_deg is None:
        v = rng.standard_normal(3)
        k = v / np.linalg.norm(v)
    else:
        cmin = np.cos(np.deg2rad(cap_deg))
        ct = rng.uniform(cmin, 1.0)
        ph = rng.uniform(0, 2 * np.pi)
        st = np.sqrt(1 - ct * ct)
        k = np.array([st * np.cos(ph), st * np.sin(ph), ct])
    H, V = _hv_basis(k)
    if elliptical:
        a = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        p = a[0] * H + a[1] * V
    else:
        t = rng.uniform(0, np.pi)
        p = np.cos(t) * H + np.sin(t) * V
    return planewave(k, p)
