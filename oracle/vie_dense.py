"""Dense FP64 oracle of the discrete volume integral equation (test infrastructure only).

The paper states the scattering problem as a volume integral equation for
the polarisation current J = -i w (eps - eps0) E (Sec. II-C, eq. 24), with the
free-space dyadic Green's function (eq. dyadicG), and solves it by method of
moments on a uniform voxel grid with FFT-accelerated products and BiCGStab.
This module writes out the discrete system the GPU path solves, in the most
direct way:

* unknown: the contrast current ``w = chi E`` per voxel and Cartesian
  component, ``chi = eps_r - 1``; J = -i w eps0 w, so eq. 24 divided by
  -i w eps0 and multiplied by chi is  w - chi * G[w] = chi * E_inc;
* pulse basis, collocation at voxel centres: off-diagonal blocks are
  ``k0^2 h^3 G(r_m - r_n)`` (midpoint rule of the volume integral);
* diagonal blocks ``s I`` with the equal-volume-sphere self term: real part
  -1/3 + 2/3 (cos x + x sin x - 1) (principal value plus depolarisation),
  imaginary part k0^3 h^3 / (6 pi) = k0^2 h^3 Im G(0), x = k0 a,
  a = h (3 / 4 pi)^(1/3).  The imaginary part equals the exact radiation
  reaction, which makes the discrete model exactly lossless (extinction equals
  scattering for real eps);
* far field (eq. 25): F(r) = lim_{R->inf} R e^{-i k0 R} E_sca
  = k0^2 h^3 / (4 pi) sum_n (I - r r) w_n exp(-i k0 r . r_n).

Arrays: vectors are complex ``(3, M)`` (component, voxel) with the voxel
index x-fastest over an ``(N1, N2, N3)`` grid; positions ``(M, 3)``.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

FOUR_PI = 4.0 * np.pi


def voxel_centres(n, h, origin):
    """Centres ``origin + h (i, j, l)`` of an (N1, N2, N3) grid, x fastest."""
    n = tuple(int(v) for v in n)
    ax = [origin[a] + h * np.arange(n[a]) for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def self_term(k0, h):
    """Diagonal coefficient s of the discrete operator (see module docstring).

    Equal-volume-sphere radius a = h (3/4pi)^(1/3), x = k0 a.  Real part:
    static depolarisation -1/3 plus the dynamic principal-value part
    2/3 (cos x + x sin x - 1).  Imaginary part: (2/9) x^3 = k0^3 h^3 / (6 pi)."""
    a = h * (3.0 / FOUR_PI) ** (1.0 / 3.0)
    x = k0 * a
    return complex(-1.0 / 3.0 + (2.0 / 3.0) * (np.cos(x) + x * np.sin(x) - 1.0),
                   (2.0 / 9.0) * x**3)


def green_dyadic(R, k0):
    """Free-space dyadic Green's function (eq. dyadicG) for separations R != 0.

    (I + grad grad / k0^2) e^{i k0 R}/(4 pi R), differentiated in closed form:
    g [ (1 + i/(kR) - 1/(kR)^2) I + (3/(kR)^2 - 3i/(kR) - 1) Rhat Rhat ].
    R: (..., 3) real.  Returns (..., 3, 3) complex."""
    R = np.asarray(R, float)
    r = np.linalg.norm(R, axis=-1)
    kr = k0 * r
    g = np.asarray(np.exp(1j * kr) / (FOUR_PI * r))
    a = np.asarray(1.0 + 1j / kr - 1.0 / kr**2)
    b = np.asarray(3.0 / kr**2 - 3j / kr - 1.0)
    u = R / np.asarray(r)[..., None]
    I = np.eye(3)
    return g[..., None, None] * (a[..., None, None] * I + b[..., None, None] * u[..., :, None] * u[..., None, :])


def incident_field(pos, k0, khat, pol):
    """Plane-wave channel e(r) = pol exp(i k0 khat . r) (e^{-i w t} convention), (3, M)."""
    ph = np.exp(1j * k0 * (pos @ np.asarray(khat, float)))
    return np.asarray(pol, complex)[:, None] * ph[None, :]


def rhs(chi, pos, k0, khat, pol):
    """Right-hand side b = chi e of the contrast-current system."""
    return chi[None, :] * incident_field(pos, k0, khat, pol)


def _green_apply_rows(pos, rows, src, x_src, h, k0, s_self=None):
    """sum_n Ghat(r_row - r_n) x_n over the sources ``src`` (indices) for the
    given rows, including the diagonal s x_row when the row is a source
    (s = self_term unless s_self is given).  Returns (3, len(rows))."""
    s = self_term(k0, h) if s_self is None else s_self
    scale = k0 * k0 * h**3
    P = pos[src]
    out = np.zeros((3, len(rows)), complex)
    src_pos = {int(v): i for i, v in enumerate(src)}
    chunk = max(1, int(4_000_000 // max(1, len(src))))
    for c0 in range(0, len(rows), chunk):
        rr = rows[c0:c0 + chunk]
        R = pos[rr][:, None, :] - P[None, :, :]  # (r, n, 3)
        r = np.linalg.norm(R, axis=-1)
        zero = r == 0.0
        r_safe = np.where(zero, 1.0, r)
        kr = k0 * r_safe
        g = np.exp(1j * kr) / (FOUR_PI * r_safe)
        a = g * (1.0 + 1j / kr - 1.0 / kr**2)
        b = g * (3.0 / kr**2 - 3j / kr - 1.0)
        a[zero] = 0.0
        b[zero] = 0.0
        u = R / r_safe[..., None]
        udotx = np.einsum("rnc,cn->rn", u, x_src)
        acc = a @ x_src.T  # (r, 3)   sum_n a x_n
        acc = acc + np.einsum("rn,rnc->rc", b * udotx, u)
        out[:, c0:c0 + len(rr)] = scale * acc.T
    for k, m in enumerate(rows):
        j = src_pos.get(int(m))
        if j is not None:
            out[:, k] += s * x_src[:, j]
    return out


def matvec_rows(chi, pos, h, k0, x, rows, s_self=None):
    """Rows of y = A x = x - chi * (Ghat x), summing directly over every voxel
    where x is non-zero (O(M) per row).  chi: (M,), x: (3, M)."""
    rows = np.asarray(rows, dtype=np.int64)
    src = np.nonzero(np.any(x != 0, axis=0))[0]
    gx = (_green_apply_rows(pos, rows, src, x[:, src], h, k0, s_self) if len(src)
          else np.zeros((3, len(rows)), complex))
    return x[:, rows] - chi[rows][None, :] * gx


def matvec(chi, pos, h, k0, x, s_self=None):
    """Full direct product y = x - chi * (Ghat x) (O(M^2); rows with chi = 0
    reduce to the identity)."""
    y = x.astype(complex).copy()
    rows = np.nonzero(chi != 0)[0]
    if len(rows):
        y[:, rows] = matvec_rows(chi, pos, h, k0, x, rows, s_self)
    return y


def green_matrix(pos, h, k0, s_self=None):
    """Dense Ghat over the given voxels, index ``comp * M + voxel`` (diagonal
    self_term unless s_self is given)."""
    M = len(pos)
    R = pos[:, None, :] - pos[None, :, :]
    eye = np.eye(M, dtype=bool)
    R[eye] = 1.0  # placeholder, overwritten below
    G = green_dyadic(R, k0) * (k0 * k0 * h**3)
    G[eye] = (self_term(k0, h) if s_self is None else s_self) * np.eye(3)
    return G.transpose(2, 0, 3, 1).reshape(3 * M, 3 * M)


def body_system(chi, pos, h, k0, s_self=None):
    """A = I - diag(chi) Ghat restricted to the body voxels (chi != 0).
    Returns (A, body_indices)."""
    body = np.nonzero(chi != 0)[0]
    G = green_matrix(pos[body], h, k0, s_self)
    c = np.tile(chi[body], 3)
    A = np.eye(3 * len(body), dtype=complex) - c[:, None] * G
    return A, body


def solve_lu(chi, pos, h, k0, khat, pol, s_self=None):
    """Exact solution of the discrete system by dense LU (w = 0 off the body).
    Returns w (3, M)."""
    A, body = body_system(chi, pos, h, k0, s_self)
    b = rhs(chi, pos, k0, khat, pol)[:, body].reshape(-1)
    wb = scipy.linalg.lu_solve(scipy.linalg.lu_factor(A), b)
    w = np.zeros((3, len(chi)), complex)
    w[:, body] = wb.reshape(3, -1)
    return w


def bicgstab(apply_A, b, tol=1e-8, maxit=5000, x0=None):
    """Textbook BiCGSTAB (van der Vorst 1992; the paper's Krylov solver,
    Sec. II-C) with conjugated inner products and shadow residual r0.

    Returns (x, iterations, relative residual history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x)
    rhat = r.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, [0.0]
    hist = [np.linalg.norm(r) / bn]
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for it in range(1, maxit + 1):
        rho = np.vdot(rhat, r)
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply_A(p)
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        if np.linalg.norm(s) / bn <= tol:
            x = x + alpha * p
            hist.append(np.linalg.norm(s) / bn)
            return x, it, hist
        t = apply_A(s)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] <= tol:
            return x, it, hist
    return x, maxit, hist


def direction(theta, phi):
    """Unit vectors r, theta-hat, phi-hat for spherical angles (radians)."""
    theta = np.asarray(theta, float)
    phi = np.asarray(phi, float)
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    r = np.stack([st * cp, st * sp, ct], -1)
    th = np.stack([ct * cp, ct * sp, -st], -1)
    ph = np.stack([-sp, cp, np.zeros_like(sp)], -1)
    return r, th, ph


def farfield_vec(w, pos, h, k0, rhat):
    """Cartesian far-field amplitude (eq. 25 with C_inf fixed so that
    F = lim R e^{-i k0 R} E_sca):  k0^2 h^3/(4 pi) (I - r r) sum_n w_n e^{-i k0 r.r_n}.
    rhat: (D, 3).  Returns (D, 3)."""
    rhat = np.atleast_2d(np.asarray(rhat, float))
    nz = np.nonzero(np.any(w != 0, axis=0))[0]
    P = pos[nz]
    W = w[:, nz]
    out = np.zeros((len(rhat), 3), complex)
    chunk = max(1, int(2_000_000 // max(1, len(nz))))
    for d0 in range(0, len(rhat), chunk):
        rh = rhat[d0:d0 + chunk]
        ph = np.exp(-1j * k0 * (rh @ P.T))  # (d, n)
        S = ph @ W.T  # (d, 3)
        S = S - rh * np.einsum("dc,dc->d", rh, S)[:, None]
        out[d0:d0 + chunk] = S
    return (k0 * k0 * h**3 / FOUR_PI) * out


def farfield(w, pos, h, k0, theta, phi):
    """(F_theta, F_phi) at the given angles (radians)."""
    r, th, ph = direction(theta, phi)
    shp = r.shape[:-1]
    F = farfield_vec(w, pos, h, k0, r.reshape(-1, 3))
    Ft = np.einsum("dc,dc->d", th.reshape(-1, 3), F).reshape(shp)
    Fp = np.einsum("dc,dc->d", ph.reshape(-1, 3), F).reshape(shp)
    return Ft, Fp


def extinction_cross_section(w, pos, h, k0, khat, pol):
    """Optical theorem: sigma_ext = (4 pi / k0) Im(pol* . F(khat))."""
    F = farfield_vec(w, pos, h, k0, np.asarray(khat, float)[None, :])[0]
    return FOUR_PI / k0 * float(np.imag(np.vdot(np.asarray(pol, complex), F)))


def scattering_cross_section(w, pos, h, k0, n_theta=None, n_phi=None):
    """sigma_sca = integral of |F|^2 over the sphere: Gauss-Legendre in cos(theta)
    times the trapezoid rule in phi (spectrally accurate for band-limited F)."""
    ext = np.ptp(pos, axis=0).max() + h
    nmin = int(2 * k0 * ext) + 12
    n_theta = n_theta or nmin
    n_phi = n_phi or 2 * nmin
    x, wt = np.polynomial.legendre.leggauss(n_theta)
    theta = np.arccos(x)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    T, P = np.meshgrid(theta, phi, indexing="ij")
    r, _, _ = direction(T, P)
    F = farfield_vec(w, pos, h, k0, r.reshape(-1, 3)).reshape(n_theta, n_phi, 3)
    I = (np.abs(F) ** 2).sum(-1)
    return float((wt[:, None] * I).sum() * (2 * np.pi / n_phi))
