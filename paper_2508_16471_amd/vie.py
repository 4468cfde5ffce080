"""ctypes binding of ``include/vie.h`` (argument marshalling only).

Every numerical step runs inside ``libvie.so`` (HIP kernels for gfx950 and
the library's host runtime).  Loading fails loudly when the library has not
been built; there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VIE_LIB selects another build of the library (the host-ASan one in tests)
LIB_PATH = os.environ.get("VIE_LIB") or os.path.join(_HERE, "libvie.so")

VIE_OK, VIE_EINVAL, VIE_ENOMEM, VIE_EDEVICE, VIE_ENOCONV, VIE_ENOTSUP, VIE_ESTATE = 0, -1, -2, -3, -4, -5, -6
VIE_FP64, VIE_MIXED, VIE_MIXED_BF16 = 0, 1, 2
VIE_NORM_R1, VIE_NORM_R2 = 0, 1
VIE_FLAG_TIMING = 1
VIE_FLAG_NO_GRAPH = 2
VIE_FLAG_CUBE_SELF = 4
VIE_FLAG_Z_WINDOW = 8
VIE_STATIC_SCRATCH_BYTES = 268435456  # size of the static scratch of vie_matvec_dev_static


class vie_c64(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class vie_body(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("origin", C.c_double * 3),
                ("eps_r", C.POINTER(C.c_double))]


class vie_options(C.Structure):
    _fields_ = [("k0", C.c_double), ("precision", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("inner_tol", C.c_double), ("warm_start", C.c_int32),
                ("flags", C.c_int32)]


class vie_planewave(C.Structure):
    _fields_ = [("khat", C.c_double * 3), ("pol", vie_c64 * 3)]


class vie_na_detector(C.Structure):
    _fields_ = [("theta0", C.c_double), ("phi0", C.c_double), ("alpha", C.c_double),
                ("pol", vie_c64 * 3)]


class vie_fgmres_options(C.Structure):
    _fields_ = [("restart", C.c_int32), ("blocks", C.c_int32 * 2), ("inner_iters", C.c_int32),
                ("inner_precision", C.c_int32)]


class vie_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("matvecs", C.c_int32), ("cycles", C.c_int32),
                ("converged", C.c_int32), ("fallback", C.c_int32), ("warm", C.c_int32),
                ("rel_res", C.c_double), ("rel_res_x0", C.c_double), ("seconds", C.c_double)]


class VieError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def lib():
    """Load libvie.so (raises if it is missing: no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libvie.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        sig = {
            "vie_setup": (C.c_int, [P(vie_body), C.c_int32, P(vie_options), P(C.c_void_p)]),
            "vie_solve": (C.c_int, [C.c_void_p, P(vie_planewave), P(C.c_int32), P(vie_stats)]),
            "vie_solve_fgmres": (C.c_int, [C.c_void_p, P(vie_planewave), P(C.c_int32),
                                           P(vie_fgmres_options), P(vie_stats)]),
            "vie_precond_apply": (C.c_int, [C.c_void_p, P(vie_fgmres_options), P(vie_c64),
                                            P(vie_c64), C.c_int32]),
            "vie_farfield": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double),
                                       C.c_int32, P(vie_c64)]),
            "hom_classical_p2": (C.c_int, [P(vie_c64), P(C.c_double)]),
            "vie_self_term": (C.c_int, [C.c_int32, C.c_double, C.c_double, P(vie_c64)]),
            "vie_grid": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_int32), P(C.c_int32),
                                   P(C.c_int32)]),
            "vie_transfer_na": (C.c_int, [C.c_void_p, C.c_int32, P(vie_na_detector), C.c_int32,
                                          C.c_int32, C.c_int32, P(vie_c64)]),
            "hom_g2": (C.c_int, [P(vie_c64), P(C.c_double), C.c_double, P(C.c_double), C.c_int32,
                                 C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double)]),
            "vie_get_current": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, P(vie_c64)]),
            "vie_matvec": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, P(vie_c64), P(vie_c64),
                                     C.c_int32]),
            "vie_matvec_dev": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                         C.c_int32]),
            "vie_matvec_dev_static": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                                C.c_void_p, C.c_int32]),
            "vie_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
            "vie_hbm_probe": (C.c_int, [C.c_int64, C.c_int32, P(C.c_double)]),
            "vie_kernel_times": (C.c_int, [C.c_void_p, P(C.c_char_p), P(C.c_double), P(C.c_int64),
                                           P(C.c_int32), C.c_int32]),
            "vie_set_options": (C.c_int, [C.c_void_p, P(vie_options)]),
            "vie_destroy": (None, [C.c_void_p]),
            "vie_strerror": (C.c_char_p, [C.c_int]),
            "vie_rt_setup": (C.c_int, [P(vie_body), C.c_double, P(C.c_void_p)]),
            "vie_rt_grid": (C.c_int, [C.c_void_p, P(C.c_int32), P(C.c_int32)]),
            "vie_rt_matvec": (C.c_int, [C.c_void_p, P(vie_c64), P(vie_c64), C.c_int32,
                                        C.c_int32]),
            "vie_rt_solve": (C.c_int, [C.c_void_p, P(vie_planewave), C.c_int32, C.c_double,
                                       C.c_int32, C.c_int32, P(vie_c64), P(vie_stats)]),
            "vie_rt_farfield": (C.c_int, [C.c_void_p, P(vie_c64), C.c_int32, P(C.c_double),
                                          P(C.c_double), C.c_int32, P(vie_c64)]),
            "vie_rt_destroy": (None, [C.c_void_p]),
            "vie_cnn_num_params": (C.c_int64, []),
            "vie_cnn_create": (C.c_int, [C.c_uint64, P(C.c_void_p)]),
            "vie_cnn_destroy": (None, [C.c_void_p]),
            "vie_cnn_params": (C.c_int, [C.c_void_p, P(C.c_float), C.c_int64, C.c_int32]),
            "vie_cnn_adam_state": (C.c_int, [C.c_void_p, P(C.c_float), P(C.c_float), C.c_int64,
                                             P(C.c_int64), C.c_int32]),
            "vie_attach_cnn": (C.c_int, [C.c_void_p, C.c_void_p]),
            "vie_cnn_sample_dev": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                             C.c_void_p, P(C.c_int32)]),
            "vie_cnn_infer_dev": (C.c_int, [C.c_void_p, P(C.c_int32), C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
            "vie_cnn_grad_dev": (C.c_int, [C.c_void_p, P(C.c_int32), C.c_void_p, C.c_void_p,
                                           P(C.c_float), P(C.c_float), C.c_void_p]),
            "vie_cnn_train_step_dev": (C.c_int, [C.c_void_p, P(C.c_int32), C.c_void_p, C.c_void_p,
                                                 C.c_float, P(C.c_float), C.c_void_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(code):
    return lib().vie_strerror(int(code)).decode()


def _check(code, where, allow=()):
    if code != VIE_OK and code not in allow:
        raise VieError(code, where)
    return code


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _cptr(a):
    return a.ctypes.data_as(C.POINTER(vie_c64))


def make_options(k0, precision=VIE_FP64, tol=1e-8, max_iter=5000, inner_tol=1e-3, warm_start=0, flags=0):
    return vie_options(float(k0), int(precision), float(tol), int(max_iter), float(inner_tol),
                       int(warm_start), int(flags))


def vie_setup(bodies, opt):
    """bodies: list of (eps_r[N3,N2,N1] float64, h, origin[3]).  Returns ctx handle."""
    arr = (vie_body * len(bodies))()
    keep = []
    for i, (eps, h, origin) in enumerate(bodies):
        e = np.ascontiguousarray(eps, dtype=np.float64)
        keep.append(e)
        arr[i].n[0], arr[i].n[1], arr[i].n[2] = e.shape[2], e.shape[1], e.shape[0]
        arr[i].h = float(h)
        for a in range(3):
            arr[i].origin[a] = float(origin[a])
        arr[i].eps_r = _dptr(e)
    ctx = C.c_void_p()
    _check(lib().vie_setup(arr, len(bodies), C.byref(opt), C.byref(ctx)), "vie_setup")
    return ctx


def planewaves(channels):
    """channels: list of (khat[3], pol[3] complex) -> vie_planewave array."""
    arr = (vie_planewave * max(1, len(channels)))()
    for i, (k, p) in enumerate(channels):
        for a in range(3):
            arr[i].khat[a] = float(k[a])
            arr[i].pol[a].re = float(np.real(p[a]))
            arr[i].pol[a].im = float(np.imag(p[a]))
    return arr


def vie_solve(ctx, channels, nrhs_per_body, allow_noconv=False):
    """Solve all right-hand sides; returns (status, list of stats dicts)."""
    pw = planewaves(channels)
    nr = (C.c_int32 * len(nrhs_per_body))(*[int(v) for v in nrhs_per_body])
    st = (vie_stats * max(1, len(channels)))()
    rc = lib().vie_solve(ctx, pw, nr, st)
    _check(rc, "vie_solve", allow=(VIE_ENOCONV,) if allow_noconv else ())
    out = [{f: getattr(st[i], f) for f, _ in vie_stats._fields_} for i in range(len(channels))]
    return rc, out


def fgmres_options(restart=30, blocks=(7, 7), inner_iters=4, inner_precision=VIE_MIXED):
    o = vie_fgmres_options()
    o.restart = int(restart)
    o.blocks[0], o.blocks[1] = int(blocks[0]), int(blocks[1])
    o.inner_iters = int(inner_iters)
    o.inner_precision = int(inner_precision)
    return o


def vie_solve_fgmres(ctx, channels, nrhs_per_body, fopt, allow_noconv=False):
    """Block-Jacobi preconditioned restarted FGMRES solve of every body; returns
    (status, list of stats dicts) like vie_solve."""
    pw = planewaves(channels)
    nr = (C.c_int32 * len(nrhs_per_body))(*[int(v) for v in nrhs_per_body])
    st = (vie_stats * max(1, len(channels)))()
    rc = lib().vie_solve_fgmres(ctx, pw, nr, C.byref(fopt), st)
    _check(rc, "vie_solve_fgmres", allow=(VIE_ENOCONV,) if allow_noconv else ())
    out = [{f: getattr(st[i], f) for f, _ in vie_stats._fields_} for i in range(len(channels))]
    return rc, out


def vie_precond_apply(ctx, fopt, r):
    """z = M^{-1} r (block-Jacobi) for host vectors r[nvec, 3, N3, N2, N1] (or one)."""
    rs = np.ascontiguousarray(r, dtype=np.complex128)
    single = rs.ndim == 4
    if single:
        rs = rs[None]
    z = np.zeros_like(rs)
    _check(lib().vie_precond_apply(ctx, C.byref(fopt), _cptr(rs), _cptr(z), rs.shape[0]),
           "vie_precond_apply")
    return z[0] if single else z


def vie_farfield(ctx, body, theta, phi, nrhs):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    F = np.zeros((nrhs, len(th), 2), dtype=np.complex128)
    _check(lib().vie_farfield(ctx, int(body), _dptr(th), _dptr(ph), len(th), _cptr(F)), "vie_farfield")
    return F


def vie_grid(ctx, body):
    """(window grid, FFT lengths, window offset in the body's grid) of a body."""
    g, f, o = (C.c_int32 * 3)(), (C.c_int32 * 3)(), (C.c_int32 * 3)()
    _check(lib().vie_grid(ctx, int(body), g, f, o), "vie_grid")
    return tuple(g), tuple(f), tuple(o)


def vie_self_term(kind, k0, h):
    """Diagonal coefficient of the discrete operator: kind 0 sphere, 1 cube."""
    out = vie_c64()
    _check(lib().vie_self_term(int(kind), float(k0), float(h), C.byref(out)), "vie_self_term")
    return complex(out.re, out.im)


def vie_rt_setup(eps, h, origin, k0):
    """Rooftop-basis operator of one body (eps_r[N3,N2,N1]).  Returns a handle."""
    e = np.ascontiguousarray(eps, dtype=np.float64)
    b = vie_body()
    b.n[0], b.n[1], b.n[2] = e.shape[2], e.shape[1], e.shape[0]
    b.h = float(h)
    for a in range(3):
        b.origin[a] = float(origin[a])
    b.eps_r = _dptr(e)
    rt = C.c_void_p()
    _check(lib().vie_rt_setup(C.byref(b), float(k0), C.byref(rt)), "vie_rt_setup")
    return rt


def vie_rt_grid(rt):
    """(padded grid E, circulant lengths P), each (x, y, z)."""
    e, f = (C.c_int32 * 3)(), (C.c_int32 * 3)()
    _check(lib().vie_rt_grid(rt, e, f), "vie_rt_grid")
    return tuple(e), tuple(f)


def vie_rt_matvec(rt, x, precision=VIE_FP64):
    """y = A x for x[nvec, 3, E3, E2, E1] (or one vector) on the padded grid."""
    xs = np.ascontiguousarray(x, dtype=np.complex128)
    single = xs.ndim == 4
    if single:
        xs = xs[None]
    y = np.zeros_like(xs)
    _check(lib().vie_rt_matvec(rt, _cptr(xs), _cptr(y), xs.shape[0], int(precision)),
           "vie_rt_matvec")
    return y[0] if single else y


def vie_rt_solve(rt, channels, tol=1e-8, max_iter=2000, allow_noconv=False, precision=VIE_FP64):
    """BiCGSTAB solves of the channels; returns (status, w[nrhs, 3, E3, E2, E1], stats)."""
    E, _ = vie_rt_grid(rt)
    pw = planewaves(channels)
    n = len(channels)
    w = np.zeros((n, 3, E[2], E[1], E[0]), dtype=np.complex128)
    st = (vie_stats * max(1, n))()
    rc = lib().vie_rt_solve(rt, pw, n, float(tol), int(max_iter), int(precision), _cptr(w), st)
    _check(rc, "vie_rt_solve", allow=(VIE_ENOCONV,) if allow_noconv else ())
    out = [{f: getattr(st[i], f) for f, _ in vie_stats._fields_} for i in range(n)]
    return rc, w, out


def vie_rt_farfield(rt, w, theta, phi):
    """(F_theta, F_phi) of solutions w[nrhs, 3, E3, E2, E1]: array [nrhs, ndir, 2]."""
    ws = np.ascontiguousarray(w, dtype=np.complex128)
    if ws.ndim == 4:
        ws = ws[None]
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    F = np.zeros((ws.shape[0], len(th), 2), dtype=np.complex128)
    _check(lib().vie_rt_farfield(rt, _cptr(ws), ws.shape[0], _dptr(th), _dptr(ph), len(th),
                                 _cptr(F)), "vie_rt_farfield")
    return F


def vie_rt_destroy(rt):
    if rt:
        lib().vie_rt_destroy(rt)


def hom_classical_p2(T):
    """Classical intensity product of the superposed channels (eq. 27)."""
    t = np.ascontiguousarray(np.asarray(T, dtype=np.complex128).reshape(4))
    p = np.zeros(1)
    _check(lib().hom_classical_p2(_cptr(t), _dptr(p)), "hom_classical_p2")
    return float(p[0])


def vie_transfer_na(ctx, body, detectors, nrhs, n_rad=8, n_az=16):
    """Aperture-averaged transfer coefficients T[nrhs, ndet]; detectors: list of
    (theta0, phi0, alpha, pol[3] complex)."""
    arr = (vie_na_detector * max(1, len(detectors)))()
    for i, (t0, p0, al, pol) in enumerate(detectors):
        arr[i].theta0, arr[i].phi0, arr[i].alpha = float(t0), float(p0), float(al)
        for a in range(3):
            arr[i].pol[a].re = float(np.real(pol[a]))
            arr[i].pol[a].im = float(np.imag(pol[a]))
    T = np.zeros((nrhs, len(detectors)), dtype=np.complex128)
    _check(lib().vie_transfer_na(ctx, int(body), arr, len(detectors), int(n_rad), int(n_az),
                                 _cptr(T)), "vie_transfer_na")
    return T


def hom_g2(T, sigma=1.2, dtau=None, norm=VIE_NORM_R1, omega=None):
    """Returns (g2, Nc_raw[ndelay], Nc_norm[ndelay])."""
    t = np.ascontiguousarray(np.asarray(T, dtype=np.complex128).reshape(4))
    d = np.ascontiguousarray(np.zeros(0) if dtau is None else dtau, dtype=np.float64)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64)
    g = np.zeros(1)
    raw = np.zeros(len(d))
    nrm = np.zeros(len(d))
    _check(lib().hom_g2(_cptr(t), None if om is None else _dptr(om), float(sigma),
                        _dptr(d) if len(d) else None, len(d), int(norm), _dptr(g),
                        _dptr(raw) if len(d) else None, _dptr(nrm) if len(d) else None), "hom_g2")
    return float(g[0]), raw, nrm


def vie_get_current(ctx, body, rhs, n):
    """Solution w = chi E as complex array (3, N3, N2, N1); n = (N1, N2, N3)."""
    w = np.zeros((3, n[2], n[1], n[0]), dtype=np.complex128)
    _check(lib().vie_get_current(ctx, int(body), int(rhs), _cptr(w)), "vie_get_current")
    return w


def vie_matvec(ctx, body, x, precision=VIE_FP64):
    """y = x - chi Ghat x for host vectors x[nvec, 3, N3, N2, N1] (or one vector)."""
    xs = np.ascontiguousarray(x, dtype=np.complex128)
    single = xs.ndim == 4
    if single:
        xs = xs[None]
    y = np.zeros_like(xs)
    _check(lib().vie_matvec(ctx, int(body), int(precision), _cptr(xs), _cptr(y), xs.shape[0]), "vie_matvec")
    return y[0] if single else y


def vie_matvec_dev(ctx, body, x_ptr, y_ptr, nvec, precision=VIE_FP64):
    _check(lib().vie_matvec_dev(ctx, int(body), int(precision), C.c_void_p(x_ptr), C.c_void_p(y_ptr),
                                int(nvec)), "vie_matvec_dev")


def vie_matvec_dev_static(ctx, body, x_ptr, y_ptr, nvec, precision=VIE_FP64):
    """vie_matvec_dev with its scratch in the library's static device array
    (allocates nothing); raises VieError(VIE_ENOTSUP) beyond that array's size."""
    _check(lib().vie_matvec_dev_static(ctx, int(body), int(precision), C.c_void_p(x_ptr),
                                       C.c_void_p(y_ptr), int(nvec)), "vie_matvec_dev_static")


def vie_hbm_probe(nbytes=4 << 30, reps=10):
    """Achievable HBM bandwidth (GB/s): dict(read=, write=, copy=)."""
    g = np.zeros(3)
    _check(lib().vie_hbm_probe(int(nbytes), int(reps), _dptr(g)), "vie_hbm_probe")
    return {"read": float(g[0]), "write": float(g[1]), "copy": float(g[2])}


def vie_set_stream(ctx, stream_ptr):
    _check(lib().vie_set_stream(ctx, C.c_void_p(stream_ptr)), "vie_set_stream")


def vie_set_options(ctx, opt):
    _check(lib().vie_set_options(ctx, C.byref(opt)), "vie_set_options")


def vie_kernel_times(ctx, reset=False):
    nk = C.c_int32(0)
    _check(lib().vie_kernel_times(ctx, None, None, None, C.byref(nk), 0), "vie_kernel_times")
    cap = nk.value
    names = (C.c_char_p * cap)()
    ms = (C.c_double * cap)()
    cnt = (C.c_int64 * cap)()
    nk = C.c_int32(cap)
    _check(lib().vie_kernel_times(ctx, names, ms, cnt, C.byref(nk), int(reset)), "vie_kernel_times")
    return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(cap, nk.value))}


# ------------------------------------------------------------ network
def vie_cnn_num_params():
    return int(lib().vie_cnn_num_params())


def vie_cnn_create(seed=0):
    net = C.c_void_p()
    _check(lib().vie_cnn_create(C.c_uint64(seed), C.byref(net)), "vie_cnn_create")
    return net


def vie_cnn_destroy(net):
    if net:
        lib().vie_cnn_destroy(net)


def vie_cnn_params(net, params=None):
    """Get (params None) or set the fp32 parameter vector."""
    n = vie_cnn_num_params()
    if params is None:
        out = np.zeros(n, dtype=np.float32)
        _check(lib().vie_cnn_params(net, out.ctypes.data_as(C.POINTER(C.c_float)), n, 0), "vie_cnn_params")
        return out
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().vie_cnn_params(net, p.ctypes.data_as(C.POINTER(C.c_float)), n, 1), "vie_cnn_params")
    return p


def vie_cnn_adam_state(net, state=None):
    """Get (state None) or set the Adam state (m, v, step) of a network."""
    n = vie_cnn_num_params()
    fp = C.POINTER(C.c_float)
    if state is None:
        m = np.zeros(n, dtype=np.float32)
        v = np.zeros(n, dtype=np.float32)
        step = C.c_int64()
        _check(lib().vie_cnn_adam_state(net, m.ctypes.data_as(fp), v.ctypes.data_as(fp), n,
                                        C.byref(step), 0), "vie_cnn_adam_state")
        return m, v, int(step.value)
    m = np.ascontiguousarray(state[0], dtype=np.float32)
    v = np.ascontiguousarray(state[1], dtype=np.float32)
    step = C.c_int64(int(state[2]))
    _check(lib().vie_cnn_adam_state(net, m.ctypes.data_as(fp), v.ctypes.data_as(fp), n,
                                    C.byref(step), 1), "vie_cnn_adam_state")
    return state


def vie_attach_cnn(ctx, net):
    _check(lib().vie_attach_cnn(ctx, net), "vie_attach_cnn")


def _dims(d):
    return (C.c_int32 * 3)(*[int(v) for v in d])


def vie_cnn_sample_dev(ctx, body, rhs, feat_ptr=0, target_ptr=0):
    """Returns box dims (d0, d1, d2); fills device tensors when pointers given."""
    d = (C.c_int32 * 3)()
    _check(lib().vie_cnn_sample_dev(ctx, int(body), int(rhs), C.c_void_p(feat_ptr or None),
                                    C.c_void_p(target_ptr or None), d), "vie_cnn_sample_dev")
    return tuple(d)


def vie_cnn_infer_dev(net, dims, feat_ptr, out_ptr, stream=0):
    _check(lib().vie_cnn_infer_dev(net, _dims(dims), C.c_void_p(feat_ptr), C.c_void_p(out_ptr),
                                   C.c_void_p(stream or None)), "vie_cnn_infer_dev")


def vie_cnn_grad_dev(net, dims, feat_ptr, target_ptr, stream=0):
    n = vie_cnn_num_params()
    g = np.zeros(n, dtype=np.float32)
    loss = C.c_float()
    _check(lib().vie_cnn_grad_dev(net, _dims(dims), C.c_void_p(feat_ptr), C.c_void_p(target_ptr),
                                  g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss),
                                  C.c_void_p(stream or None)), "vie_cnn_grad_dev")
    return float(loss.value), g


def vie_cnn_train_step_dev(net, dims, feat_ptr, target_ptr, lr, stream=0):
    loss = C.c_float()
    _check(lib().vie_cnn_train_step_dev(net, _dims(dims), C.c_void_p(feat_ptr), C.c_void_p(target_ptr),
                                        C.c_float(lr), C.byref(loss), C.c_void_p(stream or None)),
           "vie_cnn_train_step_dev")
    return float(loss.value)


def cnn_param_shapes():
    """[(W shape (27, Cout, Cin), b shape (Cout,))] of the network layers."""
    ch = [32, 32, 32, 32, 16]
    return [((27, co, ci), (co,)) for ci, co in zip(ch[:-1], ch[1:])]


def cnn_unpack(p):
    """Split the flat parameter vector into [(W, b)] (views)."""
    out, at = [], 0
    for ws, bs in cnn_param_shapes():
        nw = int(np.prod(ws))
        out.append((p[at:at + nw].reshape(ws), p[at + nw:at + nw + bs[0]]))
        at += nw + bs[0]
    return out


def vie_destroy(ctx):
    if ctx:
        lib().vie_destroy(ctx)


def vie_strerror(code):
    return strerror(code)
