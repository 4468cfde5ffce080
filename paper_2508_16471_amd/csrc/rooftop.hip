// Rooftop basis with pulse testing (Sec. II-C, eq. Js_expand): FP64 products,
// or FP32 products inside FP64 refinement.
//
// The paper expands the current in rooftops along x, y and z on the uniform
// grid and tests with pulses.  Reading taken (entries and the body surface
// are not given): the contrast current w = chi E, component i carried by
// rooftops on the faces normal to i, a full rooftop between two body cells,
// the inside half on the body surface (alpha = 1 or 1/2); the charge
// rho = div w is constant per cell, a surface face's sheet charge carried by
// its outside cell; E_sca = k0^2 A + grad phi with A = g * w, phi = g * rho,
// both collocated at face centres, midpoint weights h^3 alpha (a rooftop) and
// h^3 (a cell) off the diagonal and the cube-cell integral of g on it; grad
// phi across a face is the difference of its two cells' potentials over h;
// at a face E = W / chi_f with 1/chi_f the mean of its body sides' 1/chi.
//
// The grid is the body grid padded by one cell on every side, so every
// active face has both of its cells on the grid.  A and phi are four scalar
// convolutions with the same kernel h^3 g (self: the cube integral) over the
// padded grid: its circulant (length P >= 2 E - 1 per axis) is transformed
// once at setup, each product transforms alpha W_x, alpha W_y, alpha W_z and
// rho forward, multiplies by the spectrum and transforms back (the inverse as
// the conjugate of the forward transform of the conjugate).  The transforms
// are pruned: the forward one skips the zero padding, the inverse one
// computes only the padded grid's outputs.  The solver is
// BiCGSTAB (the paper's method) with the true residual deciding convergence.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/vie.h"
#include "fft_common.h"
#include "green.h"
#include "kernels.h"
#include "trace.h"

namespace vie {

// Circulant length of an axis of n cells: the smallest supported transform
// length (2^k >= 8 or 3 * 2^k >= 12) with P >= 2 n - 1.
static int rt_fft_length(int n) {
  const int need = std::max(8, 2 * n - 1);
  int p2 = 8, p3 = 12;
  while (p2 < need) p2 <<= 1;
  while (p3 < need) p3 <<= 1;
  return std::min(p2, p3);
}

struct RtGeom {
  int E[3];   // padded grid (body grid + 2)
  int P[3];   // circulant lengths
  int64_t m;  // E1 E2 E3
  int64_t M;  // P1 P2 P3
};

// Circulant samples of h^3 e^{i k0 r} / (4 pi r) over displacements
// [-(E-1), E-1] per axis at index d mod P, zero elsewhere; the cube integral
// at d = 0.
__global__ void k_rt_green(c64* __restrict__ work, RtGeom q, double h, double k0, double s_re,
                           double s_im) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < q.M;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int idx[3] = {(int)(e % q.P[0]), (int)((e / q.P[0]) % q.P[1]),
                        (int)(e / ((int64_t)q.P[0] * q.P[1]))};
    int d[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
      if (idx[a] <= q.E[a] - 1)
        d[a] = idx[a];
      else if (idx[a] >= q.P[a] - (q.E[a] - 1))
        d[a] = idx[a] - q.P[a];
      else
        ok = false;
    }
    c64 v = mk(0.0, 0.0);
    if (ok) {
      if (d[0] == 0 && d[1] == 0 && d[2] == 0) {
        v = mk(s_re, s_im);
      } else {
        const double r = h * sqrt((double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2]);
        double sn, cs;
        sincos(k0 * r, &sn, &cs);
        const double f = h * h * h / (4.0 * M_PI * r);
        v = mk(f * cs, f * sn);
      }
    }
    work[e] = v;
  }
}

// The kernel samples are even along every axis (they depend on |d| per
// axis), so is their transform: only the octant [0, P/2]^3 is kept,
// [z][y][x] with extents Q = P/2 + 1, scaled by s (= 1/M), with an FP32 copy.
__global__ void k_rt_octant(const c64* __restrict__ in, c64* __restrict__ out,
                            c32* __restrict__ out32, RtGeom q, double s) {
  const int Q0 = q.P[0] / 2 + 1, Q1 = q.P[1] / 2 + 1, Q2 = q.P[2] / 2 + 1;
  const int64_t n = (int64_t)Q0 * Q1 * Q2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(e % Q0), y = (int)((e / Q0) % Q1), z = (int)(e / ((int64_t)Q0 * Q1));
    const c64 v = s * in[((int64_t)z * q.P[1] + y) * q.P[0] + x];
    out[e] = v;
    out32[e] = cvt<float>(v);
  }
}

// One input field of the product over the padded grid ([E3][E2][E1]): f < 3
// the weighted current alpha W_f, f = 3 the cell charge rho.  Inactive faces
// (alpha = 0) contribute nothing.
template <typename T>
__global__ void k_rt_gather(const c64* __restrict__ x, const double* __restrict__ alpha,
                            cpx<T>* __restrict__ out, RtGeom q, int f, double inv_h) {
  const int64_t step[3] = {1, q.E[0], (int64_t)q.E[0] * q.E[1]};
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < q.m;
       c += (int64_t)gridDim.x * blockDim.x) {
    c64 v = mk(0.0, 0.0);
    if (f < 3) {
      v = alpha[f * q.m + c] * x[f * q.m + c];
    } else {
      const int pc[3] = {(int)(c % q.E[0]), (int)((c / q.E[0]) % q.E[1]),
                         (int)(c / ((int64_t)q.E[0] * q.E[1]))};
      for (int i = 0; i < 3; ++i) {
        const int64_t o = i * q.m + c;
        if (alpha[o] != 0.0) v = v + x[o];  // + face of the cell
        if (pc[i] > 0 && alpha[o - step[i]] != 0.0) v = v - x[o - step[i]];  // - face
      }
      v = inv_h * v;
    }
    out[c] = cvt<T>(v);
  }
}

// The z stage with the kernel's spectrum, one workgroup per W neighbouring x
// columns at one y of the y-transformed field t [E3][P2][P1] (rows z < E3
// non-zero): forward z transform (zero half skipped), product with the
// spectrum (1/M folded in), conjugate, forward z transform keeping rows
// z < E3.  With the y and x stages run forward afterwards and a final
// conjugate, that is the inverse transform of the product (the conjugate of
// the forward transform of the conjugate).
template <typename T, int P>
__global__ __launch_bounds__(nt_lines<T>()) void k_rt_zconv(
    const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, const cpx<T>* __restrict__ ghat,
    const cpx<T>* __restrict__ tw, int E3, int P1, int P2, int tiles) {
  constexpr int E = fft_e<P>(), TT = P / E, NT = nt_lines<T>(), W = NT / TT;
  __shared__ cpx<T> lds[W * Pad<P>::LSTR];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = b % tiles, y = b / tiles;
  const int cw = threadIdx.x % W, t = threadIdx.x / W;
  const int col = tile * W + cw;
  const bool valid = col < P1;
  const int64_t plane = (int64_t)P2 * P1;
  const int64_t base = (int64_t)y * P1 + (valid ? col : 0);
  // the spectrum's octant record of this column (mirrored x and y)
  const int Q0 = P1 / 2 + 1, Q1 = P2 / 2 + 1;
  const int xo = valid ? (col <= P1 / 2 ? col : P1 - col) : 0;
  const int yo = y <= P2 / 2 ? y : P2 - y;
  const cpx<T>* gcol = ghat + (int64_t)yo * Q0 + xo;
  const int64_t gplane = (int64_t)Q0 * Q1;
  TwReg<T, P, E> tr;
  tr.load(t, tw);
  cpx<T> v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int row = t + q * TT;
    v[q] = (q < E / 2 && valid && row < E3) ? in[base + row * plane] : mk<T>(0, 0);
  }
  line_fft<T, P, false, true, false>(v, lds + cw * Pad<P>::LSTR, t, tr);
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int z = t + q * TT;
    const cpx<T> p = v[q] * gcol[(int64_t)(z <= P / 2 ? z : P - z) * gplane];
    v[q] = mk(p.re, -p.im);
  }
  line_fft<T, P, false, false, true>(v, lds + cw * Pad<P>::LSTR, t, tr);
  if (valid) {
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int row = t + q * TT;
      if (row < E3) out[base + row * plane] = v[q];
    }
  }
}

// R[c] = conj(t) over the padded grid, t the truncated transform
// [E3][E2][P1] (the inverse transform's result).
template <typename T>
__global__ void k_rt_store(const cpx<T>* __restrict__ t, c64* __restrict__ R, RtGeom q) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < q.m;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % q.E[0]);
    const int64_t yz = c / q.E[0];  // z E2 + y
    const cpx<T> v = t[yz * q.P[0] + x];
    R[c] = mk((double)v.re, -(double)v.im);
  }
}

// y = x - chi_f (k0^2 A_i + (phi(c + e_i) - phi(c)) / h) on active faces,
// y = x on the others.  R holds A_x, A_y, A_z, phi (m each).
__global__ void k_rt_epilogue(const c64* __restrict__ x, const c64* __restrict__ R,
                              const double* __restrict__ chif, c64* __restrict__ y, RtGeom q,
                              double k0sq, double inv_h) {
  const int64_t step[3] = {1, q.E[0], (int64_t)q.E[0] * q.E[1]};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 3 * q.m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double cf = chif[e];
    if (cf == 0.0) {
      y[e] = x[e];
      continue;
    }
    const int i = (int)(e / q.m);
    const int64_t c = e - i * q.m;
    // an active face has its upper cell on the padded grid (c + e_i < m)
    const c64 grad = inv_h * (R[3 * q.m + c + step[i]] - R[3 * q.m + c]);
    const c64 Es = k0sq * R[e] + grad;
    y[e] = x[e] - cf * Es;
  }
}

// b = chi_f pol_i e^{i k0 khat . r_f}, face i of padded cell c at
// origin + h (c - 1) + (h/2) e_i.
__global__ void k_rt_rhs(c64* __restrict__ b, const double* __restrict__ chif, RtGeom q, double h,
                         double o0, double o1, double o2, double k0, double kx, double ky,
                         double kz, c64 p0, c64 p1, c64 p2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 3 * q.m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double cf = chif[e];
    if (cf == 0.0) {
      b[e] = mk(0.0, 0.0);
      continue;
    }
    const int i = (int)(e / q.m);
    const int64_t c = e - i * q.m;
    double r[3] = {o0 + h * ((int)(c % q.E[0]) - 1), o1 + h * ((int)((c / q.E[0]) % q.E[1]) - 1),
                   o2 + h * ((int)(c / ((int64_t)q.E[0] * q.E[1])) - 1)};
    r[i] += 0.5 * h;
    double sn, cs;
    sincos(k0 * (kx * r[0] + ky * r[1] + kz * r[2]), &sn, &cs);
    const c64 pol = i == 0 ? p0 : (i == 1 ? p1 : p2);
    b[e] = cf * (pol * mk(cs, sn));
  }
}

constexpr int kRtThreads = 256;
constexpr int kRtDotBlocks = 256;

// Per-block partial sums of conj(a) . b (fixed reduction order).
__global__ void __launch_bounds__(kRtThreads) k_rt_dot(const c64* __restrict__ a,
                                                       const c64* __restrict__ b, int64_t n,
                                                       c64* __restrict__ part) {
  __shared__ double sr[kRtThreads], si[kRtThreads];
  double re = 0.0, im = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const c64 p = cmulc(a[e], b[e]);
    re += p.re;
    im += p.im;
  }
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int s = kRtThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = mk(sr[0], si[0]);
}

// out = a + ca b + cc c (c nullable)
__global__ void k_rt_lin(c64* __restrict__ out, const c64* __restrict__ a, c64 cb,
                         const c64* __restrict__ b, c64 cc, const c64* __restrict__ c, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    c64 v = cfma(cb, b[e], a[e]);
    if (c) v = cfma(cc, c[e], v);
    out[e] = v;
  }
}

// BiCGSTAB scalars, kept on the device between host checks.
struct RtScal {
  c64 rho, alpha, omega, beta, rho1;
  double tol2;          // tol^2 ||b||^2 (recursive residual threshold)
  int it, max_it;       // iterations done (all cycles), cap
  int stop;             // 0 running, 1 recursive residual reached, 2 breakdown, 3 cap
};
enum { kScRho = 0, kScAlpha = 1, kScOmega = 2, kScRes = 3 };

__device__ __forceinline__ c64 rt_cdiv(c64 a, c64 b) {
  const double d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

__global__ void k_rt_sinit(RtScal* sc, double tol2, int it, int max_it) {
  RtScal S;
  S.rho = S.alpha = S.omega = S.beta = S.rho1 = mk(1.0, 0.0);
  S.tol2 = tol2;
  S.it = it;
  S.max_it = max_it;
  S.stop = 0;
  *sc = S;
}

// Reduces the dot partials of slot 0 (and 1) in a fixed order and takes one
// scalar step of the iteration:
//   kScRho:   rho1 = (rh, r); beta = (rho1 / rho)(alpha / omega)
//   kScAlpha: alpha = rho1 / (rh, v)
//   kScOmega: omega = (t, s) / (t, t); rho = rho1; one iteration done
//   kScRes:   stop when (r, r) <= tol^2 ||b||^2, or after omega = 0
// A zero denominator stops the cycle (breakdown); so does the iteration cap.
__global__ void __launch_bounds__(kRtThreads) k_rt_scal(const c64* __restrict__ part,
                                                        RtScal* __restrict__ sc, int op) {
  __shared__ double red[4][kRtThreads];
  const int i = threadIdx.x;
  const c64 a = part[i];
  const c64 b = op == kScOmega ? part[kRtDotBlocks + i] : mk(0.0, 0.0);
  red[0][i] = a.re;
  red[1][i] = a.im;
  red[2][i] = b.re;
  red[3][i] = b.im;
  __syncthreads();
  for (int st = kRtThreads / 2; st > 0; st >>= 1) {
    if (i < st)
      for (int k = 0; k < 4; ++k) red[k][i] += red[k][i + st];
    __syncthreads();
  }
  if (i != 0) return;
  RtScal S = *sc;
  if (S.stop) return;
  const c64 d0 = mk(red[0][0], red[1][0]);
  const bool zero0 = d0.re == 0.0 && d0.im == 0.0;
  if (op == kScRho) {
    if (S.it >= S.max_it) {
      S.stop = 3;
    } else if (zero0) {
      S.stop = 2;
    } else {
      S.rho1 = d0;
      S.beta = rt_cdiv(d0, S.rho) * rt_cdiv(S.alpha, S.omega);
    }
  } else if (op == kScAlpha) {
    if (zero0)
      S.stop = 2;
    else
      S.alpha = rt_cdiv(S.rho1, d0);
  } else if (op == kScOmega) {
    const double tt = red[2][0];
    S.omega = tt > 0 ? mk(d0.re / tt, d0.im / tt) : mk(0.0, 0.0);
    S.rho = S.rho1;
    S.it += 1;
  } else {
    if (d0.re <= S.tol2)
      S.stop = 1;
    else if (S.omega.re == 0.0 && S.omega.im == 0.0)
      S.stop = 2;
  }
  *sc = S;
}

// p = r + beta (p - omega v)
__global__ void k_rt_pupd(c64* __restrict__ p, const c64* __restrict__ r,
                          const c64* __restrict__ v, const RtScal* __restrict__ sc, int64_t n) {
  if (sc->stop) return;
  const c64 beta = sc->beta, om = sc->omega;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = r[e] + beta * (p[e] - om * v[e]);
}

// s = r - alpha v
__global__ void k_rt_supd(c64* __restrict__ s, const c64* __restrict__ r,
                          const c64* __restrict__ v, const RtScal* __restrict__ sc, int64_t n) {
  if (sc->stop) return;
  const c64 al = sc->alpha;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    s[e] = r[e] - al * v[e];
}

// x = x + alpha p + omega s; r = s - omega t
__global__ void k_rt_xrupd(c64* __restrict__ x, c64* __restrict__ r, const c64* __restrict__ p,
                           const c64* __restrict__ s, const c64* __restrict__ t,
                           const RtScal* __restrict__ sc, int64_t n) {
  if (sc->stop) return;
  const c64 al = sc->alpha, om = sc->omega;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const c64 se = s[e];
    x[e] = x[e] + al * p[e] + om * se;
    r[e] = se - om * t[e];
  }
}

// Far field of eq. 25: one workgroup per (right-hand side, kFarDirs
// directions), S = sum_faces alpha W_i e_i e^{-i k0 r . r_f},
// F = k0^2 h^3 / (4 pi) (t . S, p . S).  The phase factors separate along the
// axes: e^{-i k0 r . r_f} = ax[x] ay[y] az[z] e^{-i k0 r_i h / 2} with
// per-axis tables over the padded grid's cell centres, built in LDS once per
// direction, so a face costs two complex products per direction instead of
// a sincos.  Sums: per thread, then across each wave by shuffles, then over
// the waves in a fixed order.
constexpr int kFarDirs = 8;
constexpr int kFarMaxE = 130;  // padded grid of the largest body (128 + 2)

__global__ void __launch_bounds__(kRtThreads) k_rt_far(const c64* __restrict__ w,
                                                       const double* __restrict__ alpha, RtGeom q,
                                                       double h, double o0, double o1, double o2,
                                                       double k0, const double* __restrict__ th,
                                                       const double* __restrict__ ph, int ndir,
                                                       c64* __restrict__ F) {
  const int ngrp = (ndir + kFarDirs - 1) / kFarDirs;
  const int grp = blockIdx.x % ngrp;
  const int rhs = blockIdx.x / ngrp;
  const int d0 = grp * kFarDirs;
  const int nd = min(kFarDirs, ndir - d0);
  const c64* W = w + (int64_t)rhs * 3 * q.m;
  __shared__ c64 tab[kFarDirs][3][kFarMaxE];
  __shared__ c64 half[kFarDirs][3];
  __shared__ double wsum[kRtThreads / 64][kFarDirs * 6];
  const double o[3] = {o0, o1, o2};
  // per-axis phase tables e^{-i k0 r_a (o_a + h (c - 1))} and half-cell shifts
  for (int k = threadIdx.x; k < kFarDirs * 3 * kFarMaxE; k += blockDim.x) {
    const int d = k / (3 * kFarMaxE), a = (k / kFarMaxE) % 3, c = k % kFarMaxE;
    c64 v = mk(0.0, 0.0);
    if (d < nd && c < q.E[a]) {
      double st, ct, sp, cp;
      sincos(th[d0 + d], &st, &ct);
      sincos(ph[d0 + d], &sp, &cp);
      const double ra = a == 0 ? st * cp : (a == 1 ? st * sp : ct);
      double sn, cs;
      sincos(-k0 * ra * (o[a] + h * (c - 1)), &sn, &cs);
      v = mk(cs, sn);
    }
    tab[d][a][c] = v;
  }
  if (threadIdx.x < kFarDirs * 3) {
    const int d = threadIdx.x / 3, a = threadIdx.x % 3;
    c64 v = mk(1.0, 0.0);
    if (d < nd) {
      double st, ct, sp, cp;
      sincos(th[d0 + d], &st, &ct);
      sincos(ph[d0 + d], &sp, &cp);
      const double ra = a == 0 ? st * cp : (a == 1 ? st * sp : ct);
      double sn, cs;
      sincos(-k0 * ra * 0.5 * h, &sn, &cs);
      v = mk(cs, sn);
    }
    half[d][a] = v;
  }
  __syncthreads();
  double acc[kFarDirs][6];
#pragma unroll
  for (int d = 0; d < kFarDirs; ++d)
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[d][k] = 0.0;
  for (int i = 0; i < 3; ++i) {
    for (int64_t c = threadIdx.x; c < q.m; c += blockDim.x) {
      const double a = alpha[i * q.m + c];
      if (a == 0.0) continue;
      const c64 wv = a * W[i * q.m + c];
      const int cx = (int)(c % q.E[0]);
      const int cy = (int)((c / q.E[0]) % q.E[1]);
      const int cz = (int)(c / ((int64_t)q.E[0] * q.E[1]));
#pragma unroll
      for (int d = 0; d < kFarDirs; ++d) {
        const c64 pz = tab[d][0][cx] * tab[d][1][cy] * tab[d][2][cz] * half[d][i];
        const c64 v = wv * pz;
        acc[d][2 * i] += v.re;
        acc[d][2 * i + 1] += v.im;
      }
    }
  }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
  for (int d = 0; d < kFarDirs; ++d)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double v = acc[d][k];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) wsum[wave][d * 6 + k] = v;
    }
  __syncthreads();
  if (threadIdx.x < nd) {
    const int d = threadIdx.x;
    double S[6];
    for (int k = 0; k < 6; ++k) {
      double v = 0.0;
      for (int wv = 0; wv < kRtThreads / 64; ++wv) v += wsum[wv][d * 6 + k];
      S[k] = v;
    }
    double st, ct, sp, cp;
    sincos(th[d0 + d], &st, &ct);
    sincos(ph[d0 + d], &sp, &cp);
    const double tv[3] = {ct * cp, ct * sp, -st};
    const double pv[3] = {-sp, cp, 0.0};
    const double C = k0 * k0 * h * h * h / (4.0 * M_PI);
    double ftr = 0, fti = 0, fpr = 0, fpi = 0;
    for (int i = 0; i < 3; ++i) {
      ftr += tv[i] * S[2 * i];
      fti += tv[i] * S[2 * i + 1];
      fpr += pv[i] * S[2 * i];
      fpi += pv[i] * S[2 * i + 1];
    }
    F[((int64_t)rhs * ndir + d0 + d) * 2 + 0] = mk(C * ftr, C * fti);
    F[((int64_t)rhs * ndir + d0 + d) * 2 + 1] = mk(C * fpr, C * fpi);
  }
}

}  // namespace vie

using namespace vie;

struct vie_rt {
  int N[3] = {0, 0, 0};
  double h = 0, k0 = 0, origin[3] = {0, 0, 0};
  RtGeom q{};
  GroupGeom g{};
  hipStream_t stream = nullptr;
  bool poisoned = false;
  double* alpha = nullptr;  // [3][m]
  double* chif = nullptr;   // [3][m]
  c64* ghat = nullptr;      // spectrum / M on the octant [0, P/2]^3
  c32* ghat32 = nullptr;    // its FP32 copy
  c64* tw[3] = {nullptr, nullptr, nullptr};
  c32* tw32[3] = {nullptr, nullptr, nullptr};
  c64* work = nullptr;  // [M]
  c64* tmp = nullptr;   // [M]
  c64* c0 = nullptr;    // [m] gathered field
  c64* t1 = nullptr;    // [E3 E2 P1]
  c64* t2 = nullptr;    // [E3 P2 P1]
  c64* t3 = nullptr;    // [E3 P2 P1]
  c64* c1 = nullptr;    // [E3 E2 P1]
  c64* R = nullptr;     // [4][m]
  c64* vec[9] = {};     // solver vectors [3m] each
  c64* part = nullptr;  // dot partials, two slots
  RtScal* sc = nullptr; // device-resident iteration scalars
  std::vector<c64> hpart;
};

namespace {

constexpr int kRtMaxN = 128;

int blocks_for(int64_t n) {
  int64_t b = (n + kRtThreads - 1) / kRtThreads;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 4096);
}

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc((void**)p, count * sizeof(T));
}

void rt_free(vie_rt* r) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(r->alpha);
  f(r->chif);
  f(r->ghat);
  f(r->ghat32);
  for (auto* t : r->tw32) f(t);
  for (auto* t : r->tw) f(t);
  f(r->work);
  f(r->tmp);
  f(r->c0);
  f(r->t1);
  f(r->t2);
  f(r->t3);
  f(r->c1);
  f(r->R);
  for (auto* v : r->vec) f(v);
  f(r->part);
  f(r->sc);
  if (r->stream) (void)hipStreamDestroy(r->stream);
}

#define RT_HIP(call)                 \
  do {                               \
    hipError_t e_ = (call);          \
    if (e_ != hipSuccess) {          \
      r->poisoned = true;            \
      return VIE_EDEVICE;            \
    }                                \
  } while (0)

// y = A x for one full-layout vector (device pointers).  The transforms of
// the four fields run in T (FP64, or FP32 for the inner products of a mixed
// solve); gather, epilogue and y stay FP64.
template <typename T>
int rt_apply_t(vie_rt* r, const c64* x, c64* y) {
  const RtGeom& q = r->q;
  const bool f64 = sizeof(T) == 8;
  const void* tw[3];
  for (int a = 0; a < 3; ++a) tw[a] = f64 ? (const void*)r->tw[a] : (const void*)r->tw32[a];
  const cpx<T>* ghat = (const cpx<T>*)(f64 ? (const void*)r->ghat : (const void*)r->ghat32);
  cpx<T>* c0 = (cpx<T>*)r->c0;
  cpx<T>* t1 = (cpx<T>*)r->t1;
  cpx<T>* t2 = (cpx<T>*)r->t2;
  cpx<T>* t3 = (cpx<T>*)r->t3;
  cpx<T>* c1 = (cpx<T>*)r->c1;
  const double inv_h = 1.0 / r->h;
  const int lpb = lines_per_block<T>(q.P[2]);
  const int tiles = (q.P[0] + lpb - 1) / lpb;
  for (int f = 0; f < 4; ++f) {
    k_rt_gather<T><<<blocks_for(q.m), kRtThreads, 0, r->stream>>>(x, r->alpha, c0, q, f, inv_h);
    RT_HIP(hipGetLastError());
    RT_HIP(launch_fft_xy_pad(c0, t1, t2, q.E, q.P, tw, r->stream));
    auto zconv = [&]() -> hipError_t {
      VIE_DISPATCH_PZ(q.P[2], (k_rt_zconv<T, PP><<<tiles * q.P[1], nt_lines<T>(), 0, r->stream>>>(
                                  t2, t3, ghat, (const cpx<T>*)tw[2], q.E[2], q.P[0], q.P[1],
                                  tiles)));
      return hipGetLastError();
    };
    RT_HIP(zconv());
    RT_HIP(launch_fft_yx_trunc(t3, t1, c1, q.E, q.P, tw, r->stream));
    k_rt_store<T><<<blocks_for(q.m), kRtThreads, 0, r->stream>>>(c1, r->R + f * q.m, q);
    RT_HIP(hipGetLastError());
  }
  k_rt_epilogue<<<blocks_for(3 * q.m), kRtThreads, 0, r->stream>>>(x, r->R, r->chif, y, q,
                                                                   r->k0 * r->k0, inv_h);
  RT_HIP(hipGetLastError());
  return VIE_OK;
}

int rt_apply(vie_rt* r, const c64* x, c64* y, bool fp32 = false) {
  return fp32 ? rt_apply_t<float>(r, x, y) : rt_apply_t<double>(r, x, y);
}

// conj(a) . b over n entries (synchronous).
int rt_dot(vie_rt* r, const c64* a, const c64* b, int64_t n, c64* out) {
  k_rt_dot<<<kRtDotBlocks, kRtThreads, 0, r->stream>>>(a, b, n, r->part);
  RT_HIP(hipGetLastError());
  RT_HIP(hipMemcpyAsync(r->hpart.data(), r->part, kRtDotBlocks * sizeof(c64),
                        hipMemcpyDeviceToHost, r->stream));
  RT_HIP(hipStreamSynchronize(r->stream));
  c64 s = mk(0.0, 0.0);
  for (int k = 0; k < kRtDotBlocks; ++k) s = s + r->hpart[k];
  *out = s;
  return VIE_OK;
}

int rt_lin(vie_rt* r, c64* out, const c64* a, c64 cb, const c64* b, c64 cc, const c64* c,
           int64_t n) {
  k_rt_lin<<<blocks_for(n), kRtThreads, 0, r->stream>>>(out, a, cb, b, cc, c, n);
  RT_HIP(hipGetLastError());
  return VIE_OK;
}

#define RT_TRY(call)          \
  do {                        \
    int rc_ = (call);         \
    if (rc_ != VIE_OK) return rc_; \
  } while (0)

}  // namespace

extern "C" int vie_rt_setup(const vie_body* body, double k0, vie_rt** out) {
  TraceRange trace_("vie_rt_setup");
  if (!out) return VIE_EINVAL;
  *out = nullptr;
  if (!body || !body->eps_r || !(body->h > 0) || !std::isfinite(body->h) || !(k0 > 0) ||
      !std::isfinite(k0))
    return VIE_EINVAL;
  for (int a = 0; a < 3; ++a) {
    if (body->n[a] < 1) return VIE_EINVAL;
    if (!std::isfinite(body->origin[a])) return VIE_EINVAL;
  }
  for (int a = 0; a < 3; ++a)
    if (body->n[a] > kRtMaxN) return VIE_ENOTSUP;
  const int64_t nvox = (int64_t)body->n[0] * body->n[1] * body->n[2];
  for (int64_t v = 0; v < nvox; ++v)
    if (!std::isfinite(body->eps_r[v]) || body->eps_r[v] < 1.0) return VIE_EINVAL;

  vie_rt* r = new (std::nothrow) vie_rt();
  if (!r) return VIE_ENOMEM;
  for (int a = 0; a < 3; ++a) {
    r->N[a] = body->n[a];
    r->origin[a] = body->origin[a];
    r->q.E[a] = body->n[a] + 2;
    r->q.P[a] = rt_fft_length(r->q.E[a]);
    r->g.N[a] = r->q.E[a];
    r->g.P[a] = r->q.P[a];
    r->g.Q[a] = r->q.P[a] / 2 + 1;
  }
  r->h = body->h;
  r->k0 = k0;
  const RtGeom& q = r->q;
  r->q.m = (int64_t)q.E[0] * q.E[1] * q.E[2];
  r->q.M = (int64_t)q.P[0] * q.P[1] * q.P[2];
  r->g.n = r->q.m;
  r->g.nrhs = 1;
  const int64_t m = r->q.m, M = r->q.M;

  // face data: chi on the padded grid, then alpha and chi_f per face
  std::vector<double> chi(m, 0.0), alpha(3 * m, 0.0), chif(3 * m, 0.0);
  for (int z = 0; z < r->N[2]; ++z)
    for (int y = 0; y < r->N[1]; ++y)
      for (int x = 0; x < r->N[0]; ++x)
        chi[((int64_t)(z + 1) * q.E[1] + (y + 1)) * q.E[0] + (x + 1)] =
            body->eps_r[((int64_t)z * r->N[1] + y) * r->N[0] + x] - 1.0;
  const int64_t step[3] = {1, q.E[0], (int64_t)q.E[0] * q.E[1]};
  for (int i = 0; i < 3; ++i)
    for (int z = 0; z < q.E[2]; ++z)
      for (int y = 0; y < q.E[1]; ++y)
        for (int x = 0; x < q.E[0]; ++x) {
          const int pc[3] = {x, y, z};
          const int64_t c = ((int64_t)z * q.E[1] + y) * q.E[0] + x;
          const double ca = chi[c];
          const double cb = pc[i] + 1 < q.E[i] ? chi[c + step[i]] : 0.0;
          double a = 0.0, cf = 0.0;
          if (ca != 0.0 && cb != 0.0) {
            a = 1.0;
            cf = 1.0 / (0.5 * (1.0 / ca + 1.0 / cb));
          } else if (ca != 0.0) {
            a = 0.5;
            cf = ca;
          } else if (cb != 0.0) {
            a = 0.5;
            cf = cb;
          }
          alpha[i * m + c] = a;
          chif[i * m + c] = cf;
        }

  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chk(hipStreamCreate(&r->stream));
  chk(dalloc(&r->alpha, 3 * m));
  chk(dalloc(&r->chif, 3 * m));
  const int64_t noct = (int64_t)(q.P[0] / 2 + 1) * (q.P[1] / 2 + 1) * (q.P[2] / 2 + 1);
  chk(dalloc(&r->ghat, noct));
  chk(dalloc(&r->ghat32, noct));
  chk(dalloc(&r->work, M));
  chk(dalloc(&r->tmp, M));
  chk(dalloc(&r->R, 4 * m));
  chk(dalloc(&r->c0, m));
  chk(dalloc(&r->t1, (size_t)q.E[2] * q.E[1] * q.P[0]));
  chk(dalloc(&r->t2, (size_t)q.E[2] * q.P[1] * q.P[0]));
  chk(dalloc(&r->t3, (size_t)q.E[2] * q.P[1] * q.P[0]));
  chk(dalloc(&r->c1, (size_t)q.E[2] * q.E[1] * q.P[0]));
  for (auto& v : r->vec) chk(dalloc(&v, 3 * m));
  chk(dalloc(&r->part, 2 * kRtDotBlocks));
  chk(dalloc(&r->sc, 1));
  for (int a = 0; a < 3; ++a) chk(dalloc(&r->tw[a], q.P[a]));
  for (int a = 0; a < 3; ++a) chk(dalloc(&r->tw32[a], q.P[a]));
  if (e != hipSuccess) {
    rt_free(r);
    delete r;
    return e == hipErrorOutOfMemory ? VIE_ENOMEM : VIE_EDEVICE;
  }
  r->hpart.resize(kRtDotBlocks);
  for (int a = 0; a < 3; ++a) {
    std::vector<c64> t(q.P[a]);
    std::vector<c32> t32(q.P[a]);
    for (int k = 0; k < q.P[a]; ++k) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * k / q.P[a];
      t[k] = mk((double)cosl(ang), (double)sinl(ang));
      t32[k] = mk((float)cosl(ang), (float)sinl(ang));
    }
    chk(hipMemcpy(r->tw[a], t.data(), q.P[a] * sizeof(c64), hipMemcpyHostToDevice));
    chk(hipMemcpy(r->tw32[a], t32.data(), q.P[a] * sizeof(c32), hipMemcpyHostToDevice));
  }
  chk(hipMemcpy(r->alpha, alpha.data(), 3 * m * sizeof(double), hipMemcpyHostToDevice));
  chk(hipMemcpy(r->chif, chif.data(), 3 * m * sizeof(double), hipMemcpyHostToDevice));
  double s_re, s_im;
  cube_green_integral(k0, r->h, &s_re, &s_im);
  const void* tw[3] = {r->tw[0], r->tw[1], r->tw[2]};
  if (e == hipSuccess) {
    k_rt_green<<<blocks_for(M), kRtThreads, 0, r->stream>>>(r->work, q, r->h, k0, s_re, s_im);
    chk(hipGetLastError());
  }
  if (e == hipSuccess) chk(launch_fft3d_full(r->work, r->tmp, r->g, tw, r->stream));
  if (e == hipSuccess) {
    k_rt_octant<<<blocks_for(noct), kRtThreads, 0, r->stream>>>(r->tmp, r->ghat, r->ghat32, q,
                                                                   1.0 / (double)M);
    chk(hipGetLastError());
  }
  if (e == hipSuccess) chk(hipStreamSynchronize(r->stream));
  if (e != hipSuccess) {
    rt_free(r);
    delete r;
    return VIE_EDEVICE;
  }
  // the full circulant buffers serve the spectrum only
  (void)hipFree(r->work);
  (void)hipFree(r->tmp);
  r->work = r->tmp = nullptr;
  *out = r;
  return VIE_OK;
}

extern "C" int vie_rt_grid(const vie_rt* r, int32_t* ext, int32_t* fft) {
  if (!r) return VIE_EINVAL;
  for (int a = 0; a < 3; ++a) {
    if (ext) ext[a] = r->q.E[a];
    if (fft) fft[a] = r->q.P[a];
  }
  return VIE_OK;
}

extern "C" int vie_rt_matvec(vie_rt* r, const vie_c64* x, vie_c64* y, int32_t nvec,
                             int32_t precision) {
  if (!r || !x || !y || nvec < 1 || (precision != VIE_FP64 && precision != VIE_MIXED))
    return VIE_EINVAL;
  if (r->poisoned) return VIE_ESTATE;
  const int64_t n = 3 * r->q.m;
  for (int v = 0; v < nvec; ++v) {
    RT_HIP(hipMemcpyAsync(r->vec[0], x + v * n, n * sizeof(c64), hipMemcpyHostToDevice,
                          r->stream));
    RT_TRY(rt_apply(r, r->vec[0], r->vec[1], precision == VIE_MIXED));
    RT_HIP(hipMemcpyAsync(y + v * n, r->vec[1], n * sizeof(c64), hipMemcpyDeviceToHost,
                          r->stream));
    RT_HIP(hipStreamSynchronize(r->stream));
  }
  return VIE_OK;
}

extern "C" int vie_rt_solve(vie_rt* r, const vie_planewave* inc, int32_t nrhs, double tol,
                            int32_t max_iter, int32_t precision, vie_c64* w, vie_stats* stats) {
  TraceRange trace_("vie_rt_solve");
  if (!r || !inc || !w || nrhs < 1 || !(tol > 0) || !(tol < 1) || max_iter < 1 ||
      (precision != VIE_FP64 && precision != VIE_MIXED))
    return VIE_EINVAL;
  const bool mixed = precision == VIE_MIXED;
  constexpr double kInnerTol = 1e-3;  // residual reduction per refinement cycle (mixed)
  if (r->poisoned) return VIE_ESTATE;
  for (int k = 0; k < nrhs; ++k)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(inc[k].khat[a]) || !std::isfinite(inc[k].pol[a].re) ||
          !std::isfinite(inc[k].pol[a].im))
        return VIE_EINVAL;
  const RtGeom& q = r->q;
  const int64_t n = 3 * q.m;
  c64 *x = r->vec[0], *b = r->vec[1], *rr = r->vec[2], *rh = r->vec[3], *p = r->vec[4],
      *v = r->vec[5], *s = r->vec[6], *t = r->vec[7];
  const c64 zero = mk(0.0, 0.0);
  int status = VIE_OK;
  for (int k = 0; k < nrhs; ++k) {
    const auto t0 = std::chrono::steady_clock::now();
    const vie_planewave& pw = inc[k];
    k_rt_rhs<<<blocks_for(n), kRtThreads, 0, r->stream>>>(
        b, r->chif, q, r->h, r->origin[0], r->origin[1], r->origin[2], r->k0, pw.khat[0],
        pw.khat[1], pw.khat[2], mk(pw.pol[0].re, pw.pol[0].im), mk(pw.pol[1].re, pw.pol[1].im),
        mk(pw.pol[2].re, pw.pol[2].im));
    RT_HIP(hipGetLastError());
    RT_HIP(hipMemsetAsync(x, 0, n * sizeof(c64), r->stream));
    c64 bb;
    RT_TRY(rt_dot(r, b, b, n, &bb));
    const double bnorm = sqrt(bb.re);
    vie_stats st{};
    st.rel_res_x0 = 1.0;
    st.cycles = 0;
    double rel = bnorm > 0 ? 1.0 : 0.0;
    int it = 0, mv = 0;
    bool conv = bnorm == 0.0;
    while (!conv && it < max_iter) {
      // (re)start from the true residual
      if (st.cycles > 0) {
        RT_TRY(rt_apply(r, x, t));
        ++mv;
        RT_TRY(rt_lin(r, rr, b, mk(-1.0, 0.0), t, zero, nullptr, n));
      } else {
        RT_HIP(hipMemcpyAsync(rr, b, n * sizeof(c64), hipMemcpyDeviceToDevice, r->stream));
      }
      ++st.cycles;
      RT_HIP(hipMemcpyAsync(rh, rr, n * sizeof(c64), hipMemcpyDeviceToDevice, r->stream));
      RT_HIP(hipMemsetAsync(p, 0, n * sizeof(c64), r->stream));
      RT_HIP(hipMemsetAsync(v, 0, n * sizeof(c64), r->stream));
      // the cycle's target: tol ||b||, and for a mixed solve no deeper than
      // kInnerTol times its starting residual (the FP32 products' accuracy)
      double tol2 = tol * tol * bb.re;
      if (mixed) {
        c64 r0;
        RT_TRY(rt_dot(r, rr, rr, n, &r0));
        tol2 = std::max(tol2, kInnerTol * kInnerTol * r0.re);
      }
      k_rt_sinit<<<1, 1, 0, r->stream>>>(r->sc, tol2, it, max_iter);
      RT_HIP(hipGetLastError());
      // iterations run in chunks with the scalars on the device; the host
      // looks at them once per chunk (iterations after a stop are no-ops)
      constexpr int kChunk = 8;
      const int it0 = it;
      RtScal S{};
      for (;;) {
        for (int j = 0; j < kChunk; ++j) {
          k_rt_dot<<<kRtDotBlocks, kRtThreads, 0, r->stream>>>(rh, rr, n, r->part);
          k_rt_scal<<<1, kRtThreads, 0, r->stream>>>(r->part, r->sc, kScRho);
          k_rt_pupd<<<blocks_for(n), kRtThreads, 0, r->stream>>>(p, rr, v, r->sc, n);
          RT_HIP(hipGetLastError());
          RT_TRY(rt_apply(r, p, v, mixed));
          k_rt_dot<<<kRtDotBlocks, kRtThreads, 0, r->stream>>>(rh, v, n, r->part);
          k_rt_scal<<<1, kRtThreads, 0, r->stream>>>(r->part, r->sc, kScAlpha);
          k_rt_supd<<<blocks_for(n), kRtThreads, 0, r->stream>>>(s, rr, v, r->sc, n);
          RT_HIP(hipGetLastError());
          RT_TRY(rt_apply(r, s, t, mixed));
          k_rt_dot<<<kRtDotBlocks, kRtThreads, 0, r->stream>>>(t, s, n, r->part);
          k_rt_dot<<<kRtDotBlocks, kRtThreads, 0, r->stream>>>(t, t, n, r->part + kRtDotBlocks);
          k_rt_scal<<<1, kRtThreads, 0, r->stream>>>(r->part, r->sc, kScOmega);
          k_rt_xrupd<<<blocks_for(n), kRtThreads, 0, r->stream>>>(x, rr, p, s, t, r->sc, n);
          k_rt_dot<<<kRtDotBlocks, kRtThreads, 0, r->stream>>>(rr, rr, n, r->part);
          k_rt_scal<<<1, kRtThreads, 0, r->stream>>>(r->part, r->sc, kScRes);
          RT_HIP(hipGetLastError());
        }
        RT_HIP(hipMemcpyAsync(&S, r->sc, sizeof(RtScal), hipMemcpyDeviceToHost, r->stream));
        RT_HIP(hipStreamSynchronize(r->stream));
        if (S.stop) break;
      }
      it = S.it;
      mv += 2 * (it - it0);
      // true residual decides
      RT_TRY(rt_apply(r, x, t));
      ++mv;
      RT_TRY(rt_lin(r, t, b, mk(-1.0, 0.0), t, zero, nullptr, n));
      c64 r2;
      RT_TRY(rt_dot(r, t, t, n, &r2));
      rel = sqrt(r2.re) / bnorm;
      conv = rel <= tol;
      // the cap, or a cycle that could not take a single step, ends the solve;
      // otherwise restart from the true residual
      if (S.stop == 3 || it == it0) break;
    }
    RT_HIP(hipMemcpyAsync(w + k * n, x, n * sizeof(c64), hipMemcpyDeviceToHost, r->stream));
    RT_HIP(hipStreamSynchronize(r->stream));
    const double sec =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    st.iters = it;
    st.matvecs = mv;
    st.converged = conv ? 1 : 0;
    st.rel_res = rel;
    st.seconds = conv ? sec : 0.0;
    if (stats) stats[k] = st;
    if (!conv) status = VIE_ENOCONV;
  }
  return status;
}

extern "C" int vie_rt_farfield(vie_rt* r, const vie_c64* w, int32_t nrhs, const double* theta,
                               const double* phi, int32_t ndir, vie_c64* F) {
  TraceRange trace_("vie_rt_farfield");
  if (!r || !w || !theta || !phi || !F || nrhs < 1 || ndir < 1) return VIE_EINVAL;
  if (r->poisoned) return VIE_ESTATE;
  for (int d = 0; d < ndir; ++d)
    if (!std::isfinite(theta[d]) || !std::isfinite(phi[d])) return VIE_EINVAL;
  if ((int64_t)nrhs * ndir > (int64_t)1 << 30) return VIE_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (r->q.E[a] > kFarMaxE) return VIE_ENOTSUP;  // not reached: setup caps the grid
  const int64_t n = 3 * r->q.m;
  c64* dw = nullptr;
  double *dth = nullptr, *dph = nullptr;
  c64* dF = nullptr;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chk(dalloc(&dw, (size_t)nrhs * n));
  chk(dalloc(&dth, ndir));
  chk(dalloc(&dph, ndir));
  chk(dalloc(&dF, (size_t)nrhs * ndir * 2));
  if (e == hipSuccess) {
    chk(hipMemcpyAsync(dw, w, (size_t)nrhs * n * sizeof(c64), hipMemcpyHostToDevice, r->stream));
    chk(hipMemcpyAsync(dth, theta, ndir * sizeof(double), hipMemcpyHostToDevice, r->stream));
    chk(hipMemcpyAsync(dph, phi, ndir * sizeof(double), hipMemcpyHostToDevice, r->stream));
  }
  if (e == hipSuccess) {
    const int ngrp = (ndir + kFarDirs - 1) / kFarDirs;
    k_rt_far<<<nrhs * ngrp, kRtThreads, 0, r->stream>>>(dw, r->alpha, r->q, r->h, r->origin[0],
                                                        r->origin[1], r->origin[2], r->k0, dth,
                                                        dph, ndir, dF);
    chk(hipGetLastError());
  }
  if (e == hipSuccess)
    chk(hipMemcpyAsync(F, dF, (size_t)nrhs * ndir * 2 * sizeof(c64), hipMemcpyDeviceToHost,
                       r->stream));
  if (e == hipSuccess) chk(hipStreamSynchronize(r->stream));
  (void)hipFree(dw);
  (void)hipFree(dth);
  (void)hipFree(dph);
  (void)hipFree(dF);
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) return VIE_ENOMEM;
    r->poisoned = true;
    return VIE_EDEVICE;
  }
  return VIE_OK;
}

extern "C" void vie_rt_destroy(vie_rt* r) {
  if (!r) return;
  if (r->stream) (void)hipStreamSynchronize(r->stream);
  rt_free(r);
  delete r;
}
