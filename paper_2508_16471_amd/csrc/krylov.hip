// BiCGSTAB vector kernels (van der Vorst 1992, the paper's Krylov solver,
// Sec. II-C) with device-resident scalars, fused updates and two-stage
// deterministic reductions: each workgroup writes a partial sum, a
// one-workgroup-per-right-hand-side finalize kernel folds them in fixed order
// and updates alpha, omega, rho, beta and the convergence flags.  No host
// round trip is needed inside an iteration.
//
// Vectors: FP64 complex, [rhs][3][N3][N2][N1] (3n per right-hand side).
// flags[rhs] = active (iterating), flags[nrhs + rhs] = not yet converged.
#include "kernels.h"

namespace vie {

static constexpr int VT = 256;  // threads per vector-kernel workgroup

int vec_blocks_n(int64_t m) {
  int64_t b = (m + 4 * VT - 1) / (4 * VT);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

__device__ __forceinline__ void block_reduce2(c64& a, c64& b) {
  __shared__ double red[4 * (VT / 64)];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a.re += __shfl_xor(a.re, off, 64);
    a.im += __shfl_xor(a.im, off, 64);
    b.re += __shfl_xor(b.re, off, 64);
    b.im += __shfl_xor(b.im, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[wv * 4 + 0] = a.re;
    red[wv * 4 + 1] = a.im;
    red[wv * 4 + 2] = b.re;
    red[wv * 4 + 3] = b.im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c64 sa = mk(0.0, 0.0), sb = mk(0.0, 0.0);
    for (int w = 0; w < VT / 64; ++w) {
      sa.re += red[w * 4 + 0];
      sa.im += red[w * 4 + 1];
      sb.re += red[w * 4 + 2];
      sb.im += red[w * 4 + 3];
    }
    a = sa;
    b = sb;
  }
}

// Vectors are body-compressed: right-hand side r holds 3 nb values at roff[r],
// component-major.  Each kernel strides its workgroups over that range.
struct VecRange {
  int64_t base, len;
  int nb, body;
};
__device__ __forceinline__ VecRange vrange(const BodyIdx& bi, int rhs) {
  VecRange v;
  v.body = bi.rhs_body[rhs];
  v.nb = bi.nb[v.body];
  v.base = bi.roff[rhs];
  v.len = 3 * (int64_t)v.nb;
  return v;
}

// x = 0, r = rhat = b = chi pol exp(i k0 khat.r); partials (rhat.r, |r|^2)
__global__ __launch_bounds__(VT) void k_init_zero(GroupGeom g, BodyIdx bi,
                                                  const c64* __restrict__ pol,
                                                  const c64* __restrict__ ph, c64* __restrict__ x,
                                                  c64* __restrict__ r, c64* __restrict__ rh,
                                                  c64* __restrict__ partials, int vb,
                                                  int keep_x, const int* __restrict__ mask) {
  const int rhs = blockIdx.x / vb, blk = blockIdx.x % vb;
  if (mask && !mask[rhs]) return;
  const VecRange R = vrange(bi, rhs);
  const int* vox = bi.vox + bi.voff[R.body];
  const double* chic = bi.chic + bi.voff[R.body];
  const c64* p = ph + (int64_t)rhs * (g.N[0] + g.N[1] + g.N[2]);
  c64 s1 = mk(0.0, 0.0), s0 = mk(0.0, 0.0);
  for (int64_t e = (int64_t)blk * VT + threadIdx.x; e < R.len; e += (int64_t)vb * VT) {
    const int comp = (int)(e / R.nb);
    const int k = (int)(e - (int64_t)comp * R.nb);
    const int v = vox[k];
    const int i = v % g.N[0];
    const int j = (v / g.N[0]) % g.N[1];
    const int l = v / (g.N[0] * g.N[1]);
    const c64 phase = p[i] * p[g.N[0] + j] * p[g.N[0] + g.N[1] + l];
    const c64 b = chic[k] * (pol[rhs * 3 + comp] * phase);
    if (!keep_x) x[R.base + e] = mk(0.0, 0.0);
    r[R.base + e] = b;
    rh[R.base + e] = b;
    s1.re += b.re * b.re + b.im * b.im;
  }
  s0 = s1;
  block_reduce2(s0, s1);
  if (threadIdx.x == 0) {
    partials[((size_t)rhs * vb + blk) * 2 + 0] = s0;
    partials[((size_t)rhs * vb + blk) * 2 + 1] = s1;
  }
}

// p = r + beta (p - omega v); p = r at the start of a cycle
__global__ __launch_bounds__(VT) void k_update_p(BodyIdx bi, const KState* __restrict__ st,
                                                 const int* __restrict__ active,
                                                 const c64* __restrict__ r, c64* __restrict__ p,
                                                 const c64* __restrict__ v, int vb) {
  const int rhs = blockIdx.x / vb, blk = blockIdx.x % vb;
  if (!active[rhs]) return;
  const VecRange R = vrange(bi, rhs);
  const bool first = st[rhs].it_cycle == 0;
  const c64 beta = st[rhs].beta, om = st[rhs].omega;
  for (int64_t e = (int64_t)blk * VT + threadIdx.x; e < R.len; e += (int64_t)vb * VT) {
    const int64_t k = R.base + e;
    p[k] = first ? r[k] : r[k] + beta * (p[k] - om * v[k]);
  }
}

// s = r - alpha v
__global__ __launch_bounds__(VT) void k_update_s(BodyIdx bi, const KState* __restrict__ st,
                                                 const int* __restrict__ active,
                                                 const c64* __restrict__ r,
                                                 const c64* __restrict__ v, c64* __restrict__ s,
                                                 int vb) {
  const int rhs = blockIdx.x / vb, blk = blockIdx.x % vb;
  if (!active[rhs]) return;
  const VecRange R = vrange(bi, rhs);
  const c64 al = st[rhs].alpha;
  for (int64_t e = (int64_t)blk * VT + threadIdx.x; e < R.len; e += (int64_t)vb * VT) {
    const int64_t k = R.base + e;
    s[k] = r[k] - al * v[k];
  }
}

// x += alpha p + omega s; r = s - omega t; partials (rhat.r, |r|^2)
__global__ __launch_bounds__(VT) void k_update_xr(BodyIdx bi, const KState* __restrict__ st,
                                                  const int* __restrict__ active,
                                                  c64* __restrict__ x, c64* __restrict__ r,
                                                  const c64* __restrict__ p,
                                                  const c64* __restrict__ s,
                                                  const c64* __restrict__ t,
                                                  const c64* __restrict__ rh,
                                                  c64* __restrict__ partials, int vb) {
  const int rhs = blockIdx.x / vb, blk = blockIdx.x % vb;
  if (!active[rhs]) return;
  const VecRange R = vrange(bi, rhs);
  const c64 al = st[rhs].alpha, om = st[rhs].omega;
  c64 s0 = mk(0.0, 0.0), s1 = mk(0.0, 0.0);
  for (int64_t e = (int64_t)blk * VT + threadIdx.x; e < R.len; e += (int64_t)vb * VT) {
    const int64_t k = R.base + e;
    const c64 sk = s[k];
    x[k] = x[k] + al * p[k] + om * sk;
    const c64 rk = sk - om * t[k];
    r[k] = rk;
    s0 = s0 + cmulc(rh[k], rk);
    s1.re += rk.re * rk.re + rk.im * rk.im;
  }
  block_reduce2(s0, s1);
  if (threadIdx.x == 0) {
    partials[((size_t)rhs * vb + blk) * 2 + 0] = s0;
    partials[((size_t)rhs * vb + blk) * 2 + 1] = s1;
  }
}

// squared norm of every right-hand side's vector (one workgroup each)
__global__ __launch_bounds__(VT) void k_vec_norm2(BodyIdx bi, const c64* __restrict__ v,
                                                  double* __restrict__ out) {
  const int rhs = blockIdx.x;
  const VecRange R = vrange(bi, rhs);
  c64 a = mk(0.0, 0.0), b = mk(0.0, 0.0);
  for (int64_t e = threadIdx.x; e < R.len; e += VT) {
    const c64 x = v[R.base + e];
    a.re += x.re * x.re + x.im * x.im;
  }
  block_reduce2(a, b);
  if (threadIdx.x == 0) out[rhs] = a.re;
}

// body-compressed gather of a box-layout vector
__global__ __launch_bounds__(VT) void k_compress(const c64* __restrict__ box, c64* __restrict__ out,
                                                 const int* __restrict__ vox, int nb, int64_t n) {
  const int64_t m = 3 * (int64_t)nb;
  for (int64_t e = (int64_t)blockIdx.x * VT + threadIdx.x; e < m; e += (int64_t)gridDim.x * VT) {
    const int comp = (int)(e / nb);
    const int k = (int)(e - (int64_t)comp * nb);
    out[e] = box[comp * n + vox[k]];
  }
}

__device__ __forceinline__ c64 cdiv(c64 a, c64 b) {
  const double d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
__device__ __forceinline__ double cabs2(c64 a) { return a.re * a.re + a.im * a.im; }

__global__ __launch_bounds__(VT) void k_finalize(int which, int nrhs, int nblk,
                                                 const c64* __restrict__ partials,
                                                 KState* __restrict__ st, int* __restrict__ flags,
                                                 FinParams fp) {
  const int rhs = blockIdx.x;
  KState& S = st[rhs];
  // flags: [0, nrhs) active, [nrhs, 2 nrhs) not done, [2 nrhs, 3 nrhs) cycle
  // ended and waiting for its true residual
  const bool gate = (which == FIN_RESTART)   ? flags[nrhs + rhs] != 0
                    : (which == FIN_PENDING) ? flags[2 * nrhs + rhs] != 0
                    : (which == FIN_INIT)    ? true
                                             : flags[rhs] != 0;
  if (!gate) return;
  c64 a = mk(0.0, 0.0), b = mk(0.0, 0.0);
  for (int k = threadIdx.x; k < nblk; k += VT) {
    a = a + partials[((size_t)rhs * nblk + k) * 2 + 0];
    b = b + partials[((size_t)rhs * nblk + k) * 2 + 1];
  }
  block_reduce2(a, b);
  if (threadIdx.x != 0) return;
  switch (which) {
    case FIN_ALPHA: {
      const c64 rhv = a;
      // Only an exact zero (or overflow) is a breakdown: rhat . A p and
      // rhat . r carry the product of the omegas, so their ratio to
      // |rhat| |r| decays geometrically in a healthy iteration and any fixed
      // relative threshold would restart it (losing the Krylov space) for
      // no reason on slowly converging problems.
      if (cabs2(rhv) == 0.0 || !(cabs2(rhv) < 1e300)) {
        S.breakdown = 1;  // rhat . A p vanished
        S.active = 0;
        flags[rhs] = 0;
        flags[2 * nrhs + rhs] = 1;
      } else {
        S.alpha = cdiv(S.rho, rhv);
      }
      break;
    }
    case FIN_OMEGA: {
      const double tt = b.re;
      S.omega = tt > 0 ? mk(a.re / tt, a.im / tt) : mk(0.0, 0.0);
      break;
    }
    case FIN_RHO: {
      S.rho_prev = S.rho;
      S.rho = a;
      S.rnorm2 = b.re;
      S.iters += 1;
      S.it_cycle += 1;
      int stop = 0;
      if (!(S.rnorm2 <= 1e300)) {  // NaN / overflow: end the cycle, restart from x
        stop = 1;
        S.breakdown = 4;
      } else if (S.rnorm2 <= S.target2) {
        stop = 1;
      } else if (S.iters >= fp.max_iter) {
        stop = 1;
      } else if (cabs2(S.rho) == 0.0 || cabs2(S.omega) == 0.0) {
        stop = 1;
        S.breakdown = cabs2(S.omega) == 0.0 ? 3 : 2;  // omega = 0 / rhat . r vanished
      } else {
        S.beta = cdiv(S.rho, S.rho_prev) * cdiv(S.alpha, S.omega);
      }
      if (stop) {
        S.active = 0;
        flags[rhs] = 0;
        flags[2 * nrhs + rhs] = 1;
      }
      break;
    }
    case FIN_INIT:
    case FIN_RESTART:
    case FIN_PENDING: {
      if (which == FIN_INIT) {
        S.bnorm2 = b.re;
        S.iters = 0;
        S.cycles = 0;
      } else {
        S.cycles += 1;  // one FP64 residual product ran for this right-hand side
      }
      S.rnorm2 = b.re;
      S.rh2 = b.re;
      S.rho = mk(b.re, 0.0);  // rhat = r
      S.rho_prev = S.alpha = S.omega = S.beta = mk(1.0, 0.0);
      S.it_cycle = 0;
      S.breakdown = 0;
      const double done2 = fp.tol2_done * S.bnorm2;
      const double t_in = fp.tol2_inner * S.bnorm2, t_eta = fp.eta2 * S.rnorm2;
      S.target2 = t_in > t_eta ? t_in : t_eta;
      S.notdone = (S.rnorm2 > done2) || !(S.rnorm2 <= 1e300);
      // completion time: the first true residual at or below tol
      if (which == FIN_INIT) S.t_done = 0;
      if (!S.notdone && S.t_done == 0) S.t_done = wall_clock64();
      S.active = (S.notdone && S.iters < fp.max_iter && S.rnorm2 <= 1e300) ? 1 : 0;
      flags[rhs] = S.active;
      flags[nrhs + rhs] = S.notdone;
      flags[2 * nrhs + rhs] = 0;
      break;
    }
  }
}

__global__ __launch_bounds__(VT) void k_axpy_real(int64_t n, double a, const c64* __restrict__ x,
                                                  c64* __restrict__ y) {
  for (int64_t e = (int64_t)blockIdx.x * VT + threadIdx.x; e < n; e += (int64_t)gridDim.x * VT)
    y[e] = y[e] + a * x[e];
}

hipError_t launch_init_zero_guess(const GroupGeom& g, const BodyIdx& bi, int vb,
                                  const c64* pol, const c64* ph, c64* x, c64* r, c64* rh,
                                  c64* partials, int keep_x, const int* mask, hipStream_t s) {
  k_init_zero<<<vb * g.nrhs, VT, 0, s>>>(g, bi, pol, ph, x, r, rh, partials, vb, keep_x, mask);
  return hipGetLastError();
}
hipError_t launch_update_p(const GroupGeom& g, const BodyIdx& bi, int vb, const KState* st,
                           const int* active, const c64* r, c64* p, const c64* v, hipStream_t s) {
  k_update_p<<<vb * g.nrhs, VT, 0, s>>>(bi, st, active, r, p, v, vb);
  return hipGetLastError();
}
hipError_t launch_update_s(const GroupGeom& g, const BodyIdx& bi, int vb, const KState* st,
                           const int* active, const c64* r, const c64* v, c64* so,
                           hipStream_t s) {
  k_update_s<<<vb * g.nrhs, VT, 0, s>>>(bi, st, active, r, v, so, vb);
  return hipGetLastError();
}
hipError_t launch_update_xr(const GroupGeom& g, const BodyIdx& bi, int vb, const KState* st,
                            const int* active, c64* x, c64* r, const c64* p, const c64* sv,
                            const c64* t, const c64* rh, c64* partials, hipStream_t s) {
  k_update_xr<<<vb * g.nrhs, VT, 0, s>>>(bi, st, active, x, r, p, sv, t, rh, partials, vb);
  return hipGetLastError();
}
hipError_t launch_vec_norm2(int nrhs, const BodyIdx& bi, const c64* v, double* out,
                           hipStream_t s) {
  k_vec_norm2<<<nrhs, VT, 0, s>>>(bi, v, out);
  return hipGetLastError();
}
__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_stamp(unsigned long long* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = wall_clock64();
}
hipError_t launch_stamp(unsigned long long* out, hipStream_t s) {
  k_stamp<<<1, 64, 0, s>>>(out);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s) {
  if (n < 1) return hipSuccess;
  k_fill_int<<<(n + VT - 1) / VT, VT, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_compress(const c64* box, c64* comp, const int* vox, int nb, int64_t n,
                           hipStream_t s) {
  int64_t b = (3 * (int64_t)nb + VT - 1) / VT;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  k_compress<<<(int)b, VT, 0, s>>>(box, comp, vox, nb, n);
  return hipGetLastError();
}
hipError_t launch_finalize(int which, int nrhs, int nblk, const c64* partials, KState* st,
                           int* flags, const FinParams& fp, hipStream_t s) {
  k_finalize<<<nrhs, VT, 0, s>>>(which, nrhs, nblk, partials, st, flags, fp);
  return hipGetLastError();
}
hipError_t launch_axpy_real(int64_t n, double a, const c64* x, c64* y, hipStream_t s) {
  int64_t b = (n + VT - 1) / VT;
  if (b > 4096) b = 4096;
  k_axpy_real<<<(int)b, VT, 0, s>>>(n, a, x, y);
  return hipGetLastError();
}

}  // namespace vie
