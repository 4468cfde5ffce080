// Line FFTs for gfx950: register radix-2/3/4/8/12/16 DFTs and Stockham
// (self-sorting) stages exchanged through LDS.  Line lengths are 2^k or
// 3 * 2^k.
//
// A line of P points is handled by T = P / E threads, each holding E points.
// On entry thread t holds x[t + q T] (q = 0..E-1) and on exit X[t + q T], so
// the first stage reads and the last stage writes the line with unit stride
// across threads: global loads/stores of a line are coalesced without any
// reordering pass.  Intermediate stages use Stockham indexing: stage with
// sub-transform length Ns and radix R reads a[j + r P/R] and writes
// a[(j / Ns) Ns R + j % Ns + r Ns] (j = butterfly index, k = j % Ns twiddle
// exponent), which self-sorts the output.
#pragma once

#include "common.h"

namespace vie {

// exp(-2 pi i m / 16) components, m = 0..15
template <typename T>
__host__ __device__ __forceinline__ constexpr T cos16(int m) {
  constexpr double c1 = 0.92387953251128675613, c2 = 0.70710678118654752440,
                   c3 = 0.38268343236508977173;
  switch (m & 15) {
    case 0: return (T)1.0;
    case 1: return (T)c1;
    case 2: return (T)c2;
    case 3: return (T)c3;
    case 4: return (T)0.0;
    case 5: return (T)-c3;
    case 6: return (T)-c2;
    case 7: return (T)-c1;
    case 8: return (T)-1.0;
    case 9: return (T)-c1;
    case 10: return (T)-c2;
    case 11: return (T)-c3;
    case 12: return (T)0.0;
    case 13: return (T)c3;
    case 14: return (T)c2;
    default: return (T)c1;
  }
}
template <typename T>
__host__ __device__ __forceinline__ constexpr T sin16(int m) {
  return cos16<T>(m + 12);  // sin(a) = cos(a - pi/2) = cos(2 pi (m - 4)/16)
}

// multiply by W_R^m = exp(-+2 pi i m / R), R divides 16, compile-time m after unrolling
template <int R, bool INV, typename T>
__host__ __device__ __forceinline__ cpx<T> twc(cpx<T> a, int m) {
  const int mm = (m * (16 / R)) & 15;
  if (mm == 0) return a;
  if (mm == 8) return mk(-a.re, -a.im);
  if (mm == 4) return INV ? mk(-a.im, a.re) : mk(a.im, -a.re);    // * (+-i)
  if (mm == 12) return INV ? mk(a.im, -a.re) : mk(-a.im, a.re);
  const T c = cos16<T>(mm);
  const T s = INV ? sin16<T>(mm) : -sin16<T>(mm);
  return mk(a.re * c - a.im * s, a.re * s + a.im * c);
}

// exp(-2 pi i m / 12) components (steps of 30 degrees), m = 0..11
template <typename T>
__host__ __device__ __forceinline__ constexpr T cos12(int m) {
  constexpr double h3 = 0.86602540378443864676;  // sqrt(3) / 2
  switch (((m % 12) + 12) % 12) {
    case 0: return (T)1.0;
    case 1: return (T)h3;
    case 2: return (T)0.5;
    case 3: return (T)0.0;
    case 4: return (T)-0.5;
    case 5: return (T)-h3;
    case 6: return (T)-1.0;
    case 7: return (T)-h3;
    case 8: return (T)-0.5;
    case 9: return (T)0.0;
    case 10: return (T)0.5;
    default: return (T)h3;
  }
}
template <typename T>
__host__ __device__ __forceinline__ constexpr T sin12(int m) {
  return cos12<T>(m + 9);  // sin(a) = cos(a - pi/2)
}

// multiply by W_R^m for R in {3, 6, 12} (multiples of 30 degrees)
template <int R, bool INV, typename T>
__host__ __device__ __forceinline__ cpx<T> twc12(cpx<T> a, int m) {
  const int mm = (m * (12 / R)) % 12;
  if (mm == 0) return a;
  if (mm == 6) return mk(-a.re, -a.im);
  if (mm == 3) return INV ? mk(-a.im, a.re) : mk(a.im, -a.re);
  if (mm == 9) return INV ? mk(a.im, -a.re) : mk(-a.im, a.re);
  const T c = cos12<T>(mm);
  const T s = INV ? sin12<T>(mm) : -sin12<T>(mm);
  return mk(a.re * c - a.im * s, a.re * s + a.im * c);
}

// In-register DFT of R points (R in {1,2,3,4,6,8,12,16}), natural order in and out.
// HIN: inputs a[R/2..R) are known to be zero (zero-padded line);
// HOUT: only outputs a[0..R/2) are needed (truncated line; the others are
// left unspecified).  Both prune work without changing the needed values.
template <int R, bool INV, bool HIN = false, bool HOUT = false, typename T>
__host__ __device__ __forceinline__ void dft(cpx<T>* a) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    if constexpr (HIN) {
      a[1] = a[0];
    } else {
      cpx<T> t = a[0];
      a[0] = t + a[1];
      if constexpr (!HOUT) a[1] = t - a[1];
    }
  } else if constexpr (R == 3) {
    // W3 = exp(-+2 pi i / 3) = -1/2 -+ i sqrt(3)/2
    constexpr double h3 = 0.86602540378443864676;
    const cpx<T> s = a[1] + a[2], d = a[1] - a[2];
    const cpx<T> m = mk(a[0].re - (T)0.5 * s.re, a[0].im - (T)0.5 * s.im);
    // i sqrt(3)/2 d (forward output 2 adds it, output 1 subtracts it)
    const cpx<T> e = mk(-(T)h3 * d.im, (T)h3 * d.re);
    a[0] = a[0] + s;
    a[1] = INV ? m + e : m - e;
    a[2] = INV ? m - e : m + e;
  } else if constexpr (R == 4) {
    if constexpr (HIN) {
      // d1 * W4^1 = d1 * (-i) forward, (+i) inverse; a2 = a3 = 0
      const cpx<T> a0 = a[0], a1 = a[1];
      const cpx<T> e1 = INV ? mk(-a1.im, a1.re) : mk(a1.im, -a1.re);
      a[0] = a0 + a1;
      a[1] = a0 + e1;
      if constexpr (!HOUT) {
        a[2] = a0 - a1;
        a[3] = a0 - e1;
      }
    } else {
      cpx<T> s0 = a[0] + a[2], d0 = a[0] - a[2];
      cpx<T> s1 = a[1] + a[3], d1 = a[1] - a[3];
      cpx<T> e1 = INV ? mk(-d1.im, d1.re) : mk(d1.im, -d1.re);
      a[0] = s0 + s1;
      a[1] = d0 + e1;
      if constexpr (!HOUT) {
        a[2] = s0 - s1;
        a[3] = d0 - e1;
      }
    }
  } else {
    // R = R1 * R2, input index n = R2 n1 + n2, output k = k1 + R1 k2.
    // Inputs n >= R/2 are those with n1 >= R1/2; outputs k < R/2 are those
    // with k2 < R2/2 when R2 is even (for R = 6 = 2 x 3 and 12 = 4 x 3 every
    // output is computed).
    static_assert(R == 6 || R == 8 || R == 12 || R == 16, "register DFT size");
    constexpr int R1 = (R == 8 || R == 6) ? 2 : 4;
    constexpr int R2 = R / R1;
    constexpr bool HO = HOUT && (R2 % 2 == 0);
    cpx<T> y[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      cpx<T> u[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) u[n1] = a[R2 * n1 + n2];
      dft<R1, INV, HIN, false>(u);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) {
        if constexpr (R % 3 == 0)
          y[n2 * R1 + k1] = twc12<R, INV>(u[k1], n2 * k1);
        else
          y[n2 * R1 + k1] = twc<R, INV>(u[k1], n2 * k1);
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cpx<T> u[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) u[n2] = y[n2 * R1 + k1];
      dft<R2, INV, false, HO>(u);
#pragma unroll
      for (int k2 = 0; k2 < (HO ? R2 / 2 : R2); ++k2) a[k1 + R1 * k2] = u[k2];
    }
  }
}

// Stockham stages for one line.  v: the thread's E points (see file header);
// lds: this line's P-point LDS scratch; tw[m] = exp(-2 pi i m / P).
// Every thread of the workgroup must call this the same number of times
// (it contains barriers).  When the line needs more than one stage the caller
// must not touch `lds` concurrently.
template <typename T, int P, int E, int NS, bool INV>
__device__ __forceinline__ void fft_stages(cpx<T> (&v)[E], cpx<T>* lds, int t,
                                           const cpx<T>* __restrict__ tw) {
  constexpr int RAD = fft_radix<P, E, NS>();
  constexpr int NB = E / RAD;  // butterflies per thread in this stage
  constexpr int TT = P / E;    // threads per line
  constexpr bool FIRST = (NS == 1);
  constexpr bool LAST = (NS * RAD == P);
  cpx<T> u[E];
  if constexpr (FIRST) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < RAD; ++r) u[b * RAD + r] = v[b + r * NB];
  } else {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + b * TT;
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        cpx<T> x = lds[j + r * (P / RAD)];
        if (r > 0) {
          cpx<T> w = tw[(r * k * (P / (NS * RAD))) % P];
          if (INV) w.im = -w.im;
          x = x * w;
        }
        u[b * RAD + r] = x;
      }
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) dft<RAD, INV>(&u[b * RAD]);
  if constexpr (LAST) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b + r * NB] = u[b * RAD + r];
  } else {
    lds_barrier();  // previous readers of lds are done
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + b * TT;
      const int base = (j / NS) * NS * RAD + (j % NS);
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds[base + r * NS] = u[b * RAD + r];
    }
    lds_barrier();
    fft_stages<T, P, E, NS * RAD, INV>(v, lds, t, tw);
  }
}

template <typename T, int P, int E, bool INV>
__device__ __forceinline__ void fft_line(cpx<T> (&v)[E], cpx<T>* lds, int t,
                                         const cpx<T>* __restrict__ tw) {
  fft_stages<T, P, E, 1, INV>(v, lds, t, tw);
}

// Elements per thread for a P-point line (P = 2^k or 3 * 2^k).
__host__ __device__ constexpr int fft_e_of(int P) { return (P % 3 == 0) ? 12 : (P < 16 ? P : 16); }
template <int P>
constexpr int fft_e() {
  return fft_e_of(P);
}

// Radix of the Stockham stage with sub-transform length NS: the largest of
// the register DFT sizes dividing both the remaining length P / NS and the
// points per thread E (so each thread runs E / RAD whole DFTs).
__host__ __device__ constexpr int gcd_i(int a, int b) { return b == 0 ? a : gcd_i(b, a % b); }
template <int P, int E, int NS>
constexpr int fft_radix() {
  return gcd_i(P / NS, E);
}

}  // namespace vie
