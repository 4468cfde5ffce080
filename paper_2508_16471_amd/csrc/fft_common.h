// Shared building blocks of the FFT passes: padded LDS lines, per-thread
// twiddle registers, Stockham stages, launch-shape helpers, block reduction.
#pragma once

#include "fft.h"
#include "kernels.h"

namespace vie {

template <int P>
struct Pad {
  static constexpr int LSTR = P + P / 16 + 1;  // padded LDS line stride (bank spread)
};
// Line stride of the x passes, where the TT threads of one line are
// neighbouring lanes and each stage touches TT consecutive points of a line:
// a stride of TT (mod 16) points puts neighbouring lines' windows side by
// side in the banks (the odd stride of Pad suits the column passes, whose
// neighbouring lanes are different lines).
template <int P, int TT>
struct PadX {
  static constexpr int base() { return P + P / 16; }
  static constexpr int LSTR = base() + ((TT % 16) - base() % 16 + 16) % 16;
};
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

// fft_stages with padded LDS indexing: wrap the line pointer in an accessor.
template <typename T>
struct LdsLine {
  cpx<T>* p;
  __device__ __forceinline__ cpx<T>& operator[](int i) const { return p[pidx(i)]; }
};

// FP32 column pairs: lanes 2i (column c) and 2i+1 (column c+1) of one row
// of threads move 16-byte row segments [c, c+1] -- the even lane the row of
// its point 2k, the odd lane the row of its point 2k+1 -- and one lane swap
// hands each lane its own column's two points.  Half the memory
// instructions of one 8-byte access per point.
__device__ __forceinline__ float swap_pair(float x) {
  // lanes 2i <-> 2i+1 (DPP quad_perm [1,0,3,2])
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ void pair_in(const float4 f, int odd, cpx<float>& a, cpx<float>& b) {
  const float sr = odd ? f.x : f.z, si = odd ? f.y : f.w;  // the partner's point
  const float kr = odd ? f.z : f.x, ki = odd ? f.w : f.y;  // this lane's point
  const float rr = swap_pair(sr), ri = swap_pair(si);
  a = odd ? mk<float>(rr, ri) : mk<float>(kr, ki);
  b = odd ? mk<float>(kr, ki) : mk<float>(rr, ri);
}
__device__ __forceinline__ float4 pair_out(int odd, const cpx<float>& a, const cpx<float>& b) {
  const cpx<float> sd = odd ? a : b;
  const float rr = swap_pair(sd.re), ri = swap_pair(sd.im);
  const cpx<float> own = odd ? b : a;
  return odd ? make_float4(rr, ri, own.re, own.im) : make_float4(own.re, own.im, rr, ri);
}

// Packed FP16 pairs for approximate products: one register holds the same
// component of two neighbouring columns (v_pk_* arithmetic on both).
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ cpx<h2> pack2(float ar, float ai, float br, float bi) {
  return mk<h2>(h2{(_Float16)ar, (_Float16)br}, h2{(_Float16)ai, (_Float16)bi});
}
// negate both halves of re and im when neg (sign bits flipped)
__device__ __forceinline__ cpx<h2> negif(cpx<h2> a, bool neg) {
  const unsigned m = neg ? 0x80008000u : 0u;
  return mk<h2>(__builtin_bit_cast(h2, __builtin_bit_cast(unsigned, a.re) ^ m),
                __builtin_bit_cast(h2, __builtin_bit_cast(unsigned, a.im) ^ m));
}
// a packed pair's two points as (re_a, im_a, re_b, im_b)
__device__ __forceinline__ float4 unpack2(cpx<h2> h) {
  return make_float4((float)h.re.x, (float)h.im.x, (float)h.re.y, (float)h.im.y);
}
__device__ __forceinline__ cpx<h2> hscale(cpx<h2> a, h2 s) { return mk<h2>(a.re * s, a.im * s); }

// Twiddles of a thread's butterflies, loaded once per kernel into registers
// and reused by every line the thread transforms (forward and inverse).
// Stage with sub-length NS and radix RAD (not the first): butterfly b of
// thread t has j = t + b TT, k = j % NS and multiplies input r by
// W_{NS RAD}^{r k} = tw[r k P / (NS RAD)].
template <int P, int E, int NS>
constexpr int tw_count() {
  constexpr int RAD = fft_radix<P, E, NS>();
  constexpr int here = (NS == 1) ? 0 : (E / RAD) * (RAD - 1);
  if constexpr (NS * RAD == P)
    return here;
  else
    return here + tw_count<P, E, NS * RAD>();
}

template <typename T, int P, int E, int NS, int OFF>
__device__ __forceinline__ void tw_load(cpx<T>* w, int t, const cpx<T>* __restrict__ tw) {
  constexpr int RAD = fft_radix<P, E, NS>();
  constexpr int NB = E / RAD, TT = P / E;
  constexpr int here = (NS == 1) ? 0 : NB * (RAD - 1);
  if constexpr (NS != 1) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int k = (t + b * TT) % NS;
#pragma unroll
      for (int r = 1; r < RAD; ++r) w[OFF + b * (RAD - 1) + r - 1] = tw[r * k * (P / (NS * RAD))];
    }
  }
  if constexpr (NS * RAD != P) tw_load<T, P, E, NS * RAD, OFF + here>(w, t, tw);
}

// Lines longer than 512 points read their twiddles from the global table at
// every stage instead (too many to keep in registers; the table is small and
// stays in cache).
template <int P>
constexpr bool tw_global() {
  return P > 512;
}
template <typename T, int P, int E, bool G = tw_global<P>()>
struct TwReg {
  static constexpr int N = tw_count<P, E, 1>() > 0 ? tw_count<P, E, 1>() : 1;
  cpx<T> w[N];
  __device__ __forceinline__ void load(int t, const cpx<T>* __restrict__ tw) {
    tw_load<T, P, E, 1, 0>(w, t, tw);
  }
};
template <typename T, int P, int E>
struct TwReg<T, P, E, true> {
  const cpx<T>* w;
  __device__ __forceinline__ void load(int, const cpx<T>* __restrict__ tw) { w = tw; }
};

// HIN: the line's upper half (points P/2..P) is zero on entry (every thread
// holds it as v[E/2..E)); HOUT: only the lower half is needed on exit.  The
// first / last stage's DFTs are pruned accordingly.
// GTW: w is the global twiddle table (tw[m] = W_P^m) instead of the
// thread's register twiddles.
template <typename T, int P, int E, int NS, bool INV, int OFF, bool HIN = false, bool HOUT = false,
          bool GTW = false>
__device__ __forceinline__ void fft_stages_p(cpx<T> (&v)[E], LdsLine<T> lds, int t,
                                             const cpx<T>* __restrict__ w) {
  constexpr int RAD = fft_radix<P, E, NS>();
  constexpr int NB = E / RAD;
  constexpr int TT = P / E;
  constexpr bool FIRST = (NS == 1);
  constexpr bool LAST = (NS * RAD == P);
  constexpr int here = FIRST ? 0 : NB * (RAD - 1);
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
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        cpx<T> x = lds[j + r * (P / RAD)];
        if (r > 0) {
          cpx<T> ww;
          if constexpr (GTW)
            ww = w[r * (j % NS) * (P / (NS * RAD))];
          else
            ww = w[OFF + b * (RAD - 1) + r - 1];
          if (INV) ww.im = -ww.im;
          x = x * ww;
        }
        u[b * RAD + r] = x;
      }
    }
  }
  // the first stage has one DFT per thread (RAD = E) holding points t + q P/E:
  // its inputs q >= E/2 are the zero half; in the last stage the needed
  // outputs q = b + r NB < E/2 are the DFT outputs r < RAD/2
  static_assert(!FIRST || NB == 1, "first stage: one DFT per thread");
  constexpr bool PIN = HIN && FIRST;
  constexpr bool POUT = HOUT && LAST;
#pragma unroll
  for (int b = 0; b < NB; ++b) dft<RAD, INV, PIN, POUT>(&u[b * RAD]);
  if constexpr (LAST) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b + r * NB] = u[b * RAD + r];
  } else {
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + b * TT;
      const int base = (j / NS) * NS * RAD + (j % NS);
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds[base + r * NS] = u[b * RAD + r];
    }
    lds_barrier();
    fft_stages_p<T, P, E, NS * RAD, INV, OFF + here, HIN, HOUT, GTW>(v, lds, t, w);
  }
}

template <typename T, int P, bool INV, bool HIN = false, bool HOUT = false>
__device__ __forceinline__ void line_fft(cpx<T> (&v)[fft_e<P>()], cpx<T>* line, int t,
                                         const TwReg<T, P, fft_e<P>()>& tr) {
  fft_stages_p<T, P, fft_e<P>(), 1, INV, 0, HIN, HOUT, tw_global<P>()>(v, LdsLine<T>{line}, t,
                                                                       tr.w);
}

template <typename T>
constexpr int nt_lines() {
  return sizeof(T) == 8 ? 128 : 256;  // threads per workgroup of single-line passes
}
// Threads per workgroup of a single-line pass of length P: nt_lines, or one
// whole line when its P / E threads are more than that (lines above 512).
template <typename T>
constexpr int nt_lines_p(int P) {
  return nt_lines<T>() > P / fft_e_of(P) ? nt_lines<T>() : P / fft_e_of(P);
}


__device__ __forceinline__ void block_sum2(c64& a, c64& b, double* red) {
  // wave64 butterfly then across waves through LDS (fixed order: deterministic)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a.re += __shfl_xor(a.re, off, 64);
    a.im += __shfl_xor(a.im, off, 64);
    b.re += __shfl_xor(b.re, off, 64);
    b.im += __shfl_xor(b.im, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    red[wv * 4 + 0] = a.re;
    red[wv * 4 + 1] = a.im;
    red[wv * 4 + 2] = b.re;
    red[wv * 4 + 3] = b.im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c64 sa = mk(0.0, 0.0), sb = mk(0.0, 0.0);
    for (int w = 0; w < nw; ++w) {
      sa.re += red[w * 4 + 0];
      sa.im += red[w * 4 + 1];
      sb.re += red[w * 4 + 2];
      sb.im += red[w * 4 + 3];
    }
    a = sa;
    b = sb;
  }
}


template <typename T>
constexpr int lines_per_block(int P) {
  return nt_lines_p<T>(P) / (P / fft_e_of(P));
}

// Line lengths of the x and y passes: 2^k (8..4096) and 3 * 2^k (12..6144).
#define VIE_DISPATCH_P(P_, CALL)                         \
  switch (P_) {                                          \
    case 8: { constexpr int PP = 8; CALL; break; }       \
    case 12: { constexpr int PP = 12; CALL; break; }     \
    case 16: { constexpr int PP = 16; CALL; break; }     \
    case 24: { constexpr int PP = 24; CALL; break; }     \
    case 32: { constexpr int PP = 32; CALL; break; }     \
    case 48: { constexpr int PP = 48; CALL; break; }     \
    case 64: { constexpr int PP = 64; CALL; break; }     \
    case 96: { constexpr int PP = 96; CALL; break; }     \
    case 128: { constexpr int PP = 128; CALL; break; }   \
    case 192: { constexpr int PP = 192; CALL; break; }   \
    case 256: { constexpr int PP = 256; CALL; break; }   \
    case 384: { constexpr int PP = 384; CALL; break; }   \
    case 512: { constexpr int PP = 512; CALL; break; }   \
    case 768: { constexpr int PP = 768; CALL; break; }   \
    case 1024: { constexpr int PP = 1024; CALL; break; } \
    case 1536: { constexpr int PP = 1536; CALL; break; } \
    case 2048: { constexpr int PP = 2048; CALL; break; } \
    case 3072: { constexpr int PP = 3072; CALL; break; } \
    case 4096: { constexpr int PP = 4096; CALL; break; } \
    case 6144: { constexpr int PP = 6144; CALL; break; } \
    default: return hipErrorInvalidValue;                \
  }

// Line lengths of the z passes: 2^k (8..512) and 3 * 2^k (12..384).
#define VIE_DISPATCH_PZ(P_, CALL)                      \
  switch (P_) {                                        \
    case 8: { constexpr int PP = 8; CALL; break; }     \
    case 12: { constexpr int PP = 12; CALL; break; }   \
    case 16: { constexpr int PP = 16; CALL; break; }   \
    case 24: { constexpr int PP = 24; CALL; break; }   \
    case 32: { constexpr int PP = 32; CALL; break; }   \
    case 48: { constexpr int PP = 48; CALL; break; }   \
    case 64: { constexpr int PP = 64; CALL; break; }   \
    case 96: { constexpr int PP = 96; CALL; break; }   \
    case 128: { constexpr int PP = 128; CALL; break; } \
    case 192: { constexpr int PP = 192; CALL; break; } \
    case 256: { constexpr int PP = 256; CALL; break; } \
    case 384: { constexpr int PP = 384; CALL; break; } \
    case 512: { constexpr int PP = 512; CALL; break; } \
    default: return hipErrorInvalidValue;              \
  }


}  // namespace vie
