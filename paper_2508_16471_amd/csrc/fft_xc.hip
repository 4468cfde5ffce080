// x passes of the operator product for body-compressed vectors.
//
// The unknowns of the discrete system are the contrast currents of the body
// voxels (3 N_b values; chi = 0 elsewhere, where the solution vanishes).  The
// solver stores its vectors over those unknowns only, component-major,
// voxels in ascending box order: v[rhs][comp][k], k < N_b(body).  An x-line
// (y, z) owns the contiguous range line_ptr[zy] .. line_ptr[zy+1] of a body's
// voxels, so the forward x pass scatters a line's voxels into its LDS line
// (zeros elsewhere) before transforming, and the inverse x pass gathers the
// convolution at the line's voxels after transforming.  The y and z passes
// and their scratch are unchanged (full FFT box).
#include "fft_common.h"
#include "kernels.h"

namespace vie {

// ---------------------------------------------------------------- X forward
// H (FP32 only): the transformed lines are stored as packed FP16 column
// pairs scaled by hs (cpx<h2> per pair of neighbouring points of a line);
// lanes t and t + 1 of a line exchange one point per pair of registers.
template <typename T, int P, typename TI, bool H = false>
__global__ __launch_bounds__(nt_lines_p<T>(P)) void k_fft_x_fwd_c(
    const cpx<TI>* __restrict__ xc, void* __restrict__ outv, const cpx<T>* __restrict__ tw,
    BodyIdx bi, int N1, int N2, int N3, int blocks_per_rhs, const int* __restrict__ active,
    float hs) {
  constexpr int E = fft_e<P>(), TT = P / E, NT = nt_lines_p<T>(P), L = NT / TT,
                LS = PadX<P, P / fft_e<P>()>::LSTR;
  __shared__ cpx<T> lds[L * LS];
  // Hardware order (consecutive blocks go to consecutive XCDs): the lines of
  // one right-hand side spread over every XCD, so inactive right-hand sides
  // leave none idle, and concurrently running blocks touch neighbouring lines.
  const int b = blockIdx.x;
  const int rhs = b / blocks_per_rhs, blk = b % blocks_per_rhs;
  if (active && !active[rhs]) return;
  const int lines_per_rhs = 3 * N2 * N3, lpc = N2 * N3;
  const int li = threadIdx.x / TT, t = threadIdx.x % TT;
  const int line = blk * L + li;
  const bool valid = line < lines_per_rhs;
  const int lc = valid ? line : 0;
  const int comp = lc / lpc, zy = lc % lpc;
  const int body = bi.rhs_body[rhs];
  const int nb = bi.nb[body];
  const int* vox = bi.vox + bi.voff[body];
  const int* lp = bi.line_ptr + (int64_t)body * (lpc + 1);
  const cpx<TI>* xv = xc + bi.roff[rhs] + (int64_t)comp * nb;
  TwReg<T, P, E> tr;
  tr.load(t, tw);
  cpx<T>* myl = lds + li * LS;
  // zero the line's first P/2 points (the padded half is never read)
#pragma unroll
  for (int q = 0; q < E / 2; ++q) myl[pidx(t + q * TT)] = mk<T>(0, 0);
  lds_barrier();
  if (valid) {
    // a line holds at most P/2 voxels, so at most E/2 per thread: all their
    // loads are issued before the first LDS write
    const int k0 = lp[zy] + t, k1 = lp[zy + 1];
    const int base = zy * N1;
    int kv[E / 2];
    cpx<TI> xr[E / 2];
#pragma unroll
    for (int i = 0; i < E / 2; ++i) {
      const int k = k0 + i * TT;
      if (k < k1) {
        kv[i] = vox[k];
        xr[i] = xv[k];
      }
    }
#pragma unroll
    for (int i = 0; i < E / 2; ++i)
      if (k0 + i * TT < k1) myl[pidx(kv[i] - base)] = cvt<T>(xr[i]);
  }
  lds_barrier();
  cpx<T> v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) v[q] = (q < E / 2) ? myl[pidx(t + q * TT)] : mk<T>(0, 0);
  line_fft<T, P, false, true>(v, myl, t, tr);  // upper half is zero padding
  if constexpr (H) {
    static_assert(sizeof(T) == 4 && TT % 2 == 0, "packed lines need FP32 and lane pairs");
    // pair q/2 of lane pair (t, t + 1): points t + q TT (even lane's) and
    // t + 1 + q TT; the even lane stores it for even q, the odd lane for odd q
    const int odd = t & 1;
    cpx<h2>* o = reinterpret_cast<cpx<h2>*>(outv) + ((size_t)rhs * lines_per_rhs + lc) * (P / 2);
#pragma unroll
    for (int q = 0; q < E; q += 2) {
      const float4 f = pair_out(odd, v[q], v[q + 1]);
      if (valid) o[(t - odd + (q + odd) * TT) >> 1] = pack2(f.x * hs, f.y * hs, f.z * hs, f.w * hs);
    }
  } else if (valid) {
    cpx<T>* o = reinterpret_cast<cpx<T>*>(outv) + ((size_t)rhs * lines_per_rhs + line) * P;
#pragma unroll
    for (int q = 0; q < E; ++q) o[t + q * TT] = v[q];
  }
}

// ------------------------------------------------ X inverse + epilogue
// TX: storage of the input vector (the epilogue's x), TIO of the output.
// H (FP32 only): A holds packed FP16 column pairs (see the forward pass);
// the convolution is scaled by hs before the epilogue.
template <typename T, int P, int MODE, typename TIO, typename TX = TIO, bool H = false>
__global__ __launch_bounds__(nt_lines_p<T>(P)) void k_fft_x_inv_c(
    const void* __restrict__ Av, const cpx<TX>* __restrict__ xin, cpx<TIO>* __restrict__ yout,
    const cpx<T>* __restrict__ tw, BodyIdx bi, int N1, int N2, int N3, int blocks_per_rhs,
    c64* __restrict__ aux, c64* __restrict__ partials, const c64* __restrict__ pol,
    const c64* __restrict__ ph, const int* __restrict__ active, float hs) {
  constexpr int E = fft_e<P>(), TT = P / E, NT = nt_lines_p<T>(P), L = NT / TT,
                LS = PadX<P, P / fft_e<P>()>::LSTR;
  __shared__ cpx<T> lds[L * LS];
  __shared__ double red[4 * (NT / 64 + 1)];
  // Hardware order (consecutive blocks go to consecutive XCDs): the lines of
  // one right-hand side spread over every XCD, so inactive right-hand sides
  // leave none idle, and concurrently running blocks touch neighbouring lines.
  const int b = blockIdx.x;
  const int rhs = b / blocks_per_rhs, blk = b % blocks_per_rhs;
  if (active && !active[rhs]) return;
  const int lines_per_rhs = 3 * N2 * N3, lpc = N2 * N3;
  const int li = threadIdx.x / TT, t = threadIdx.x % TT;
  const int line = blk * L + li;
  const bool valid = line < lines_per_rhs;
  const int lc = valid ? line : 0;
  const size_t gl = (size_t)rhs * lines_per_rhs + lc;
  TwReg<T, P, E> tr;
  tr.load(t, tw);
  cpx<T> v[E];
  if constexpr (H) {
    static_assert(sizeof(T) == 4 && TT % 2 == 0, "packed lines need FP32 and lane pairs");
    // the even lane loads pair q/2 for even q, the odd lane for odd q; one
    // exchange hands each lane its own point of both
    const int odd = t & 1;
    const cpx<h2>* src = reinterpret_cast<const cpx<h2>*>(Av) + gl * (P / 2);
#pragma unroll
    for (int q = 0; q < E; q += 2) {
      float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
      if (valid) f = unpack2(src[(t - odd + (q + odd) * TT) >> 1]);
      pair_in(f, odd, v[q], v[q + 1]);
    }
  } else {
    const cpx<T>* src = reinterpret_cast<const cpx<T>*>(Av) + gl * P;
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = valid ? src[t + q * TT] : mk<T>(0, 0);
  }
  cpx<T>* myl = lds + li * LS;
  line_fft<T, P, true, false, true>(v, myl, t, tr);  // only x < N1 is used
  lds_barrier();  // every thread has left the FFT's last LDS read
#pragma unroll
  for (int q = 0; q < E / 2; ++q) myl[pidx(t + q * TT)] = v[q];
  lds_barrier();
  const int comp = lc / lpc, zy = lc % lpc;
  const int body = bi.rhs_body[rhs];
  const int nb = bi.nb[body];
  const int* vox = bi.vox + bi.voff[body];
  const double* chic = bi.chic + bi.voff[body];
  const int* lp = bi.line_ptr + (int64_t)body * (lpc + 1);
  const int64_t vb = bi.roff[rhs] + (int64_t)comp * nb;
  c64 s0 = mk(0.0, 0.0), s1 = mk(0.0, 0.0);
  if (valid) {
    const int k1 = lp[zy + 1];
    const int base = zy * N1;
    c64 phyz = mk(0.0, 0.0), pc = mk(0.0, 0.0);
    const c64* phr = ph + (int64_t)rhs * (N1 + N2 + N3);
    if (MODE == EPI_RESID) {
      const int y = zy % N2, z = zy / N2;
      phyz = phr[N1 + y] * phr[N1 + N2 + z];
      pc = pol[rhs * 3 + comp];
    }
    // a line holds at most P/2 voxels, so at most E/2 per thread: all their
    // loads are issued before the first use
    const int k0 = lp[zy] + t;
    int kv[E / 2];
    double cv[E / 2];
    cpx<TX> xr[E / 2];
#pragma unroll
    for (int i = 0; i < E / 2; ++i) {
      const int k = k0 + i * TT;
      if (k < k1) {
        kv[i] = vox[k];
        cv[i] = chic[k];
        xr[i] = xin[vb + k];
      }
    }
#pragma unroll
    for (int i = 0; i < E / 2; ++i) {
      const int k = k0 + i * TT;
      if (k >= k1) continue;
      const int xi = kv[i] - base;
      c64 conv = cvt<double>(myl[pidx(xi)]);
      if constexpr (H) conv = (double)hs * conv;
      const double c = cv[i];
      const int64_t gi = vb + k;
      const c64 xv = cvt<double>(xr[i]);
      const c64 y = xv - c * conv;
      if (MODE == EPI_RESID) {
        const c64 e = pc * (phyz * phr[xi]);
        const c64 r = c * e - y;
        yout[gi] = cvt<TIO>(r);
        aux[gi] = r;
        s1.re += r.re * r.re + r.im * r.im;
      } else {
        yout[gi] = cvt<TIO>(y);
        if (MODE == EPI_RHV) {
          s0 = s0 + cmulc(aux[gi], y);
        } else if (MODE == EPI_TS) {
          s0 = s0 + cmulc(y, xv);
          s1.re += y.re * y.re + y.im * y.im;
        }
      }
    }
  }
  if (MODE != EPI_PLAIN) {
    block_sum2(s0, s1, red);
    if (threadIdx.x == 0) {
      c64* pp = partials + ((size_t)rhs * blocks_per_rhs + blk) * 2;
      pp[0] = s0;
      pp[1] = s1;
    }
  }
}

// ================================================================ launchers
// Packed FP16 lines need an even number of threads per line (P >= 24).
template <int P>
constexpr bool packed_lines_ok() {
  return (P / fft_e_of(P)) % 2 == 0;
}
bool x_packed_ok(int P1) { return (P1 / fft_e_of(P1)) % 2 == 0; }

template <typename T>
hipError_t x_fwd_c(const GroupGeom& g, const void* xc, int in32, cpx<T>* A, const cpx<T>* tw,
                   const BodyIdx& bi, const int* active, hipStream_t s, float hs) {
  const int lines = 3 * g.N[1] * g.N[2];
  const int L = lines_per_block<T>(g.P[0]);
  const int bpr = (lines + L - 1) / L;
  const dim3 grid(bpr * g.nrhs);
  if (hs > 0.f) {  // packed FP16 output from bfloat16 input (FP32 arithmetic)
    if constexpr (sizeof(T) == 4) {
      if (in32 != 2) return hipErrorInvalidValue;
      VIE_DISPATCH_P(g.P[0], ({
                       if constexpr (packed_lines_ok<PP>()) {
                         k_fft_x_fwd_c<T, PP, __bf16, true><<<grid, nt_lines_p<T>(PP), 0, s>>>(
                             (const cb16*)xc, A, tw, bi, g.N[0], g.N[1], g.N[2], bpr, active, hs);
                       } else {
                         return hipErrorInvalidValue;
                       }
                     }));
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (in32 == 2) {  // bfloat16 input (FP32 products only)
    if constexpr (sizeof(T) == 4) {
      VIE_DISPATCH_P(g.P[0], (k_fft_x_fwd_c<T, PP, __bf16><<<grid, nt_lines_p<T>(PP), 0, s>>>(
                                 (const cb16*)xc, A, tw, bi, g.N[0], g.N[1], g.N[2], bpr, active,
                                 0.f)));
    } else {
      return hipErrorInvalidValue;
    }
  } else if (in32) {
    VIE_DISPATCH_P(g.P[0], (k_fft_x_fwd_c<T, PP, float><<<grid, nt_lines_p<T>(PP), 0, s>>>(
                               (const c32*)xc, A, tw, bi, g.N[0], g.N[1], g.N[2], bpr, active,
                               0.f)));
  } else {
    VIE_DISPATCH_P(g.P[0], (k_fft_x_fwd_c<T, PP, double><<<grid, nt_lines_p<T>(PP), 0, s>>>(
                               (const c64*)xc, A, tw, bi, g.N[0], g.N[1], g.N[2], bpr, active,
                               0.f)));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t x_inv_c(const GroupGeom& g, const cpx<T>* A, const void* x, void* y, int io32,
                   const cpx<T>* tw, const BodyIdx& bi, EpiArgs& e, const int* active,
                   hipStream_t s, float hs) {
  const int lines = 3 * g.N[1] * g.N[2];
  const int L = lines_per_block<T>(g.P[0]);
  const int bpr = (lines + L - 1) / L;
  e.part_blocks = bpr;
  const dim3 grid(bpr * g.nrhs);
  if (hs > 0.f) {  // packed FP16 input lines, bfloat16 x, FP32 y, plain epilogue
    if constexpr (sizeof(T) == 4) {
      if (io32 != 2 || e.mode != EPI_PLAIN) return hipErrorInvalidValue;
      VIE_DISPATCH_P(g.P[0], ({
                       if constexpr (packed_lines_ok<PP>()) {
                         k_fft_x_inv_c<T, PP, EPI_PLAIN, float, __bf16, true>
                             <<<grid, nt_lines_p<T>(PP), 0, s>>>(
                                 A, (const cb16*)x, (c32*)y, tw, bi, g.N[0], g.N[1], g.N[2], bpr,
                                 e.aux, e.partials, e.pol, e.ph, active, hs);
                       } else {
                         return hipErrorInvalidValue;
                       }
                     }));
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (io32) {  // FP32 output (input FP32, or bfloat16 for io32 = 2): the plain product only
    if (e.mode != EPI_PLAIN) return hipErrorInvalidValue;
    if (io32 == 2) {
      if constexpr (sizeof(T) == 4) {
        VIE_DISPATCH_P(g.P[0], (k_fft_x_inv_c<T, PP, EPI_PLAIN, float, __bf16>
                                <<<grid, nt_lines_p<T>(PP), 0, s>>>(
                                    A, (const cb16*)x, (c32*)y, tw, bi, g.N[0], g.N[1], g.N[2],
                                    bpr, e.aux, e.partials, e.pol, e.ph, active, 0.f)));
      } else {
        return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
    VIE_DISPATCH_P(g.P[0], (k_fft_x_inv_c<T, PP, EPI_PLAIN, float><<<grid, nt_lines_p<T>(PP), 0, s>>>(
                               A, (const c32*)x, (c32*)y, tw, bi, g.N[0], g.N[1], g.N[2], bpr,
                               e.aux, e.partials, e.pol, e.ph, active, 0.f)));
    return hipGetLastError();
  }
#define VIE_XINVC(MODE_)                                                                      \
  VIE_DISPATCH_P(g.P[0], (k_fft_x_inv_c<T, PP, MODE_, double><<<grid, nt_lines_p<T>(PP), 0, s>>>(   \
                             A, (const c64*)x, (c64*)y, tw, bi, g.N[0], g.N[1], g.N[2], bpr,  \
                             e.aux, e.partials, e.pol, e.ph, active, 0.f)))
  switch (e.mode) {
    case EPI_PLAIN: VIE_XINVC(EPI_PLAIN); break;
    case EPI_RHV: VIE_XINVC(EPI_RHV); break;
    case EPI_TS: VIE_XINVC(EPI_TS); break;
    case EPI_RESID: VIE_XINVC(EPI_RESID); break;
    default: return hipErrorInvalidValue;
  }
#undef VIE_XINVC
  return hipGetLastError();
}

template hipError_t x_fwd_c<double>(const GroupGeom&, const void*, int, c64*, const c64*,
                                    const BodyIdx&, const int*, hipStream_t, float);
template hipError_t x_fwd_c<float>(const GroupGeom&, const void*, int, c32*, const c32*,
                                   const BodyIdx&, const int*, hipStream_t, float);
template hipError_t x_inv_c<double>(const GroupGeom&, const c64*, const void*, void*, int,
                                    const c64*, const BodyIdx&, EpiArgs&, const int*, hipStream_t,
                                    float);
template hipError_t x_inv_c<float>(const GroupGeom&, const c32*, const void*, void*, int,
                                   const c32*, const BodyIdx&, EpiArgs&, const int*, hipStream_t,
                                   float);

}  // namespace vie
