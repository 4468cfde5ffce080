// FFT passes of the VIE operator product y = x - chi * IFFT(Ghat^ . FFT(pad x))[0:N]
// (the FFT-accelerated matrix-vector product of the paper's Sec. II-C).
//
// Data flow for one right-hand side (3 Cartesian components):
//   x [3][N3][N2][N1]  --X fwd (pad N1->P1)-->  A [3][N3][N2][P1]
//   A --Y fwd (pad N2->P2)-->                    B [3][N3][P2][P1]
//   B --Z fwd (pad N3->P3), 3x3 spectral multiply, Z inv, keep N3--> B (in place)
//   B --Y inv (keep N2)-->                        A
//   A --X inv (keep N1), epilogue y = x - chi conv (+ fused dot products)--> y
// Padded halves are never stored: the first stage of each forward FFT skips
// the zero inputs, the last stage of each inverse FFT skips the discarded
// outputs.  The 3x3 symmetric spectrum is stored on the octant
// [0, P/2]^3 only; the other octants follow from the per-axis parity of each
// Green component.
#include <type_traits>

#include "fft_common.h"
#include "kernels.h"

namespace vie {

// ---------------------------------------------------------------- X forward
// One workgroup: L consecutive x-lines of one right-hand side.
template <typename TI, typename T, int P, bool PAD>
__global__ __launch_bounds__(nt_lines_p<T>(P)) void k_fft_x_fwd(
    const cpx<TI>* __restrict__ x, cpx<T>* __restrict__ out, const cpx<T>* __restrict__ tw, int N1,
    int lines_per_rhs, int blocks_per_rhs, const int* __restrict__ active) {
  constexpr int E = fft_e<P>(), TT = P / E, NT = nt_lines_p<T>(P), L = NT / TT;
  __shared__ cpx<T> lds[L * Pad<P>::LSTR];
  // Hardware order (consecutive blocks go to consecutive XCDs): the lines of
  // one right-hand side spread over every XCD, so inactive right-hand sides
  // leave none idle, and concurrently running blocks touch neighbouring lines.
  const int b = blockIdx.x;
  const int rhs = b / blocks_per_rhs, blk = b % blocks_per_rhs;
  if (active && !active[rhs]) return;
  const int li = threadIdx.x / TT, t = threadIdx.x % TT;
  const int line = blk * L + li;
  const bool valid = line < lines_per_rhs;
  const size_t gl = (size_t)rhs * lines_per_rhs + (valid ? line : 0);
  const cpx<TI>* xin = x + gl * N1;
  TwReg<T, P, E> tr;
  tr.load(t, tw);
  cpx<T> v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int idx = t + q * TT;
    if ((!PAD || q < E / 2) && valid && idx < N1)
      v[q] = cvt<T>(xin[idx]);
    else
      v[q] = mk<T>(0, 0);
  }
  line_fft<T, P, false, PAD>(v, lds + li * Pad<P>::LSTR, t, tr);
  if (valid) {
    cpx<T>* o = out + gl * P;
#pragma unroll
    for (int q = 0; q < E; ++q) o[t + q * TT] = v[q];
  }
}

// ------------------------------------------------------ strided (Y, or Z)
// Lines run along a strided axis; W = NT/TT neighbouring columns (unit stride)
// per workgroup so every row access is a contiguous W-element run.
// Slab s = (rhs, comp, z) with z split as (z / zl, z % zl); each side
// addresses element (row, col) of a slab at
//   rhs*rs + comp*cs + (z/zl)*zhs + (z%zl)*zls + row*row_stride + col.
// The z split lets a buffer keep zl consecutive z planes next to each other
// (blocked layout), so that both the y pass and the z pass touch only a few
// memory pages per workgroup.
struct SideAddr {
  int64_t rs, cs, zhs, zls, row;
};
struct StridedArgs {
  int n_in_rows, n_out_rows, ncols, tiles, ncomp, nz, zl;
  SideAddr in, out;
};

__device__ __forceinline__ int64_t slab_base(const SideAddr& a, int rhs, int comp, int z, int zl) {
  return rhs * a.rs + comp * a.cs + (z / zl) * a.zhs + (z % zl) * a.zls;
}

template <typename T, int P, bool PAD, bool TRUNC, bool INV, int NTB = nt_lines<T>()>
__global__ __launch_bounds__(NTB) void k_fft_strided(
    const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, const cpx<T>* __restrict__ tw,
    StridedArgs a, const int* __restrict__ active) {
  constexpr int E = fft_e<P>(), TT = P / E, NT = NTB, W = NT / TT;
  __shared__ cpx<T> lds[W * Pad<P>::LSTR];
  // XCD-contiguous ranges of the logical order below (neighbouring column
  // tiles of one slab share an XCD), with the right-hand side innermost so
  // that every XCD holds an equal share of each right-hand side and
  // inactive ones leave no XCD idle.
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int per_rhs = a.ncomp * a.nz;
  const int nrhs_l = gridDim.x / (a.tiles * per_rhs);
  const int rhs = b % nrhs_l, rest = b / nrhs_l;
  const int tile = rest % a.tiles, cz = rest / a.tiles;
  if (active && !active[rhs]) return;
  const int comp = cz / a.nz, z = cz % a.nz;
  const int cw = threadIdx.x % W, t = threadIdx.x / W;
  const int col = tile * W + cw;
  const bool valid = col < a.ncols;
  const cpx<T>* pin = in + slab_base(a.in, rhs, comp, z, a.zl) + (valid ? col : 0);
  TwReg<T, P, E> tr;
  tr.load(t, tw);
  cpx<T> v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int row = t + q * TT;
    if ((!PAD || q < E / 2) && valid && row < a.n_in_rows)
      v[q] = pin[(int64_t)row * a.in.row];
    else
      v[q] = mk<T>(0, 0);
  }
  line_fft<T, P, INV, PAD, TRUNC>(v, lds + cw * Pad<P>::LSTR, t, tr);
  if (valid) {
    cpx<T>* po = out + slab_base(a.out, rhs, comp, z, a.zl) + col;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int row = t + q * TT;
      if ((!TRUNC || q < E / 2) && row < a.n_out_rows) po[(int64_t)row * a.out.row] = v[q];
    }
  }
}

// ----------------------------------------------- Z fused with the spectrum
// Workgroup: W neighbouring xi_x columns at one xi_y of one right-hand side.
// Each thread owns one column's points t + q TT for all three Cartesian
// components (registers), transforms them one after another through the
// column's LDS line (forward, pad N3 -> P), applies the symmetric 3x3
// spectrum point by point in registers (six unique entries per point, sign
// from each component's parity on mirrored axes), transforms back and keeps
// z < N3.  In place on B.
// Launch shapes tried by the autotuner: (points per thread E, threads NT).
// W = NT E / P columns per workgroup; LDS = W padded lines.
struct ZShape {
  int e, nt;
};
template <typename T>
constexpr ZShape zshape(int v) {
  // FP32: 3 x 16 complex in registers / 3 x 8; FP64: 3 x 8 / 3 x 4.  Every
  // shape keeps W = NT E / P >= 16 (FP32) or 8 (FP64) columns per workgroup,
  // so each row access is a full 128-byte run.
  return sizeof(T) == 4 ? (v == 0 ? ZShape{16, 256} : ZShape{8, 512})
                        : (v == 0 ? ZShape{8, 256} : ZShape{4, 512});
}
static constexpr int kZVariants = 3;  // shapes 0 and 1 above, 2 the register-lean kernel
template <int P, int E0>
constexpr int zcap() {
  return (P % 3 == 0) ? (E0 >= 8 ? 12 : 6) : (E0 < P ? E0 : P);
}

struct ZArgs {
  int N3, P1, P2, Q1, Q2, Q3, tiles_x, nrhs, zl;
  int64_t comp_stride, rhs_stride, zhs, zls;  // blocked layout of B (see StridedArgs)
};

// Stockham stages with an explicit points-per-thread E (may differ from fft_e<P>).
template <typename T, int P, int E, bool INV, bool HIN = false, bool HOUT = false>
__device__ __forceinline__ void line_fft_e(cpx<T> (&v)[E], cpx<T>* line, int t,
                                           const TwReg<T, P, E>& tr) {
  fft_stages_p<T, P, E, 1, INV, 0, HIN, HOUT>(v, LdsLine<T>{line}, t, tr.w);
}

// The six spectrum components of one frequency: one contiguous record.
template <typename T>
__device__ __forceinline__ void load_g6(const cpx<T>* __restrict__ sp, cpx<T> (&g)[6]) {
  if constexpr (sizeof(T) == 4) {
    const float4* p4 = reinterpret_cast<const float4*>(sp);
    const float4 a = p4[0], b = p4[1], c = p4[2];
    g[0] = mk<T>(a.x, a.y);
    g[1] = mk<T>(a.z, a.w);
    g[2] = mk<T>(b.x, b.y);
    g[3] = mk<T>(b.z, b.w);
    g[4] = mk<T>(c.x, c.y);
    g[5] = mk<T>(c.z, c.w);
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) g[k] = sp[k];
  }
}


// FAST: the z block is 16, the blocked layout holds exactly P/2 rows (N3
// rounded up to a multiple of 16 equals P/2) and the column tiles cover P1
// exactly, so the blocked offsets are shifts and no column needs a bounds
// test.  ZP (FAST with N3 < P/2): rows N3 .. P/2-1 of the layout are padding
// that nothing else reads; they are taken as zeros and never stored.
template <typename T, int P, int E, int NT, bool FAST, bool ZP>
__device__ __forceinline__ void z_green_body(cpx<T>* __restrict__ B,
                                             const cpx<T>* __restrict__ spec,
                                             const cpx<T>* __restrict__ tw, const ZArgs& a,
                                             const int* __restrict__ active) {
  constexpr int TT = P / E, W = NT / TT, LS = Pad<P>::LSTR;
  __shared__ cpx<T> lds[W * LS];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  // Block order (innermost first): right-hand side, +-xi_y mirror, x tile
  // taken in mirror pairs (k, tiles-1-k), y octant row.  Blocks that read the
  // same spectrum slice are adjacent, hence resident on one XCD together.
  const int rhs = b % a.nrhs;
  const int u = b / a.nrhs;
  const int m = u & 1;
  const int it = (u >> 1) % a.tiles_x;
  const int yp = (u >> 1) / a.tiles_x;
  if (m && (yp == 0 || 2 * yp == a.P2)) return;  // self-mirrored row: one block only
  const int xy = m ? a.P2 - yp : yp;
  const int tile = (it & 1) ? a.tiles_x - 1 - (it >> 1) : (it >> 1);
  if (active && !active[rhs]) return;
  const int cw = threadIdx.x % W, t = threadIdx.x / W;
  const int xx = tile * W + cw;
  // FP32 with shift addressing, 16 points per thread: rows move as 16-byte
  // column-pair segments; every column of such a launch is valid (FAST
  // launches need P1 % W == 0)
  constexpr bool PAIR = FAST && sizeof(T) == 4 && (E == 16 || E == 12);
  const bool valid = PAIR || xx < a.P1;
  // B[rhs][comp][z / zl][xi_y][z % zl][xi_x]; one base pointer per component,
  // offsets within a component fit in 32 bits (the setup checks that a
  // component of B has fewer than 2^31 elements)
  cpx<T>* col = B + rhs * a.rhs_stride + (int64_t)xy * a.zl * a.P1 + (valid ? xx : 0);
  cpx<T>* col1 = col + a.comp_stride;
  cpx<T>* col2 = col1 + a.comp_stride;
  int zoff[E / 2];
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int z = t + q * TT;
    if constexpr (FAST)
      zoff[q] = (z >> 4) * (int)a.zhs + (z & 15) * (int)a.zls;
    else
      zoff[q] = (z / a.zl) * (int)a.zhs + (z % a.zl) * (int)a.zls;
  }
  TwReg<T, P, E> tr;
  tr.load(t, tw);
  const int odd = cw & 1;
  cpx<T> v0[E], v1[E], v2[E];
  if constexpr (PAIR) {
    const float* cp = reinterpret_cast<const float*>(col - odd);
    const float* cp1 = reinterpret_cast<const float*>(col1 - odd);
    const float* cp2 = reinterpret_cast<const float*>(col2 - odd);
#pragma unroll
    for (int k = 0; k < E / 4; ++k) {
      const int zr = t + (2 * k + odd) * TT;  // this lane's row: point 2k (even) or 2k+1 (odd)
      const int off = 2 * ((zr >> 4) * (int)a.zhs + (zr & 15) * (int)a.zls);
      float4 f0 = *reinterpret_cast<const float4*>(cp + off);
      float4 f1 = *reinterpret_cast<const float4*>(cp1 + off);
      float4 f2 = *reinterpret_cast<const float4*>(cp2 + off);
      if (ZP && zr >= a.N3) f0 = f1 = f2 = make_float4(0.f, 0.f, 0.f, 0.f);
      pair_in(f0, odd, v0[2 * k], v0[2 * k + 1]);
      pair_in(f1, odd, v1[2 * k], v1[2 * k + 1]);
      pair_in(f2, odd, v2[2 * k], v2[2 * k + 1]);
    }
#pragma unroll
    for (int q = E / 2; q < E; ++q) v0[q] = v1[q] = v2[q] = mk<T>(0, 0);
  } else {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int z = t + q * TT;
      if (q < E / 2 && valid && ((FAST && !ZP) || z < a.N3)) {
        v0[q] = col[zoff[q]];
        v1[q] = col1[zoff[q]];
        v2[q] = col2[zoff[q]];
      } else {
        v0[q] = v1[q] = v2[q] = mk<T>(0, 0);
      }
    }
  }
  cpx<T>* line = lds + cw * LS;
  // z < N3 <= P/2: the upper half of every line is zero padding
  line_fft_e<T, P, E, false, true, false>(v0, line, t, tr);
  line_fft_e<T, P, E, false, true, false>(v1, line, t, tr);
  // octant coordinates and mirror flags; spectrum layout [yo][zo][xo][ab]
  const int xm = xx > a.P1 / 2, ym = xy > a.P2 / 2;
  const int xo = xm ? a.P1 - xx : xx, yo = ym ? a.P2 - xy : xy;
  // paired FP32 launches up to P = 256: the first ZPF spectrum records are
  // requested before the last forward transform, so their latency overlaps it
  constexpr int ZPF = (PAIR && P <= 256) ? 2 : 0;
  cpx<T> gpre[ZPF > 0 ? ZPF : 1][6];
  {
    const cpx<T>* s0 = spec + ((int64_t)yo * a.Q3 * a.Q1 + (valid ? xo : 0)) * 6;
#pragma unroll
    for (int q = 0; q < ZPF; ++q) {
      const int z = t + q * TT;
      load_g6<T>(s0 + (z > P / 2 ? P - z : z) * 6 * a.Q1, gpre[q]);
    }
  }
  line_fft_e<T, P, E, false, true, false>(v2, line, t, tr);
  const cpx<T>* sxy = spec + ((int64_t)yo * a.Q3 * a.Q1 + (valid ? xo : 0)) * 6;
  const int zstep = 6 * a.Q1;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int z = t + q * TT;
    const int zm = z > P / 2;
    const int zo = zm ? P - z : z;
    cpx<T> gg[6];
    if (q < ZPF) {
#pragma unroll
      for (int k = 0; k < 6; ++k) gg[k] = gpre[q < ZPF ? q : 0][k];
    } else {
      load_g6<T>(sxy + zo * zstep, gg);
    }
    const cpx<T> gxx = gg[0], gyy = gg[3], gzz = gg[5];
    cpx<T> gxy = gg[1], gxz = gg[2], gyz = gg[4];
    // G_ab is odd along axis e iff exactly one of a, b equals e
    if (xm ^ ym) gxy = mk<T>(-gxy.re, -gxy.im);
    if (xm ^ zm) gxz = mk<T>(-gxz.re, -gxz.im);
    if (ym ^ zm) gyz = mk<T>(-gyz.re, -gyz.im);
    const cpx<T> ix = v0[q], iy = v1[q], iz = v2[q];
    v0[q] = cfma(gxz, iz, cfma(gxy, iy, gxx * ix));
    v1[q] = cfma(gyz, iz, cfma(gyy, iy, gxy * ix));
    v2[q] = cfma(gzz, iz, cfma(gyz, iy, gxz * ix));
  }
  // only z < N3 <= P/2 is stored
  line_fft_e<T, P, E, true, false, true>(v0, line, t, tr);
  line_fft_e<T, P, E, true, false, true>(v1, line, t, tr);
  line_fft_e<T, P, E, true, false, true>(v2, line, t, tr);
  if constexpr (PAIR) {
    float* cp = reinterpret_cast<float*>(col - odd);
    float* cp1 = reinterpret_cast<float*>(col1 - odd);
    float* cp2 = reinterpret_cast<float*>(col2 - odd);
#pragma unroll
    for (int k = 0; k < E / 4; ++k) {
      const int zr = t + (2 * k + odd) * TT;
      const int off = 2 * ((zr >> 4) * (int)a.zhs + (zr & 15) * (int)a.zls);
      // the lane swaps run on every lane; padding rows are not stored
      const float4 o0 = pair_out(odd, v0[2 * k], v0[2 * k + 1]);
      const float4 o1 = pair_out(odd, v1[2 * k], v1[2 * k + 1]);
      const float4 o2 = pair_out(odd, v2[2 * k], v2[2 * k + 1]);
      if (!ZP || zr < a.N3) {
        *reinterpret_cast<float4*>(cp + off) = o0;
        *reinterpret_cast<float4*>(cp1 + off) = o1;
        *reinterpret_cast<float4*>(cp2 + off) = o2;
      }
    }
    return;
  }
  if (valid) {
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int z = t + q * TT;
      if ((FAST && !ZP) || z < a.N3) {
        col[zoff[q]] = v0[q];
        col1[zoff[q]] = v1[q];
        col2[zoff[q]] = v2[q];
      }
    }
  }
}

template <typename T, int P, int E, int NT, bool FAST, bool ZP = false>
__global__ __launch_bounds__(NT) void k_fft_z_green(
    cpx<T>* __restrict__ B, const cpx<T>* __restrict__ spec, const cpx<T>* __restrict__ tw,
    ZArgs a, const int* __restrict__ active) {
  z_green_body<T, P, E, NT, FAST, ZP>(B, spec, tw, a, active);
}

// ------------------------------------------------ X inverse + epilogue
struct XinvArgs {
  int N1, N2, N3, lines_per_rhs, lines_per_comp, blocks_per_rhs;
  int64_t n;
};

template <typename T, int P, int MODE>
__global__ __launch_bounds__(nt_lines_p<T>(P)) void k_fft_x_inv(
    const cpx<T>* __restrict__ A, const c64* __restrict__ xin, c64* __restrict__ yout,
    const double* __restrict__ chi, const int* __restrict__ rhs_body,
    const cpx<T>* __restrict__ tw, XinvArgs a, c64* __restrict__ aux, c64* __restrict__ partials,
    const c64* __restrict__ pol, const c64* __restrict__ ph, const int* __restrict__ active) {
  constexpr int E = fft_e<P>(), TT = P / E, NT = nt_lines_p<T>(P), L = NT / TT;
  __shared__ cpx<T> lds[L * Pad<P>::LSTR];
  __shared__ double red[4 * (NT / 64 + 1)];
  // hardware order (see the forward x pass)
  const int b = blockIdx.x;
  const int rhs = b / a.blocks_per_rhs, blk = b % a.blocks_per_rhs;
  if (active && !active[rhs]) return;
  const int li = threadIdx.x / TT, t = threadIdx.x % TT;
  const int line = blk * L + li;
  const bool valid = line < a.lines_per_rhs;
  const int lc = valid ? line : 0;
  const size_t gl = (size_t)rhs * a.lines_per_rhs + lc;
  TwReg<T, P, E> tr;
  tr.load(t, tw);
  cpx<T> v[E];
  {
    const cpx<T>* src = A + gl * P;
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = valid ? src[t + q * TT] : mk<T>(0, 0);
  }
  line_fft<T, P, true, false, true>(v, lds + li * Pad<P>::LSTR, t, tr);  // only x < N1 kept
  const int comp = lc / a.lines_per_comp, sp = lc % a.lines_per_comp;  // sp = z*N2 + y
  const double* chib = chi + (int64_t)rhs_body[rhs] * a.n + (int64_t)sp * a.N1;
  c64 s0 = mk(0.0, 0.0), s1 = mk(0.0, 0.0);
  c64 phyz = mk(0.0, 0.0), pc = mk(0.0, 0.0);
  if (MODE == EPI_RESID && valid) {
    const c64* phr = ph + (int64_t)rhs * (a.N1 + a.N2 + a.N3);
    const int y = sp % a.N2, z = sp / a.N2;
    phyz = phr[a.N1 + y] * phr[a.N1 + a.N2 + z];
    pc = pol[rhs * 3 + comp];
  }
  if (valid) {
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int xi = t + q * TT;
      if (xi < a.N1) {
        const size_t gi = gl * a.N1 + xi;
        const double c = chib[xi];
        const c64 conv = cvt<double>(v[q]);
        const c64 xv = xin[gi];
        const c64 y = xv - c * conv;
        if (MODE == EPI_RESID) {
          const c64 e = pc * (phyz * ph[(int64_t)rhs * (a.N1 + a.N2 + a.N3) + xi]);
          const c64 r = c * e - y;
          yout[gi] = r;
          aux[gi] = r;
          s1.re += r.re * r.re + r.im * r.im;
        } else {
          yout[gi] = y;
          if (MODE == EPI_RHV) {
            s0 = s0 + cmulc(aux[gi], y);
          } else if (MODE == EPI_TS) {
            s0 = s0 + cmulc(y, xv);
            s1.re += y.re * y.re + y.im * y.im;
          }
        }
      }
    }
  }
  if (MODE != EPI_PLAIN) {
    block_sum2(s0, s1, red);
    if (threadIdx.x == 0) {
      c64* pp = partials + ((size_t)rhs * a.blocks_per_rhs + blk) * 2;
      pp[0] = s0;
      pp[1] = s1;
    }
  }
}

// ================================================================ launchers
template <typename T>
static hipError_t x_fwd(const GroupGeom& g, const c64* x, cpx<T>* A, const cpx<T>* tw,
                        const int* active, hipStream_t s) {
  const int lines = 3 * g.N[1] * g.N[2];
  const int L = lines_per_block<T>(g.P[0]);
  const int bpr = (lines + L - 1) / L;
  const dim3 grid(bpr * g.nrhs);
  VIE_DISPATCH_P(g.P[0], (k_fft_x_fwd<double, T, PP, true><<<grid, nt_lines_p<T>(PP), 0, s>>>(
                             x, A, tw, g.N[0], lines, bpr, active)));
  return hipGetLastError();
}

// Scratch layouts: A[rhs][comp][z][y][xi_x] (x pass side),
// B[rhs][comp][z / zl][xi_y][z % zl][xi_x] (z pass side).
static SideAddr side_A(const GroupGeom& g, int zl) {
  SideAddr s;
  const int64_t plane = (int64_t)g.N[1] * g.P[0];
  s.row = g.P[0];
  s.zls = plane;
  s.zhs = plane * zl;
  s.cs = plane * g.N[2];
  s.rs = s.cs * 3;
  return s;
}
static SideAddr side_B(const GroupGeom& g, int zl) {
  SideAddr s;
  const int nzh = (g.N[2] + zl - 1) / zl;
  s.row = (int64_t)zl * g.P[0];
  s.zls = g.P[0];
  s.zhs = (int64_t)g.P[1] * zl * g.P[0];
  s.cs = s.zhs * nzh;
  s.rs = s.cs * 3;
  return s;
}
int z_block(const GroupGeom& g) { return g.N[2] < 16 ? g.N[2] : 16; }
int64_t bufB_elems(const GroupGeom& g) {
  const int zl = z_block(g);
  return side_B(g, zl).rs;  // per right-hand side
}

// Workgroup size of the y passes: enough threads that each row access is a
// 128-byte run of columns, at least nt_lines; long lines (P > 512) are capped
// at 1024 threads and about 150 KB of LDS (W padded lines), so they get fewer
// columns per workgroup.
template <typename T, int P>
constexpr int y_threads() {
  constexpr int tt = P / fft_e<P>();
  int v = (int)(128 / sizeof(cpx<T>)) * tt;
  if (v < nt_lines<T>()) v = nt_lines<T>();
  while (v > tt && (v > 1024 || (v / tt) * Pad<P>::LSTR * (int)sizeof(cpx<T>) > 150 * 1024))
    v /= 2;
  return v < tt ? tt : v;
}

template <typename T, int PP>
static void y_launch(const GroupGeom& g, const cpx<T>* in, cpx<T>* out, const cpx<T>* tw,
                     bool inverse, const int* active, hipStream_t s) {
  const int P1 = g.P[0], N2 = g.N[1], N3 = g.N[2];
  const int zl = z_block(g);
  constexpr int ntY = y_threads<T, PP>();
  constexpr int W = ntY / (PP / fft_e<PP>());
  StridedArgs a;
  a.ncols = P1;
  a.ncomp = 3;
  a.nz = N3;
  a.zl = zl;
  a.tiles = (P1 + W - 1) / W;
  const SideAddr A = side_A(g, zl), B = side_B(g, zl);
  if (!inverse) {
    a.n_in_rows = N2;
    a.n_out_rows = PP;
    a.in = A;
    a.out = B;
  } else {
    a.n_in_rows = PP;
    a.n_out_rows = N2;
    a.in = B;
    a.out = A;
  }
  const dim3 grid(a.tiles * 3 * N3 * g.nrhs);
  if (!inverse)
    k_fft_strided<T, PP, true, false, false, ntY><<<grid, ntY, 0, s>>>(in, out, tw, a, active);
  else
    k_fft_strided<T, PP, false, true, true, ntY><<<grid, ntY, 0, s>>>(in, out, tw, a, active);
}

template <typename T>
static hipError_t y_pass(const GroupGeom& g, const cpx<T>* in, cpx<T>* out, const cpx<T>* tw,
                         bool inverse, const int* active, hipStream_t s) {
  VIE_DISPATCH_P(g.P[1], (y_launch<T, PP>(g, in, out, tw, inverse, active, s)));
  return hipGetLastError();
}

// Register-lean z pass (autotuner shape 2, FAST layouts only): one column
// per lane at E points (8 FP32, 4 FP64; 6 for 3 * 2^k lines) of all three
// components, 256 threads, registers capped at 128 so that four waves share
// each SIMD (twice the FP32 16-point shape) and memory and transform phases
// of different workgroups overlap.  The spectrum record of the next point is
// requested while the current one is multiplied (the first one before the
// last forward transform); the empty asm statements keep the compiler from
// issuing every point's loads at once.  Block order, octant lookup and signs
// as the other shapes.
template <typename T>
constexpr int lean_e(int P) {
  return sizeof(T) == 4 ? (P % 3 == 0 ? 6 : 8) : (P % 3 == 0 ? 6 : 4);
}
constexpr int kLeanThreads = 256;
template <typename T, int P, bool ZP>
__global__ __launch_bounds__(kLeanThreads) __attribute__((amdgpu_waves_per_eu(4))) void
k_fft_z_green_lean(cpx<T>* __restrict__ B, const cpx<T>* __restrict__ spec,
                   const cpx<T>* __restrict__ tw, ZArgs a, const int* __restrict__ active) {
  constexpr int E = lean_e<T>(P), TT = P / E, W = kLeanThreads / TT, LS = Pad<P>::LSTR;
  __shared__ cpx<T> lds[W * LS];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int rhs = b % a.nrhs;
  const int u = b / a.nrhs;
  const int m = u & 1;
  const int it = (u >> 1) % a.tiles_x;
  const int yp = (u >> 1) / a.tiles_x;
  if (m && (yp == 0 || 2 * yp == a.P2)) return;  // self-mirrored row: one block only
  const int xy = m ? a.P2 - yp : yp;
  const int tile = (it & 1) ? a.tiles_x - 1 - (it >> 1) : (it >> 1);
  if (active && !active[rhs]) return;
  const int cw = threadIdx.x % W, t = threadIdx.x / W;
  const int xx = tile * W + cw;  // the tiles cover P1 exactly
  cpx<T>* col = B + rhs * a.rhs_stride + (int64_t)xy * a.zl * a.P1 + xx;
  cpx<T>* col1 = col + a.comp_stride;
  cpx<T>* col2 = col1 + a.comp_stride;
  const int zhs = (int)a.zhs, zls = (int)a.zls;
  TwReg<T, P, E> tr;
  tr.load(t, tw);
  cpx<T> v0[E], v1[E], v2[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    v0[q] = v1[q] = v2[q] = mk<T>(0, 0);
    const int z = t + q * TT;
    if (q < E / 2 && (!ZP || z < a.N3)) {  // padding rows are neither read nor written
      const int off = (z >> 4) * zhs + (z & 15) * zls;
      v0[q] = col[off];
      v1[q] = col1[off];
      v2[q] = col2[off];
    }
  }
  const int xm = xx > a.P1 / 2, ym = xy > a.P2 / 2;
  const int xo = xm ? a.P1 - xx : xx, yo = ym ? a.P2 - xy : xy;
  const cpx<T>* sxy = spec + ((int64_t)yo * a.Q3 * a.Q1 + xo) * 6;
  auto rec = [&](int q) {
    const int z = t + q * TT;
    return sxy + (int64_t)(z > P / 2 ? P - z : z) * 6 * a.Q1;
  };
  cpx<T>* line = lds + cw * LS;
  line_fft_e<T, P, E, false, true, false>(v0, line, t, tr);
  line_fft_e<T, P, E, false, true, false>(v1, line, t, tr);
  cpx<T> gn[6];
  load_g6<T>(rec(0), gn);
  asm volatile("" ::: "memory");
  line_fft_e<T, P, E, false, true, false>(v2, line, t, tr);
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int zm = t + q * TT > P / 2;
    cpx<T> gg[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gg[k] = gn[k];
    if (q + 1 < E) load_g6<T>(rec(q + 1), gn);
    asm volatile("" ::: "memory");
    const cpx<T> gxx = gg[0], gyy = gg[3], gzz = gg[5];
    cpx<T> gxy = gg[1], gxz = gg[2], gyz = gg[4];
    // G_ab is odd along axis e iff exactly one of a, b equals e
    if (xm ^ ym) gxy = mk<T>(-gxy.re, -gxy.im);
    if (xm ^ zm) gxz = mk<T>(-gxz.re, -gxz.im);
    if (ym ^ zm) gyz = mk<T>(-gyz.re, -gyz.im);
    const cpx<T> ix = v0[q], iy = v1[q], iz = v2[q];
    v0[q] = cfma(gxz, iz, cfma(gxy, iy, gxx * ix));
    v1[q] = cfma(gyz, iz, cfma(gyy, iy, gxy * ix));
    v2[q] = cfma(gzz, iz, cfma(gyz, iy, gxz * ix));
  }
  line_fft_e<T, P, E, true, false, true>(v0, line, t, tr);
  line_fft_e<T, P, E, true, false, true>(v1, line, t, tr);
  line_fft_e<T, P, E, true, false, true>(v2, line, t, tr);
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int z = t + q * TT;
    if (!ZP || z < a.N3) {
      const int off = (z >> 4) * zhs + (z & 15) * zls;
      col[off] = v0[q];
      col1[off] = v1[q];
      col2[off] = v2[q];
    }
  }
}

template <typename T, int PP, int V>
static void z_launch(const GroupGeom& g, ZArgs a, cpx<T>* B, const cpx<T>* spec,
                     const cpx<T>* tw, const int* active, hipStream_t s) {
  if constexpr (V == 2) {
    // FP64 3 * 2^k lines would spill at the register cap: they keep shape 0
    if constexpr (PP >= 32 && PP <= 128 && (sizeof(T) == 4 || PP % 3 != 0)) {
      constexpr int W = kLeanThreads / (PP / lean_e<T>(PP));
      if (a.zl == 16 && 2 * ((a.N3 + 15) / 16) * 16 == PP && g.P[0] % W == 0) {
        a.tiles_x = g.P[0] / W;
        const dim3 grid((g.P[1] / 2 + 1) * 2 * a.tiles_x * g.nrhs);
        if (2 * a.N3 == PP)
          k_fft_z_green_lean<T, PP, false><<<grid, kLeanThreads, 0, s>>>(B, spec, tw, a, active);
        else
          k_fft_z_green_lean<T, PP, true><<<grid, kLeanThreads, 0, s>>>(B, spec, tw, a, active);
        return;
      }
    }
    z_launch<T, PP, 0>(g, a, B, spec, tw, active, s);  // layouts the lean kernel does not take
    return;
  } else {
  constexpr ZShape sh = zshape<T>(V);
  constexpr int E = zcap<PP, sh.e>();
  constexpr int W = sh.nt / (PP / E);
  a.tiles_x = (g.P[0] + W - 1) / W;
  const dim3 grid((g.P[1] / 2 + 1) * 2 * a.tiles_x * g.nrhs);
  if constexpr (PP >= 32) {
    // FAST: the blocked layout holds exactly PP/2 rows (see z_green_body)
    if (a.zl == 16 && 2 * ((a.N3 + 15) / 16) * 16 == PP && g.P[0] % W == 0) {
      if (2 * a.N3 == PP)
        k_fft_z_green<T, PP, E, sh.nt, true, false><<<grid, sh.nt, 0, s>>>(B, spec, tw, a, active);
      else
        k_fft_z_green<T, PP, E, sh.nt, true, true><<<grid, sh.nt, 0, s>>>(B, spec, tw, a, active);
      return;
    }
  }
  k_fft_z_green<T, PP, E, sh.nt, false><<<grid, sh.nt, 0, s>>>(B, spec, tw, a, active);
  }
}

template <typename T>
static hipError_t z_pass(const GroupGeom& g, cpx<T>* B, const cpx<T>* spec, const cpx<T>* tw,
                         const int* active, hipStream_t s, int variant) {
  ZArgs a;
  a.N3 = g.N[2];
  a.P1 = g.P[0];
  a.P2 = g.P[1];
  a.Q1 = g.Q[0];
  a.Q2 = g.Q[1];
  a.Q3 = g.Q[2];
  a.nrhs = g.nrhs;
  a.zl = z_block(g);
  const SideAddr sb = side_B(g, a.zl);
  a.comp_stride = sb.cs;
  a.rhs_stride = sb.rs;
  a.zhs = sb.zhs;
  a.zls = sb.zls;
  VIE_DISPATCH_PZ(g.P[2], ({
                   switch (variant) {
                     case 1: z_launch<T, PP, 1>(g, a, B, spec, tw, active, s); break;
                     case 2: z_launch<T, PP, 2>(g, a, B, spec, tw, active, s); break;
                     default: z_launch<T, PP, 0>(g, a, B, spec, tw, active, s); break;
                   }
                 }));
  return hipGetLastError();
}

// ------------------------------- approximate products: packed FP16 passes
// The block solves of the block-Jacobi preconditioner only approximate its
// inverse, so their products may run the y and z passes in FP16 arithmetic
// on packed pairs (v_pk_fma_f16 and friends: two columns per register, twice
// the FP32 rate) with both scratch buffers in FP16: a cpx<h2> holds columns
// 2p and 2p + 1 of one row, so the FP32 layouts apply with every stride
// halved and pair indices for columns.  The x passes transform in FP32 and
// convert at the scratch side.
//
// Range: the input is a unit-norm basis vector x.  Each forward pass scales
// its input by a power of two h_d <= 1 / sqrt(N_d) (N_d the box extent along
// the axis), so by Cauchy-Schwarz every forward value of component b is at
// most the 2-norm of x_b over the lines it sums (|sum of N_d terms| <=
// sqrt(N_d) times their 2-norm), hence within one.  The spectrum copy is
// scaled by gs = 2^-ceil(log2 max|G|) (entries within one), so a product
// point is at most 3.  The inverse passes are unnormalised; with Parseval
// along each axis the values after the inverse z pass are at most
// sqrt(3) P3 / sqrt(N3), after the inverse y pass at most
// sqrt(3) P2 P3 / sqrt(N2 N3) -- a few hundred for these grids, far inside
// the FP16 range.  The FP32 inverse x pass scales back by 1 / (h1 h2 h3 gs).
//
// The spectrum copy is pair-packed: record (yo, zo, p) holds the six
// entries of columns 2p and 2p + 1 as packed halves (octant lookups and the
// x-mirror signs already applied), scaled by gs.

// y pass on packed pairs (the forward pass scales its input by hs).
template <int P, bool INV, int NTB>
__global__ __launch_bounds__(NTB) void k_fft_y_h2(const cpx<h2>* __restrict__ in,
                                                 cpx<h2>* __restrict__ out,
                                                 const cpx<h2>* __restrict__ tw, StridedArgs a,
                                                 float hs, const int* __restrict__ active) {
  constexpr int E = fft_e<P>(), TT = P / E, W = NTB / TT;
  __shared__ cpx<h2> lds[W * Pad<P>::LSTR];
  // block order as the FP32 strided pass
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int per_rhs = a.ncomp * a.nz;
  const int nrhs_l = gridDim.x / (a.tiles * per_rhs);
  const int rhs = b % nrhs_l, rest = b / nrhs_l;
  const int tile = rest % a.tiles, cz = rest / a.tiles;
  if (active && !active[rhs]) return;
  const int comp = cz / a.nz, z = cz % a.nz;
  const int cw = threadIdx.x % W, t = threadIdx.x / W;
  const int col = tile * W + cw;
  const bool valid = col < a.ncols;
  const cpx<h2>* pin = in + slab_base(a.in, rhs, comp, z, a.zl) + (valid ? col : 0);
  TwReg<h2, P, E> tr;
  tr.load(t, tw);
  const h2 sc = {(_Float16)hs, (_Float16)hs};
  cpx<h2> v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int row = t + q * TT;
    if ((INV || q < E / 2) && valid && row < a.n_in_rows) {
      v[q] = pin[(int64_t)row * a.in.row];
      if constexpr (!INV) v[q] = hscale(v[q], sc);
    } else {
      v[q] = mk<h2>(h2{0, 0}, h2{0, 0});
    }
  }
  line_fft<h2, P, INV, !INV, INV>(v, lds + cw * Pad<P>::LSTR, t, tr);
  if (valid) {
    cpx<h2>* po = out + slab_base(a.out, rhs, comp, z, a.zl) + col;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int row = t + q * TT;
      if ((!INV || q < E / 2) && row < a.n_out_rows) po[(int64_t)row * a.out.row] = v[q];
    }
  }
}

// Fused x and y passes of the packed path: one workgroup per (right-hand
// side, component, z) plane keeps the plane's x-transformed lines in LDS as
// packed pairs (N2 rows of P1 / 2 pairs), so the x-y scratch never goes to
// HBM.  Forward: the plane's x lines are scattered from the compressed
// bfloat16 vector and transformed in FP32 (L1 lines at a time), converted
// into the plane (scale h1), then the column pairs are transformed along y in
// packed FP16 (W2 at a time, scale h2) and written to the y/z scratch.
// Inverse: the reverse, ending in the compressed product epilogue
// y = x - chi (conv / (h1 h2 h3 gs)).  The x and y phases share one LDS
// buffer for their transform lines.
template <int P1, int P2>
struct XYShape {
  static constexpr int NT = 256;
  // 8 points per thread on 128-point lines (16 threads a line): fewer lines
  // in flight per phase, so three workgroups share a CU
  static constexpr int E1 = P1 == 128 ? 8 : fft_e<P1>(), TT1 = P1 / E1, L1 = NT / TT1;
  static constexpr int E2 = P2 == 128 ? 8 : fft_e<P2>(), TT2 = P2 / E2, W2 = NT / TT2;
  static constexpr int PS = P1 / 2;               // packed pairs per plane row
  static constexpr int NBX = (P2 / 2 + L1 - 1) / L1;  // x-line batches (N2 <= P2 / 2)
  static constexpr int NP = P1 / 2;               // column pairs
  static constexpr int PLANE = (P2 / 2) * PS;     // rows N2 <= P2 / 2
  static constexpr int XLS = PadX<P1, TT1>::LSTR;  // x-line stride
  static constexpr int XB = L1 * XLS * (int)sizeof(c32);
  static constexpr int YB = W2 * Pad<P2>::LSTR * (int)sizeof(cpx<h2>);
  static constexpr int UB = XB > YB ? XB : YB;
  static_assert(NT % TT1 == 0 && NT % TT2 == 0 && TT1 % 2 == 0, "fused x-y shape");
};

// NRM: the input is an FP32 work vector, normalised per right-hand side
// (see MatvecArgs::npart) into the bfloat16 vector vout on the way in.
template <int P1, int P2, bool NRM>
__global__ __launch_bounds__(256) void k_fft_xy_fwd_h2(
    const void* __restrict__ xcv, cpx<h2>* __restrict__ B, const c32* __restrict__ tw1,
    const cpx<h2>* __restrict__ tw2, BodyIdx bi, int N1, int N2, int N3, SideAddr sb, int zl,
    float hs1, float hs2, const int* __restrict__ active, const double* __restrict__ npart,
    int nblk, double* __restrict__ nrm, int ldn, cb16* __restrict__ vout) {
  using TXI = typename std::conditional<NRM, c32, cb16>::type;
  using S = XYShape<P1, P2>;
  __shared__ cpx<h2> plane[S::PLANE];
  __shared__ __align__(16) char ubuf[S::UB];
  const int nrhs = gridDim.x / (3 * N3);
  const int rhs = blockIdx.x % nrhs, cz = blockIdx.x / nrhs;
  if (active && !active[rhs]) return;
  const int comp = cz / N3, z = cz % N3;
  const int body = bi.rhs_body[rhs];
  const int nb = bi.nb[body];
  const int* vox = bi.vox + bi.voff[body];
  const int* lp = bi.line_ptr + (int64_t)body * (N2 * N3 + 1);
  const TXI* xv = reinterpret_cast<const TXI*>(xcv) + bi.roff[rhs] + (int64_t)comp * nb;
  cb16* vo = NRM ? vout + bi.roff[rhs] + (int64_t)comp * nb : nullptr;
  double sc = 1.0;
  if constexpr (NRM) {
    // ||w||^2 of this right-hand side: every wave sums the partials in the
    // order of the separate reduction (lane-strided, then a fixed butterfly)
    double t2 = 0.0;
    for (int k = threadIdx.x & 63; k < nblk; k += 64) t2 += npart[(int64_t)rhs * nblk + k];
    for (int mk = 32; mk >= 1; mk >>= 1) t2 += __shfl_xor(t2, mk);
    sc = t2 > 0.0 ? 1.0 / sqrt(t2) : 0.0;
    if (comp == 0 && z == 0 && threadIdx.x == 0) nrm[(int64_t)rhs * ldn] = t2;
  }
  {  // x: FP32 lines into the plane, S::L1 lines a batch
    constexpr int E = S::E1, TT = S::TT1;
    const int li = threadIdx.x / TT, t = threadIdx.x % TT, odd = t & 1;
    cpx<float>* myl = reinterpret_cast<cpx<float>*>(ubuf) + li * S::XLS;
    TwReg<float, P1, E> tr;
    tr.load(t, tw1);
    // the line pointers of this thread's line in every batch, in one round of
    // loads; each batch's voxels (at most P1 / 2 a line, so E / 2 a thread)
    // are requested while the previous batch is transformed
    int lpa[S::NBX], lpb[S::NBX];
#pragma unroll
    for (int n = 0; n < S::NBX; ++n) {
      const int y = n * S::L1 + li;
      lpa[n] = lpb[n] = 0;
      if (y < N2) {
        lpa[n] = lp[z * N2 + y];
        lpb[n] = lp[z * N2 + y + 1];
      }
    }
    int kv[E / 2];
    TXI xr[E / 2];
    auto fetch = [&](int n) {
      const int k0 = lpa[n] + t, k1 = lpb[n];
#pragma unroll
      for (int i = 0; i < E / 2; ++i) {
        const int k = k0 + i * TT;
        if (k < k1) {
          kv[i] = vox[k];
          xr[i] = xv[k];
        }
      }
    };
    fetch(0);
#pragma unroll
    for (int n = 0; n < S::NBX; ++n) {
      if (n * S::L1 >= N2) break;
      const int y = n * S::L1 + li;
      const bool valid = y < N2;
      lds_barrier();  // the previous lines' last transform stage has read the buffer
#pragma unroll
      for (int q = 0; q < E / 2; ++q) myl[pidx(t + q * TT)] = mk<float>(0, 0);
      lds_barrier();
      {
        const int k0 = lpa[n] + t, k1 = lpb[n], base = (z * N2 + y) * N1;
#pragma unroll
        for (int i = 0; i < E / 2; ++i) {
          if (k0 + i * TT >= k1) continue;
          if constexpr (NRM) {
            // the basis vector as stored (bfloat16 through FP32) is what is multiplied
            const c64 wn = sc * cvt<double>(xr[i]);
            cb16 b16;
            b16.re = (__bf16)(float)wn.re;
            b16.im = (__bf16)(float)wn.im;
            vo[k0 + i * TT] = b16;
            myl[pidx(kv[i] - base)] = cvt<float>(b16);
          } else {
            myl[pidx(kv[i] - base)] = cvt<float>(xr[i]);
          }
        }
      }
      lds_barrier();
      if (n + 1 < S::NBX) fetch(n + 1);
      cpx<float> v[E];
#pragma unroll
      for (int q = 0; q < E; ++q) v[q] = (q < E / 2) ? myl[pidx(t + q * TT)] : mk<float>(0, 0);
      line_fft_e<float, P1, E, false, true, false>(v, myl, t, tr);
      // lanes t, t + 1 hold neighbouring points: one exchange packs a pair
#pragma unroll
      for (int q = 0; q < E; q += 2) {
        const float4 f = pair_out(odd, v[q], v[q + 1]);
        if (valid)
          plane[y * S::PS + ((t - odd + (q + odd) * TT) >> 1)] =
              pack2(f.x * hs1, f.y * hs1, f.z * hs1, f.w * hs1);
      }
    }
  }
  lds_barrier();  // the plane is complete and the line buffer free
  {  // y: packed column pairs from the plane to the y/z scratch
    constexpr int E = S::E2, TT = S::TT2;
    const int cw = threadIdx.x % S::W2, t = threadIdx.x / S::W2;
    cpx<h2>* myl = reinterpret_cast<cpx<h2>*>(ubuf) + cw * Pad<P2>::LSTR;
    TwReg<h2, P2, E> tr;
    tr.load(t, tw2);
    const h2 sc = {(_Float16)hs2, (_Float16)hs2};
    cpx<h2>* po = B + slab_base(sb, rhs, comp, z, zl);
    for (int p0 = 0; p0 < S::NP; p0 += S::W2) {
      const int p = p0 + cw;
      const bool valid = p < S::NP;
      cpx<h2> v[E];
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int row = t + q * TT;
        v[q] = (q < E / 2 && valid && row < N2) ? hscale(plane[row * S::PS + p], sc)
                                               : mk<h2>(h2{0, 0}, h2{0, 0});
      }
      line_fft_e<h2, P2, E, false, true, false>(v, myl, t, tr);
      if (valid) {
#pragma unroll
        for (int q = 0; q < E; ++q) po[(int64_t)(t + q * TT) * sb.row + p] = v[q];
      }
    }
  }
}

template <int P1, int P2>
__global__ __launch_bounds__(256) void k_fft_yx_inv_h2(
    const cpx<h2>* __restrict__ B, const cb16* __restrict__ xin, c32* __restrict__ yout,
    const c32* __restrict__ tw1, const cpx<h2>* __restrict__ tw2, BodyIdx bi, int N1, int N2,
    int N3, SideAddr sb, int zl, float hs, const int* __restrict__ active) {
  using S = XYShape<P1, P2>;
  __shared__ cpx<h2> plane[S::PLANE];
  __shared__ __align__(16) char ubuf[S::UB];
  const int nrhs = gridDim.x / (3 * N3);
  const int rhs = blockIdx.x % nrhs, cz = blockIdx.x / nrhs;
  if (active && !active[rhs]) return;
  const int comp = cz / N3, z = cz % N3;
  // The epilogue's operands of this thread's x line in every batch (line
  // pointers first, in one round; then each batch's voxels, at most P1 / 2 a
  // line, so E1 / 2 a thread) are requested ahead: the first batch's before
  // the y phase, each next one while the current batch is finished.
  const int body = bi.rhs_body[rhs];
  const int nb = bi.nb[body];
  const int* vox = bi.vox + bi.voff[body];
  const double* chic = bi.chic + bi.voff[body];
  const int* lp = bi.line_ptr + (int64_t)body * (N2 * N3 + 1);
  const int64_t vb = bi.roff[rhs] + (int64_t)comp * nb;
  const int lix = threadIdx.x / S::TT1, tx = threadIdx.x % S::TT1;
  int lpa[S::NBX], lpb[S::NBX];
#pragma unroll
  for (int n = 0; n < S::NBX; ++n) {
    const int y = n * S::L1 + lix;
    lpa[n] = lpb[n] = 0;
    if (y < N2) {
      lpa[n] = lp[z * N2 + y];
      lpb[n] = lp[z * N2 + y + 1];
    }
  }
  int kv[S::E1 / 2];
  double cv[S::E1 / 2];
  cb16 xr[S::E1 / 2];
  auto fetch = [&](int n) {
    const int k0 = lpa[n] + tx, k1 = lpb[n];
#pragma unroll
    for (int i = 0; i < S::E1 / 2; ++i) {
      const int k = k0 + i * S::TT1;
      if (k < k1) {
        kv[i] = vox[k];
        cv[i] = chic[k];
        xr[i] = xin[vb + k];
      }
    }
  };
  fetch(0);
  {  // inverse y: packed column pairs from the y/z scratch into the plane (rows < N2)
    constexpr int E = S::E2, TT = S::TT2;
    const int cw = threadIdx.x % S::W2, t = threadIdx.x / S::W2;
    cpx<h2>* myl = reinterpret_cast<cpx<h2>*>(ubuf) + cw * Pad<P2>::LSTR;
    TwReg<h2, P2, E> tr;
    tr.load(t, tw2);
    const cpx<h2>* pin = B + slab_base(sb, rhs, comp, z, zl);
    for (int p0 = 0; p0 < S::NP; p0 += S::W2) {
      const int p = p0 + cw;
      const bool valid = p < S::NP;
      cpx<h2> v[E];
#pragma unroll
      for (int q = 0; q < E; ++q)
        v[q] = valid ? pin[(int64_t)(t + q * TT) * sb.row + p] : mk<h2>(h2{0, 0}, h2{0, 0});
      line_fft_e<h2, P2, E, true, false, true>(v, myl, t, tr);
      if (valid) {
#pragma unroll
        for (int q = 0; q < E / 2; ++q) {
          const int row = t + q * TT;
          if (row < N2) plane[row * S::PS + p] = v[q];
        }
      }
    }
  }
  lds_barrier();  // the plane is complete and the line buffer free
  {  // inverse x in FP32 and the compressed epilogue, L1 lines at a time
    constexpr int E = S::E1, TT = S::TT1;
    const int li = lix, t = tx, odd = t & 1;
    cpx<float>* myl = reinterpret_cast<cpx<float>*>(ubuf) + li * S::XLS;
    TwReg<float, P1, E> tr;
    tr.load(t, tw1);
#pragma unroll
    for (int n = 0; n < S::NBX; ++n) {
      if (n * S::L1 >= N2) break;
      const int y = n * S::L1 + li;
      const bool valid = y < N2;
      cpx<float> v[E];
#pragma unroll
      for (int q = 0; q < E; q += 2) {
        float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid) f = unpack2(plane[y * S::PS + ((t - odd + (q + odd) * TT) >> 1)]);
        pair_in(f, odd, v[q], v[q + 1]);
      }
      line_fft_e<float, P1, E, true, false, true>(v, myl, t, tr);  // only x < N1 is used
      lds_barrier();  // every thread has left the transform's last LDS read
#pragma unroll
      for (int q = 0; q < E / 2; ++q) myl[pidx(t + q * TT)] = v[q];
      lds_barrier();
      {
        const int k0 = lpa[n] + t, k1 = lpb[n], base = (z * N2 + y) * N1;
#pragma unroll
        for (int i = 0; i < E / 2; ++i) {
          const int k = k0 + i * TT;
          if (k >= k1) continue;
          const c64 conv = (double)hs * cvt<double>(myl[pidx(kv[i] - base)]);
          const c64 r = cvt<double>(xr[i]) - cv[i] * conv;
          yout[vb + k] = cvt<float>(r);
        }
      }
      if (n + 1 < S::NBX) fetch(n + 1);
    }
  }
}

__device__ __forceinline__ void load_g6h(const cpx<h2>* __restrict__ r, cpx<h2> (&g)[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = r[k];
}

// z pass fused with the spectrum on packed pairs, in place on the packed
// y/z scratch: each lane takes one column pair at its rows (8 bytes per
// row), scales the input by hs; layout conditions as the FAST paired FP32
// shape (z block 16, P/2 rows, column tiles covering P1).  At most 128
// registers: two 8-wave workgroups per CU.
template <int P, int E, int NT, bool ZP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_fft_z_green_h2(
    cpx<h2>* __restrict__ B, const cpx<h2>* __restrict__ spec, const cpx<h2>* __restrict__ tw,
    ZArgs a, float hs, const int* __restrict__ active) {
  constexpr int TT = P / E, WP = NT / TT, LS = Pad<P>::LSTR;
  __shared__ cpx<h2> lds[WP * LS];
  // block order as the FP32 z pass (right-hand side innermost, y mirror
  // pairs, x tiles in mirror pairs)
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int rhs = b % a.nrhs;
  const int u = b / a.nrhs;
  const int m = u & 1;
  const int it = (u >> 1) % a.tiles_x;
  const int yp = (u >> 1) / a.tiles_x;
  if (m && (yp == 0 || 2 * yp == a.P2)) return;
  const int xy = m ? a.P2 - yp : yp;
  const int tile = (it & 1) ? a.tiles_x - 1 - (it >> 1) : (it >> 1);
  if (active && !active[rhs]) return;
  const int cw = threadIdx.x % WP, t = threadIdx.x / WP;
  const int x0 = tile * 2 * WP + 2 * cw;  // the pair's even column
  // FP32-layout strides are multiples of P1, so every halved one is exact
  cpx<h2>* hp0 = B + (rhs * a.rhs_stride + (int64_t)xy * a.zl * a.P1 + x0) / 2;
  cpx<h2>* hp1 = hp0 + a.comp_stride / 2;
  cpx<h2>* hp2 = hp1 + a.comp_stride / 2;
  const int zhs = (int)(a.zhs / 2), zls = (int)(a.zls / 2);
  TwReg<h2, P, E> tr;
  tr.load(t, tw);
  const h2 sc = {(_Float16)hs, (_Float16)hs};
  const cpx<h2> zero = mk<h2>(h2{0, 0}, h2{0, 0});
  cpx<h2> v0[E], v1[E], v2[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    v0[q] = v1[q] = v2[q] = zero;
    if (q < E / 2) {
      // rows below P/2 exist in the blocked layout; padding rows (never
      // written) are not read
      const int z = t + q * TT;
      if (!ZP || z < a.N3) {
        const int off = (z >> 4) * zhs + (z & 15) * zls;
        v0[q] = hscale(hp0[off], sc);
        v1[q] = hscale(hp1[off], sc);
        v2[q] = hscale(hp2[off], sc);
      }
    }
  }
  const int ym = xy > a.P2 / 2;
  const int yo = ym ? a.P2 - xy : xy;
  const int npair = a.P1 / 2;
  const cpx<h2>* sp = spec + ((int64_t)yo * a.Q3 * npair + x0 / 2) * 6;
  auto rec = [&](int q) {
    const int z = t + q * TT;
    return sp + (int64_t)(z > P / 2 ? P - z : z) * 6 * npair;
  };
  cpx<h2>* line = lds + cw * LS;
  line_fft_e<h2, P, E, false, true, false>(v0, line, t, tr);
  line_fft_e<h2, P, E, false, true, false>(v1, line, t, tr);
  // the first point's record is requested before the last forward
  // transform, each next one while the current point is multiplied (the
  // empty asm statements keep the compiler from issuing every point's loads
  // at once, which would hold 12 registers per point)
  cpx<h2> gn[6];
  load_g6h(rec(0), gn);
  asm volatile("" ::: "memory");
  line_fft_e<h2, P, E, false, true, false>(v2, line, t, tr);
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int z = t + q * TT;
    const int zm = z > P / 2;
    cpx<h2> gg[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gg[k] = gn[k];
    if (q + 1 < E) load_g6h(rec(q + 1), gn);
    asm volatile("" ::: "memory");
    // x signs are in the record; G_ab is odd along y (z) iff exactly one of
    // a, b is y (z)
    const cpx<h2> gxx = gg[0], gyy = gg[3], gzz = gg[5];
    const cpx<h2> gxy = negif(gg[1], ym), gxz = negif(gg[2], zm), gyz = negif(gg[4], ym ^ zm);
    const cpx<h2> ix = v0[q], iy = v1[q], iz = v2[q];
    v0[q] = cfma(gxz, iz, cfma(gxy, iy, gxx * ix));
    v1[q] = cfma(gyz, iz, cfma(gyy, iy, gxy * ix));
    v2[q] = cfma(gzz, iz, cfma(gyz, iy, gxz * ix));
  }
  line_fft_e<h2, P, E, true, false, true>(v0, line, t, tr);
  line_fft_e<h2, P, E, true, false, true>(v1, line, t, tr);
  line_fft_e<h2, P, E, true, false, true>(v2, line, t, tr);
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int z = t + q * TT;
    if (!ZP || z < a.N3) {
      const int off = (z >> 4) * zhs + (z & 15) * zls;
      hp0[off] = v0[q];
      hp1[off] = v1[q];
      hp2[off] = v2[q];
    }
  }
}

// 8 points per thread (6 for 3 * 2^k lines), 256 threads: 32 column pairs
// per workgroup (256-byte row runs); the packed data of three components stay
// within the 128-register cap (four 4-wave workgroups per CU).
constexpr int kZH2Threads = 256;
template <int P>
constexpr int zh2_e() {
  return P % 3 == 0 ? 6 : 8;
}
template <int P>
static int zh2_pairs() {
  return kZH2Threads / (P / zh2_e<P>());
}

bool x_packed_ok(int P1);

// Whether a grid takes the packed-FP16 passes: the z pass's shape (z block
// 16, P3 = 32 .. 128 with P3 / 2 rows in the blocked layout, column-pair
// tiles covering P1) and an even number of threads per x line.
bool h16_ok(const GroupGeom& g) {
  const int zl = z_block(g);
  if (zl != 16 || 2 * ((g.N[2] + 15) / 16) * 16 != g.P[2]) return false;
  if (!x_packed_ok(g.P[0])) return false;
  int wp = 0;
  switch (g.P[2]) {
    case 32: wp = zh2_pairs<32>(); break;
    case 48: wp = zh2_pairs<48>(); break;
    case 64: wp = zh2_pairs<64>(); break;
    case 96: wp = zh2_pairs<96>(); break;
    case 128: wp = zh2_pairs<128>(); break;
    default: return false;
  }
  return g.P[0] % (2 * wp) == 0;
}

// FP32-layout addresses in units of packed pairs
static SideAddr halved(SideAddr s) {
  s.rs /= 2;
  s.cs /= 2;
  s.zhs /= 2;
  s.zls /= 2;
  s.row /= 2;
  return s;
}

template <int PP>
static void y_launch_h2(const GroupGeom& g, const cpx<h2>* in, cpx<h2>* out, const cpx<h2>* tw,
                        bool inverse, float hs, const int* active, hipStream_t s) {
  const int N2 = g.N[1], N3 = g.N[2];
  const int zl = z_block(g);
  constexpr int ntY = y_threads<h2, PP>();
  constexpr int W = ntY / (PP / fft_e<PP>());
  StridedArgs a;
  a.ncols = g.P[0] / 2;
  a.ncomp = 3;
  a.nz = N3;
  a.zl = zl;
  a.tiles = (a.ncols + W - 1) / W;
  const SideAddr A = halved(side_A(g, zl)), B = halved(side_B(g, zl));
  if (!inverse) {
    a.n_in_rows = N2;
    a.n_out_rows = PP;
    a.in = A;
    a.out = B;
  } else {
    a.n_in_rows = PP;
    a.n_out_rows = N2;
    a.in = B;
    a.out = A;
  }
  const dim3 grid(a.tiles * 3 * N3 * g.nrhs);
  if (!inverse)
    k_fft_y_h2<PP, false, ntY><<<grid, ntY, 0, s>>>(in, out, tw, a, hs, active);
  else
    k_fft_y_h2<PP, true, ntY><<<grid, ntY, 0, s>>>(in, out, tw, a, 1.f, active);
}

static hipError_t y_pass_h2(const GroupGeom& g, const cpx<h2>* in, cpx<h2>* out,
                            const cpx<h2>* tw, bool inverse, float hs, const int* active,
                            hipStream_t s) {
  VIE_DISPATCH_P(g.P[1], (y_launch_h2<PP>(g, in, out, tw, inverse, hs, active, s)));
  return hipGetLastError();
}

// The fused x-y passes take FFT lengths 64, 96 and 128 along x and y (the
// plane and one set of transform lines fit a quarter of the LDS).
static bool xy_len_ok(int p) { return p == 64 || p == 96 || p == 128; }
bool xy_fused_ok(const GroupGeom& g) { return xy_len_ok(g.P[0]) && xy_len_ok(g.P[1]); }

#define VIE_DISPATCH_XY(P_, CALL)                    \
  switch (P_) {                                      \
    case 64: { constexpr int PP = 64; CALL; break; } \
    case 96: { constexpr int PP = 96; CALL; break; } \
    case 128: { constexpr int PP = 128; CALL; break; } \
    default: return hipErrorInvalidValue;            \
  }

// m.npart set: normalising FP32 input (see MatvecArgs), else bfloat16 input
static hipError_t xy_fwd_h2(const GroupGeom& g, const void* xc, cpx<h2>* B, const c32* tw1,
                            const cpx<h2>* tw2, const BodyIdx& bi, float hs1, float hs2,
                            const MatvecArgs& m, hipStream_t s) {
  if (!xy_fused_ok(g)) return hipErrorInvalidValue;
  const int zl = z_block(g);
  const SideAddr sb = halved(side_B(g, zl));
  const dim3 grid(g.nrhs * 3 * g.N[2]);
  VIE_DISPATCH_XY(g.P[0], ({
                    constexpr int Q1 = PP;
                    VIE_DISPATCH_XY(g.P[1], ({
                                      if (m.npart)
                                        k_fft_xy_fwd_h2<Q1, PP, true><<<grid, 256, 0, s>>>(
                                            xc, B, tw1, tw2, bi, g.N[0], g.N[1], g.N[2], sb, zl,
                                            hs1, hs2, m.active, m.npart, m.nblk, m.nrm, m.ldn,
                                            (cb16*)m.vout);
                                      else
                                        k_fft_xy_fwd_h2<Q1, PP, false><<<grid, 256, 0, s>>>(
                                            xc, B, tw1, tw2, bi, g.N[0], g.N[1], g.N[2], sb, zl,
                                            hs1, hs2, m.active, nullptr, 0, nullptr, 0, nullptr);
                                    }));
                  }));
  return hipGetLastError();
}

static hipError_t yx_inv_h2(const GroupGeom& g, const cpx<h2>* B, const void* x, void* y,
                            const c32* tw1, const cpx<h2>* tw2, const BodyIdx& bi, float hs,
                            const int* active, hipStream_t s) {
  if (!xy_fused_ok(g)) return hipErrorInvalidValue;
  const int zl = z_block(g);
  const SideAddr sb = halved(side_B(g, zl));
  const dim3 grid(g.nrhs * 3 * g.N[2]);
  VIE_DISPATCH_XY(g.P[0], ({
                    constexpr int Q1 = PP;
                    VIE_DISPATCH_XY(g.P[1], (k_fft_yx_inv_h2<Q1, PP><<<grid, 256, 0, s>>>(
                                                B, (const cb16*)x, (c32*)y, tw1, tw2, bi, g.N[0],
                                                g.N[1], g.N[2], sb, zl, hs, active)));
                  }));
  return hipGetLastError();
}
#undef VIE_DISPATCH_XY

static hipError_t z_pass_h2(const GroupGeom& g, cpx<h2>* B, const cpx<h2>* spec,
                            const cpx<h2>* tw, float hs, const int* active, hipStream_t s) {
  if (!h16_ok(g)) return hipErrorInvalidValue;
  ZArgs a;
  a.N3 = g.N[2];
  a.P1 = g.P[0];
  a.P2 = g.P[1];
  a.Q1 = g.Q[0];
  a.Q2 = g.Q[1];
  a.Q3 = g.Q[2];
  a.nrhs = g.nrhs;
  a.zl = z_block(g);
  const SideAddr sb = side_B(g, a.zl);  // FP32-layout strides (halved in the kernel)
  a.comp_stride = sb.cs;
  a.rhs_stride = sb.rs;
  a.zhs = sb.zhs;
  a.zls = sb.zls;
#define VIE_ZH2(P_)                                                                           \
  case P_: {                                                                                  \
    a.tiles_x = g.P[0] / (2 * zh2_pairs<P_>());                                               \
    const dim3 grid((g.P[1] / 2 + 1) * 2 * a.tiles_x * g.nrhs);                               \
    if (2 * a.N3 == P_)                                                                       \
      k_fft_z_green_h2<P_, zh2_e<P_>(), kZH2Threads, false>                                   \
          <<<grid, kZH2Threads, 0, s>>>(B, spec, tw, a, hs, active);                          \
    else                                                                                      \
      k_fft_z_green_h2<P_, zh2_e<P_>(), kZH2Threads, true>                                    \
          <<<grid, kZH2Threads, 0, s>>>(B, spec, tw, a, hs, active);                          \
    break;                                                                                    \
  }
  switch (g.P[2]) {
    VIE_ZH2(32)
    VIE_ZH2(48)
    VIE_ZH2(64)
    VIE_ZH2(96)
    VIE_ZH2(128)
    default: return hipErrorInvalidValue;
  }
#undef VIE_ZH2
  return hipGetLastError();
}

// FP16 tables of the packed passes: the pair-packed spectrum (scaled by gs,
// x-mirror signs applied: entries xy and xz are odd along x), and the y and
// z twiddles splatted to both halves.
__global__ void k_spec_pairs(const c32* __restrict__ in, cpx<h2>* __restrict__ out, int P1,
                             int Q1, int64_t nyz, float gs) {
  const int npair = P1 / 2;
  const int64_t n = nyz * npair * 6;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int ab = (int)(i % 6);
    const int p = (int)((i / 6) % npair);
    const int64_t yz = i / (6 * npair);
    float re[2], im[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int x = 2 * p + h;
      const int xm = x > P1 / 2;
      const int xo = xm ? P1 - x : x;
      const c32 v = in[(yz * Q1 + xo) * 6 + ab];
      const float sg = (xm && (ab == 1 || ab == 2)) ? -gs : gs;
      re[h] = v.re * sg;
      im[h] = v.im * sg;
    }
    out[i] = pack2(re[0], im[0], re[1], im[1]);
  }
}
__global__ void k_tw_h2(const c32* __restrict__ in, cpx<h2>* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const _Float16 re = (_Float16)in[i].re, im = (_Float16)in[i].im;
    out[i] = mk<h2>(h2{re, re}, h2{im, im});
  }
}
// max |re|, |im| over n complex values into *out (float bits, atomic max)
__global__ void k_absmax(const c32* __restrict__ in, int64_t n, unsigned* __restrict__ out) {
  float mx = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    mx = fmaxf(mx, fmaxf(fabsf(in[i].re), fabsf(in[i].im)));
  for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(mx));
}

hipError_t launch_spec_absmax(const void* spec32, int64_t n, unsigned* dmax, hipStream_t s) {
  k_absmax<<<512, 256, 0, s>>>((const c32*)spec32, n, dmax);
  return hipGetLastError();
}
hipError_t launch_spec_pairs(const void* spec32, void* spec16, const GroupGeom& g, float gs,
                             hipStream_t s) {
  k_spec_pairs<<<1024, 256, 0, s>>>((const c32*)spec32, (cpx<h2>*)spec16, g.P[0], g.Q[0],
                                    (int64_t)g.Q[1] * g.Q[2], gs);
  return hipGetLastError();
}
hipError_t launch_tw_h2(const void* tw32, void* tw16, int n, hipStream_t s) {
  k_tw_h2<<<(n + 255) / 256, 256, 0, s>>>((const c32*)tw32, (cpx<h2>*)tw16, n);
  return hipGetLastError();
}

int part_blocks_xinv(const GroupGeom& g, int precision) {
  const int lines = 3 * g.N[1] * g.N[2];
  const int L = precision == 0 ? lines_per_block<double>(g.P[0]) : lines_per_block<float>(g.P[0]);
  return (lines + L - 1) / L;
}

template <typename T>
static hipError_t x_inv(const GroupGeom& g, const cpx<T>* A, const c64* x, c64* y,
                        const double* chi, const int* rhs_body, const cpx<T>* tw, EpiArgs& e,
                        const int* active, hipStream_t s) {
  XinvArgs a;
  a.N1 = g.N[0];
  a.N2 = g.N[1];
  a.N3 = g.N[2];
  a.lines_per_comp = g.N[1] * g.N[2];
  a.lines_per_rhs = 3 * a.lines_per_comp;
  const int L = lines_per_block<T>(g.P[0]);
  a.blocks_per_rhs = (a.lines_per_rhs + L - 1) / L;
  a.n = g.n;
  e.part_blocks = a.blocks_per_rhs;
  const dim3 grid(a.blocks_per_rhs * g.nrhs);
#define VIE_XINV(MODE_)                                                                    \
  VIE_DISPATCH_P(g.P[0], (k_fft_x_inv<T, PP, MODE_><<<grid, nt_lines_p<T>(PP), 0, s>>>(       \
                             A, x, y, chi, rhs_body, tw, a, e.aux, e.partials, e.pol, e.ph, \
                             active)))
  switch (e.mode) {
    case EPI_PLAIN: VIE_XINV(EPI_PLAIN); break;
    case EPI_RHV: VIE_XINV(EPI_RHV); break;
    case EPI_TS: VIE_XINV(EPI_TS); break;
    case EPI_RESID: VIE_XINV(EPI_RESID); break;
    default: return hipErrorInvalidValue;
  }
#undef VIE_XINV
  return hipGetLastError();
}

// hs > 0: packed FP16 lines on the scratch side (see the x passes)
template <typename T>
hipError_t x_fwd_c(const GroupGeom& g, const void* xc, int in32, cpx<T>* A, const cpx<T>* tw,
                   const BodyIdx& bi, const int* active, hipStream_t s, float hs = 0.f);
template <typename T>
hipError_t x_inv_c(const GroupGeom& g, const cpx<T>* A, const void* x, void* y, int io32,
                   const cpx<T>* tw, const BodyIdx& bi, EpiArgs& e, const int* active,
                   hipStream_t s, float hs = 0.f);

template <typename T>
static hipError_t matvec_t(const MatvecArgs& m, const void* xv, void* yv, EpiArgs& e,
                           hipStream_t s, void (*cb)(int, bool, void*), void* u) {
  // FP32 vectors only with body-compressed FP32 passes and the plain epilogue
  if (m.io32 && (!m.bi || sizeof(T) != 4 || e.mode != EPI_PLAIN)) return hipErrorInvalidValue;
  const c64* x = (const c64*)xv;
  c64* y = (c64*)yv;
  const GroupGeom& g = *m.g;
  cpx<T>* A = (cpx<T>*)m.bufA;
  cpx<T>* B = (cpx<T>*)m.bufB;
  const cpx<T>* tw0 = (const cpx<T>*)m.tw[0];
  const cpx<T>* tw1 = (const cpx<T>*)m.tw[1];
  const cpx<T>* tw2 = (const cpx<T>*)m.tw[2];
  hipError_t err;
  int base = sizeof(T) == 8 ? 0 : 5;
#define STEP(K, CALL)              \
  if (cb) cb(base + K, true, u);   \
  err = CALL;                      \
  if (cb) cb(base + K, false, u);  \
  if (err != hipSuccess) return err;
  if (m.spec16) {  // approximate products: packed FP16 y and z passes, FP16 scratch
    if constexpr (sizeof(T) == 4) {
      if (!m.bi || m.io32 != 2 || e.mode != EPI_PLAIN) return hipErrorInvalidValue;
      cpx<h2>* Ah = (cpx<h2>*)m.bufA;
      cpx<h2>* Bh = (cpx<h2>*)m.bufB;
      const cpx<h2>* twy = (const cpx<h2>*)m.tw16[0];
      const cpx<h2>* twz = (const cpx<h2>*)m.tw16[1];
      base = kH16Kind0;
      if (xy_fused_ok(g)) {  // x and y fused per plane: no x-y scratch traffic
        STEP(5, xy_fwd_h2(g, xv, Bh, (const c32*)tw0, twy, *m.bi, m.hs[0], m.hs[1], m, s));
        STEP(2, z_pass_h2(g, Bh, (const cpx<h2>*)m.spec16, twz, m.hs[2], m.active, s));
        // with a normalised input the epilogue's x is the stored bfloat16 vector
        STEP(6, yx_inv_h2(g, Bh, m.npart ? m.vout : xv, yv, (const c32*)tw0, twy, *m.bi, m.hout,
                          m.active, s));
        return hipSuccess;
      }
      if (m.npart) return hipErrorInvalidValue;
      STEP(0, x_fwd_c<T>(g, xv, m.io32, A, tw0, *m.bi, m.active, s, m.hs[0]));
      STEP(1, y_pass_h2(g, Ah, Bh, twy, false, m.hs[1], m.active, s));
      STEP(2, z_pass_h2(g, Bh, (const cpx<h2>*)m.spec16, twz, m.hs[2], m.active, s));
      STEP(3, y_pass_h2(g, Bh, Ah, twy, true, 1.f, m.active, s));
      STEP(4, x_inv_c<T>(g, A, xv, yv, m.io32, tw0, *m.bi, e, m.active, s, m.hout));
      return hipSuccess;
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (m.bi) {
    STEP(0, x_fwd_c<T>(g, xv, m.io32, A, tw0, *m.bi, m.active, s));
  } else {
    STEP(0, x_fwd<T>(g, x, A, tw0, m.active, s));
  }
  STEP(1, y_pass<T>(g, A, B, tw1, false, m.active, s));
  STEP(2, z_pass<T>(g, B, (const cpx<T>*)m.spec, tw2, m.active, s, m.zvar));
  STEP(3, y_pass<T>(g, B, A, tw1, true, m.active, s));
  if (m.bi) {
    STEP(4, x_inv_c<T>(g, A, xv, yv, m.io32, tw0, *m.bi, e, m.active, s));
  } else {
    STEP(4, x_inv<T>(g, A, x, y, m.chi, m.rhs_body, tw0, e, m.active, s));
  }
#undef STEP
  return hipSuccess;
}

int z_variants(int) { return kZVariants; }

hipError_t launch_z_only(const MatvecArgs& m, int precision, hipStream_t s) {
  const GroupGeom& g = *m.g;
  if (precision == 0)
    return z_pass<double>(g, (c64*)m.bufB, (const c64*)m.spec, (const c64*)m.tw[2], m.active, s,
                          m.zvar);
  return z_pass<float>(g, (c32*)m.bufB, (const c32*)m.spec, (const c32*)m.tw[2], m.active, s,
                       m.zvar);
}

hipError_t launch_matvec(const MatvecArgs& a, int precision, const void* x, void* y, EpiArgs& epi,
                         hipStream_t s, void (*cb)(int, bool, void*), void* u) {
  return precision == 0 ? matvec_t<double>(a, x, y, epi, s, cb, u)
                        : matvec_t<float>(a, x, y, epi, s, cb, u);
}

// ------------------------------------------- full (unpadded) FP64 3-D FFT
// Forward transform of work[P3][P2][P1]; the result lands in tmp.
hipError_t launch_fft3d_full(c64* work, c64* tmp, const GroupGeom& g, const void* twv[3],
                             hipStream_t s) {
  const int P1 = g.P[0], P2 = g.P[1], P3 = g.P[2];
  const c64* tw0 = (const c64*)twv[0];
  const c64* tw1 = (const c64*)twv[1];
  const c64* tw2 = (const c64*)twv[2];
  {  // x lines: work -> tmp
    const int lines = P2 * P3;
    const int L = lines_per_block<double>(P1);
    const int bpr = (lines + L - 1) / L;
    VIE_DISPATCH_P(P1, (k_fft_x_fwd<double, double, PP, false><<<bpr, nt_lines_p<double>(PP), 0, s>>>(
                           work, tmp, tw0, P1, lines, bpr, nullptr)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {  // y lines: tmp -> work, slabs = z planes
    StridedArgs a;
    a.n_in_rows = a.n_out_rows = P2;
    a.ncols = P1;
    a.ncomp = 1;
    a.nz = P3;
    a.zl = 1;
    const int W = lines_per_block<double>(P2);
    a.tiles = (P1 + W - 1) / W;
    a.in.row = a.out.row = P1;
    a.in.zhs = a.out.zhs = (int64_t)P2 * P1;
    a.in.zls = a.out.zls = a.in.cs = a.out.cs = a.in.rs = a.out.rs = 0;
    VIE_DISPATCH_P(P2, (k_fft_strided<double, PP, false, false, false, nt_lines_p<double>(PP)>
                        <<<a.tiles * P3, nt_lines_p<double>(PP), 0, s>>>(tmp, work, tw1, a, nullptr)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {  // z lines: work -> tmp, slabs = y rows
    StridedArgs a;
    a.n_in_rows = a.n_out_rows = P3;
    a.ncols = P1;
    a.ncomp = 1;
    a.nz = P2;
    a.zl = 1;
    const int W = lines_per_block<double>(P3);
    a.tiles = (P1 + W - 1) / W;
    a.in.row = a.out.row = (int64_t)P2 * P1;
    a.in.zhs = a.out.zhs = P1;
    a.in.zls = a.out.zls = a.in.cs = a.out.cs = a.in.rs = a.out.rs = 0;
    VIE_DISPATCH_PZ(P3, (k_fft_strided<double, PP, false, false, false>
                         <<<a.tiles * P2, nt_lines<double>(), 0, s>>>(work, tmp, tw2, a, nullptr)));
  }
  return hipGetLastError();
}


// ---------------------------- pruned x and y transforms of one field
// For a field non-zero only on the first E[a] points of each axis
// (E[a] <= P[a] / 2), the x and y stages of its forward 3-D transform, and
// the y and x stages of a forward transform that keeps only the first E[1]
// y and E[2] z outputs; both skip the zero halves like the operator's passes.
template <typename T>
static hipError_t px_pass(const cpx<T>* src, cpx<T>* dst, int n1, bool pad, const int E[3],
                          const int P[3], const cpx<T>* tw0, hipStream_t s) {
  const int P1 = P[0];
  const int lines = E[1] * E[2];
  const int L = lines_per_block<T>(P1);
  const int bpr = (lines + L - 1) / L;
  if (pad) {
    VIE_DISPATCH_P(P1, (k_fft_x_fwd<T, T, PP, true><<<bpr, nt_lines_p<T>(PP), 0, s>>>(
                           src, dst, tw0, n1, lines, bpr, nullptr)));
  } else {
    VIE_DISPATCH_P(P1, (k_fft_x_fwd<T, T, PP, false><<<bpr, nt_lines_p<T>(PP), 0, s>>>(
                           src, dst, tw0, n1, lines, bpr, nullptr)));
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t py_pass(const cpx<T>* src, cpx<T>* dst, int rin, int rout, bool pad,
                          const int E[3], const int P[3], const cpx<T>* tw1, hipStream_t s) {
  const int P1 = P[0], P2 = P[1];
  StridedArgs a;
  a.n_in_rows = rin;
  a.n_out_rows = rout;
  a.ncols = P1;
  a.ncomp = 1;
  a.nz = E[2];
  a.zl = 1;
  const int W = lines_per_block<T>(P2);
  a.tiles = (P1 + W - 1) / W;
  a.in.row = a.out.row = P1;
  a.in.zhs = (int64_t)rin * P1;
  a.out.zhs = (int64_t)rout * P1;
  a.in.zls = a.out.zls = a.in.cs = a.out.cs = a.in.rs = a.out.rs = 0;
  if (pad) {
    VIE_DISPATCH_P(P2, (k_fft_strided<T, PP, true, false, false, nt_lines_p<T>(PP)>
                        <<<a.tiles * E[2], nt_lines_p<T>(PP), 0, s>>>(src, dst, tw1, a, nullptr)));
  } else {
    VIE_DISPATCH_P(P2, (k_fft_strided<T, PP, false, true, false, nt_lines_p<T>(PP)>
                        <<<a.tiles * E[2], nt_lines_p<T>(PP), 0, s>>>(src, dst, tw1, a, nullptr)));
  }
  return hipGetLastError();
}

static bool pruned_ok(const int E[3], const int P[3]) {
  for (int a = 0; a < 3; ++a)
    if (E[a] < 1 || 2 * E[a] > P[a]) return false;
  return true;
}

template <typename T>
static hipError_t xy_pad_t(const cpx<T>* in, cpx<T>* t1, cpx<T>* out, const int E[3],
                           const int P[3], const void* tw[3], hipStream_t s) {
  if (!pruned_ok(E, P)) return hipErrorInvalidValue;
  hipError_t e = px_pass<T>(in, t1, E[0], true, E, P, (const cpx<T>*)tw[0], s);
  if (e != hipSuccess) return e;
  return py_pass<T>(t1, out, E[1], P[1], true, E, P, (const cpx<T>*)tw[1], s);
}

template <typename T>
static hipError_t yx_trunc_t(const cpx<T>* in, cpx<T>* t1, cpx<T>* out, const int E[3],
                             const int P[3], const void* tw[3], hipStream_t s) {
  if (!pruned_ok(E, P)) return hipErrorInvalidValue;
  hipError_t e = py_pass<T>(in, t1, P[1], E[1], false, E, P, (const cpx<T>*)tw[1], s);
  if (e != hipSuccess) return e;
  return px_pass<T>(t1, out, P[0], false, E, P, (const cpx<T>*)tw[0], s);
}

hipError_t launch_fft_xy_pad(const c64* in, c64* t1, c64* out, const int E[3], const int P[3],
                             const void* tw[3], hipStream_t s) {
  return xy_pad_t<double>(in, t1, out, E, P, tw, s);
}
hipError_t launch_fft_xy_pad(const c32* in, c32* t1, c32* out, const int E[3], const int P[3],
                             const void* tw[3], hipStream_t s) {
  return xy_pad_t<float>(in, t1, out, E, P, tw, s);
}
hipError_t launch_fft_yx_trunc(const c64* in, c64* t1, c64* out, const int E[3], const int P[3],
                               const void* tw[3], hipStream_t s) {
  return yx_trunc_t<double>(in, t1, out, E, P, tw, s);
}
hipError_t launch_fft_yx_trunc(const c32* in, c32* t1, c32* out, const int E[3], const int P[3],
                               const void* tw[3], hipStream_t s) {
  return yx_trunc_t<float>(in, t1, out, E, P, tw, s);
}

}  // namespace vie
