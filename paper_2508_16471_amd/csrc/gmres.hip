// Segmented multi-vector kernels of the flexible GMRES driver (Arnoldi with
// classical Gram-Schmidt and selective reorthogonalisation, solution update) and the permutation
// between a body's vector and its block-ordered copy (block-Jacobi
// preconditioner).  All work is HBM-bound streaming over FP64 complex vectors:
// one coalesced 16-byte load per element per vector, reductions through
// per-workgroup partials summed in a fixed order.
#include <algorithm>

#include "gmres.h"
#include "kernels.h"

namespace vie {

namespace {

constexpr int GT = 256;      // threads per workgroup (4 waves)
constexpr int GU = 8;        // basis vectors per pass of the multi-dot
constexpr int kMaxVec = 256; // coefficients a multi-axpy holds in LDS

__device__ __forceinline__ c64 shfl_xor_c(c64 v, int m) {
  return mk(__shfl_xor(v.re, m), __shfl_xor(v.im, m));
}

__device__ __forceinline__ c64 ld64(const c64* p) { return *p; }
__device__ __forceinline__ c64 ld64(const c32* p) { return cvt<double>(*p); }
__device__ __forceinline__ c64 ld64(const cb16* p) {
  const cb16 v = *p;
  return mk((double)(float)v.re, (double)(float)v.im);
}
__device__ __forceinline__ void st(cb16* p, c64 v) {
  cb16 o;
  o.re = (__bf16)(float)v.re;
  o.im = (__bf16)(float)v.im;
  *p = o;
}
__device__ __forceinline__ void st(c64* p, c64 v) { *p = v; }
__device__ __forceinline__ void st(c32* p, c64 v) { *p = cvt<float>(v); }
// v as stored in a T vector (rounded to FP32 for c32), without a reload
__device__ __forceinline__ c64 stored(const c64*, c64 v) { return v; }
__device__ __forceinline__ c64 stored(const c32*, c64 v) { return cvt<double>(cvt<float>(v)); }

template <typename TV, typename TW>
__global__ __launch_bounds__(GT) void k_seg_mdot(SegSet S, const TV* __restrict__ V,
                                                 int64_t stride, int nv,
                                                 const TW* __restrict__ w,
                                                 c64* __restrict__ partials) {
  const int s = blockIdx.y, blk = blockIdx.x;
  if (S.active && !S.active[s]) return;
  const int64_t off = S.off[s];
  const int len = S.len[s];
  __shared__ c64 red[GT / 64][GU];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i0 = 0; i0 < nv; i0 += GU) {
    c64 acc[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) acc[u] = mk(0.0, 0.0);
    // two elements per iteration (twice the loads in flight), then the tail
    const int step = S.nblk * GT;
    int e = blk * GT + threadIdx.x;
    for (; e + step < len; e += 2 * step) {
      const c64 wa = ld64(w + off + e), wb = ld64(w + off + e + step);
#pragma unroll
      for (int u = 0; u < GU; ++u)
        if (i0 + u < nv) {
          const TV* vu = V + (int64_t)(i0 + u) * stride + off + e;
          acc[u] = acc[u] + cmulc(ld64(vu), wa);
          acc[u] = acc[u] + cmulc(ld64(vu + step), wb);
        }
    }
    if (e < len) {
      const c64 we = ld64(w + off + e);
#pragma unroll
      for (int u = 0; u < GU; ++u)
        if (i0 + u < nv) acc[u] = acc[u] + cmulc(ld64(V + (int64_t)(i0 + u) * stride + off + e), we);
    }
    // Reduce-scatter across the wave: at each of the first three steps a
    // lane keeps half of its sums (the half selected by that lane bit) and
    // adds its partner's copy of them, so 4 + 2 + 1 exchanges replace 3 x 8;
    // the last three steps sum the one remaining value.  Lane 8 v then holds
    // the wave's sum for basis vector v (v = lane bits 5, 4, 3).
    static_assert(GU == 8, "reduce-scatter over 8 sums");
#pragma unroll
    for (int h = 4, m = 32; h >= 1; h >>= 1, m >>= 1) {
      const bool up = (lane & m) != 0;
#pragma unroll
      for (int u = 0; u < h; ++u) {
        const c64 keep = up ? acc[h + u] : acc[u], give = up ? acc[u] : acc[h + u];
        acc[u] = keep + shfl_xor_c(give, m);
      }
    }
#pragma unroll
    for (int m = 4; m >= 1; m >>= 1) acc[0] = acc[0] + shfl_xor_c(acc[0], m);
    if ((lane & 7) == 0) red[wv][lane >> 3] = acc[0];
    __syncthreads();
    if (threadIdx.x < GU && i0 + (int)threadIdx.x < nv) {
      c64 t = red[0][threadIdx.x];
      for (int k = 1; k < GT / 64; ++k) t = t + red[k][threadIdx.x];
      partials[((int64_t)s * nv + i0 + threadIdx.x) * S.nblk + blk] = t;
    }
    __syncthreads();
  }
}

// One wave per (segment, coefficient): lane l sums partials l, l + 64, ...,
// then a fixed butterfly across the wave.
__global__ __launch_bounds__(64) void k_seg_sum_c(SegSet S, int nv,
                                                  const c64* __restrict__ partials,
                                                  c64* __restrict__ out, int ldo) {
  const int i = blockIdx.x, s = blockIdx.y;
  c64 t = mk(0.0, 0.0);
  if (!(S.active && !S.active[s]))
    for (int k = threadIdx.x; k < S.nblk; k += 64)
      t = t + partials[((int64_t)s * nv + i) * S.nblk + k];
  for (int m = 32; m >= 1; m >>= 1) t = t + shfl_xor_c(t, m);
  if (threadIdx.x == 0) out[(int64_t)s * ldo + i] = t;
}

template <typename TV, typename TW>
__global__ __launch_bounds__(GT) void k_seg_maxpy(SegSet S, const TV* __restrict__ V,
                                                  int64_t stride, int nv,
                                                  const int* __restrict__ nv_seg,
                                                  const c64* __restrict__ coef, int ldc,
                                                  TW* __restrict__ w,
                                                  double* __restrict__ partials) {
  const int s = blockIdx.y, blk = blockIdx.x;
  if (S.active && !S.active[s]) return;
  const int64_t off = S.off[s];
  const int len = S.len[s];
  int n = nv;
  if (nv_seg) n = min(n, nv_seg[s]);
  __shared__ c64 cf[kMaxVec];
  __shared__ double red[GT / 64];
  for (int i = threadIdx.x; i < n; i += GT) cf[i] = coef[(int64_t)s * ldc + i];
  __syncthreads();
  double nr = 0.0;
  for (int e = blk * GT + threadIdx.x; e < len; e += S.nblk * GT) {
    c64 a = ld64(w + off + e);
    for (int i = 0; i < n; ++i) a = a - cf[i] * ld64(V + (int64_t)i * stride + off + e);
    if (n > 0) {
      st(w + off + e, a);
      a = stored(w, a);  // the norm of what is stored (rounded when w is FP32)
    }
    nr += a.re * a.re + a.im * a.im;
  }
  if (!partials) return;
  for (int m = 32; m >= 1; m >>= 1) nr += __shfl_xor(nr, m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nr;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int k = 1; k < GT / 64; ++k) t += red[k];
    partials[(int64_t)s * S.nblk + blk] = t;
  }
}

__global__ __launch_bounds__(64) void k_seg_sum_r(SegSet S, const double* __restrict__ partials,
                                                  double* __restrict__ out, int ldn) {
  const int s = blockIdx.x;
  if (S.active && !S.active[s]) return;
  double t = 0.0;
  for (int k = threadIdx.x; k < S.nblk; k += 64) t += partials[(int64_t)s * S.nblk + k];
  for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m);
  if (threadIdx.x == 0) out[(int64_t)s * ldn] = t;
}

__global__ void k_seg_reorth_flags(SegSet S, const double* __restrict__ before,
                                   const double* __restrict__ after, int ldn, double eta2,
                                   int* __restrict__ act2) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S.nseg) return;
  const bool on = !S.active || S.active[s];
  act2[s] = (on && eta2 > 0.0 && after[(int64_t)s * ldn] < eta2 * before[s]) ? 1 : 0;
}

// SUM: norm2 is first reduced here from the norm partials of the multi-axpy
// (every wave in the order of k_seg_sum_r, so the result is the same bits),
// and workgroup 0 stores it at norm2[s * ldn].
template <typename TS, typename TD, bool SUM = false>
__global__ __launch_bounds__(GT) void k_seg_normalize(SegSet S, const TS* __restrict__ src,
                                                      double* __restrict__ norm2, int ldn,
                                                      TD* __restrict__ dst,
                                                      const double* __restrict__ npart) {
  const int s = blockIdx.y, blk = blockIdx.x;
  if (S.active && !S.active[s]) return;
  const int64_t off = S.off[s];
  const int len = S.len[s];
  double n2;
  if constexpr (SUM) {
    double t = 0.0;
    for (int k = threadIdx.x & 63; k < S.nblk; k += 64) t += npart[(int64_t)s * S.nblk + k];
    for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m);
    n2 = t;
    if (blk == 0 && threadIdx.x == 0) norm2[(int64_t)s * ldn] = t;
  } else {
    n2 = norm2[(int64_t)s * ldn];
  }
  const double sc = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
  for (int e = blk * GT + threadIdx.x; e < len; e += S.nblk * GT)
    st(dst + off + e, sc * ld64(src + off + e));
}

template <typename TV>
__global__ __launch_bounds__(GT) void k_seg_lincomb(SegSet S, const TV* __restrict__ V,
                                                    int64_t stride, int nv,
                                                    const int* __restrict__ nv_seg,
                                                    const c64* __restrict__ coef, int ldc,
                                                    c64* __restrict__ x) {
  const int s = blockIdx.y, blk = blockIdx.x;
  if (S.active && !S.active[s]) return;
  const int64_t off = S.off[s];
  const int len = S.len[s];
  int n = nv;
  if (nv_seg) n = min(n, nv_seg[s]);
  __shared__ c64 cf[kMaxVec];
  for (int i = threadIdx.x; i < n; i += GT) cf[i] = coef[(int64_t)s * ldc + i];
  __syncthreads();
  for (int e = blk * GT + threadIdx.x; e < len; e += S.nblk * GT) {
    c64 a = mk(0.0, 0.0);
    for (int i = 0; i < n; ++i) a = a - cf[i] * ld64(V + (int64_t)i * stride + off + e);
    x[off + e] = a;
  }
}

// The same combination written straight into the outer vectors' order (the
// permutation's scatter fused): element e of segment s, whose right-hand side
// is q = seg_rhs[s], goes to dst[qoff[q] + perm[qpoff[q] + off[s] - qoff[q] + e]].
template <typename TV, typename TD>
__global__ __launch_bounds__(GT) void k_seg_lincomb_perm(
    SegSet S, const TV* __restrict__ V, int64_t stride, int nv, const int* __restrict__ nv_seg,
    const c64* __restrict__ coef, int ldc, const int* __restrict__ seg_rhs,
    const int64_t* __restrict__ qoff, const int64_t* __restrict__ qpoff,
    const int* __restrict__ perm, TD* __restrict__ dst) {
  const int s = blockIdx.y, blk = blockIdx.x;
  if (S.active && !S.active[s]) return;
  const int64_t off = S.off[s];
  const int len = S.len[s];
  const int q = seg_rhs[s];
  const int64_t qo = qoff[q];
  const int* pm = perm + qpoff[q] + (off - qo);
  int n = nv;
  if (nv_seg) n = min(n, nv_seg[s]);
  __shared__ c64 cf[kMaxVec];
  for (int i = threadIdx.x; i < n; i += GT) cf[i] = coef[(int64_t)s * ldc + i];
  __syncthreads();
  for (int e = blk * GT + threadIdx.x; e < len; e += S.nblk * GT) {
    c64 a = mk(0.0, 0.0);
    for (int i = 0; i < n; ++i) a = a - cf[i] * ld64(V + (int64_t)i * stride + off + e);
    st(dst + qo + pm[e], a);
  }
}

__global__ void k_seg_act_map(int nseg, const int* __restrict__ seg_rhs,
                              const int* __restrict__ act_rhs, int* __restrict__ act_seg) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nseg) act_seg[s] = act_rhs[seg_rhs[s]] ? 1 : 0;
}

template <typename TS, typename TD>
__global__ __launch_bounds__(GT) void k_permute(const int64_t* __restrict__ qoff,
                                                const int64_t* __restrict__ qpoff,
                                                const int* __restrict__ qlen,
                                                const int* __restrict__ perm,
                                                const TS* __restrict__ src,
                                                TD* __restrict__ dst, int scatter,
                                                const int* __restrict__ act) {
  const int q = blockIdx.y;
  if (act && !act[q]) return;
  const int64_t base = qoff[q];
  const int* pm = perm + qpoff[q];
  const int n = qlen[q];
  for (int j = blockIdx.x * GT + threadIdx.x; j < n; j += gridDim.x * GT) {
    const int p = pm[j];
    if (scatter)
      st(dst + base + p, ld64(src + base + j));
    else
      st(dst + base + j, ld64(src + base + p));
  }
}

// ------------------------------------------------ GMRES least squares
__device__ __forceinline__ c64 conjc(c64 a) { return mk(a.re, -a.im); }
__device__ __forceinline__ double cabs2(c64 a) { return hypot(a.re, a.im); }

// Apply the previous j rotations to column j (col[0..j]), form the rotation
// that annihilates the subdiagonal hn, update g; returns |g[j+1]|.  The entry
// each rotation hands to the next stays in a register, so the loads of the
// rotations and of the column do not wait on the previous rotation's store.
__device__ double ls_add(int j, c64* __restrict__ col, double* __restrict__ cs,
                         c64* __restrict__ sn, c64* __restrict__ g, double hn) {
  c64 carry = col[0];
  for (int i = 0; i < j; ++i) {
    const c64 a = carry, b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    carry = cs[i] * b - conjc(sn[i]) * a;
  }
  const c64 a = carry;
  const double aa = cabs2(a);
  const double rho = hypot(aa, hn);
  double c;
  c64 sv;
  if (rho == 0.0) {
    c = 1.0;
    sv = mk(0.0, 0.0);
  } else if (aa == 0.0) {
    c = 0.0;
    sv = mk(1.0, 0.0);
  } else {
    c = aa / rho;
    sv = mk(a.re / aa * hn / rho, a.im / aa * hn / rho);  // (a / |a|) hn / rho
  }
  cs[j] = c;
  sn[j] = sv;
  col[j] = c * a + hn * sv;
  const c64 gj = g[j];
  g[j] = c * gj;
  g[j + 1] = mk(0.0, 0.0) - conjc(sv) * gj;
  return cabs2(g[j + 1]);
}

// y[0..k) from R y = g (columns of R at stride ldr), written as -y into out.
__device__ void ls_backsolve(int k, const c64* __restrict__ R, int ldr, const c64* __restrict__ g,
                             c64* __restrict__ out) {
  for (int i = k - 1; i >= 0; --i) {
    c64 t = g[i];
    for (int l = i + 1; l < k; ++l) t = t + R[(size_t)l * ldr + i] * out[l];  // out = -y
    const c64 d = R[(size_t)i * ldr + i];
    const double dd = d.re * d.re + d.im * d.im;
    const c64 y = dd > 0 ? (1.0 / dd) * cmulc(d, t) : mk(0.0, 0.0);
    out[i] = mk(-y.re, -y.im);
  }
}

__global__ void k_ls_cycle_init(int nseg, int maxit, const KState* __restrict__ st,
                                int* __restrict__ act, int* __restrict__ steps,
                                int* __restrict__ mc, int* __restrict__ cycles, LsBufs L) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nseg) return;
  const int nd = st[q].notdone;
  act[q] = (nd && steps[q] < maxit) ? 1 : 0;
  if (nd) cycles[q] += 1;
  L.nst[q] = 0;
  mc[q] = min(L.m, maxit - steps[q]);
  L.g[(size_t)q * L.ldr] = mk(sqrt(fmax(st[q].rnorm2, 0.0)), 0.0);
}

__global__ __launch_bounds__(256) void k_ls_step(int nseg, int j, const c64* __restrict__ H1,
                                                 const c64* __restrict__ H2, int use_h2, int ldh,
                                                 const double* __restrict__ NR, int ldn,
                                                 const KState* __restrict__ st, double half_tol,
                                                 int* __restrict__ act, int* __restrict__ steps,
                                                 const int* __restrict__ mc, LsBufs L,
                                                 int* __restrict__ any) {
  int live = 0;
  for (int q = threadIdx.x; q < nseg; q += blockDim.x) {
    if (!act[q]) continue;
    c64* col = L.R + ((size_t)q * L.m + j) * L.ldr;
    const c64* h1 = H1 + ((size_t)j * nseg + q) * ldh;
    const c64* h2 = H2 + ((size_t)j * nseg + q) * ldh;
    for (int i = 0; i <= j; ++i) col[i] = use_h2 ? h1[i] + h2[i] : h1[i];
    const double hn = sqrt(fmax(NR[(size_t)q * ldn + j + 1], 0.0));
    const double est = ls_add(j, col, L.cs + (size_t)q * L.m, L.sn + (size_t)q * L.m,
                              L.g + (size_t)q * L.ldr, hn);
    L.nst[q] = j + 1;
    steps[q] += 1;
    const bool stop = est <= half_tol * sqrt(fmax(st[q].bnorm2, 0.0)) || j + 1 >= mc[q] ||
                      hn <= 1e-14 * sqrt(fmax(st[q].rnorm2, 0.0));
    if (stop)
      act[q] = 0;
    else
      live = 1;
  }
  live = __syncthreads_or(live);
  if (threadIdx.x == 0) any[0] = live;
}

__global__ void k_ls_solve(int nseg, LsBufs L, c64* __restrict__ coef, int ldc,
                           int* __restrict__ nvs, int* __restrict__ act) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nseg) return;
  const int n = L.nst[q];
  nvs[q] = n;
  act[q] = n > 0 ? 1 : 0;
  if (n > 0)
    ls_backsolve(n, L.R + (size_t)q * L.m * L.ldr, L.ldr, L.g + (size_t)q * L.ldr,
                 coef + (size_t)q * ldc);
}

__global__ void k_ls_full(int nseg, int k, const c64* __restrict__ H1, const c64* __restrict__ H2,
                          int use_h2, int ldh, const double* __restrict__ NR, int ldn,
                          const int* __restrict__ act, LsBufs L, c64* __restrict__ coef, int ldc,
                          int* __restrict__ nvs) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  nvs[s] = 0;
  if (!act[s]) return;
  const double beta = sqrt(fmax(NR[(size_t)s * ldn], 0.0));
  if (!(beta > 0)) return;
  c64* R = L.R + (size_t)s * L.m * L.ldr;
  c64* g = L.g + (size_t)s * L.ldr;
  double* cs = L.cs + (size_t)s * L.m;
  c64* sn = L.sn + (size_t)s * L.m;
  g[0] = mk(beta, 0.0);
  int steps = 0;
  for (int j = 0; j < k; ++j) {
    c64* col = R + (size_t)j * L.ldr;
    const c64* h1 = H1 + ((size_t)j * nseg + s) * ldh;
    const c64* h2 = H2 + ((size_t)j * nseg + s) * ldh;
    for (int i = 0; i <= j; ++i) col[i] = use_h2 ? h1[i] + h2[i] : h1[i];
    const double hn = sqrt(fmax(NR[(size_t)s * ldn + j + 1], 0.0));
    ls_add(j, col, cs, sn, g, hn);
    steps = j + 1;
    if (hn <= 1e-14 * beta) break;
  }
  ls_backsolve(steps, R, L.ldr, g, coef + (size_t)s * ldc);
  nvs[s] = steps;
}

__global__ __launch_bounds__(256) void k_any_notdone(int n, const KState* __restrict__ st,
                                                     const int* __restrict__ steps, int maxit,
                                                     int* __restrict__ any) {
  int live = 0;
  for (int q = threadIdx.x; q < n; q += blockDim.x)
    if (st[q].notdone && steps[q] < maxit) live = 1;
  live = __syncthreads_or(live);
  if (threadIdx.x == 0) any[0] = live;
}

}  // namespace

int seg_blocks(int64_t max_len) {
  int64_t b = (max_len + 4 * GT - 1) / (4 * GT);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 256));
}

hipError_t launch_seg_mdot(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                           const void* w, int w32, c64* partials, c64* out, int ldo,
                           hipStream_t st) {
  if (S.nseg < 1 || nv < 1) return hipSuccess;
  const dim3 grid(S.nblk, S.nseg);
  if (v32 == 2 && w32)
    k_seg_mdot<<<grid, GT, 0, st>>>(S, (const cb16*)V, stride, nv, (const c32*)w, partials);
  else if (v32 == 2)
    return hipErrorInvalidValue;  // a bfloat16 basis comes with an FP32 work vector
  else if (v32 && w32)
    k_seg_mdot<<<grid, GT, 0, st>>>(S, (const c32*)V, stride, nv, (const c32*)w, partials);
  else if (v32)
    k_seg_mdot<<<grid, GT, 0, st>>>(S, (const c32*)V, stride, nv, (const c64*)w, partials);
  else if (w32)
    k_seg_mdot<<<grid, GT, 0, st>>>(S, (const c64*)V, stride, nv, (const c32*)w, partials);
  else
    k_seg_mdot<<<grid, GT, 0, st>>>(S, (const c64*)V, stride, nv, (const c64*)w, partials);
  k_seg_sum_c<<<dim3(nv, S.nseg), 64, 0, st>>>(S, nv, partials, out, ldo);
  return hipGetLastError();
}

hipError_t launch_seg_maxpy(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                            const int* nv_seg, const c64* coef, int ldc, void* w, int w32,
                            double* partials, double* norm2, int ldn, hipStream_t st,
                            bool defer) {
  if (S.nseg < 1) return hipSuccess;
  if (nv < 0 || nv > kMaxVec) return hipErrorInvalidValue;
  double* pn = (norm2 || defer) ? partials : nullptr;
  const dim3 grid(S.nblk, S.nseg);
  if (v32 == 2 && w32)
    k_seg_maxpy<<<grid, GT, 0, st>>>(S, (const cb16*)V, stride, nv, nv_seg, coef, ldc, (c32*)w, pn);
  else if (v32 == 2)
    return hipErrorInvalidValue;
  else if (v32 && w32)
    k_seg_maxpy<<<grid, GT, 0, st>>>(S, (const c32*)V, stride, nv, nv_seg, coef, ldc, (c32*)w, pn);
  else if (v32)
    k_seg_maxpy<<<grid, GT, 0, st>>>(S, (const c32*)V, stride, nv, nv_seg, coef, ldc, (c64*)w, pn);
  else if (w32)
    k_seg_maxpy<<<grid, GT, 0, st>>>(S, (const c64*)V, stride, nv, nv_seg, coef, ldc, (c32*)w, pn);
  else
    k_seg_maxpy<<<grid, GT, 0, st>>>(S, (const c64*)V, stride, nv, nv_seg, coef, ldc, (c64*)w, pn);
  if (norm2 && !defer) k_seg_sum_r<<<S.nseg, 64, 0, st>>>(S, partials, norm2, ldn);
  return hipGetLastError();
}

hipError_t launch_seg_reorth_flags(const SegSet& S, const double* before, const double* after,
                                  int ldn, double eta2, int* act2, hipStream_t st) {
  if (S.nseg < 1) return hipSuccess;
  k_seg_reorth_flags<<<(S.nseg + 63) / 64, 64, 0, st>>>(S, before, after, ldn, eta2, act2);
  return hipGetLastError();
}

hipError_t launch_seg_normalize(const SegSet& S, const void* src, int s32, const double* norm2,
                                int ldn, void* dst, int d32, hipStream_t st) {
  if (S.nseg < 1) return hipSuccess;
  const dim3 grid(S.nblk, S.nseg);
  double* n2 = const_cast<double*>(norm2);  // read only without SUM
  if (d32 == 2 && s32)
    k_seg_normalize<<<grid, GT, 0, st>>>(S, (const c32*)src, n2, ldn, (cb16*)dst, nullptr);
  else if (d32 == 2)
    k_seg_normalize<<<grid, GT, 0, st>>>(S, (const c64*)src, n2, ldn, (cb16*)dst, nullptr);
  else if (s32 && d32)
    k_seg_normalize<<<grid, GT, 0, st>>>(S, (const c32*)src, n2, ldn, (c32*)dst, nullptr);
  else if (s32)
    k_seg_normalize<<<grid, GT, 0, st>>>(S, (const c32*)src, n2, ldn, (c64*)dst, nullptr);
  else if (d32)
    k_seg_normalize<<<grid, GT, 0, st>>>(S, (const c64*)src, n2, ldn, (c32*)dst, nullptr);
  else
    k_seg_normalize<<<grid, GT, 0, st>>>(S, (const c64*)src, n2, ldn, (c64*)dst, nullptr);
  return hipGetLastError();
}

hipError_t launch_seg_normalize_sum(const SegSet& S, const void* src, int s32,
                                    const double* npart, double* norm2, int ldn, void* dst,
                                    int d32, hipStream_t st) {
  if (S.nseg < 1) return hipSuccess;
  if (!s32) return hipErrorInvalidValue;  // FP32 work vectors only
  const dim3 grid(S.nblk, S.nseg);
  if (d32 == 2)
    k_seg_normalize<c32, cb16, true>
        <<<grid, GT, 0, st>>>(S, (const c32*)src, norm2, ldn, (cb16*)dst, npart);
  else if (d32)
    k_seg_normalize<c32, c32, true>
        <<<grid, GT, 0, st>>>(S, (const c32*)src, norm2, ldn, (c32*)dst, npart);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_permute(int nrep, const int64_t* qoff, const int64_t* qpoff, const int* qlen,
                          int maxlen, const int* perm, const void* src, int s32, void* dst,
                          int d32, int scatter, const int* act, hipStream_t st) {
  if (nrep < 1 || maxlen < 1) return hipSuccess;
  const dim3 grid(std::min((maxlen + GT - 1) / GT, 4096), nrep);
  if (s32 && d32)
    k_permute<<<grid, GT, 0, st>>>(qoff, qpoff, qlen, perm, (const c32*)src, (c32*)dst, scatter, act);
  else if (s32)
    k_permute<<<grid, GT, 0, st>>>(qoff, qpoff, qlen, perm, (const c32*)src, (c64*)dst, scatter, act);
  else if (d32)
    k_permute<<<grid, GT, 0, st>>>(qoff, qpoff, qlen, perm, (const c64*)src, (c32*)dst, scatter, act);
  else
    k_permute<<<grid, GT, 0, st>>>(qoff, qpoff, qlen, perm, (const c64*)src, (c64*)dst, scatter, act);
  return hipGetLastError();
}

hipError_t launch_seg_lincomb_perm(const SegSet& S, const void* V, int v32, int64_t stride,
                                   int nv, const int* nv_seg, const c64* coef, int ldc,
                                   const int* seg_rhs, const int64_t* qoff, const int64_t* qpoff,
                                   const int* perm, void* dst, int d32, hipStream_t st) {
  if (S.nseg < 1) return hipSuccess;
  if (nv < 0 || nv > kMaxVec) return hipErrorInvalidValue;
  const dim3 grid(S.nblk, S.nseg);
#define VIE_LCP(TV_, TD_)                                                                       \
  k_seg_lincomb_perm<<<grid, GT, 0, st>>>(S, (const TV_*)V, stride, nv, nv_seg, coef, ldc,      \
                                          seg_rhs, qoff, qpoff, perm, (TD_*)dst)
  if (v32 == 2) {
    if (d32) VIE_LCP(cb16, c32); else VIE_LCP(cb16, c64);
  } else if (v32) {
    if (d32) VIE_LCP(c32, c32); else VIE_LCP(c32, c64);
  } else {
    if (d32) VIE_LCP(c64, c32); else VIE_LCP(c64, c64);
  }
#undef VIE_LCP
  return hipGetLastError();
}

hipError_t launch_seg_lincomb(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                              const int* nv_seg, const c64* coef, int ldc, c64* x,
                              hipStream_t st) {
  if (S.nseg < 1) return hipSuccess;
  if (nv < 0 || nv > kMaxVec) return hipErrorInvalidValue;
  if (v32 == 2)
    k_seg_lincomb<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, (const cb16*)V, stride, nv, nv_seg, coef,
                                                       ldc, x);
  else if (v32)
    k_seg_lincomb<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, (const c32*)V, stride, nv, nv_seg, coef,
                                                       ldc, x);
  else
    k_seg_lincomb<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, (const c64*)V, stride, nv, nv_seg, coef,
                                                       ldc, x);
  return hipGetLastError();
}

hipError_t launch_seg_act_map(int nseg, const int* seg_rhs, const int* act_rhs, int* act_seg,
                              hipStream_t st) {
  if (nseg < 1) return hipSuccess;
  k_seg_act_map<<<(nseg + 255) / 256, 256, 0, st>>>(nseg, seg_rhs, act_rhs, act_seg);
  return hipGetLastError();
}

hipError_t launch_ls_cycle_init(int nseg, int maxit, const KState* st, int* act, int* steps,
                                int* mc, int* cycles, const LsBufs& L, hipStream_t s) {
  if (nseg < 1) return hipSuccess;
  k_ls_cycle_init<<<(nseg + 255) / 256, 256, 0, s>>>(nseg, maxit, st, act, steps, mc, cycles, L);
  return hipGetLastError();
}

hipError_t launch_ls_step(int nseg, int j, const c64* H1, const c64* H2, int use_h2, int ldh,
                          const double* NR, int ldn, const KState* st, double half_tol,
                          int* act, int* steps, const int* mc, const LsBufs& L, int* any,
                          hipStream_t s) {
  if (nseg < 1) return hipSuccess;
  if (j < 0 || j >= L.m) return hipErrorInvalidValue;
  k_ls_step<<<1, 256, 0, s>>>(nseg, j, H1, H2, use_h2, ldh, NR, ldn, st, half_tol, act, steps, mc,
                              L, any);
  return hipGetLastError();
}

hipError_t launch_ls_solve(int nseg, const LsBufs& L, c64* coef, int ldc, int* nvs, int* act,
                           hipStream_t s) {
  if (nseg < 1) return hipSuccess;
  k_ls_solve<<<(nseg + 63) / 64, 64, 0, s>>>(nseg, L, coef, ldc, nvs, act);
  return hipGetLastError();
}

hipError_t launch_ls_full(int nseg, int k, const c64* H1, const c64* H2, int use_h2, int ldh,
                          const double* NR, int ldn, const int* act, const LsBufs& L, c64* coef,
                          int ldc, int* nvs, hipStream_t s) {
  if (nseg < 1) return hipSuccess;
  if (k < 1 || k > L.m) return hipErrorInvalidValue;
  k_ls_full<<<(nseg + 63) / 64, 64, 0, s>>>(nseg, k, H1, H2, use_h2, ldh, NR, ldn, act, L, coef,
                                             ldc, nvs);
  return hipGetLastError();
}

hipError_t launch_any_notdone(int n, const KState* st, const int* steps, int maxit, int* any,
                              hipStream_t s) {
  k_any_notdone<<<1, 256, 0, s>>>(n, st, steps, maxit, any);
  return hipGetLastError();
}

}  // namespace vie
