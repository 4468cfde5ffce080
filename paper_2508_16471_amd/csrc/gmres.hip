// Segmented multi-vector kernels of the flexible GMRES driver (Arnoldi with
// classical Gram-Schmidt and selective reorthogonalisation, solution update) and the permutation
// between a body's vector and its block-ordered copy (block-Jacobi
// preconditioner).  All work is HBM-bound streaming over FP64 complex vectors:
// one coalesced 16-byte load per element per vector, reductions through
// per-workgroup partials summed in a fixed order.
#include <algorithm>

#include "gmres.h"

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
__device__ __forceinline__ void st(c64* p, c64 v) { *p = v; }
__device__ __forceinline__ void st(c32* p, c64 v) { *p = cvt<float>(v); }

template <typename TV>
__global__ __launch_bounds__(GT) void k_seg_mdot(SegSet S, const TV* __restrict__ V,
                                                 int64_t stride, int nv,
                                                 const c64* __restrict__ w,
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
    for (int e = blk * GT + threadIdx.x; e < len; e += S.nblk * GT) {
      const c64 we = w[off + e];
#pragma unroll
      for (int u = 0; u < GU; ++u)
        if (i0 + u < nv) acc[u] = acc[u] + cmulc(ld64(V + (int64_t)(i0 + u) * stride + off + e), we);
    }
#pragma unroll
    for (int u = 0; u < GU; ++u)
      for (int m = 32; m >= 1; m >>= 1) acc[u] = acc[u] + shfl_xor_c(acc[u], m);
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < GU; ++u) red[wv][u] = acc[u];
    }
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

template <typename TV>
__global__ __launch_bounds__(GT) void k_seg_maxpy(SegSet S, const TV* __restrict__ V,
                                                  int64_t stride, int nv,
                                                  const int* __restrict__ nv_seg,
                                                  const c64* __restrict__ coef, int ldc,
                                                  c64* __restrict__ w,
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
    c64 a = w[off + e];
    for (int i = 0; i < n; ++i) a = a - cf[i] * ld64(V + (int64_t)i * stride + off + e);
    if (n > 0) w[off + e] = a;
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

template <typename TD>
__global__ __launch_bounds__(GT) void k_seg_normalize(SegSet S, const c64* __restrict__ src,
                                                      const double* __restrict__ norm2, int ldn,
                                                      TD* __restrict__ dst) {
  const int s = blockIdx.y, blk = blockIdx.x;
  if (S.active && !S.active[s]) return;
  const int64_t off = S.off[s];
  const int len = S.len[s];
  const double n2 = norm2[(int64_t)s * ldn];
  const double sc = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
  for (int e = blk * GT + threadIdx.x; e < len; e += S.nblk * GT) st(dst + off + e, sc * src[off + e]);
}

template <typename TS>
__global__ __launch_bounds__(GT) void k_seg_widen(SegSet S, const TS* __restrict__ src,
                                                  c64* __restrict__ dst) {
  const int s = blockIdx.y, blk = blockIdx.x;
  if (S.active && !S.active[s]) return;
  const int64_t off = S.off[s];
  const int len = S.len[s];
  for (int e = blk * GT + threadIdx.x; e < len; e += S.nblk * GT) dst[off + e] = ld64(src + off + e);
}

template <typename TS, typename TD>
__global__ __launch_bounds__(GT) void k_permute(const int64_t* __restrict__ qoff,
                                                const int64_t* __restrict__ qpoff,
                                                const int* __restrict__ qlen,
                                                const int* __restrict__ perm,
                                                const TS* __restrict__ src,
                                                TD* __restrict__ dst, int scatter) {
  const int q = blockIdx.y;
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

}  // namespace

int seg_blocks(int64_t max_len) {
  int64_t b = (max_len + 4 * GT - 1) / (4 * GT);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 256));
}

hipError_t launch_seg_mdot(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                           const c64* w, c64* partials, c64* out, int ldo, hipStream_t st) {
  if (S.nseg < 1 || nv < 1) return hipSuccess;
  if (v32)
    k_seg_mdot<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, (const c32*)V, stride, nv, w, partials);
  else
    k_seg_mdot<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, (const c64*)V, stride, nv, w, partials);
  k_seg_sum_c<<<dim3(nv, S.nseg), 64, 0, st>>>(S, nv, partials, out, ldo);
  return hipGetLastError();
}

hipError_t launch_seg_maxpy(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                            const int* nv_seg, const c64* coef, int ldc, c64* w,
                            double* partials, double* norm2, int ldn, hipStream_t st) {
  if (S.nseg < 1) return hipSuccess;
  if (nv < 0 || nv > kMaxVec) return hipErrorInvalidValue;
  double* pn = norm2 ? partials : nullptr;
  if (v32)
    k_seg_maxpy<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, (const c32*)V, stride, nv, nv_seg, coef,
                                                     ldc, w, pn);
  else
    k_seg_maxpy<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, (const c64*)V, stride, nv, nv_seg, coef,
                                                     ldc, w, pn);
  if (norm2) k_seg_sum_r<<<S.nseg, 64, 0, st>>>(S, partials, norm2, ldn);
  return hipGetLastError();
}

hipError_t launch_seg_reorth_flags(const SegSet& S, const double* before, const double* after,
                                  int ldn, double eta2, int* act2, hipStream_t st) {
  if (S.nseg < 1) return hipSuccess;
  k_seg_reorth_flags<<<(S.nseg + 63) / 64, 64, 0, st>>>(S, before, after, ldn, eta2, act2);
  return hipGetLastError();
}

hipError_t launch_seg_normalize(const SegSet& S, const c64* src, const double* norm2, int ldn,
                                void* dst, int d32, hipStream_t st) {
  if (S.nseg < 1) return hipSuccess;
  if (d32)
    k_seg_normalize<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, src, norm2, ldn, (c32*)dst);
  else
    k_seg_normalize<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, src, norm2, ldn, (c64*)dst);
  return hipGetLastError();
}

hipError_t launch_seg_widen(const SegSet& S, const void* src, int s32, c64* dst, hipStream_t st) {
  if (S.nseg < 1) return hipSuccess;
  if (s32)
    k_seg_widen<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, (const c32*)src, dst);
  else
    k_seg_widen<<<dim3(S.nblk, S.nseg), GT, 0, st>>>(S, (const c64*)src, dst);
  return hipGetLastError();
}

hipError_t launch_permute(int nrep, const int64_t* qoff, const int64_t* qpoff, const int* qlen,
                          int maxlen, const int* perm, const void* src, int s32, void* dst,
                          int d32, int scatter, hipStream_t st) {
  if (nrep < 1 || maxlen < 1) return hipSuccess;
  const dim3 grid(std::min((maxlen + GT - 1) / GT, 4096), nrep);
  if (s32 && d32)
    k_permute<<<grid, GT, 0, st>>>(qoff, qpoff, qlen, perm, (const c32*)src, (c32*)dst, scatter);
  else if (s32)
    k_permute<<<grid, GT, 0, st>>>(qoff, qpoff, qlen, perm, (const c32*)src, (c64*)dst, scatter);
  else if (d32)
    k_permute<<<grid, GT, 0, st>>>(qoff, qpoff, qlen, perm, (const c64*)src, (c32*)dst, scatter);
  else
    k_permute<<<grid, GT, 0, st>>>(qoff, qpoff, qlen, perm, (const c64*)src, (c64*)dst, scatter);
  return hipGetLastError();
}

}  // namespace vie
