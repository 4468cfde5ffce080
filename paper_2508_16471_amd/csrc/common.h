// Shared device/host definitions of the MI355X VIE library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vie {

// Interleaved complex; 2*sizeof(T) alignment so a value moves in one
// dwordx4 (FP64) or dwordx2 (FP32) memory instruction.
template <typename T>
struct __align__(2 * sizeof(T)) cpx {
  T re, im;
};
using c64 = cpx<double>;
using c32 = cpx<float>;
using cb16 = cpx<__bf16>;  // storage only (Arnoldi basis of the block solves)

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T r, T i) {
  cpx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return mk(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return mk(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) {
  return mk(s * a.re, s * a.im);
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// fused a + s*b  (s complex)
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cfma(cpx<T> s, cpx<T> b, cpx<T> a) {
  return mk(a.re + s.re * b.re - s.im * b.im, a.im + s.re * b.im + s.im * b.re);
}

template <typename D, typename S>
__host__ __device__ __forceinline__ cpx<D> cvt(cpx<S> a) {
  return mk((D)a.re, (D)a.im);
}

// Workgroup barrier for LDS exchanges: orders LDS accesses only, so global
// loads issued before it (prefetches) stay in flight across it, unlike
// __syncthreads, whose fence also waits for every outstanding global access.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroups are handed to the 8 XCDs round-robin (block b -> XCD b % 8) and
// each XCD has its own L2.  Remapping the linear block id makes neighbouring
// tiles (which share cache lines or spectrum entries) run on one XCD at about
// the same time.  Bijective for any nblocks.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  constexpr int NX = 8;
  int q = nblocks / NX, r = nblocks % NX;
  int x = b % NX, i = b / NX;
  // XCD x owns logical tiles [start(x), start(x) + count(x))
  int start = x * q + (x < r ? x : r);
  int count = q + (x < r ? 1 : 0);
  return (i < count) ? start + i : b;  // i < count always holds for b < nblocks
}

}  // namespace vie
