// Launchers of the segmented multi-vector kernels used by the flexible GMRES
// driver and its block-Jacobi preconditioner.
//
// A segment is one independent vector of a batched solve (one right-hand
// side, or one block of one right-hand side): elements [off[s], off[s] +
// len[s]) of every vector.  A multi-vector holds nv vectors at base + i *
// stride.  Reductions go through per-workgroup partials summed in a fixed
// order, so results do not depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace vie {

struct SegSet {
  const int64_t* off;  // [nseg] first element of each segment (device)
  const int* len;      // [nseg] elements (device)
  const int* active;   // [nseg] (device) or nullptr: segments with 0 are skipped
  int nseg;
  int nblk;            // workgroups per segment, from seg_blocks()
};

int seg_blocks(int64_t max_len);

// Multi-vectors V may be stored in FP64 (v32 = 0: c64) or FP32 (v32 = 1:
// c32); arithmetic and the vectors w, x are FP64 either way.

// out[s * ldo + i] = sum_e conj(V_i[e]) w[e] over segment s, for i < nv
// (zero for skipped segments).  partials: nseg * nv * nblk c64.
hipError_t launch_seg_mdot(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                           const c64* w, c64* partials, c64* out, int ldo, hipStream_t st);

// w[e] -= sum_{i < n_s} coef[s * ldc + i] V_i[e] with n_s = nv, or
// min(nv, nv_seg[s]) when nv_seg is given.  With norm2 != nullptr also
// norm2[s * ldn] = ||w_s||^2 after the update (partials: nseg * nblk doubles).
// nv = 0 only measures the norm.
hipError_t launch_seg_maxpy(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                            const int* nv_seg, const c64* coef, int ldc, c64* w,
                            double* partials, double* norm2, int ldn, hipStream_t st);

// act2[s] = 1 where segment s is active and after[s * ldn] < eta2 * before[s]
// (too much cancellation in a Gram-Schmidt pass: orthogonalise again).
hipError_t launch_seg_reorth_flags(const SegSet& S, const double* before, const double* after,
                                  int ldn, double eta2, int* act2, hipStream_t st);

// dst = src / sqrt(norm2[s * ldn]) per segment (zero where norm2 is 0),
// stored in FP32 when d32.
hipError_t launch_seg_normalize(const SegSet& S, const c64* src, const double* norm2, int ldn,
                                void* dst, int d32, hipStream_t st);

// dst = src (FP32 when s32) as FP64, per active segment.
hipError_t launch_seg_widen(const SegSet& S, const void* src, int s32, c64* dst, hipStream_t st);

// Permutation of each of nrep vectors (vector q: qlen[q] elements at qoff[q],
// its permutation at perm + qpoff[q]; maxlen >= every qlen):
//   gather  (scatter == 0): dst[qoff + j] = src[qoff + perm[j]]
//   scatter (scatter != 0): dst[qoff + perm[j]] = src[qoff + j]
// src is FP32 when s32, dst when d32.
hipError_t launch_permute(int nrep, const int64_t* qoff, const int64_t* qpoff, const int* qlen,
                          int maxlen, const int* perm, const void* src, int s32, void* dst,
                          int d32, int scatter, hipStream_t st);

}  // namespace vie
