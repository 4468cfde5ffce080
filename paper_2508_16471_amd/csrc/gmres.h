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

struct KState;

struct SegSet {
  const int64_t* off;  // [nseg] first element of each segment (device)
  const int* len;      // [nseg] elements (device)
  const int* active;   // [nseg] (device) or nullptr: segments with 0 are skipped
  int nseg;
  int nblk;            // workgroups per segment, from seg_blocks()
};

int seg_blocks(int64_t max_len);

// Multi-vectors V may be stored in FP64 (v32 = 0: c64), FP32 (v32 = 1:
// c32) or bfloat16 (v32 = 2: cb16, with an FP32 w); arithmetic is FP64 either
// way.  The normalisation writes a bfloat16 destination for d32 = 2.

// out[s * ldo + i] = sum_e conj(V_i[e]) w[e] over segment s, for i < nv
// (zero for skipped segments); w is FP32 when w32.  partials: nseg * nv * nblk
// c64.
hipError_t launch_seg_mdot(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                           const void* w, int w32, c64* partials, c64* out, int ldo,
                           hipStream_t st);

// w[e] -= sum_{i < n_s} coef[s * ldc + i] V_i[e] with n_s = nv, or
// min(nv, nv_seg[s]) when nv_seg is given (w FP32 when w32, arithmetic FP64).
// With norm2 != nullptr also norm2[s * ldn] = ||w_s||^2 of the stored result
// (partials: nseg * nblk doubles).  nv = 0 only measures the norm.  defer:
// only the partials are written (launch_seg_normalize_sum reduces them).
hipError_t launch_seg_maxpy(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                            const int* nv_seg, const c64* coef, int ldc, void* w, int w32,
                            double* partials, double* norm2, int ldn, hipStream_t st,
                            bool defer = false);

// act2[s] = 1 where segment s is active and after[s * ldn] < eta2 * before[s]
// (too much cancellation in a Gram-Schmidt pass: orthogonalise again).
hipError_t launch_seg_reorth_flags(const SegSet& S, const double* before, const double* after,
                                  int ldn, double eta2, int* act2, hipStream_t st);

// dst = src / sqrt(norm2[s * ldn]) per segment (zero where norm2 is 0);
// src is FP32 when s32, dst when d32.
hipError_t launch_seg_normalize(const SegSet& S, const void* src, int s32, const double* norm2,
                                int ldn, void* dst, int d32, hipStream_t st);
// The same after a deferred multi-axpy: norm2[s * ldn] is reduced from its
// partials npart first (same result as the non-deferred sum) and stored; FP32
// src only.
hipError_t launch_seg_normalize_sum(const SegSet& S, const void* src, int s32,
                                    const double* npart, double* norm2, int ldn, void* dst,
                                    int d32, hipStream_t st);

// x[e] = -sum_{i < n_s} coef[s * ldc + i] V_i[e] over every active segment
// (n_s = min(nv, nv_seg[s]); x = 0 where n_s = 0).
hipError_t launch_seg_lincomb(const SegSet& S, const void* V, int v32, int64_t stride, int nv,
                              const int* nv_seg, const c64* coef, int ldc, c64* x,
                              hipStream_t st);

// The same combination scattered into the outer vectors' order: element e
// of segment s (right-hand side q = seg_rhs[s]) goes to
// dst[qoff[q] + perm[qpoff[q] + off[s] - qoff[q] + e]] (dst FP32 when d32).
hipError_t launch_seg_lincomb_perm(const SegSet& S, const void* V, int v32, int64_t stride,
                                   int nv, const int* nv_seg, const c64* coef, int ldc,
                                   const int* seg_rhs, const int64_t* qoff, const int64_t* qpoff,
                                   const int* perm, void* dst, int d32, hipStream_t st);

// Permutation of each of nrep vectors (vector q: qlen[q] elements at qoff[q],
// its permutation at perm + qpoff[q]; maxlen >= every qlen):
//   gather  (scatter == 0): dst[qoff + j] = src[qoff + perm[j]]
//   scatter (scatter != 0): dst[qoff + perm[j]] = src[qoff + j]
// src is FP32 when s32, dst when d32; vectors with act[q] == 0 are skipped
// (act may be nullptr).
hipError_t launch_permute(int nrep, const int64_t* qoff, const int64_t* qpoff, const int* qlen,
                          int maxlen, const int* perm, const void* src, int s32, void* dst,
                          int d32, int scatter, const int* act, hipStream_t st);

// act_seg[s] = act_rhs[seg_rhs[s]] (activity of every segment from that of
// its right-hand side).
hipError_t launch_seg_act_map(int nseg, const int* seg_rhs, const int* act_rhs, int* act_seg,
                              hipStream_t st);

// ---------------------------------------------------------------------------
// Least-squares part of GMRES on the device: the Hessenberg matrix of every
// segment reduced column by column by complex Givens rotations (c real,
// s complex), then the triangular solve.  One thread per segment; the
// Hessenberg columns come from the Arnoldi kernels above: column j of all
// segments at H + j * nseg * ldh, entry i of segment s at [s * ldh + i]
// (H1 + H2 when both Gram-Schmidt passes ran, use_h2), the subdiagonal as
// sqrt(NR[s * ldn + j + 1]).
struct LsBufs {
  c64* R;      // [nseg][m][ldr] rotated columns, entry i of column j at j * ldr + i
  double* cs;  // [nseg][m]
  c64* sn;     // [nseg][m]
  c64* g;      // [nseg][ldr] rotated right-hand side beta e_1
  int* nst;    // [nseg] columns taken in the current cycle
  int ldr;     // m + 1
  int m;
};

// Start of an outer cycle: act[q] = notdone && steps[q] < maxit;
// cycles[q] += notdone; nst = 0; mc[q] = min(m, maxit - steps[q]);
// g = (||r_q||, 0, ...), with ||r_q||^2 = st[q].rnorm2.
hipError_t launch_ls_cycle_init(int nseg, int maxit, const KState* st, int* act, int* steps,
                                int* mc, int* cycles, const LsBufs& L, hipStream_t s);
// Step j of every active segment: append column j; the segment leaves the
// cycle (act = 0) once its residual estimate |g[j+1]| <= half_tol ||b||
// (||b||^2 = st[q].bnorm2), it has taken mc[q] columns, or the subdiagonal
// is <= 1e-14 ||r_cycle||.  steps[q] counts the columns of every cycle.
// any[0] = 1 while some segment is still active.
hipError_t launch_ls_step(int nseg, int j, const c64* H1, const c64* H2, int use_h2, int ldh,
                          const double* NR, int ldn, const KState* st, double half_tol,
                          int* act, int* steps, const int* mc, const LsBufs& L, int* any,
                          hipStream_t s);
// End of a cycle: y from R y = g over the nst columns, coef[s * ldc + i] = -y_i,
// nvs = nst, act[s] = (nst > 0).
hipError_t launch_ls_solve(int nseg, const LsBufs& L, c64* coef, int ldc, int* nvs, int* act,
                           hipStream_t s);
// Whole k-step GMRES least squares of every active segment (the block
// solves): beta = sqrt(NR[s * ldn]); columns j < k until the subdiagonal is
// <= 1e-14 beta; coef = -y, nvs = columns used (0 for inactive segments or
// beta = 0).
hipError_t launch_ls_full(int nseg, int k, const c64* H1, const c64* H2, int use_h2, int ldh,
                          const double* NR, int ldn, const int* act, const LsBufs& L, c64* coef,
                          int ldc, int* nvs, hipStream_t s);
// any[0] = 1 if some q < n has st[q].notdone && steps[q] < maxit.
hipError_t launch_any_notdone(int n, const KState* st, const int* steps, int maxit, int* any,
                              hipStream_t s);

}  // namespace vie
