// Internal launcher interface between the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "common.h"

namespace vie {

// Per-right-hand-side BiCGSTAB state, resident in device memory.
struct KState {
  c64 rho, rho_prev, alpha, omega, beta;
  double bnorm2;   // ||b||^2
  double rnorm2;   // ||r||^2 (recursive inside a cycle, true after a restart)
  double target2;  // stop the current cycle when rnorm2 <= target2
  int active;      // 1 while this right-hand side iterates
  int it_cycle;    // iterations in the current cycle
  int iters;       // total iterations
  int breakdown;   // why the last cycle broke down: 0 no, 1 rhat.Ap, 2 rhat.r, 3 omega, 4 overflow
  int notdone;     // 1 while the true residual is above tol
  double rh2;      // ||rhat||^2 (shadow residual of the current cycle)
  int cycles;      // FP64 true-residual products (restarts) so far
  int pad_;
  unsigned long long t_done;  // device wall clock when the true residual first met tol (0: not)
};

// Epilogue of the inverse-x pass (y = x - chi * conv, then):
enum EpiMode {
  EPI_PLAIN = 0,  // y only
  EPI_RHV = 1,    // partial sum conj(rhat) . y          (v = A p)
  EPI_TS = 2,     // partial sums conj(y) . x, |y|^2       (t = A s)
  EPI_RESID = 3   // r = b - y, rhat = r, partial |r|^2    (restart)
};

// Geometry of one group of right-hand sides sharing a grid and spectrum.
struct GroupGeom {
  int N[3];     // grid
  int P[3];     // FFT lengths (powers of two >= 2N - 1)
  int Q[3];     // octant extents P/2 + 1
  int64_t n;    // N1 N2 N3
  int nrhs;     // right-hand sides in the group
};

// Body-compressed vectors: the solver stores each right-hand side's vectors
// over its body's voxels only, v[rhs][comp][k] at roff[rhs] + comp nb + k.
struct BodyIdx {
  const int* vox;        // concatenated body-voxel linear indices (ascending per body)
  const int* line_ptr;   // [body][N2 N3 + 1] start of each x-line in the body's list
  const double* chic;    // chi at the body voxels (same order as vox)
  const int* nb;         // [body] body voxels
  const int* voff;       // [body] offset of the body's lists in vox / chic
  const int64_t* roff;   // [rhs] offset of the right-hand side's vector
  const int* rhs_body;   // [rhs] body of each right-hand side
};

// Device pointers used by one operator product of a group.
struct MatvecArgs {
  const GroupGeom* g;
  const double* chi;       // [body][n]
  const int* rhs_body;     // [nrhs] body index of each right-hand side
  const void* spec;        // octant spectrum, c64 or c32 per precision
  const void* tw[3];       // twiddle tables per axis (c64 or c32)
  void* bufA;              // x-transformed scratch [nrhs][3][N3][N2][P1]
  void* bufB;              // y-transformed scratch [nrhs][3][N3/zl][P2][zl][P1]
  const int* active;       // [nrhs] or nullptr
  int zvar = 0;            // launch shape of the z pass (autotuned per group/precision)
  const BodyIdx* bi = nullptr;  // non-null: x and y are body-compressed
  int io32 = 0;  // compressed x and y stored in FP32 (FP32 passes, plain epilogue only);
                 // 2: x stored in bfloat16, y in FP32
  // Approximate products (FP32, bfloat16 x, FP32 y, plain epilogue): with
  // spec16 set the y and z passes run in packed FP16 arithmetic on FP16
  // scratch (see h16_ok for the grids this takes): spec16 the scaled
  // pair-packed spectrum, tw16 the splatted y and z twiddles, hs the forward
  // scales along x, y, z, hout the inverse x pass's scale back.
  const void* spec16 = nullptr;
  const void* tw16[2] = {nullptr, nullptr};
  float hs[3] = {0.f, 0.f, 0.f};
  float hout = 0.f;
  // Fused packed passes only (xy_fused_ok), with npart set: x is an FP32 work
  // vector w; right-hand side q of it is scaled by 1 / ||w_q|| (||w_q||^2
  // summed from the nblk partials npart[q nblk ..] in a fixed order and
  // stored at nrm[q ldn]) and rounded to bfloat16, that vector is stored at
  // vout (bfloat16) and multiplied: the normalisation of an Arnoldi step
  // done inside the next product
  const double* npart = nullptr;
  int nblk = 0;
  double* nrm = nullptr;
  int ldn = 0;
  void* vout = nullptr;
};

// precision 0: FP64 passes, 1: FP32 passes (input/output vectors are FP64)
// epilogue extras: aux (rhat for EPI_RHV, rhat output for EPI_RESID),
// partials [nrhs][blocks][2] (c64), pol/phase tables for EPI_RESID.
struct EpiArgs {
  int mode;
  c64* aux;
  c64* partials;
  int part_blocks;  // filled by the launcher: blocks per right-hand side
  const c64* pol;   // [nrhs][3]
  const c64* ph;    // [nrhs][N1 + N2 + N3]  exp(i k0 khat_a (o_a + h idx))
};

int part_blocks_xinv(const GroupGeom& g, int precision);
int z_block(const GroupGeom& g);        // z planes kept adjacent in the y/z scratch
int64_t bufB_elems(const GroupGeom& g);  // y/z scratch elements per right-hand side
int vec_blocks(const GroupGeom& g);

// x, y: c64 vectors, or c32 when a.io32.
hipError_t launch_matvec(const MatvecArgs& a, int precision, const void* x, void* y, EpiArgs& epi,
                         hipStream_t s, void (*ev_cb)(int kind, bool begin, void* u), void* u);
int z_variants(int precision);  // z-pass launch shapes (0 = FP64, 1 = FP32)
// z pass alone on bufB (autotuning; contents are scratch)
hipError_t launch_z_only(const MatvecArgs& a, int precision, hipStream_t s);
// Packed-FP16 y and z passes of approximate FP32 products: whether the grid
// takes them, and their tables: max |re|, |im| of an FP32 octant spectrum (n
// complex values) as float bits atomically maxed into *dmax (zeroed by the
// caller), the pair-packed FP16 copy scaled by gs (Q2 Q3 P1/2 6 packed
// pairs, 8 bytes each), the splatted FP16 twiddles of n points.
bool h16_ok(const GroupGeom& g);
// timing kinds of their passes: the five separate ones (26..30), then the
// fused x-y forward and inverse passes (31, 32) of grids xy_fused_ok takes
static constexpr int kH16Kind0 = 26;
bool xy_fused_ok(const GroupGeom& g);
hipError_t launch_spec_absmax(const void* spec32, int64_t n, unsigned* dmax, hipStream_t s);
hipError_t launch_spec_pairs(const void* spec32, void* spec16, const GroupGeom& g, float gs,
                             hipStream_t s);
hipError_t launch_tw_h2(const void* tw32, void* tw16, int n, hipStream_t s);

// Green spectrum: sample the circulant kernel of component ab into
// work[P3][P2][P1] (c64).
hipError_t launch_green_sample(c64* work, const GroupGeom& g, int ab, double h, double k0,
                               hipStream_t s);
// In-place unpadded 3-D FFT of one P3 x P2 x P1 c64 array (forward).
hipError_t launch_fft3d_full(c64* work, c64* tmp, const GroupGeom& g, const void* tw[3],
                             hipStream_t s);
// Pruned x and y stages of the forward 3-D FFT of one field (FP64 or FP32),
// with E[a] <= P[a] / 2.  xy_pad: input non-zero on the first E[a] points
// per axis, in [E3][E2][E1] -> t1 [E3][E2][P1] -> out [E3][P2][P1].
// yx_trunc: the y and x stages of a transform keeping the first E[1] y
// outputs, in [E3][P2][P1] -> t1 [E3][E2][P1] -> out [E3][E2][P1] (all P1 x
// outputs).  tw: the twiddle tables of the field's precision.
hipError_t launch_fft_xy_pad(const c64* in, c64* t1, c64* out, const int E[3], const int P[3],
                             const void* tw[3], hipStream_t s);
hipError_t launch_fft_xy_pad(const c32* in, c32* t1, c32* out, const int E[3], const int P[3],
                             const void* tw[3], hipStream_t s);
hipError_t launch_fft_yx_trunc(const c64* in, c64* t1, c64* out, const int E[3], const int P[3],
                               const void* tw[3], hipStream_t s);
hipError_t launch_fft_yx_trunc(const c32* in, c32* t1, c32* out, const int E[3], const int P[3],
                               const void* tw[3], hipStream_t s);
// Octant compression with 1/M scaling into spec64 (and spec32 if non-null).
hipError_t launch_octant(const c64* work, c64* spec64, c32* spec32, const GroupGeom& g, int ab,
                         hipStream_t s);

// Krylov vector kernels on body-compressed FP64 vectors (3 nb per rhs).
// vb = vec_blocks(max 3 nb) workgroups per right-hand side.
int vec_blocks_n(int64_t max_len);
// b = chi pol e^{i k0 khat.r}; r = rhat = b; x = 0 unless keep_x; partials |b|^2.
// mask (nullable): only right-hand sides with mask[rhs] != 0.
hipError_t launch_init_zero_guess(const GroupGeom& g, const BodyIdx& bi, int vb,
                                  const c64* pol, const c64* ph, c64* x, c64* r, c64* rh,
                                  c64* partials, int keep_x, const int* mask, hipStream_t s);
hipError_t launch_update_p(const GroupGeom& g, const BodyIdx& bi, int vb, const KState* st,
                           const int* active, const c64* r, c64* p, const c64* v, hipStream_t s);
hipError_t launch_update_s(const GroupGeom& g, const BodyIdx& bi, int vb, const KState* st,
                           const int* active, const c64* r, const c64* v, c64* s_out,
                           hipStream_t s);
hipError_t launch_update_xr(const GroupGeom& g, const BodyIdx& bi, int vb, const KState* st,
                            const int* active, c64* x, c64* r, const c64* p, const c64* sv,
                            const c64* t, const c64* rh, c64* partials, hipStream_t s);
// Finalize reductions (one workgroup per right-hand side, fixed order):
// FIN_RESTART acts on the right-hand sides not done; FIN_PENDING (the same
// restart) on those whose cycle has ended and waits for its true residual.
enum FinWhich {
  FIN_ALPHA = 0,
  FIN_OMEGA = 1,
  FIN_RHO = 2,
  FIN_INIT = 3,
  FIN_RESTART = 4,
  FIN_PENDING = 5
};
struct FinParams {
  double tol2_done;   // converged when ||r_true||^2 <= tol2_done ||b||^2
  double tol2_inner;  // a cycle may stop at ||r||^2 <= tol2_inner ||b||^2 ...
  double eta2;        // ... or at ||r||^2 <= eta2 ||r_cycle_start||^2 (larger of the two)
  int max_iter;
};
hipError_t launch_finalize(int which, int nrhs, int nblk, const c64* partials, KState* st,
                           int* active, const FinParams& fp, hipStream_t s);
hipError_t launch_axpy_real(int64_t n, double a, const c64* x, c64* y, hipStream_t s);

// Far field (eq. 25) on FP64 MFMA.  The body voxels are grouped into aligned
// blocks of 16 voxels.  The block shape (bx x by x bz) is chosen per band of
// z layers to minimise empty slots (a slab and the fins on it want different
// shapes); bands with the same shape form one group of whole tiles of 16.
struct FarGroup {
  int shape[3];
  int tile0, ntiles;
};
struct FarBlocks {
  std::vector<FarGroup> groups;
  int nblk = 0, ntiles = 0;
  std::vector<int> org;  // [ntiles*16][4] block origin (i, j, k, 0) in voxels
  std::vector<int> vi;   // [ntiles*16][16] compressed voxel index at offset u, -1 empty
};
void far_blocks_build(const int* vox, int nb, const int N[3], FarBlocks& fb);
// Total K-split count over the groups, and packed-operand size (c64).
int far_split_total(const FarBlocks& fb, int nd);
size_t far_pack_elems(int ntiles);
// F[rhs][dir][2] = (F_theta, F_phi) for nr right-hand sides of one body; w
// body-compressed with per-rhs offsets roff (host values), blk_vi / blk_org the
// device copies of fb.vi / fb.org; dirs[nd][9] = (r, theta-hat, phi-hat).
// Scratch: Wd far_pack_elems(ntiles) c64, part far_split_total(..)*nd*3 c64.
hipError_t launch_farfield_mfma(const c64* w, const int64_t* roff_host, int nr, int nb,
                                const FarBlocks& fb, const int* blk_vi, const int* blk_org,
                                const double* dirs, int nd, double k0, double h,
                                const double* origin, c64* Wd, c64* part, c64* F,
                                hipStream_t s);
// ||v_rhs||^2 of body-compressed vectors into out[nrhs] (device).
hipError_t launch_vec_norm2(int nrhs, const BodyIdx& bi, const c64* v, double* out,
                            hipStream_t s);
// p[i] = v for i < n (device ints), by a kernel (no memset node when captured).
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s);
// *out = the device wall clock (constant rate, hipDeviceAttributeWallClockRate
// kHz) when the stream reaches this launch
hipError_t launch_stamp(unsigned long long* out, hipStream_t s);
// Gather a box-layout vector [3][n] into body-compressed storage [3][nb].
hipError_t launch_compress(const c64* box, c64* comp, const int* vox, int nb, int64_t n,
                           hipStream_t s);

}  // namespace vie
