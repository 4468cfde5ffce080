/*
 * vie.h -- C ABI of the MI355X FFT-VIE / far-field / two-photon library.
 *
 * Problem (arXiv 2508.16471, Sec. II-C): a lossless dielectric body of
 * piecewise-constant permittivity eps_r in vacuum, lit by plane-wave input
 * channels (e^{-i w t} convention).  The polarisation current
 * J = -i w (eps - eps0) E (eq. Js_def) solves the volume integral equation
 * eq. 24 with the free-space dyadic Green's function (eq. dyadicG).  The
 * library discretises it on the body's uniform voxel grid (pulse basis,
 * centre collocation, equal-volume-sphere self term) in the contrast-current
 * unknown w = chi E, chi = eps_r - 1:
 *
 *     w_m - chi_m sum_n Ghat_mn w_n = chi_m e_m,
 *     Ghat_mn = k0^2 h^3 G(r_m - r_n) (m != n),  Ghat_mm = s I,
 *     s = -1/3 + 2/3 (cos x + x sin x - 1) + i k0^3 h^3 / (6 pi),
 *     x = k0 h (3 / 4 pi)^(1/3),
 *
 * or, with VIE_FLAG_CUBE_SELF, the voxel's own singular integral (the paper
 * leaves the self-term integral open):
 *
 *     s_cube = -1/3 + (2 k0^2 / 3) integral over the cube of e^{i k0 r} / (4 pi r) dV
 *
 * (-1/3: the cube's static principal value; its imaginary part equals the
 * radiation reaction k0^3 h^3 / (6 pi) only to leading order in k0 h, so that
 * discrete model is not exactly lossless),
 *
 * solves it with BiCGSTAB around an FFT-accelerated product (Sec. II-C),
 * evaluates the far-field amplitude of eq. 25,
 *     F(r) = k0^2 h^3 / (4 pi) (I - r r) sum_n w_n exp(-i k0 r . r_n)
 * (so that E_sca ~ F e^{i k0 R} / R), and the two-photon observables g2
 * (eq. 10) and the coincidence number Nc(dtau) (eqs. 18-22).
 * J^s follows from w as J^s = -i w eps0 w.
 *
 * Conventions
 *   - Lengths in any unit, the same for h, origin and 1/k0.
 *   - Grids: n[3] = (N1, N2, N3) voxels, x fastest in memory; voxel (i,j,l)
 *     is centred at origin + h (i, j, l).
 *   - Complex vectors of a body are [component 0..2][z][y][x], interleaved
 *     (re, im) doubles: 3 * N1 * N2 * N3 vie_c64 per right-hand side.
 *   - Every pointer argument is owned by the caller; host pointers unless
 *     the function name ends in _dev (then device pointers on the current
 *     HIP device, and the call is asynchronous on the context's stream).
 *   - Errors are negative return codes; nothing is thrown across the ABI.
 *     After VIE_EINVAL / VIE_ENOTSUP the context stays usable.  After
 *     VIE_EDEVICE the context is poisoned: later calls return VIE_ESTATE and
 *     the caller must vie_destroy() it.
 *   - A context is not thread-safe; use one per host thread.
 *
 * Environment
 *   - VIE_LOG: progress and tuning lines on stderr.
 *   - VIE_ZVAR=<k>: use z-pass launch shape k instead of timing them.
 *   - VIE_DETERMINISTIC=1: use shape 0 instead of timing, so that results are
 *     bit-for-bit the same from run to run and context to context (every
 *     reduction has a fixed order; the timed shape choice is the only
 *     run-dependent decision).
 *   - VIE_TUNE_CACHE=<file>: reuse the timed shape choices recorded in the
 *     file (lines "zshape P1 P2 P3 N1 N2 N3 precision nrhs shape") and append
 *     new ones; an unreadable or unwritable file is ignored.
 */
#ifndef VIE_H
#define VIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vie_ctx vie_ctx;
typedef struct { double re, im; } vie_c64;

enum vie_status {
  VIE_OK = 0,
  VIE_EINVAL = -1,  /* invalid argument (shape, range, NaN, NULL)            */
  VIE_ENOMEM = -2,  /* device or host allocation failed                      */
  VIE_EDEVICE = -3, /* HIP runtime error; context poisoned                   */
  VIE_ENOCONV = -4, /* a right-hand side missed tol within max_iter          */
  VIE_ENOTSUP = -5, /* valid but unsupported request (e.g. grid too large)   */
  VIE_ESTATE = -6   /* call on a poisoned / unprepared context               */
};

/* VIE_MIXED_BF16 (inner_precision of vie_solve_fgmres only): FP32 block
 * products as VIE_MIXED, with the block solves' Arnoldi basis stored in
 * bfloat16 (8-bit significand; dots and updates in FP64, work vector FP32).
 * The block solves only approximate M^{-1}, so the basis' rounding (a few
 * 1e-3 relative) leaves the preconditioner about as good while the basis
 * traffic halves; the FP64 outer residual still decides convergence.
 * Where the block grid allows it (16-layer z tiles, padded z length 32, 48,
 * 64, 96 or 128, and an even number of threads per x line), the block
 * products' y and z transforms and the Green tensor product run in packed
 * FP16 on FP16 scratch (two columns per register); the x transforms stay
 * FP32 and convert at the scratch side, fused with the y transforms per z
 * plane where the x and y lengths are 64, 96 or 128.  Each forward transform
 * scales its input by a power of two at most 1/sqrt(extent), the spectrum by
 * a power of two that brings its largest modulus into [1/2, 1), so no
 * intermediate overflows for the unit-norm basis vectors the block solves
 * multiply; the result is scaled back exactly in FP32. */
enum { VIE_FP64 = 0, VIE_MIXED = 1, VIE_MIXED_BF16 = 2 };
enum { VIE_NORM_R1 = 0, VIE_NORM_R2 = 1 };
enum {
  VIE_FLAG_TIMING = 1,  /* record per-kernel HIP-event durations (disables graphs) */
  VIE_FLAG_NO_GRAPH = 2, /* launch every BiCGSTAB iteration eagerly instead of    */
                         /* replaying a captured hipGraph of VIE_GRAPH_ITERS       */
                         /* iterations (results are identical either way)          */
  VIE_FLAG_CUBE_SELF = 4, /* self term of the exact cube cell instead of the       */
                          /* equal-volume sphere (see below); read by vie_setup,   */
                          /* vie_set_options may not change it                     */
  VIE_FLAG_Z_WINDOW = 8   /* compute each grid group on the window of z layers     */
                          /* that holds its bodies (see vie_grid); read by         */
                          /* vie_setup, vie_set_options may not change it          */
};
enum { VIE_GRAPH_ITERS = 8 };

/* One body on its own uniform grid (eq. 24's volume V, discretised). */
typedef struct {
  int32_t n[3];        /* voxels per axis: N1, N2 in 1..3072, N3 in 1..256,      */
                       /* N1 N2 N3 < 2^31                                       */
  double h;            /* voxel edge > 0                                        */
  double origin[3];    /* centre of voxel (0,0,0)                               */
  const double *eps_r; /* host, N1*N2*N3 relative permittivities, x fastest,   */
                       /* finite and >= 1 (lossless, eps_r = 1 is background);  */
                       /* copied during vie_setup                               */
} vie_body;

typedef struct {
  double k0;          /* free-space wavenumber > 0                              */
  int32_t precision;  /* VIE_FP64: FP64 FFT product; VIE_MIXED: FP32 FFT       */
                      /* product inside FP64 iterative refinement               */
  double tol;         /* stop when ||b - A w|| / ||b|| <= tol, measured with    */
                      /* the FP64 operator (A = I - chi Ghat, b = chi e)        */
  int32_t max_iter;   /* BiCGSTAB iterations per right-hand side (all cycles)   */
  double inner_tol;   /* MIXED: residual reduction per refinement cycle (1e-3) */
  int32_t warm_start; /* 1: start from the loaded network's prediction (with    */
                      /* residual check and fallback to w = 0)                  */
  int32_t flags;      /* VIE_FLAG_* bits                                        */
} vie_options;

/* Incident channel e(r) = pol exp(i k0 khat . r); |khat| = 1, pol . khat = 0. */
typedef struct {
  double khat[3];
  vie_c64 pol[3];
} vie_planewave;

typedef struct {
  int32_t iters;      /* BiCGSTAB iterations (all refinement cycles)            */
  int32_t matvecs;    /* operator products (FP32 and FP64)                      */
  int32_t cycles;     /* refinement / restart cycles                            */
  int32_t converged;  /* 1 if rel_res <= tol                                    */
  int32_t fallback;   /* 1 if a warm start was rejected and w = 0 was used      */
  int32_t warm;       /* 1 if the warm start was used                           */
  double rel_res;     /* final true ||b - A w|| / ||b|| (FP64 operator)         */
  double rel_res_x0;  /* true relative residual of the initial guess            */
  double seconds;     /* completion time: device wall-clock seconds from the   */
                      /* start of this call's device work to the FP64 residual */
                      /* check that first found rel_res <= tol (groups solved  */
                      /* earlier in the call included); 0 if not converged     */
} vie_stats;

/* Set up a context for n_bodies bodies: copies eps_r (chi = eps_r - 1) to
 * the device, builds the FP64 (and FP32) octant spectrum of the circulant
 * embedding of Ghat for each distinct (grid, h, k0), allocates Krylov and FFT
 * workspaces.  Returns VIE_EINVAL on bad shapes/values, VIE_ENOTSUP if a
 * grid exceeds the limits of vie_body.n (FFT lines of up to 6144 points
 * along x and y, 512 along z) or one component of the y/z scratch would
 * exceed 2^31 elements. */
int vie_setup(const vie_body *bodies, int32_t n_bodies, const vie_options *opt,
              vie_ctx **out);

/* Solve eq. 24 (discretised as above) for every right-hand side: body b gets
 * nrhs_per_body[b] channels taken in order from inc[].  All right-hand sides
 * of all bodies are advanced together (batched kernels); each one restarts
 * (FP64 true residual, then a new refinement cycle) as soon as its own cycle
 * ends, while the others keep iterating, and stops costing work once
 * converged.  stats (caller array, one entry per right-hand side, may be
 * NULL) report iterations, the final FP64 true residual and the completion
 * time.  Solutions stay on the device (vie_get_current,
 * vie_farfield).  Returns VIE_ENOCONV if any right-hand side missed tol
 * (stats and the best iterate are still filled in). */
int vie_solve(vie_ctx *ctx, const vie_planewave *inc, const int32_t *nrhs_per_body,
              vie_stats *stats);

/* Block preconditioner of the paper's large metasurface solve (Sec. III-B:
 * BiCGStab with a preconditioner over 7 x 7 blocks), here as block Jacobi
 * over a lateral partition, with restarted flexible GMRES (Saad 1993) as the
 * outer method because the block solves are inexact.
 *   Partition: x part p of bx holds voxels [floor(p N1 / bx),
 *   floor((p + 1) N1 / bx)), y alike; a block is one (x part, y part) pair over
 *   the full z extent.  M = the operator with every coupling between two
 *   different blocks dropped; z = M^{-1} v is approximated on every block by
 *   inner_iters steps of GMRES from zero (the minimal-residual element of that
 *   Krylov space of the block's own operator).
 * blocks = {0, 0} turns the preconditioner off (plain restarted GMRES). */
typedef struct {
  int32_t restart;         /* Arnoldi steps per cycle, 1..128                      */
  int32_t blocks[2];       /* bx, by: each 1..64 and at most N1 (N2); or {0, 0}    */
  int32_t inner_iters;     /* GMRES steps of every block solve, 1..64              */
  int32_t inner_precision; /* VIE_FP64 / VIE_MIXED: block products in FP64 / FP32; */
                           /* VIE_MIXED_BF16: bfloat16 basis, FP16 y/z passes  */
} vie_fgmres_options;

/* Solve like vie_solve (same channels, stats, solution storage and return
 * codes, all bodies and grids of the context batched) with right-
 * preconditioned restarted FGMRES.  Start: w = 0, or with warm_start the
 * network's guess under the same residual check and fallback as vie_solve.
 * The Arnoldi products use the context's precision; every cycle ends with the
 * FP64 true residual, which alone decides convergence (tol and max_iter of the
 * context: max_iter caps the Arnoldi steps).  stats: iters = Arnoldi steps,
 * cycles = FP64 residual products, matvecs = iters + cycles (the block
 * products, inner_iters per step, are not counted).  VIE_EINVAL for options
 * out of range for any grid of the context.  The first call with a new
 * partition builds the block sub-problems of every body (one spectrum per
 * group on the common cropped block grid). */
int vie_solve_fgmres(vie_ctx *ctx, const vie_planewave *inc, const int32_t *nrhs_per_body,
                     const vie_fgmres_options *opt, vie_stats *stats);

/* Apply the preconditioner alone: z = M^{-1} r (as defined above, blocks
 * required) for nvec host vectors r[nvec][3][N3][N2][N1] of the context's
 * only body; z has the same layout and is 0 off the body (entries of r off
 * the body are ignored).  VIE_EINVAL for blocks = {0, 0} or bad options. */
int vie_precond_apply(vie_ctx *ctx, const vie_fgmres_options *opt, const vie_c64 *r, vie_c64 *z,
                      int32_t nvec);

/* Far-field amplitude (eq. 25, normalisation above) of every right-hand
 * side of `body` at ndir directions (theta, phi in radians):
 * F[(rhs * ndir + d) * 2 + {0,1}] = (F_theta, F_phi) with
 * theta-hat = (cos t cos p, cos t sin p, -sin t), phi-hat = (-sin p, cos p, 0).
 * Host arrays. */
int vie_farfield(vie_ctx *ctx, int32_t body, const double *theta, const double *phi,
                 int32_t ndir, vie_c64 *F);

/* Two-photon observables of two populated channels from the 2x2 transfer
 * coefficients T = (T_a1, T_a2, T_b1, T_b2) (eqs. field_transfer1/2; T_aj is
 * detector a's projected far-field amplitude for channel j, eq. Eproj).
 * Channel weights omega[2] (NULL: equal) are the omega_kj of the field
 * operators (eqs. 8-9): every coefficient of channel j is first multiplied by
 * sqrt(omega[j]), t_aj = sqrt(w_j) T_aj, t_bj = sqrt(w_j) T_bj.  Then
 *   g2 (eq. 10) = |t_a1 t_b2 + t_a2 t_b1|^2 / (G1_a G1_b),
 *     G1_a = |t_a1|^2 + |t_a2|^2, G1_b = |t_b1|^2 + |t_b2|^2;
 *   Nc_raw[k] = sigma sqrt(pi) (|A_d|^2 + |A_e|^2 + 2 Re(A_d A_e*) c_k),
 *     A_d = t_a1 t_b2, A_e = t_a2 t_b1, c_k = exp(-dtau_k^2 / sigma^2)
 *     (eqs. 19-22 with K = 1 and baseband Gaussian wavepackets);
 *   Nc_norm = Nc_raw / D_c with D_c = sigma sqrt(pi) (|A_d|^2 + |A_e|^2)
 *     (VIE_NORM_R1, -> 1 at large delay, eq. 18) or
 *     D_c = sigma sqrt(pi) G1_a G1_b (VIE_NORM_R2, Nc_norm(0) = g2 for any
 *     weights).
 * A dark detector (zero denominator) gives NaN and VIE_OK.  VIE_EINVAL for
 * non-finite T, non-positive or non-finite weights, and sigma <= 0 when
 * delays are asked for.  Host arrays; g2, Nc_raw, Nc_norm may each be NULL. */
int hom_g2(const vie_c64 T[4], const double *omega, double sigma, const double *dtau,
           int32_t ndelay, int32_t norm, double *g2, double *Nc_raw, double *Nc_norm);

/* The grid a body is computed on.  With VIE_FLAG_Z_WINDOW a group of bodies
 * sharing (n, h) computes on a window of z layers of their grid: as many
 * layers as the tallest body's z extent, placed per body over its voxels.  Voxels
 * outside have chi = 0, so the system for the body's unknowns (and every
 * solve, current and far field) is that of the full grid.  Box vectors at the
 * ABI (vie_matvec, vie_get_current) stay in the body's grid; vie_matvec then
 * applies the operator to x restricted to the window and passes the
 * components outside it through (y = x there).  Without the flag the window
 * is the whole grid.  grid[3] = window voxels (N1, N2, N3w), fft[3] =
 * circulant lengths, offset[3] = (0, 0, first z layer of the window in the
 * body's grid).  Any pointer may be NULL. */
int vie_grid(vie_ctx *ctx, int32_t body, int32_t *grid, int32_t *fft, int32_t *offset);

/* Diagonal coefficient s of the discrete operator for voxel edge h (host
 * arithmetic): kind 0 = the default equal-volume-sphere term, kind 1 = the
 * exact cube cell (VIE_FLAG_CUBE_SELF), both as defined at the top of this
 * header.  VIE_EINVAL for another kind or non-positive / non-finite k0, h. */
int vie_self_term(int32_t kind, double k0, double h, vie_c64 *s);

/* ---------------------------------------------------------------------------
 * Rooftop basis with pulse testing (Sec. II-C, eq. Js_expand): the paper's
 * own discretisation, beside the pulse-basis operator above (FP64, or FP32
 * products inside FP64 refinement).
 *   Unknown w = chi E, component i expanded in rooftops on the faces normal
 *   to i of the body grid padded by one cell per side ("padded grid", E =
 *   n + 2 cells per axis; padded cell c is centred at origin + h (c - 1)).
 *   A face is active if one of its two cells is a body cell (eps_r != 1):
 *   between two body cells it carries a full rooftop (weight alpha = 1), on
 *   the body surface the inside half (alpha = 1/2).  Charge per cell
 *   rho = div w; E_sca = k0^2 A + grad phi, A = g * w, phi = g * rho,
 *   g = e^{i k0 r} / (4 pi r), collocated at face centres: midpoint weights
 *   h^3 alpha (rooftop) and h^3 (cell), the integral of g over the cube cell
 *   for a rooftop's and a cell's own term; grad phi = difference of the
 *   face's two cell potentials over h.  At an active face
 *       W - chi_f (k0^2 A_i + grad_i phi) = chi_f e_i(r_f),
 *   1/chi_f = the mean of 1/chi over the face's body sides.
 *   Far field (eq. 25, the normalisation above):
 *       F(r) = k0^2 h^3 / (4 pi) (I - r r) sum_faces alpha W_i e_i e^{-i k0 r . r_f}.
 * Vectors: [component 0..2][z][y][x] over the padded grid, 3 E1 E2 E3
 * vie_c64 each; entry c of component i is the face between padded cells c
 * and c + e_i (r_f = centre of c + (h/2) e_i).  Entries of inactive faces are
 * ignored on input (they do not couple) and passed through by the product
 * (y = x there); solutions are zero there.  Host arrays, caller-owned. */
typedef struct vie_rt vie_rt;

/* Build the operator of one body (n: 1..128 per axis, VIE_ENOTSUP above;
 * eps_r as vie_body) at wavenumber k0: face data, the spectrum of the scalar
 * kernel's circulant (length P >= 2 E - 1 per axis; kept on its octant,
 * (P1/2 + 1)(P2/2 + 1)(P3/2 + 1) complex doubles and an FP32 copy), transform
 * scratch (2 E3 P2 P1 + 2 E3 E2 P1 complex), fields and solver vectors
 * (36 E1 E2 E3 complex); setup needs two P1 P2 P3 complex arrays for the
 * duration of the call.  VIE_EINVAL on bad values. */
int vie_rt_setup(const vie_body *body, double k0, vie_rt **out);

/* Padded grid E[3] and circulant lengths P[3]; either may be NULL. */
int vie_rt_grid(const vie_rt *rt, int32_t *ext, int32_t *fft);

/* y = A x for nvec vectors (layout above).  precision VIE_FP64: FP64
 * transforms; VIE_MIXED: FP32 transforms and spectrum (gather, epilogue and
 * y in FP64). */
int vie_rt_matvec(vie_rt *rt, const vie_c64 *x, vie_c64 *y, int32_t nvec, int32_t precision);

/* Solve for nrhs plane-wave channels (b = chi_f e(r_f)) with BiCGSTAB from
 * w = 0 (scalars on the device, the host checking them every 8 iterations),
 * restarted from the FP64 true residual when the recursive one reaches its
 * target or the iteration breaks down (a zero denominator); the true residual
 * ||b - A w|| / ||b|| <= tol decides.  precision VIE_FP64: FP64 products;
 * VIE_MIXED: FP32 products inside FP64 iterative refinement, every cycle
 * reducing its starting residual by 1e-3 (or to tol), the vectors and dots
 * FP64.  w: nrhs vectors.  stats (nullable, one per channel): iters (all
 * cycles), matvecs, cycles, converged, rel_res; seconds = host wall time of
 * the channel's solve (0 if not converged).  VIE_ENOCONV if a channel missed
 * tol in max_iter iterations (its best iterate is still returned). */
int vie_rt_solve(vie_rt *rt, const vie_planewave *inc, int32_t nrhs, double tol,
                 int32_t max_iter, int32_t precision, vie_c64 *w, vie_stats *stats);

/* Far field of nrhs solutions w at ndir directions, laid out as vie_farfield:
 * F[(rhs * ndir + d) * 2 + {0,1}] = (F_theta, F_phi). */
int vie_rt_farfield(vie_rt *rt, const vie_c64 *w, int32_t nrhs, const double *theta,
                    const double *phi, int32_t ndir, vie_c64 *F);

void vie_rt_destroy(vie_rt *rt);

/* Classical comparison observable (eq. 27): for deterministic fields, the
 * product of the two detectors' intensities of the coherent superposition of
 * both channels' responses, P2 = |T_a1 + T_a2|^2 |T_b1 + T_b2|^2 (T ordered
 * as in hom_g2, unit channel amplitudes).  VIE_EINVAL for NULL or non-finite
 * input.  Host arrays. */
int hom_classical_p2(const vie_c64 T[4], double *p2);

/* Detector with a finite aperture (the aperture-collected field operator,
 * eq. NAfield).  Under the narrowband approximation of Sec. II the collected
 * field of channel j is a transfer coefficient like the point detector's
 * (eq. Eproj), averaged over the aperture:
 *   T_NA = (1 / Omega) * integral over the cone of p . F(r) dOmega(r),
 * with a uniform angular sensitivity W = 1 / Omega on the cone of half-angle
 * `alpha` (radians, 0 <= alpha <= pi; Omega = 2 pi (1 - cos alpha)) about the
 * axis direction (theta0, phi0), and a fixed detection polarisation `pol`
 * (complex Cartesian 3-vector, taken unconjugated like c_theta, c_phi of the
 * point detector).  F is the Cartesian far field of eq. 25.  alpha = 0 is the
 * point detector on the axis, with c_theta = pol . theta0-hat and
 * c_phi = pol . phi0-hat.  The g2 and coincidences of such detectors follow
 * from hom_g2 with these coefficients. */
typedef struct {
  double theta0, phi0; /* cone axis */
  double alpha;        /* cone half-angle; NA = sin(alpha) in vacuum */
  vie_c64 pol[3];      /* detection polarisation */
} vie_na_detector;

/* T[rhs * ndet + a] for every right-hand side of `body` and every detector
 * det[a].  Quadrature: n_rad Gauss-Legendre nodes in the cosine of the angle
 * from the axis on [cos alpha, 1] times n_az equally spaced azimuths (exact
 * for a single dipole with n_rad >= 2, n_az >= 3); the far field at all
 * nodes comes from the same MFMA projection as vie_farfield.  Host arrays.
 * VIE_EINVAL for non-finite input, alpha outside [0, pi], n_rad outside
 * [1, 256], n_az outside [1, 1024] or more than 2^22 nodes in all;
 * VIE_ESTATE before a solve. */
int vie_transfer_na(vie_ctx *ctx, int32_t body, const vie_na_detector *det, int32_t ndet,
                    int32_t n_rad, int32_t n_az, vie_c64 *T);

/* Copy the solution w = chi E of (body, rhs) to host memory w[3*N1*N2*N3]. */
int vie_get_current(vie_ctx *ctx, int32_t body, int32_t rhs, vie_c64 *w);

/* Apply the discrete operator y = x - chi Ghat x of `body` to nvec host
 * vectors x[nvec][3][N3][N2][N1] (precision VIE_FP64 or VIE_MIXED). */
int vie_matvec(vie_ctx *ctx, int32_t body, int32_t precision, const vie_c64 *x, vie_c64 *y,
               int32_t nvec);

/* Same on device buffers (asynchronous on the context's stream). */
int vie_matvec_dev(vie_ctx *ctx, int32_t body, int32_t precision, const void *x_dev,
                   void *y_dev, int32_t nvec);

/* Allocation-free variant of vie_matvec_dev, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, layout and result (the
 * same kernels; the z-pass launch shape is the one the context has tuned for
 * this grid, else the default).  The call allocates nothing, copies nothing
 * from host memory and records no memset: its scratch (FFT work arrays, a
 * table of nvec ints and, with the z window, two window copies of the
 * vectors) lives in a static device array of VIE_STATIC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends.  Bytes
 * needed, each term rounded up to 256, with c = 16 (VIE_FP64) or 8
 * (VIE_MIXED), window grid (N1, N2, N3) and FFT lengths (P1, P2, P3) as
 * reported by vie_grid, and n the window's voxel count:
 *   nvec * 3 * N3 * N2 * P1 * c  +  nvec * 3 * Z * P2 * P1 * c  +  4 nvec
 *   [+ 2 * nvec * 3 * n * 16 when the window is smaller than the grid],
 * Z = N3 rounded up to a multiple of min(16, N3).
 * VIE_ENOTSUP when that exceeds the limit (nothing is launched).  Every call
 * on one GPU, from any context or thread, shares that GPU's array: calls
 * whose work overlaps in time on one GPU (different streams, or different
 * host threads) race and give wrong results; calls on one stream are ordered
 * and safe.  Nothing in the array must start at zero (every element a call
 * reads, it has written first). */
#define VIE_STATIC_SCRATCH_BYTES 268435456
int vie_matvec_dev_static(vie_ctx *ctx, int32_t body, int32_t precision, const void *x_dev,
                          void *y_dev, int32_t nvec);

/* Use the given hipStream_t for all later device work (NULL: library's own). */
int vie_set_stream(vie_ctx *ctx, void *hip_stream);

/* Per-kernel-kind durations recorded with HIP events while VIE_FLAG_TIMING is
 * set: names[k] (static strings), total milliseconds ms[k] and launch counts
 * cnt[k] for k < *nkinds (in: capacity, out: number of kinds).  Kinds: the
 * five product passes per precision ("fft_x_fwd_f64" ... "fft_x_inv_f32"),
 * Krylov vector work, reductions, far field, setup, network; the same five
 * passes of the block solves of vie_solve_fgmres ("block_fft_..."), its
 * Arnoldi vector kernels ("arnoldi"), and the five packed-FP16 passes
 * ("fft_x_fwd_h16" ... "fft_x_inv_h16", and "block_fft_..._h16").  Call with
 * *nkinds = 0 to learn the number of kinds.  reset != 0 clears the
 * accumulators after reading. */
int vie_kernel_times(vie_ctx *ctx, const char **names, double *ms, int64_t *cnt,
                     int32_t *nkinds, int32_t reset);

/* Achievable HBM bandwidth of the current device (measurement aid): streaming
 * read, write and copy kernels over a buffer of `bytes` (1 MiB .. 64 GiB; the
 * copy uses two such buffers), each timed over `reps` launches after one
 * warm-up with HIP events on the null stream.  gbps[0] = read, gbps[1] =
 * write, gbps[2] = copy (read + write bytes), in 1e9 bytes/s.  Allocates and
 * frees its buffers; VIE_EINVAL for out-of-range sizes, VIE_ENOMEM when the
 * buffers do not fit. */
int vie_hbm_probe(int64_t bytes, int32_t reps, double *gbps);

/* Change option fields that do not affect setup (tol, max_iter, precision,
 * inner_tol, warm_start, flags).  k0 must match the setup value. */
int vie_set_options(vie_ctx *ctx, const vie_options *opt);

/* ------------------------------------------------------------------------
 * Learned warm start (a data-driven initial guess for the BiCGSTAB solve of
 * eq. 24; the paper's own acceleration is a block preconditioner, Sec. II-C).
 * A 4-layer 3x3x3 convolutional network (32 -> 32 -> 32 -> 32 -> 16 channels,
 * ReLU between layers, bf16 weights and activations, fp32 accumulation)
 * evaluated on each body's bounding box plus a 4-voxel halo, channels-last.
 * Input channels: chi/4, then the Krylov vectors b, A b, A^2 b, A^3 b (FP32
 * products), each divided by its own rms over the body voxels (re, im of x, y,
 * z, six channels per vector), zeros; b = chi e.  Outputs 0..5: the predicted
 * w/s (re, im of x, y, z), s = rms of |b| over the body voxels.  The solver
 * uses x0 = s * output only if ||b - A x0|| < ||b|| (FP64 operator), else
 * x0 = 0 (vie_stats.fallback).
 * Parameters (fp32, host): per layer W[27][Cout][Cin] (tap (dz+1)*9 +
 * (dy+1)*3 + (dx+1)) followed by b[Cout].  Device tensors: features
 * [d2][d1][d0][32] bf16, targets [d2][d1][d0][6] fp32, outputs
 * [d2][d1][d0][16] fp32 (dims = (d0, d1, d2)).  Loss: masked relative L2
 * sum_body |out - t|^2 / sum_body |t|^2 over outputs 0..5 (mask: chi > 0).
 * ------------------------------------------------------------------------ */
typedef struct vie_cnn vie_cnn;

/* Number of fp32 parameters of the network. */
int64_t vie_cnn_num_params(void);
/* Create a network with seeded He-normal weights on the current device. */
int vie_cnn_create(uint64_t seed, vie_cnn **out);
void vie_cnn_destroy(vie_cnn *net);
/* set != 0: load n = vie_cnn_num_params() host fp32 parameters (resets the
 * optimiser state); set == 0: read them back. */
int vie_cnn_params(vie_cnn *net, float *params, int64_t n, int32_t set);
/* Adam optimiser state for checkpoints: set == 0 reads the first and second
 * moments m, v (n = vie_cnn_num_params() host fp32 each, parameter order)
 * and the step count; set != 0 loads them (after vie_cnn_params, which
 * resets them), so that training resumes exactly where it was saved.
 * VIE_EINVAL for non-finite moments, v < 0 or step < 0. */
int vie_cnn_adam_state(vie_cnn *net, float *m, float *v, int64_t n, int64_t *step, int32_t set);
/* Use net for warm starts of ctx (vie_options.warm_start = 1); NULL detaches.
 * The network must outlive its use by ctx. */
int vie_attach_cnn(vie_ctx *ctx, vie_cnn *net);
/* Training sample of (body, rhs) from the last vie_solve: writes the box dims
 * to dims[3]; when feat / target are non-NULL, fills the device tensors with
 * the input features and the solution w/s (the target). */
int vie_cnn_sample_dev(vie_ctx *ctx, int32_t body, int32_t rhs, void *feat_dev,
                       void *target_dev, int32_t *dims);
/* Forward pass on device tensors (stream: hipStream_t or NULL). */
int vie_cnn_infer_dev(vie_cnn *net, const int32_t *dims, const void *feat_dev, void *out_dev,
                      void *stream);
/* Forward + backward: loss and the gradient of every parameter (host fp32
 * array of vie_cnn_num_params(); may be NULL); parameters unchanged. */
int vie_cnn_grad_dev(vie_cnn *net, const int32_t *dims, const void *feat_dev,
                     const void *target_dev, float *grad_host, float *loss, void *stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with learning rate lr. */
int vie_cnn_train_step_dev(vie_cnn *net, const int32_t *dims, const void *feat_dev,
                           const void *target_dev, float lr, float *loss, void *stream);

void vie_destroy(vie_ctx *ctx);
const char *vie_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* VIE_H */
