// Host runtime and C ABI (include/vie.h): contexts, spectrum setup, the
// BiCGSTAB / iterative-refinement driver, far field, two-photon observables.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/vie.h"
#include "cnn.h"
#include "gmres.h"
#include "green.h"
#include "kernels.h"
#include "trace.h"

using namespace vie;

namespace {

// ------------------------------------------------------------ device memory
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // grow-only; contents are not preserved
  hipError_t reserve(size_t b) {
    if (b <= bytes) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = b;
    return hipSuccess;
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

constexpr int kMaxNxy = 3072, kMaxNz = 256;  // voxels per axis (FFT lines 6144 / 512)

// Circulant length of an axis with n voxels: the smallest supported FFT
// length (2^k >= 8, or 3 * 2^k >= 12) that holds every displacement,
// P >= 2n - 1.
int fft_length(int n) {
  const int need = std::max(8, 2 * n - 1);
  int p2 = 8;
  while (p2 < need) p2 <<= 1;
  int p3 = 12;
  while (p3 < need) p3 <<= 1;
  return std::min(p2, p3);
}

struct BodyRec {
  int group;       // group index
  int slot;        // body index inside the group
  int nb;          // body voxels (chi != 0)
  int zoff = 0;    // first z layer of the body's grid inside the group's compute window
  double origin[3];  // centre of the compute window's voxel (0, 0, 0)
  int rhs0 = 0, nrhs = 0;  // right-hand sides of this body inside the group (last solve)
};

struct Group {
  GroupGeom g;     // compute grid: the bodies' grid cut to a window of z layers
  int N0[3];       // the bodies' grid as given
  int64_t n0;      // N0[0] N0[1] N0[2]
  double h;
  std::vector<int> bodies;       // body ids
  DevBuf chi;                    // double[nb][n]
  DevBuf spec64, spec32;         // octant spectra [Q2][Q3][Q1][6] (see k_octant)
  DevBuf tw64[3], tw32[3];       // twiddles per axis
  // body-compressed index data of every body of the group (see BodyIdx)
  DevBuf vox_all, chic_all, line_ptr_all, nb_arr, voff_arr;
  std::vector<int> vox_host, nb_host, voff_host;
  int max_nb = 0;
  // per-solve storage (capacity in right-hand sides / compressed elements)
  int cap = 0;
  int64_t vec_cap = 0;
  DevBuf roff;                   // int64 [cap] vector offset of each right-hand side
  std::vector<int64_t> roff_host;
  BodyIdx bi;
  DevBuf x, r, rh, p, v, s, t;   // c64, body-compressed, all right-hand sides
  DevBuf mask;                   // int [cap] scratch mask
  DevBuf knorm;                  // double [4][cap] norms of the network's Krylov inputs
  std::vector<double> knorm_host;
  // learned warm start: per body, network box = bounding box + 4-voxel halo
  std::vector<int> box_lo, box_d;        // [slot][3]
  std::vector<double> res_x0;            // per rhs: relative residual of the initial guess
  std::vector<int> fallback, warm_used;  // per rhs
  bool samples_ready = false;            // r = b and v = A b hold for every rhs
  DevBuf bufA, bufB;             // FFT scratch (sized for FP64)
  DevBuf boxX, boxY;             // compute-window copies of box-layout product vectors
  DevBuf partials;               // c64 [cap][maxblk][2]
  DevBuf state;                  // KState [cap]
  DevBuf flags;                  // int [2][cap]
  DevBuf rhs_body, pol, ph;      // per right-hand side
  DevBuf dirs, part, F, wd;      // far-field scratch
  // far-field voxel blocks per body (built on first use; the body never changes)
  struct Far {
    FarBlocks fb;
    DevBuf vi, org;
  };
  std::vector<std::unique_ptr<Far>> far;  // [slot]
  // captured BiCGSTAB iterations (replayed while every pointer and the shape
  // they were captured with are unchanged)
  struct IterGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> key;
    ~IterGraph() {
      if (exec) (void)hipGraphExecDestroy(exec);
    }
  } iter_graph;
  int zvar[2] = {-1, -1};        // autotuned z-pass shape per precision (-1: not yet)
  int zvar_nrhs[2] = {0, 0};     // right-hand-side count it was tuned for
  // packed-FP16 y and z passes of approximate FP32 products (block solves):
  // tables, spectrum scale gs, forward scales along x, y, z, scale back, on/off
  DevBuf spec16, tw16y, tw16z, gmax;
  float zh_gs = 0.f, hs[3] = {0.f, 0.f, 0.f}, hout = 0.f;
  int zh = 0;
};

struct TimedEvent {
  int kind;
  hipEvent_t a, b;
};

// Device storage of one batched Arnoldi process over nseg segments: basis V
// (m + 1 vectors), preconditioned vectors Z (flexible variant, m vectors),
// the work vector, both Gram-Schmidt passes of every Hessenberg column
// H[j][s][i] (i <= j; column j of all segments contiguous, so one plain copy
// brings it to the host) and the squared norms NR[s][j] (NR[s][0] = ||r||^2).
struct ArnoldiBufs {
  DevBuf V, Z, w, H1, H2, NR, dpart, npart, off, len, act, nvs, coef;
  DevBuf W2, act2;  // ||w||^2 before orthogonalisation, reorthogonalisation flags
  // least squares on the device (LsBufs) and the per-segment step counters
  DevBuf lsR, lscs, lssn, lsg, lsnst, mc, steps, cycles, anyf;
  int ls_m = 0;     // columns the least-squares buffers hold
  int v32 = 0;      // V and Z stored in FP32 (mixed precision) instead of FP64; 2: V in
                    // bfloat16 (block solves), w FP32
  // captured step chunks of the outer FGMRES (graph per first step, valid
  // while `key` matches every pointer and size the capture used)
  std::vector<hipGraphExec_t> chunk_exec;
  std::vector<const void*> chunk_key;
  ~ArnoldiBufs() { clear_graphs(); }
  void clear_graphs() {
    for (auto e : chunk_exec)
      if (e) (void)hipGraphExecDestroy(e);
    chunk_exec.clear();
  }
  // address of vector j of a multi-vector with `stride` elements per vector
  void* at(const DevBuf& b, int64_t j, int64_t stride) const {
    const size_t es = v32 == 2 ? sizeof(cb16) : v32 ? sizeof(c32) : sizeof(c64);
    return (char*)b.p + (size_t)j * stride * es;
  }
  LsBufs ls() const {
    LsBufs L;
    L.R = lsR.as<c64>();
    L.cs = lscs.as<double>();
    L.sn = lssn.as<c64>();
    L.g = lsg.as<c64>();
    L.nst = lsnst.as<int>();
    L.m = ls_m;
    L.ldr = ls_m + 1;
    return L;
  }
};

// Block-Jacobi preconditioner of one group: every body split into bx x by
// lateral blocks, each non-empty block one body of a sub-context on a common
// cropped grid, so that the block solves of all blocks, bodies and
// right-hand sides run as one batched product.
struct BlockPrec {
  int bx = 0, by = 0;
  vie_ctx* sub = nullptr;        // owned; its stream is set to the parent's per use
  int nsub = 0;                  // sub-context bodies (non-empty blocks of all bodies)
  std::vector<int> first_blk;    // [slot] first sub-context body of each body of the group
  std::vector<int> nblk_of;      // [slot] its non-empty blocks
  std::vector<int64_t> boff;     // [sub body] element offset in its body's permuted vector
  std::vector<int> blen;         // [sub body] elements (3 nb of the block)
  std::vector<int64_t> poff;     // [slot] offset of the body's permutation in perm
  DevBuf perm;                   // int, per body: permuted position -> body vector position
  // binding of the current right-hand sides
  std::vector<int> bound_rb;     // body slot of every right-hand side
  std::vector<int64_t> bound_roff;
  std::vector<int> seg_rhs;      // [segment] right-hand side
  DevBuf seg_rhs_dev, ones;      // device copy of seg_rhs; [rhs] all-active flags
  int nseg = 0, maxlen = 1, maxqlen = 1;
  int64_t tot = 0;               // elements of all right-hand sides' vectors
  DevBuf qoff, qpoff, qlen;      // [rhs] vector offset, permutation offset, elements
  ArnoldiBufs ab;
  DevBuf R;                      // permuted input
  ~BlockPrec() {
    if (sub) vie_destroy(sub);
  }
};

}  // namespace

// Timing kinds: the product passes, vector work and setup of the context's
// own groups (0..14), the product passes of the block solves run on a
// block-Jacobi sub-context (15..24, same order as 0..9), the Arnoldi
// vector kernels of FGMRES (25), and the packed-FP16 passes of approximate
// FP32 products (26..32 the context's own: the five passes in the order of
// 0..4, then the fused x-y forward and inverse passes; 33..39 the block
// solves').
static const char* kKindNames[] = {
    "fft_x_fwd_f64",       "fft_y_fwd_f64",       "fft_z_green_f64",       "fft_y_inv_f64",
    "fft_x_inv_f64",       "fft_x_fwd_f32",       "fft_y_fwd_f32",         "fft_z_green_f32",
    "fft_y_inv_f32",       "fft_x_inv_f32",       "krylov_vec",            "finalize",
    "farfield",            "init",                "cnn_forward",           "block_fft_x_fwd_f64",
    "block_fft_y_fwd_f64", "block_fft_z_green_f64", "block_fft_y_inv_f64", "block_fft_x_inv_f64",
    "block_fft_x_fwd_f32", "block_fft_y_fwd_f32", "block_fft_z_green_f32", "block_fft_y_inv_f32",
    "block_fft_x_inv_f32", "arnoldi",               "fft_x_fwd_h16",         "fft_y_fwd_h16",
    "fft_z_h16",           "fft_y_inv_h16",       "fft_x_inv_h16",         "fft_xy_fwd_h16",
    "fft_yx_inv_h16",      "block_fft_x_fwd_h16", "block_fft_y_fwd_h16",   "block_fft_z_h16",
    "block_fft_y_inv_h16", "block_fft_x_inv_h16", "block_fft_xy_fwd_h16",  "block_fft_yx_inv_h16"};
static constexpr int kNumKinds = 40;
static constexpr int kBlockKind0 = 15, kArnoldiKind = 25, kBlockH16Kind0 = 33;
static_assert(kH16Kind0 == 26, "timing kind table");

struct vie_cnn {
  vie::Cnn c;
};

struct vie_ctx {
  vie_options opt;
  int dev = 0;             // HIP device current at setup
  vie_cnn* cnn = nullptr;  // warm-start network (not owned)
  DevBuf feat;             // network input workspace (bf16)
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  bool poisoned = false;
  std::vector<std::unique_ptr<BodyRec>> bodies;
  std::vector<std::unique_ptr<Group>> groups;
  // timing
  std::vector<hipEvent_t> ev_pool;
  std::vector<TimedEvent> ev_live;
  double kind_ms[kNumKinds] = {0};
  int64_t kind_cnt[kNumKinds] = {0};
  // pinned flag mirrors for lagged convergence checks
  int* hflags[2] = {nullptr, nullptr};
  int hflags_cap = 0;
  hipEvent_t flag_ev[2] = {nullptr, nullptr};
  // flexible GMRES and its block-Jacobi preconditioner (built on first use)
  std::unique_ptr<ArnoldiBufs> fgm;
  std::vector<std::unique_ptr<BlockPrec>> bj;  // [group]
  // device wall clock: its rate, and the stamp taken at the start of a solve call
  double clock_khz = 0;
  DevBuf t_call;
};

// ------------------------------------------------ allocation-free scratch
// Scratch of vie_matvec_dev_static: a file-scope device array, one copy per
// GPU, that exists from the code object's load to the end of the process.
// Host code never passes `scratch` itself to a kernel (on the host it is a
// stand-in, not a device address): vie_setup looks up each device's address
// of it once, with that device current, and the entry point uses that.
static __device__ __align__(256) unsigned char scratch[VIE_STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];      // device address per device
static hipError_t g_scratch_err[kMaxDevices];  // result of the look-up
static bool g_scratch_done[kMaxDevices];

// Look up the current device's address of `scratch` (first call per device).
static hipError_t scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
    g_scratch_done[dev] = true;
  }
  return g_scratch_err[dev];
}

// --------------------------------------------------------------- utilities
#define VIE_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      if (getenv("VIE_LOG"))                                                          \
        fprintf(stderr, "vie: %s failed: %s (%s:%d)\n", #call, hipGetErrorString(e_), \
                __FILE__, __LINE__);                                                  \
      return e_ == hipErrorOutOfMemory ? VIE_ENOMEM : fail_device(ctx);               \
    }                                                                                 \
  } while (0)

static int fail_device(vie_ctx* ctx) {
  if (ctx) ctx->poisoned = true;
  return VIE_EDEVICE;
}

static hipEvent_t ev_get(vie_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static void timing_cb(int kind, bool begin, void* u) {
  vie_ctx* c = (vie_ctx*)u;
  if (begin) {
    TimedEvent t;
    t.kind = kind;
    t.a = ev_get(c);
    t.b = ev_get(c);
    if (!t.a || !t.b) return;
    (void)hipEventRecord(t.a, c->stream);
    c->ev_live.push_back(t);
  } else {
    if (c->ev_live.empty()) return;
    TimedEvent& t = c->ev_live.back();
    (void)hipEventRecord(t.b, c->stream);
  }
}

static bool timing_on(vie_ctx* c) { return (c->opt.flags & VIE_FLAG_TIMING) != 0; }

static void timing_collect(vie_ctx* c) {
  if (c->ev_live.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& t : c->ev_live) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      c->kind_ms[t.kind] += ms;
      c->kind_cnt[t.kind] += 1;
    }
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->ev_live.clear();
}

template <typename F>
static hipError_t timed(vie_ctx* c, int kind, F&& f) {
  if (timing_on(c)) timing_cb(kind, true, c);
  hipError_t e = f();
  if (timing_on(c)) timing_cb(kind, false, c);
  return e;
}

static void make_twiddles(int P, std::vector<c64>& t64, std::vector<c32>& t32) {
  t64.resize(P);
  t32.resize(P);
  for (int m = 0; m < P; ++m) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / P;
    t64[m] = mk((double)cosl(a), (double)sinl(a));
    t32[m] = mk((float)cosl(a), (float)sinl(a));
  }
}

static bool valid_options(const vie_options* o) {
  if (!o) return false;
  if (!(o->k0 > 0) || !isfinite(o->k0)) return false;
  if (o->precision != VIE_FP64 && o->precision != VIE_MIXED) return false;
  if (!(o->tol > 0) || !(o->tol < 1)) return false;
  if (o->max_iter < 1) return false;
  if (o->precision == VIE_MIXED && !(o->inner_tol > 0 && o->inner_tol < 1)) return false;
  return true;
}

// ------------------------------------------------------------------ setup
static int build_spectrum(vie_ctx* ctx, Group& G) {
  const GroupGeom& g = G.g;
  const size_t M = (size_t)g.P[0] * g.P[1] * g.P[2];
  const size_t oct = (size_t)g.Q[0] * g.Q[1] * g.Q[2];
  DevBuf work, tmp;
  VIE_HIP(work.reserve(M * sizeof(c64)));
  VIE_HIP(tmp.reserve(M * sizeof(c64)));
  VIE_HIP(G.spec64.reserve(6 * oct * sizeof(c64)));
  VIE_HIP(G.spec32.reserve(6 * oct * sizeof(c32)));
  const void* tw[3] = {G.tw64[0].p, G.tw64[1].p, G.tw64[2].p};
  for (int ab = 0; ab < 6; ++ab) {
    if (ctx->opt.flags & VIE_FLAG_CUBE_SELF) {
      double sr, si;
      self_term_cube(ctx->opt.k0, G.h, &sr, &si);
      VIE_HIP(launch_green_sample_self(work.as<c64>(), g, ab, G.h, ctx->opt.k0, sr, si,
                                       ctx->stream));
    } else {
      VIE_HIP(launch_green_sample(work.as<c64>(), g, ab, G.h, ctx->opt.k0, ctx->stream));
    }
    VIE_HIP(launch_fft3d_full(work.as<c64>(), tmp.as<c64>(), g, tw, ctx->stream));
    VIE_HIP(launch_octant(tmp.as<c64>(), G.spec64.as<c64>(), G.spec32.as<c32>(), g, ab,
                          ctx->stream));
  }
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  return VIE_OK;
}

extern "C" int vie_setup(const vie_body* bodies, int32_t n_bodies, const vie_options* opt,
                         vie_ctx** out) {
  TraceRange trace_("vie_setup");
  if (!out) return VIE_EINVAL;
  *out = nullptr;
  if (!bodies || n_bodies < 1 || !valid_options(opt)) return VIE_EINVAL;
  for (int b = 0; b < n_bodies; ++b) {
    const vie_body& B = bodies[b];
    if (!B.eps_r || !(B.h > 0) || !isfinite(B.h)) return VIE_EINVAL;
    for (int a = 0; a < 3; ++a) {
      if (B.n[a] < 1) return VIE_EINVAL;
      if (!isfinite(B.origin[a])) return VIE_EINVAL;
    }
    // x and y lines up to 6144 points (3072 voxels), z lines up to 512 (256)
    if (B.n[0] > kMaxNxy || B.n[1] > kMaxNxy || B.n[2] > kMaxNz) return VIE_ENOTSUP;
    const int64_t n = (int64_t)B.n[0] * B.n[1] * B.n[2];
    if (n >= ((int64_t)1 << 31)) return VIE_ENOTSUP;  // voxel indices are 32-bit
    for (int64_t i = 0; i < n; ++i)
      if (!(B.eps_r[i] >= 1.0) || !isfinite(B.eps_r[i])) return VIE_EINVAL;
  }
  vie_ctx* ctx = new (std::nothrow) vie_ctx();
  if (!ctx) return VIE_ENOMEM;
  ctx->opt = *opt;
  int rc = VIE_OK;
  auto bail = [&](int code) {
    vie_destroy(ctx);
    return code;
  };
  auto hip_fail = [&](hipError_t e, const char* what) {
    if (getenv("VIE_LOG"))
      fprintf(stderr, "vie: vie_setup: %s failed: %s\n", what, hipGetErrorString(e));
    return bail(e == hipErrorOutOfMemory ? VIE_ENOMEM : VIE_EDEVICE);
  };
  hipError_t he;
  if ((he = hipGetDevice(&ctx->dev)) != hipSuccess) return hip_fail(he, "hipGetDevice");
  if ((he = hipStreamCreate(&ctx->own_stream)) != hipSuccess) return hip_fail(he, "hipStreamCreate");
  ctx->stream = ctx->own_stream;
  {
    const hipError_t se = scratch_init(ctx->dev);
    if (se != hipSuccess) {
      if (getenv("VIE_LOG"))
        fprintf(stderr, "vie: hipGetSymbolAddress(scratch) failed on device %d: %s\n", ctx->dev,
                hipGetErrorString(se));
      return bail(VIE_EDEVICE);
    }
  }
  {  // device wall clock for the solves' completion times
    int khz = 0;
    if ((he = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->dev)) != hipSuccess)
      return hip_fail(he, "hipDeviceGetAttribute");
    ctx->clock_khz = khz;
    if ((he = ctx->t_call.reserve(sizeof(unsigned long long))) != hipSuccess)
      return hip_fail(he, "hipMalloc");
  }
  // Group bodies by (n, h).  With VIE_FLAG_Z_WINDOW a group computes on a
  // window of its grid in z: the layers that hold body voxels of any of its
  // bodies, clipped to the grid.
  // Voxels outside the window have chi = 0 in every body, so they neither act
  // on the body nor are acted on: the discrete system for the body's unknowns
  // is the same, on a shorter circulant.  Each body sits in the window at its
  // own offset zoff.  Without the flag the window is the whole grid.
  std::map<std::vector<int64_t>, int> key2g;
  std::vector<int> gi_of(n_bodies), zlo_of(n_bodies), zhi_of(n_bodies);
  for (int b = 0; b < n_bodies; ++b) {
    const vie_body& B = bodies[b];
    int64_t hb;
    memcpy(&hb, &B.h, sizeof(hb));
    std::vector<int64_t> key = {B.n[0], B.n[1], B.n[2], hb};
    auto it = key2g.find(key);
    if (it == key2g.end()) {
      gi_of[b] = (int)ctx->groups.size();
      key2g[key] = gi_of[b];
      auto G = std::make_unique<Group>();
      G->h = B.h;
      for (int a = 0; a < 3; ++a) G->N0[a] = B.n[a];
      G->n0 = (int64_t)B.n[0] * B.n[1] * B.n[2];
      G->g.nrhs = 0;
      ctx->groups.push_back(std::move(G));
    } else {
      gi_of[b] = it->second;
    }
    const int64_t plane = (int64_t)B.n[0] * B.n[1];
    int zmin = B.n[2], zmax = -1;
    for (int64_t i = 0; i < (int64_t)plane * B.n[2]; ++i)
      if (B.eps_r[i] != 1.0) {
        const int z = (int)(i / plane);
        zmin = std::min(zmin, z);
        zmax = std::max(zmax, z);
      }
    if (zmax < 0) zmin = zmax = 0;  // no body voxel: a one-layer window
    zlo_of[b] = zmin;
    zhi_of[b] = zmax + 1;
    if (!(opt->flags & VIE_FLAG_Z_WINDOW)) {
      zlo_of[b] = 0;
      zhi_of[b] = B.n[2];
    }
  }
  std::vector<int> win(ctx->groups.size(), 1);
  for (int b = 0; b < n_bodies; ++b)
    win[gi_of[b]] = std::max(win[gi_of[b]], zhi_of[b] - zlo_of[b]);
  for (size_t gi = 0; gi < ctx->groups.size(); ++gi) {
    Group& G = *ctx->groups[gi];
    G.g.N[0] = G.N0[0];
    G.g.N[1] = G.N0[1];
    G.g.N[2] = win[gi];
    for (int a = 0; a < 3; ++a) {
      G.g.P[a] = fft_length(G.g.N[a]);
      G.g.Q[a] = G.g.P[a] / 2 + 1;
    }
    G.g.n = (int64_t)G.g.N[0] * G.g.N[1] * G.g.N[2];
    // one component of the y/z scratch must be addressable with 32-bit offsets
    const int64_t zl = G.g.N[2] < 16 ? G.g.N[2] : 16;
    if (((G.g.N[2] + zl - 1) / zl) * zl * G.g.P[1] * G.g.P[0] >= ((int64_t)1 << 31)) {
      vie_destroy(ctx);
      return VIE_ENOTSUP;
    }
  }
  std::vector<std::vector<double>> chi_host(ctx->groups.size());
  for (int b = 0; b < n_bodies; ++b) {
    const vie_body& B = bodies[b];
    const int gi = gi_of[b];
    Group& G = *ctx->groups[gi];
    auto rec = std::make_unique<BodyRec>();
    rec->group = gi;
    rec->slot = (int)G.bodies.size();
    rec->zoff = std::max(0, std::min(zlo_of[b], G.N0[2] - G.g.N[2]));
    for (int a = 0; a < 3; ++a) rec->origin[a] = B.origin[a];
    rec->origin[2] += B.h * rec->zoff;
    G.bodies.push_back(b);
    std::vector<double>& ch = chi_host[gi];
    const int64_t n = G.g.n;
    const int64_t shift = (int64_t)G.g.N[0] * G.g.N[1] * rec->zoff;
    std::vector<int> vox;
    ch.resize((size_t)(rec->slot + 1) * n);
    for (int64_t i = 0; i < n; ++i) {
      const double c = B.eps_r[i + shift] - 1.0;
      ch[(size_t)rec->slot * n + i] = c;
      if (c != 0.0) vox.push_back((int)i);
    }
    rec->nb = (int)vox.size();
    G.voff_host.push_back((int)G.vox_host.size());
    G.nb_host.push_back(rec->nb);
    G.max_nb = std::max(G.max_nb, rec->nb);
    G.vox_host.insert(G.vox_host.end(), vox.begin(), vox.end());
    {  // network box: bounding box of the body voxels with a 4-voxel halo,
       // clipped to the body's grid (not the window: layers outside the window
       // hold no body voxel, so their features are zero as on the full grid)
      const int* N = G.g.N;
      const int off[3] = {0, 0, rec->zoff};
      int lo[3] = {N[0], N[1], N[2]}, hi[3] = {0, 0, 0};
      for (int v : vox) {
        const int c[3] = {v % N[0], (v / N[0]) % N[1], v / (N[0] * N[1])};
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::min(lo[a], c[a]);
          hi[a] = std::max(hi[a], c[a] + 1);
        }
      }
      for (int a = 0; a < 3; ++a) {
        if (vox.empty()) {
          lo[a] = 0;
          hi[a] = 1;
        }
        lo[a] = std::max(0, lo[a] + off[a] - 4) - off[a];
        hi[a] = std::min(G.N0[a], hi[a] + off[a] + 4) - off[a];
        G.box_lo.push_back(lo[a]);
        G.box_d.push_back(hi[a] - lo[a]);
      }
    }
    ctx->bodies.push_back(std::move(rec));
  }
  for (size_t gi = 0; gi < ctx->groups.size(); ++gi) {
    Group& G = *ctx->groups[gi];
    // compressed index data: line pointers and chi at body voxels
    const int nl = G.g.N[1] * G.g.N[2];
    const int nbod = (int)G.bodies.size();
    std::vector<int> lp((size_t)nbod * (nl + 1), 0);
    std::vector<double> chic(G.vox_host.size());
    for (int sl = 0; sl < nbod; ++sl) {
      const int* vx = G.vox_host.data() + G.voff_host[sl];
      int* L = lp.data() + (size_t)sl * (nl + 1);
      for (int k = 0; k < G.nb_host[sl]; ++k) {
        L[vx[k] / G.g.N[0] + 1] += 1;
        chic[G.voff_host[sl] + k] = chi_host[gi][(size_t)sl * G.g.n + vx[k]];
      }
      for (int z = 0; z < nl; ++z) L[z + 1] += L[z];
    }
    auto up = [&](DevBuf& d, const void* src, size_t bytes) {
      if (d.reserve(std::max<size_t>(bytes, 8)) != hipSuccess) return VIE_ENOMEM;
      hipError_t ue;
      if (bytes && (ue = hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice)) != hipSuccess) {
        if (getenv("VIE_LOG"))
          fprintf(stderr, "vie: vie_setup: hipMemcpy failed: %s\n", hipGetErrorString(ue));
        return VIE_EDEVICE;
      }
      return VIE_OK;
    };
    int urc;
    if ((urc = up(G.vox_all, G.vox_host.data(), G.vox_host.size() * sizeof(int))) != VIE_OK ||
        (urc = up(G.chic_all, chic.data(), chic.size() * sizeof(double))) != VIE_OK ||
        (urc = up(G.line_ptr_all, lp.data(), lp.size() * sizeof(int))) != VIE_OK ||
        (urc = up(G.nb_arr, G.nb_host.data(), G.nb_host.size() * sizeof(int))) != VIE_OK ||
        (urc = up(G.voff_arr, G.voff_host.data(), G.voff_host.size() * sizeof(int))) != VIE_OK)
      return bail(urc);
    if (G.chi.reserve(chi_host[gi].size() * sizeof(double)) != hipSuccess) return bail(VIE_ENOMEM);
    if ((he = hipMemcpy(G.chi.p, chi_host[gi].data(), chi_host[gi].size() * sizeof(double),
                        hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(he, "hipMemcpy");
    for (int a = 0; a < 3; ++a) {
      std::vector<c64> t64;
      std::vector<c32> t32;
      make_twiddles(G.g.P[a], t64, t32);
      if (G.tw64[a].reserve(t64.size() * sizeof(c64)) != hipSuccess ||
          G.tw32[a].reserve(t32.size() * sizeof(c32)) != hipSuccess)
        return bail(VIE_ENOMEM);
      if ((he = hipMemcpy(G.tw64[a].p, t64.data(), t64.size() * sizeof(c64),
                          hipMemcpyHostToDevice)) != hipSuccess ||
          (he = hipMemcpy(G.tw32[a].p, t32.data(), t32.size() * sizeof(c32),
                          hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(he, "hipMemcpy");
    }
    rc = build_spectrum(ctx, G);
    if (rc != VIE_OK) return bail(rc);
  }
  for (int k = 0; k < 2; ++k)
    if ((he = hipEventCreateWithFlags(&ctx->flag_ev[k], hipEventDisableTiming)) != hipSuccess)
      return hip_fail(he, "hipEventCreateWithFlags");
  *out = ctx;
  return VIE_OK;
}

extern "C" void vie_destroy(vie_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto& P : ctx->bj)
    if (P && P->sub) P->sub->stream = P->sub->own_stream;
  ctx->bj.clear();
  ctx->fgm.reset();
  ctx->groups.clear();
  ctx->bodies.clear();
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto& t : ctx->ev_live) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (int k = 0; k < 2; ++k) {
    if (ctx->hflags[k]) (void)hipHostFree(ctx->hflags[k]);
    if (ctx->flag_ev[k]) (void)hipEventDestroy(ctx->flag_ev[k]);
  }
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
  delete ctx;
}

extern "C" int vie_set_stream(vie_ctx* ctx, void* s) {
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  ctx->stream = s ? (hipStream_t)s : ctx->own_stream;
  return VIE_OK;
}

extern "C" int vie_set_options(vie_ctx* ctx, const vie_options* opt) {
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (!valid_options(opt) || opt->k0 != ctx->opt.k0) return VIE_EINVAL;
  if ((opt->flags ^ ctx->opt.flags) & (VIE_FLAG_CUBE_SELF | VIE_FLAG_Z_WINDOW))
    return VIE_EINVAL;  // fixed at setup
  ctx->opt = *opt;
  return VIE_OK;
}

// -------------------------------------------------------------- workspace
static int vec_blocks_group(const Group& G) { return vec_blocks_n(3 * (int64_t)G.max_nb); }

// Krylov vectors of all right-hand sides (body-compressed, vec_len elements).
static int ensure_vectors(vie_ctx* ctx, Group& G, int64_t vec_len) {
  if (vec_len <= G.vec_cap) return VIE_OK;
  DevBuf* vs[] = {&G.x, &G.r, &G.rh, &G.p, &G.v, &G.s, &G.t};
  for (DevBuf* b : vs) VIE_HIP(b->reserve((size_t)vec_len * sizeof(c64)));
  G.vec_cap = vec_len;
  return VIE_OK;
}

// Scratch and per-right-hand-side arrays for nrhs right-hand sides.
static int ensure_solve_storage(vie_ctx* ctx, Group& G, int nrhs) {
  if (nrhs <= G.cap) return VIE_OK;
  const size_t a = (size_t)3 * G.g.N[2] * G.g.N[1] * G.g.P[0] * sizeof(c64);
  const size_t bb = (size_t)bufB_elems(G.g) * sizeof(c64);
  VIE_HIP(G.bufA.reserve(a * nrhs));
  VIE_HIP(G.bufB.reserve(bb * nrhs));
  const int maxblk = std::max(std::max(part_blocks_xinv(G.g, 0), part_blocks_xinv(G.g, 1)),
                              vec_blocks_group(G));
  VIE_HIP(G.partials.reserve((size_t)nrhs * maxblk * 2 * sizeof(c64)));
  VIE_HIP(G.state.reserve((size_t)nrhs * sizeof(KState)));
  VIE_HIP(G.flags.reserve((size_t)3 * nrhs * sizeof(int)));  // active, not done, pending
  VIE_HIP(G.rhs_body.reserve((size_t)nrhs * sizeof(int)));
  VIE_HIP(G.pol.reserve((size_t)nrhs * 3 * sizeof(c64)));
  VIE_HIP(G.ph.reserve((size_t)nrhs * (G.g.N[0] + G.g.N[1] + G.g.N[2]) * sizeof(c64)));
  VIE_HIP(G.roff.reserve((size_t)nrhs * sizeof(int64_t)));
  VIE_HIP(G.mask.reserve((size_t)nrhs * sizeof(int)));
  VIE_HIP(G.knorm.reserve((size_t)4 * nrhs * sizeof(double)));
  G.cap = nrhs;
  return VIE_OK;
}

static int ensure_hflags(vie_ctx* ctx, int n) {
  if (n <= ctx->hflags_cap) return VIE_OK;
  for (int k = 0; k < 2; ++k) {
    if (ctx->hflags[k]) (void)hipHostFree(ctx->hflags[k]);
    ctx->hflags[k] = nullptr;
    VIE_HIP(hipHostMalloc((void**)&ctx->hflags[k], (size_t)n * sizeof(int)));
  }
  ctx->hflags_cap = n;
  return VIE_OK;
}

static MatvecArgs matvec_args(Group& G, int precision, const int* active) {
  MatvecArgs m;
  m.zvar = G.zvar[precision] < 0 ? 0 : G.zvar[precision];
  m.g = &G.g;
  m.chi = G.chi.as<double>();
  m.rhs_body = G.rhs_body.as<int>();
  m.spec = precision == 0 ? G.spec64.p : G.spec32.p;
  for (int a = 0; a < 3; ++a) m.tw[a] = precision == 0 ? G.tw64[a].p : G.tw32[a].p;
  if (precision == 1 && G.zh) {
    m.spec16 = G.spec16.p;
    m.tw16[0] = G.tw16y.p;
    m.tw16[1] = G.tw16z.p;
    for (int d = 0; d < 3; ++d) m.hs[d] = G.hs[d];
    m.hout = G.hout;
  }
  m.bufA = G.bufA.p;
  m.bufB = G.bufB.p;
  m.active = active;
  return m;
}

// Tuned z shapes kept across processes (VIE_TUNE_CACHE=<file>): one line
// per decision, "zshape P1 P2 P3 N1 N2 N3 precision nrhs variant", read once
// per process and path, appended to after every new tuning.
using TuneKey = std::array<int, 8>;
static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_tune;
static std::string g_tune_path;

static void tune_cache_load(const char* path) {
  if (g_tune_path == path) return;
  g_tune.clear();
  g_tune_path = path;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char tag[16];
  TuneKey k;
  int v;
  while (fscanf(f, "%15s %d %d %d %d %d %d %d %d %d", tag, &k[0], &k[1], &k[2], &k[3], &k[4],
                &k[5], &k[6], &k[7], &v) == 10)
    if (strcmp(tag, "zshape") == 0) g_tune[k] = v;
  fclose(f);
}

static void tune_cache_store(const char* path, const TuneKey& k, int v) {
  g_tune[k] = v;
  FILE* f = fopen(path, "a");
  if (!f) return;  // the cache is an optimisation: an unwritable file is ignored
  fprintf(f, "zshape %d %d %d %d %d %d %d %d %d\n", k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7],
          v);
  fclose(f);
}

// Autotuner: time every z-pass launch shape on this group's scratch with the
// current right-hand-side count and keep the fastest, by a clear margin.
// VIE_ZVAR=<k> forces shape k; VIE_DETERMINISTIC=1 fixes shape 0, so that
// results do not depend on timing (every reduction already has a fixed
// order); VIE_TUNE_CACHE=<file> reuses and records decisions.
static hipError_t tune_z(vie_ctx* ctx, Group& G, int precision) {
  if (G.zvar[precision] >= 0 && G.zvar_nrhs[precision] == G.g.nrhs) return hipSuccess;
  const char* force = getenv("VIE_ZVAR");
  const char* det = getenv("VIE_DETERMINISTIC");
  if (force || (det && atoi(det) != 0)) {
    G.zvar[precision] =
        force ? std::max(0, std::min(z_variants(precision) - 1, atoi(force))) : 0;
    G.zvar_nrhs[precision] = G.g.nrhs;
    return hipSuccess;
  }
  const char* cache = getenv("VIE_TUNE_CACHE");
  const TuneKey key = {G.g.P[0], G.g.P[1], G.g.P[2], G.g.N[0],
                       G.g.N[1], G.g.N[2], precision, G.g.nrhs};
  if (cache && *cache) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load(cache);
    auto it = g_tune.find(key);
    if (it != g_tune.end() && it->second >= 0 && it->second < z_variants(precision)) {
      G.zvar[precision] = it->second;
      G.zvar_nrhs[precision] = G.g.nrhs;
      return hipSuccess;
    }
  }
  hipError_t e = hipMemsetAsync(G.bufB.p, 0, G.bufB.bytes, ctx->stream);
  if (e != hipSuccess) return e;
  hipEvent_t a = nullptr, b = nullptr;
  if ((e = hipEventCreate(&a)) != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return e;
  }
  float best = 1e30f;
  int bestv = 0;
  for (int v = 0; v < z_variants(precision) && e == hipSuccess; ++v) {
    MatvecArgs m = matvec_args(G, precision, nullptr);
    m.zvar = v;
    e = launch_z_only(m, precision, ctx->stream);  // warm-up
    if (e != hipSuccess) break;
    (void)hipEventRecord(a, ctx->stream);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_z_only(m, precision, ctx->stream);
    (void)hipEventRecord(b, ctx->stream);
    if (e != hipSuccess) break;
    e = hipEventSynchronize(b);
    float ms = 0;
    // a later shape must beat the best so far by 3 % (timing noise would
    // otherwise flip between near-equal shapes from run to run)
    if (e == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess && ms < 0.97f * best) {
      best = ms;
      bestv = v;
    }
    if (getenv("VIE_LOG"))
      fprintf(stderr, "vie: tune z pass P=%dx%dx%d prec=%d nrhs=%d variant %d: %.4f ms\n",
              G.g.P[0], G.g.P[1], G.g.P[2], precision, G.g.nrhs, v, ms / 3);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e == hipSuccess) {
    G.zvar[precision] = bestv;
    G.zvar_nrhs[precision] = G.g.nrhs;
    if (cache && *cache) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      tune_cache_load(cache);
      tune_cache_store(cache, key, bestv);
    }
  }
  return e;
}

// x, y: c64 vectors, or c32 with io32 (FP32 product, compressed, plain).
static hipError_t run_matvec(vie_ctx* ctx, Group& G, int precision, const void* x, void* y,
                             EpiArgs& e, const int* active, bool compressed = true,
                             int io32 = 0) {
  hipError_t te = tune_z(ctx, G, precision);
  if (te != hipSuccess) return te;
  MatvecArgs m = matvec_args(G, precision, active);
  if (compressed) m.bi = &G.bi;
  m.io32 = io32;
  return launch_matvec(m, precision, x, y, e, ctx->stream, timing_on(ctx) ? timing_cb : nullptr,
                       ctx);
}

// Packed fused product of the block solves whose input is the FP32 work
// vector w normalised on the way in (MatvecArgs::npart): the normalised
// bfloat16 vector goes to vout, ||w||^2 of every right-hand side to
// nrm[q ldn], the product to y (FP32).
static hipError_t run_matvec_nrm(vie_ctx* ctx, Group& G, const void* w, void* y, void* vout,
                                 const double* npart, int nblk, double* nrm, int ldn,
                                 const int* active) {
  hipError_t te = tune_z(ctx, G, 1);
  if (te != hipSuccess) return te;
  MatvecArgs m = matvec_args(G, 1, active);
  m.bi = &G.bi;
  m.io32 = 2;
  m.npart = npart;
  m.nblk = nblk;
  m.nrm = nrm;
  m.ldn = ldn;
  m.vout = vout;
  EpiArgs e{EPI_PLAIN, nullptr, nullptr, 0, nullptr, nullptr};
  return launch_matvec(m, 1, w, y, e, ctx->stream, timing_on(ctx) ? timing_cb : nullptr, ctx);
}

// ------------------------------------------------------ learned warm start
// Krylov inputs of the network for every right-hand side, r holding b after
// the init kernel: v = A r, s = A v, t = A s (FP32 products), and the squared
// norm of each of r, v, s, t (host copy in knorm_host[k * nrhs + q]).
static int krylov_inputs(vie_ctx* ctx, Group& G) {
  const int nrhs = G.g.nrhs;
  c64* vec[4] = {G.r.as<c64>(), G.v.as<c64>(), G.s.as<c64>(), G.t.as<c64>()};
  for (int k = 0; k < 3; ++k) {
    EpiArgs e{EPI_PLAIN, nullptr, nullptr, 0, nullptr, nullptr};
    VIE_HIP(run_matvec(ctx, G, 1, vec[k], vec[k + 1], e, nullptr));
  }
  for (int k = 0; k < 4; ++k)
    VIE_HIP(launch_vec_norm2(nrhs, G.bi, vec[k], G.knorm.as<double>() + (size_t)k * nrhs,
                             ctx->stream));
  G.knorm_host.resize((size_t)4 * nrhs);
  VIE_HIP(hipMemcpyAsync(G.knorm_host.data(), G.knorm.p, G.knorm_host.size() * sizeof(double),
                         hipMemcpyDeviceToHost, ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  return VIE_OK;
}

static int ensure_feat(vie_ctx* ctx, size_t vox) {
  VIE_HIP(ctx->feat.reserve(vox * kCnnIn * sizeof(uint16_t)));
  return VIE_OK;
}

// Features of right-hand side q (body slot sl) into feat (bf16 [box][32]).
static int build_features(vie_ctx* ctx, Group& G, int q, int sl, void* feat) {
  const int* d = &G.box_d[3 * sl];
  const int* lo = &G.box_lo[3 * sl];
  const int nb = G.nb_host[sl];
  const int nrhs = G.g.nrhs;
  const c64* vec[4] = {G.r.as<c64>() + G.roff_host[q], G.v.as<c64>() + G.roff_host[q],
                       G.s.as<c64>() + G.roff_host[q], G.t.as<c64>() + G.roff_host[q]};
  double inv[4];
  for (int k = 0; k < 4; ++k) {
    const double n2 = G.knorm_host[(size_t)k * nrhs + q];
    inv[k] = nb > 0 && n2 > 0 ? 1.0 / sqrt(n2 / nb) : 0.0;
  }
  VIE_HIP(launch_cnn_features((bf16raw*)feat, d, lo, G.g.N, G.vox_all.as<int>() + G.voff_host[sl],
                              G.chic_all.as<double>() + G.voff_host[sl], nb, vec, inv,
                              ctx->stream));
  return VIE_OK;
}

static int predict_x0(vie_ctx* ctx, Group& G) {
  if (!ctx->cnn) return VIE_ESTATE;
  int rc = krylov_inputs(ctx, G);
  if (rc != VIE_OK) return rc;
  const int nrhs = G.g.nrhs;
  std::vector<KState> hs(nrhs);
  VIE_HIP(hipMemcpyAsync(hs.data(), G.state.p, nrhs * sizeof(KState), hipMemcpyDeviceToHost,
                         ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<int> slot_of(nrhs, 0);
  for (int b : G.bodies) {
    BodyRec& B = *ctx->bodies[b];
    for (int q = 0; q < B.nrhs; ++q) slot_of[B.rhs0 + q] = B.slot;
  }
  Cnn& net = ctx->cnn->c;
  for (int q = 0; q < nrhs; ++q) {
    const int sl = slot_of[q];
    const int* d = &G.box_d[3 * sl];
    const size_t nv = (size_t)d[0] * d[1] * d[2];
    if ((rc = ensure_feat(ctx, nv)) != VIE_OK) return rc;
    VIE_HIP(cnn_ensure_ws(net, nv));
    if ((rc = build_features(ctx, G, q, sl, ctx->feat.p)) != VIE_OK) return rc;
    VIE_HIP(timed(ctx, 14, [&] {
      return cnn_forward(net, d, (const bf16raw*)ctx->feat.p, net.out, ctx->stream);
    }));
    const int nb = G.nb_host[sl];
    const double s = nb > 0 && hs[q].bnorm2 > 0 ? sqrt(hs[q].bnorm2 / nb) : 0.0;
    VIE_HIP(launch_cnn_gather(G.x.as<c64>() + G.roff_host[q], net.out, d, &G.box_lo[3 * sl],
                              G.g.N, G.vox_all.as<int>() + G.voff_host[sl], nb, s, ctx->stream));
  }
  return VIE_OK;
}

// ---------------------------------------------------------------- solver
// Restarted BiCGSTAB with FP64 vectors.  Each cycle iterates on the current
// residual r with the FP64 (VIE_FP64) or FP32 (VIE_MIXED) product until the
// recursive residual drops below max((tol/2)^2 ||b||^2, eta^2 ||r_start||^2),
// then recomputes the true residual with the FP64 product and restarts.
// With VIE_MIXED this is FP64 iterative refinement around an FP32-product
// inner solver; with VIE_FP64 the restart only confirms convergence.
// Learned warm start after the zero-guess init (r = b, KState as after
// FIN_INIT): the network's guess x0 for every right-hand side, its true
// residual, and x0 = 0 again wherever ||b - A x0|| >= ||b||.  Leaves x, r, rhat
// and KState / flags as after a restart; records res_x0, fallback, warm_used.
static int warm_start_init(vie_ctx* ctx, Group& G, const FinParams& fp,
                           std::vector<int>& fallback_out) {
  const GroupGeom& g = G.g;
  const int nrhs = g.nrhs;
  KState* st = G.state.as<KState>();
  int* flags = G.flags.as<int>();
  int* active = flags;
  int* notdone = flags + nrhs;
  c64* part = G.partials.as<c64>();
  const int vb = vec_blocks_group(G);
  const BodyIdx& bi = G.bi;
  c64 *x = G.x.as<c64>(), *r = G.r.as<c64>(), *rh = G.rh.as<c64>();
  const c64* pol = G.pol.as<c64>();
  const c64* ph = G.ph.as<c64>();
  // network prediction x0 for every right-hand side (r = b after init)
  int rc0 = predict_x0(ctx, G);
  if (rc0 != VIE_OK) return rc0;
  // true residual of the initial guess; reject guesses with ||r0|| >= ||b||
  EpiArgs e{EPI_RESID, rh, part, 0, pol, ph};
  VIE_HIP(run_matvec(ctx, G, 0, x, r, e, notdone));
  VIE_HIP(timed(ctx, 11, [&] {
    return launch_finalize(FIN_RESTART, nrhs, e.part_blocks, part, st, flags, fp, ctx->stream);
  }));
  std::vector<KState> hs(nrhs);
  VIE_HIP(hipMemcpyAsync(hs.data(), st, nrhs * sizeof(KState), hipMemcpyDeviceToHost,
                         ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<int> mask(nrhs, 0);
  bool any = false;
  for (int i = 0; i < nrhs; ++i) {
    G.warm_used[i] = 1;
    G.res_x0[i] = hs[i].bnorm2 > 0 ? sqrt(hs[i].rnorm2 / hs[i].bnorm2) : 0.0;
    if (hs[i].bnorm2 > 0 && !(hs[i].rnorm2 < hs[i].bnorm2)) {
      mask[i] = 1;
      any = true;
      G.fallback[i] = 1;
      fallback_out[i] = 1;
    }
  }
  if (any) {
    // fall back to x0 = 0 for the rejected right-hand sides only
    int* dmask = G.mask.as<int>();
    VIE_HIP(hipMemcpyAsync(dmask, mask.data(), nrhs * sizeof(int), hipMemcpyHostToDevice,
                           ctx->stream));
    VIE_HIP(launch_init_zero_guess(g, bi, vb, pol, ph, x, r, rh, part, 0, dmask, ctx->stream));
    VIE_HIP(hipMemcpyAsync(notdone, mask.data(), nrhs * sizeof(int), hipMemcpyHostToDevice,
                           ctx->stream));
    VIE_HIP(launch_finalize(FIN_RESTART, nrhs, vb, part, st, flags, fp, ctx->stream));
    VIE_HIP(hipMemcpyAsync(hs.data(), st, nrhs * sizeof(KState), hipMemcpyDeviceToHost,
                           ctx->stream));
    VIE_HIP(hipStreamSynchronize(ctx->stream));
    std::vector<int> nd(nrhs), ac(nrhs);
    for (int i = 0; i < nrhs; ++i) {
      nd[i] = hs[i].notdone;
      ac[i] = hs[i].active;
    }
    VIE_HIP(hipMemcpyAsync(notdone, nd.data(), nrhs * sizeof(int), hipMemcpyHostToDevice,
                           ctx->stream));
    VIE_HIP(hipMemcpyAsync(active, ac.data(), nrhs * sizeof(int), hipMemcpyHostToDevice,
                           ctx->stream));
    VIE_HIP(hipStreamSynchronize(ctx->stream));  // nd, ac are about to go out of scope
  }
  return VIE_OK;
}

static int solve_group(vie_ctx* ctx, Group& G, bool warm, std::vector<int>& fallback_out) {
  TraceRange trace_("solve_group");
  const GroupGeom& g = G.g;
  const int nrhs = g.nrhs;
  const int prec = ctx->opt.precision == VIE_MIXED ? 1 : 0;
  FinParams fp;
  fp.tol2_done = ctx->opt.tol * ctx->opt.tol;
  fp.tol2_inner = 0.25 * fp.tol2_done;
  fp.eta2 = prec ? ctx->opt.inner_tol * ctx->opt.inner_tol : 0.0;
  fp.max_iter = ctx->opt.max_iter;
  KState* st = G.state.as<KState>();
  int* flags = G.flags.as<int>();
  int* active = flags;
  c64* part = G.partials.as<c64>();
  const int vb = vec_blocks_group(G);
  const BodyIdx& bi = G.bi;
  c64 *x = G.x.as<c64>(), *r = G.r.as<c64>(), *rh = G.rh.as<c64>(), *p = G.p.as<c64>(),
      *v = G.v.as<c64>(), *s = G.s.as<c64>(), *t = G.t.as<c64>();
  const c64* pol = G.pol.as<c64>();
  const c64* ph = G.ph.as<c64>();
  fallback_out.assign(nrhs, 0);

  VIE_HIP(timed(ctx, 13, [&] {
    return launch_init_zero_guess(g, bi, vb, pol, ph, x, r, rh, part, warm ? 1 : 0, nullptr,
                                  ctx->stream);
  }));
  VIE_HIP(timed(ctx, 11, [&] {
    return launch_finalize(FIN_INIT, nrhs, vb, part, st, flags, fp, ctx->stream);
  }));
  G.res_x0.assign(nrhs, 1.0);
  G.fallback.assign(nrhs, 0);
  G.warm_used.assign(nrhs, 0);
  if (warm) {
    int rcw = warm_start_init(ctx, G, fp, fallback_out);
    if (rcw != VIE_OK) return rcw;
  }
  int rc = ensure_hflags(ctx, 3 * nrhs);
  if (rc != VIE_OK) return rc;

  // one BiCGSTAB iteration for every active right-hand side
  auto iteration = [&]() -> hipError_t {
    hipError_t he;
    if ((he = timed(ctx, 10, [&] {
           return launch_update_p(g, bi, vb, st, active, r, p, v, ctx->stream);
         })) != hipSuccess)
      return he;
    EpiArgs e1{EPI_RHV, rh, part, 0, pol, ph};
    if ((he = run_matvec(ctx, G, prec, p, v, e1, active)) != hipSuccess) return he;
    if ((he = timed(ctx, 11, [&] {
           return launch_finalize(FIN_ALPHA, nrhs, e1.part_blocks, part, st, flags, fp,
                                  ctx->stream);
         })) != hipSuccess)
      return he;
    if ((he = timed(ctx, 10, [&] {
           return launch_update_s(g, bi, vb, st, active, r, v, s, ctx->stream);
         })) != hipSuccess)
      return he;
    EpiArgs e2{EPI_TS, nullptr, part, 0, pol, ph};
    if ((he = run_matvec(ctx, G, prec, s, t, e2, active)) != hipSuccess) return he;
    if ((he = timed(ctx, 11, [&] {
           return launch_finalize(FIN_OMEGA, nrhs, e2.part_blocks, part, st, flags, fp,
                                  ctx->stream);
         })) != hipSuccess)
      return he;
    if ((he = timed(ctx, 10, [&] {
           return launch_update_xr(g, bi, vb, st, active, x, r, p, s, t, rh, part, ctx->stream);
         })) != hipSuccess)
      return he;
    return timed(ctx, 11, [&] {
      return launch_finalize(FIN_RHO, nrhs, vb, part, st, flags, fp, ctx->stream);
    });
  };
  // Graph mode: capture VIE_GRAPH_ITERS iterations once and replay them.  Every
  // launch reads its scalars from device state and skips inactive right-hand
  // sides, so replaying past convergence changes nothing.  The capture holds
  // only kernel launches (the autotuner, which clears memory, runs first).
  const bool use_graph = !timing_on(ctx) && !(ctx->opt.flags & VIE_FLAG_NO_GRAPH);
  const int per_launch = use_graph ? VIE_GRAPH_ITERS : 1;
  if (use_graph) {
    VIE_HIP(tune_z(ctx, G, prec));
    std::vector<const void*> key = {x, r, rh, p, v, s, t, part, st, flags, pol, ph,
                                    G.bufA.p, G.bufB.p, G.roff.p, G.rhs_body.p,
                                    (const void*)ctx->stream,
                                    (const void*)(intptr_t)nrhs, (const void*)(intptr_t)prec,
                                    (const void*)(intptr_t)G.zvar[prec],
                                    (const void*)(intptr_t)fp.max_iter};
    double fpd[3] = {fp.tol2_done, fp.tol2_inner, fp.eta2};
    for (double d : fpd) {
      intptr_t bits = 0;
      memcpy(&bits, &d, sizeof(d) < sizeof(bits) ? sizeof(d) : sizeof(bits));
      key.push_back((const void*)bits);
    }
    if (!G.iter_graph.exec || G.iter_graph.key != key) {
      if (G.iter_graph.exec) (void)hipGraphExecDestroy(G.iter_graph.exec);
      G.iter_graph.exec = nullptr;
      hipGraph_t graph = nullptr;
      VIE_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      hipError_t ce = hipSuccess;
      for (int i = 0; i < VIE_GRAPH_ITERS && ce == hipSuccess; ++i) ce = iteration();
      hipError_t ee = hipStreamEndCapture(ctx->stream, &graph);
      if (ce == hipSuccess) ce = ee;
      if (ce == hipSuccess) ce = hipGraphInstantiate(&G.iter_graph.exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      VIE_HIP(ce);
      G.iter_graph.key = key;
    }
  }

  // Each right-hand side restarts on its own: when its cycle ends (the
  // recursive residual met the cycle target, or a breakdown) its pending flag
  // is set on the device, and the next check runs the FP64 true-residual
  // product and the restart for the pending right-hand sides only, while the
  // others keep iterating.  The host reads the flags one chunk late (the copy
  // after chunk k - 1 is read once chunk k is queued).  A restart queued
  // right after that copy covers every right-hand side pending in it (the
  // device gates the restart on its own pending flags, which only iterations
  // set), so a restart is queued only when the flags read are not already
  // covered by one.
  int* pending = flags + 2 * nrhs;
  bool restart_queued = false;  // a restart was queued right after the copy being read
  bool have_prev = false;       // a flag copy of the previous chunk is in flight
  int prev = 0;                 // its slot
  auto queue_restart = [&]() -> hipError_t {
    EpiArgs e{EPI_RESID, rh, part, 0, pol, ph};
    hipError_t he = run_matvec(ctx, G, 0, x, r, e, pending);
    if (he != hipSuccess) return he;
    return timed(ctx, 11, [&] {
      return launch_finalize(FIN_PENDING, nrhs, e.part_blocks, part, st, flags, fp, ctx->stream);
    });
  };
  for (int64_t k = 0;; ++k) {
    if (use_graph) {
      VIE_HIP(hipGraphLaunch(G.iter_graph.exec, ctx->stream));
    } else {
      VIE_HIP(iteration());
    }
    const int slot = (int)(k & 1);
    VIE_HIP(hipMemcpyAsync(ctx->hflags[slot], flags, 3 * nrhs * sizeof(int),
                           hipMemcpyDeviceToHost, ctx->stream));
    VIE_HIP(hipEventRecord(ctx->flag_ev[slot], ctx->stream));
    if (!have_prev) {
      have_prev = true;
      prev = slot;
      continue;
    }
    const int* hf = ctx->hflags[prev];
    VIE_HIP(hipEventSynchronize(ctx->flag_ev[prev]));
    prev = slot;
    bool any_active = false, any_pending = false;
    for (int i = 0; i < nrhs; ++i) {
      any_active |= hf[i] != 0;
      any_pending |= hf[2 * nrhs + i] != 0;
    }
    if (!any_active) {
      // nothing iterated in the chunk read (nor in the one queued after it,
      // unless a restart came between): restart what is pending and read the
      // flags after it directly, instead of replaying empty chunks meanwhile
      if (any_pending && !restart_queued) VIE_HIP(queue_restart());
      int* now = ctx->hflags[slot ^ 1];
      VIE_HIP(hipMemcpyAsync(now, flags, 3 * nrhs * sizeof(int), hipMemcpyDeviceToHost,
                             ctx->stream));
      VIE_HIP(hipStreamSynchronize(ctx->stream));
      bool act = false;
      for (int i = 0; i < nrhs; ++i) act |= now[i] != 0 || now[2 * nrhs + i] != 0;
      if (!act) break;  // all done (or out of steps)
      have_prev = false;  // the copy in flight predates the restart
      restart_queued = false;
    } else {
      const bool need = any_pending && !restart_queued;
      restart_queued = false;
      if (need) {
        VIE_HIP(queue_restart());
        restart_queued = true;
      }
    }
    if (k * per_launch > 4 * ((int64_t)ctx->opt.max_iter + 2)) break;
    if ((k & 63) == 63 && getenv("VIE_LOG")) {
      KState h0;
      VIE_HIP(hipMemcpyAsync(&h0, st, sizeof(KState), hipMemcpyDeviceToHost, ctx->stream));
      VIE_HIP(hipStreamSynchronize(ctx->stream));
      fprintf(stderr, "vie: %lld iterations launched, rhs 0: %d steps, %d restarts, rel res %.3e\n",
              (long long)((k + 1) * per_launch), h0.iters, h0.cycles,
              h0.bnorm2 > 0 ? sqrt(h0.rnorm2 / h0.bnorm2) : 0.0);
    }
  }
  return VIE_OK;
}

static void planewave_tables(const vie_planewave& pw, const Group& G, const double* origin,
                             double k0, c64* pol, c64* ph) {
  for (int c = 0; c < 3; ++c) pol[c] = mk(pw.pol[c].re, pw.pol[c].im);
  int off = 0;
  for (int a = 0; a < 3; ++a) {
    for (int i = 0; i < G.g.N[a]; ++i) {
      const double ang = k0 * pw.khat[a] * (origin[a] + G.h * i);
      ph[off + i] = mk(cos(ang), sin(ang));
    }
    off += G.g.N[a];
  }
}

// Check the incident channels of a solve; first[b] = index of body b's first
// channel in inc.
static int check_channels(vie_ctx* ctx, const vie_planewave* inc, const int32_t* nrhs_per_body,
                          std::vector<int>& first) {
  const int nb = (int)ctx->bodies.size();
  int total = 0;
  first.assign(nb, 0);
  for (int b = 0; b < nb; ++b) {
    if (nrhs_per_body[b] < 0) return VIE_EINVAL;
    first[b] = total;
    total += nrhs_per_body[b];
  }
  for (int i = 0; i < total; ++i) {
    const vie_planewave& w = inc[i];
    const double kn = sqrt(w.khat[0] * w.khat[0] + w.khat[1] * w.khat[1] + w.khat[2] * w.khat[2]);
    if (!(fabs(kn - 1.0) < 1e-9)) return VIE_EINVAL;
    for (int c = 0; c < 3; ++c)
      if (!isfinite(w.pol[c].re) || !isfinite(w.pol[c].im)) return VIE_EINVAL;
  }
  return VIE_OK;
}

// Bind the right-hand sides of one solve to group G: per-body ranges,
// storage, vector offsets, compressed-index pointers, plane-wave tables.
static int bind_rhs(vie_ctx* ctx, Group& G, const vie_planewave* inc,
                    const int32_t* nrhs_per_body, const std::vector<int>& first) {
  int nr = 0;
  for (int b : G.bodies) {
    BodyRec& B = *ctx->bodies[b];
    B.rhs0 = nr;
    B.nrhs = nrhs_per_body[b];
    nr += B.nrhs;
  }
  G.g.nrhs = nr;
  if (nr == 0) return VIE_OK;
  int rc = ensure_solve_storage(ctx, G, nr);
  if (rc != VIE_OK) return rc;
  G.roff_host.assign(nr, 0);
  int64_t vlen = 0;
  for (int b : G.bodies) {
    BodyRec& B = *ctx->bodies[b];
    for (int q = 0; q < B.nrhs; ++q) {
      G.roff_host[B.rhs0 + q] = vlen;
      vlen += 3 * (int64_t)B.nb;
    }
  }
  rc = ensure_vectors(ctx, G, std::max<int64_t>(vlen, 1));
  if (rc != VIE_OK) return rc;
  VIE_HIP(hipMemcpyAsync(G.roff.p, G.roff_host.data(), nr * sizeof(int64_t),
                         hipMemcpyHostToDevice, ctx->stream));
  G.bi.vox = G.vox_all.as<int>();
  G.bi.line_ptr = G.line_ptr_all.as<int>();
  G.bi.chic = G.chic_all.as<double>();
  G.bi.nb = G.nb_arr.as<int>();
  G.bi.voff = G.voff_arr.as<int>();
  G.bi.roff = G.roff.as<int64_t>();
  G.bi.rhs_body = G.rhs_body.as<int>();
  const int L = G.g.N[0] + G.g.N[1] + G.g.N[2];
  std::vector<int> rb(nr);
  std::vector<c64> pol((size_t)nr * 3), ph((size_t)nr * L);
  for (int b : G.bodies) {
    BodyRec& B = *ctx->bodies[b];
    for (int q = 0; q < B.nrhs; ++q) {
      const int gi = B.rhs0 + q;
      rb[gi] = B.slot;
      if (inc)
        planewave_tables(inc[first[b] + q], G, B.origin, ctx->opt.k0, &pol[(size_t)gi * 3],
                         &ph[(size_t)gi * L]);
    }
  }
  VIE_HIP(hipMemcpyAsync(G.rhs_body.p, rb.data(), nr * sizeof(int), hipMemcpyHostToDevice,
                         ctx->stream));
  VIE_HIP(hipMemcpyAsync(G.pol.p, pol.data(), pol.size() * sizeof(c64), hipMemcpyHostToDevice,
                         ctx->stream));
  VIE_HIP(hipMemcpyAsync(G.ph.p, ph.data(), ph.size() * sizeof(c64), hipMemcpyHostToDevice,
                         ctx->stream));
  // the host tables must outlive the copies
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  return VIE_OK;
}

// Seconds from the call's start stamp t0 to the residual check that found S
// converged, on the device wall clock (0 if not converged).
static double done_seconds(const vie_ctx* ctx, const KState& S, bool conv,
                           unsigned long long t0) {
  if (!conv || S.t_done < t0 || !(ctx->clock_khz > 0)) return 0.0;
  return (double)(S.t_done - t0) / (ctx->clock_khz * 1e3);
}

extern "C" int vie_solve(vie_ctx* ctx, const vie_planewave* inc, const int32_t* nrhs_per_body,
                         vie_stats* stats) {
  TraceRange trace_("vie_solve");
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (!inc || !nrhs_per_body) return VIE_EINVAL;
  std::vector<int> first;
  int rc = check_channels(ctx, inc, nrhs_per_body, first);
  if (rc != VIE_OK) return rc;
  if (ctx->opt.warm_start && !ctx->cnn) return VIE_EINVAL;  // warm start needs vie_attach_cnn
  VIE_HIP(launch_stamp(ctx->t_call.as<unsigned long long>(), ctx->stream));
  for (auto& Gp : ctx->groups) {
    Group& G = *Gp;
    rc = bind_rhs(ctx, G, inc, nrhs_per_body, first);
    if (rc != VIE_OK) return rc;
    if (G.g.nrhs == 0) continue;
    std::vector<int> fb;
    G.samples_ready = false;
    rc = solve_group(ctx, G, ctx->opt.warm_start != 0, fb);
    if (rc != VIE_OK) return rc;
  }
  // statistics
  bool all_conv = true;
  unsigned long long t0 = 0;
  VIE_HIP(hipMemcpyAsync(&t0, ctx->t_call.p, sizeof(t0), hipMemcpyDeviceToHost, ctx->stream));
  for (auto& Gp : ctx->groups) {
    Group& G = *Gp;
    if (G.g.nrhs == 0) continue;
    std::vector<KState> hs(G.g.nrhs);
    VIE_HIP(hipMemcpyAsync(hs.data(), G.state.p, hs.size() * sizeof(KState),
                           hipMemcpyDeviceToHost, ctx->stream));
    VIE_HIP(hipStreamSynchronize(ctx->stream));
    for (int b : G.bodies) {
      BodyRec& B = *ctx->bodies[b];
      for (int q = 0; q < B.nrhs; ++q) {
        const KState& S = hs[B.rhs0 + q];
        const double rel = S.bnorm2 > 0 ? sqrt(S.rnorm2 / S.bnorm2) : 0.0;
        const bool conv = !S.notdone;
        all_conv &= conv;
        if (stats) {
          vie_stats& o = stats[first[b] + q];
          o.iters = S.iters;
          o.matvecs = 2 * S.iters + S.cycles;
          o.cycles = S.cycles;
          o.converged = conv;
          o.fallback = G.fallback.empty() ? 0 : G.fallback[B.rhs0 + q];
          o.warm = G.warm_used.empty() ? 0 : G.warm_used[B.rhs0 + q];
          o.rel_res = rel;
          o.rel_res_x0 = G.res_x0.empty() ? 1.0 : G.res_x0[B.rhs0 + q];
          o.seconds = done_seconds(ctx, S, conv, t0);
        }
      }
    }
  }
  timing_collect(ctx);
  return all_conv ? VIE_OK : VIE_ENOCONV;
}

// ------------------------------------------------- flexible GMRES (FGMRES)
// Restarted FGMRES with right preconditioning (Saad 1993) and the block
// preconditioner of the paper's large metasurface solve (Sec. III-B, 7 x 7
// blocks), read as block Jacobi over a lateral partition with inexact block
// solves: k steps of GMRES from zero on every block.  The block solves of all
// blocks, bodies and right-hand sides of a group run as one batched product
// on a sub-context.

static bool valid_fgmres(const vie_fgmres_options* fo, const GroupGeom& g) {
  if (!fo) return false;
  if (fo->restart < 1 || fo->restart > 128) return false;
  if (fo->blocks[0] == 0 && fo->blocks[1] == 0) return true;
  for (int a = 0; a < 2; ++a)
    if (fo->blocks[a] < 1 || fo->blocks[a] > 64 || fo->blocks[a] > g.N[a]) return false;
  if (fo->inner_iters < 1 || fo->inner_iters > 64) return false;
  return fo->inner_precision == VIE_FP64 || fo->inner_precision == VIE_MIXED ||
         fo->inner_precision == VIE_MIXED_BF16;
}

// Storage of an Arnoldi process of m steps over nseg segments of at most
// maxlen elements, total elements per vector.
static int arnoldi_alloc(vie_ctx* ctx, ArnoldiBufs& A, int nseg, int maxlen, int64_t total, int m,
                         bool flexible) {
  const int nblk = seg_blocks(maxlen);
  const size_t vb = (size_t)std::max<int64_t>(total, 1) * sizeof(c64);
  VIE_HIP(A.V.reserve((size_t)(m + 1) * vb));
  if (flexible) VIE_HIP(A.Z.reserve((size_t)m * vb));
  VIE_HIP(A.w.reserve(vb));
  VIE_HIP(A.H1.reserve((size_t)nseg * m * (m + 1) * sizeof(c64)));
  VIE_HIP(A.H2.reserve((size_t)nseg * m * (m + 1) * sizeof(c64)));
  VIE_HIP(A.NR.reserve((size_t)nseg * (m + 1) * sizeof(double)));
  VIE_HIP(A.dpart.reserve((size_t)nseg * (m + 1) * nblk * sizeof(c64)));
  VIE_HIP(A.npart.reserve((size_t)nseg * nblk * sizeof(double)));
  VIE_HIP(A.off.reserve((size_t)nseg * sizeof(int64_t)));
  VIE_HIP(A.len.reserve((size_t)nseg * sizeof(int)));
  VIE_HIP(A.act.reserve((size_t)nseg * sizeof(int)));
  VIE_HIP(A.nvs.reserve((size_t)nseg * sizeof(int)));
  VIE_HIP(A.coef.reserve((size_t)nseg * (m + 1) * sizeof(c64)));
  VIE_HIP(A.W2.reserve((size_t)nseg * sizeof(double)));
  VIE_HIP(A.act2.reserve((size_t)nseg * sizeof(int)));
  VIE_HIP(A.lsR.reserve((size_t)nseg * m * (m + 1) * sizeof(c64)));
  VIE_HIP(A.lscs.reserve((size_t)nseg * m * sizeof(double)));
  VIE_HIP(A.lssn.reserve((size_t)nseg * m * sizeof(c64)));
  VIE_HIP(A.lsg.reserve((size_t)nseg * (m + 1) * sizeof(c64)));
  VIE_HIP(A.lsnst.reserve((size_t)nseg * sizeof(int)));
  VIE_HIP(A.mc.reserve((size_t)nseg * sizeof(int)));
  VIE_HIP(A.steps.reserve((size_t)nseg * sizeof(int)));
  VIE_HIP(A.cycles.reserve((size_t)nseg * sizeof(int)));
  VIE_HIP(A.anyf.reserve(sizeof(int)));
  A.ls_m = m;
  return VIE_OK;
}

static int arnoldi_tables(vie_ctx* ctx, ArnoldiBufs& A, const std::vector<int64_t>& off,
                          const std::vector<int>& len) {
  VIE_HIP(hipMemcpyAsync(A.off.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                         ctx->stream));
  VIE_HIP(hipMemcpyAsync(A.len.p, len.data(), len.size() * sizeof(int), hipMemcpyHostToDevice,
                         ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  return VIE_OK;
}

// Step j of the Arnoldi process after the caller has put the product into w:
// classical Gram-Schmidt against V_0..V_j (coefficients in H1), repeated
// (coefficients in H2, zero where skipped; only when eta2 > 0, otherwise H2 is
// neither written nor read) for the segments whose squared norm
// fell below eta2 times its value before the pass (eta2 = 1/2: the "twice is
// enough" criterion of Daniel, Gragg, Kaufman and Stewart 1976; eta2 = 0: one
// pass); ||w||^2 into NR[s][j+1], V_{j+1} = w / ||w||.
// nonorm (single pass, FP32 w): w_{j+1} is not normalised here; its norm
// partials stay for the next product, which normalises it on the way in, or
// for the last step (j = m - 1, whose vector is not needed) its norm is
// reduced into NR.
static hipError_t arnoldi_orth(vie_ctx* ctx, ArnoldiBufs& A, const SegSet& S, int64_t stride,
                               int m, int j, double eta2, bool nonorm = false) {
  const void* V = A.V.p;
  const int v32 = A.v32;       // basis storage (0 FP64, 1 FP32, 2 bfloat16)
  const int w32 = v32 ? 1 : 0;
  void* w = A.w.p;  // FP32 when the basis is not FP64 (the products then write FP32)
  const int ldh = m + 1;
  c64* h1 = A.H1.as<c64>() + (size_t)j * S.nseg * (m + 1);
  c64* h2 = A.H2.as<c64>() + (size_t)j * S.nseg * (m + 1);
  double* nr = A.NR.as<double>() + j + 1;
  double* npart = A.npart.as<double>();
  SegSet S2 = S;
  S2.active = A.act2.as<int>();
  hipError_t e;
  if (eta2 > 0 && (e = launch_seg_maxpy(S, nullptr, 0, 0, 0, nullptr, nullptr, 0, w, w32, npart,
                                         A.W2.as<double>(), 1, ctx->stream)) != hipSuccess)
    return e;
  if ((e = launch_seg_mdot(S, V, v32, stride, j + 1, w, w32, A.dpart.as<c64>(), h1, ldh,
                           ctx->stream)) != hipSuccess)
    return e;
  // one pass with an FP32 work vector: the normalisation reduces the norm
  const bool defer = eta2 <= 0 && w32;
  if (nonorm) {
    if (!defer) return hipErrorInvalidValue;
    return launch_seg_maxpy(S, V, v32, stride, j + 1, nullptr, h1, ldh, w, w32, npart, nr, m + 1,
                            ctx->stream, j + 1 < m);
  }
  if ((e = launch_seg_maxpy(S, V, v32, stride, j + 1, nullptr, h1, ldh, w, w32, npart, nr, m + 1,
                            ctx->stream, defer)) != hipSuccess)
    return e;
  if (defer)
    return launch_seg_normalize_sum(S, w, w32, npart, nr, m + 1, A.at(A.V, j + 1, stride), v32,
                                    ctx->stream);
  if (eta2 > 0) {  // otherwise there is no second pass (and H2 is not read)
    if ((e = launch_seg_reorth_flags(S, A.W2.as<double>(), nr, m + 1, eta2, A.act2.as<int>(),
                                     ctx->stream)) != hipSuccess)
      return e;
    if ((e = launch_seg_mdot(S2, V, v32, stride, j + 1, w, w32, A.dpart.as<c64>(), h2, ldh,
                             ctx->stream)) != hipSuccess)
      return e;
    if ((e = launch_seg_maxpy(S2, V, v32, stride, j + 1, nullptr, h2, ldh, w, w32, npart, nr, m + 1,
                              ctx->stream)) != hipSuccess)
      return e;
  }
  return launch_seg_normalize(S, w, w32, nr, m + 1, A.at(A.V, j + 1, stride), v32, ctx->stream);
}

// Block partition of every body of group G into bx x by lateral blocks:
// x part p covers voxels [floor(p N1 / bx), floor((p + 1) N1 / bx)), y alike,
// every block the full z extent.  Each non-empty block becomes one body of a
// sub-context: its voxels cropped to their own bounding box and placed at the
// origin of a common grid (the largest box extent per axis over all blocks);
// the other voxels of that grid have eps = 1.  Couplings depend on voxel
// offsets only, so the block's operator is exactly the full operator
// restricted to the block, and the crop keeps the ascending voxel order of
// the body's vector.
static int bj_build(vie_ctx* ctx, int gi, const vie_fgmres_options* fo) {
  const int bx = fo->blocks[0], by = fo->blocks[1];
  if ((int)ctx->bj.size() <= gi) ctx->bj.resize(gi + 1);
  std::unique_ptr<BlockPrec>& slotp = ctx->bj[gi];
  if (slotp && slotp->bx == bx && slotp->by == by) return VIE_OK;
  if (slotp && slotp->sub) slotp->sub->stream = slotp->sub->own_stream;
  slotp.reset();
  Group& G = *ctx->groups[gi];
  const int N1 = G.g.N[0], N2 = G.g.N[1];
  const int nbod = (int)G.bodies.size();
  std::vector<double> chic(G.vox_host.size());
  if (!chic.empty()) {
    VIE_HIP(hipMemcpyAsync(chic.data(), G.chic_all.p, chic.size() * sizeof(double),
                           hipMemcpyDeviceToHost, ctx->stream));
    VIE_HIP(hipStreamSynchronize(ctx->stream));
  }
  auto parts = [](int n, int np, std::vector<int>& of) {
    of.assign(n, 0);
    for (int p = 0; p < np; ++p) {
      const int lo = (int)((int64_t)p * n / np), hi = (int)((int64_t)(p + 1) * n / np);
      for (int i = lo; i < hi; ++i) of[i] = p;
    }
  };
  std::vector<int> px, py;
  parts(N1, bx, px);
  parts(N2, by, py);
  const size_t nbl = (size_t)bx * by;
  // members (indices into the body's voxel list) and bounding box of every block
  std::vector<std::vector<int>> members((size_t)nbod * nbl);
  std::vector<int> blo(members.size() * 3, INT32_MAX), bhi(members.size() * 3, -1);
  int ext[3] = {1, 1, 1};
  for (int sl = 0; sl < nbod; ++sl) {
    const int* vx = G.vox_host.data() + G.voff_host[sl];
    for (int k = 0; k < G.nb_host[sl]; ++k) {
      const int v = vx[k];
      const int c[3] = {v % N1, (v / N1) % N2, v / (N1 * N2)};
      const size_t id = (size_t)sl * nbl + px[c[0]] + (size_t)bx * py[c[1]];
      members[id].push_back(k);
      for (int a = 0; a < 3; ++a) {
        blo[id * 3 + a] = std::min(blo[id * 3 + a], c[a]);
        bhi[id * 3 + a] = std::max(bhi[id * 3 + a], c[a]);
      }
    }
  }
  for (size_t id = 0; id < members.size(); ++id)
    if (!members[id].empty())
      for (int a = 0; a < 3; ++a) ext[a] = std::max(ext[a], bhi[id * 3 + a] - blo[id * 3 + a] + 1);
  auto P = std::make_unique<BlockPrec>();
  P->bx = bx;
  P->by = by;
  std::vector<std::vector<double>> eps;
  std::vector<int> perm;
  for (int sl = 0; sl < nbod; ++sl) {
    const int nb = G.nb_host[sl];
    const int* vx = G.vox_host.data() + G.voff_host[sl];
    const double* ch = chic.data() + G.voff_host[sl];
    P->first_blk.push_back((int)eps.size());
    P->poff.push_back((int64_t)perm.size());
    perm.resize(perm.size() + 3 * (size_t)nb);
    int* pm = perm.data() + P->poff.back();
    int64_t acc = 0;
    for (size_t t = 0; t < nbl; ++t) {
      const size_t id = (size_t)sl * nbl + t;
      const std::vector<int>& mem = members[id];
      if (mem.empty()) continue;
      const int x0 = blo[id * 3], y0 = blo[id * 3 + 1], z0 = blo[id * 3 + 2];
      eps.emplace_back((size_t)ext[0] * ext[1] * ext[2], 1.0);
      std::vector<double>& e = eps.back();
      const int nbb = (int)mem.size();
      for (int u = 0; u < nbb; ++u) {
        const int v = vx[mem[u]];
        const int i = v % N1 - x0, j = (v / N1) % N2 - y0, kz = v / (N1 * N2) - z0;
        e[i + (size_t)ext[0] * (j + (size_t)ext[1] * kz)] = 1.0 + ch[mem[u]];
        for (int c = 0; c < 3; ++c) pm[acc + (int64_t)c * nbb + u] = c * nb + mem[u];
      }
      P->boff.push_back(acc);
      P->blen.push_back(3 * nbb);
      acc += 3 * nbb;
    }
    P->nblk_of.push_back((int)eps.size() - P->first_blk.back());
  }
  P->nsub = (int)eps.size();
  if (P->nsub > 0) {
    std::vector<vie_body> bodies(P->nsub);
    for (int b = 0; b < P->nsub; ++b) {
      for (int a = 0; a < 3; ++a) {
        bodies[b].n[a] = ext[a];
        bodies[b].origin[a] = 0.0;
      }
      bodies[b].h = G.h;
      bodies[b].eps_r = eps[b].data();
    }
    vie_options so = ctx->opt;
    so.precision = VIE_MIXED;
    so.inner_tol = 1e-3;
    so.warm_start = 0;
    so.flags = VIE_FLAG_NO_GRAPH | (ctx->opt.flags & VIE_FLAG_CUBE_SELF);  // same operator
    int rc = vie_setup(bodies.data(), P->nsub, &so, &P->sub);
    if (rc != VIE_OK) return rc;
    // the sub-context's compressed order must be the block order used above
    if (P->sub->groups.size() != 1) return VIE_EDEVICE;
    for (int b = 0; b < P->nsub; ++b)
      if (3 * P->sub->bodies[b]->nb != P->blen[b] || P->sub->bodies[b]->slot != b)
        return VIE_EDEVICE;
  }
  VIE_HIP(P->perm.reserve(std::max<size_t>(perm.size(), 1) * sizeof(int)));
  if (!perm.empty())
    VIE_HIP(hipMemcpy(P->perm.p, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice));
  slotp = std::move(P);
  return VIE_OK;
}

// Segment tables of the block solves for right-hand sides of body slots rb[q]
// at vector offsets roff[q]: one segment per (right-hand side, block of its
// body).
static int bj_bind(vie_ctx* ctx, Group& G, BlockPrec& P, const std::vector<int>& rb,
                   const std::vector<int64_t>& roff, int k) {
  if (P.nsub == 0) return VIE_OK;
  if (P.bound_rb == rb && P.bound_roff == roff) return VIE_OK;
  vie_ctx* sub = P.sub;
  sub->stream = ctx->stream;
  Group& Gp = *sub->groups[0];
  const int nrhs = (int)rb.size();
  std::vector<int64_t> off, qoff(nrhs), qpoff(nrhs);
  std::vector<int> len, srb, qlen(nrhs);
  P.seg_rhs.clear();
  P.maxlen = 1;
  P.maxqlen = 1;
  int64_t tot = 0;
  for (int q = 0; q < nrhs; ++q) {
    const int sl = rb[q];
    qoff[q] = roff[q];
    qpoff[q] = P.poff[sl];
    qlen[q] = 3 * G.nb_host[sl];
    P.maxqlen = std::max(P.maxqlen, qlen[q]);
    tot = std::max<int64_t>(tot, roff[q] + qlen[q]);
    for (int t = 0; t < P.nblk_of[sl]; ++t) {
      const int sb = P.first_blk[sl] + t;
      off.push_back(roff[q] + P.boff[sb]);
      len.push_back(P.blen[sb]);
      srb.push_back(sb);
      P.seg_rhs.push_back(q);
      P.maxlen = std::max(P.maxlen, P.blen[sb]);
    }
  }
  const int nseg = (int)off.size();
  P.nseg = nseg;
  P.tot = tot;
  if (nseg > 0) {
    Gp.g.nrhs = nseg;
    int rc = ensure_solve_storage(sub, Gp, nseg);
    if (rc != VIE_OK) return rc;
    Gp.roff_host = off;
    VIE_HIP(hipMemcpyAsync(Gp.roff.p, off.data(), nseg * sizeof(int64_t), hipMemcpyHostToDevice,
                           ctx->stream));
    VIE_HIP(hipMemcpyAsync(Gp.rhs_body.p, srb.data(), nseg * sizeof(int), hipMemcpyHostToDevice,
                           ctx->stream));
    Gp.bi.vox = Gp.vox_all.as<int>();
    Gp.bi.line_ptr = Gp.line_ptr_all.as<int>();
    Gp.bi.chic = Gp.chic_all.as<double>();
    Gp.bi.nb = Gp.nb_arr.as<int>();
    Gp.bi.voff = Gp.voff_arr.as<int>();
    Gp.bi.roff = Gp.roff.as<int64_t>();
    Gp.bi.rhs_body = Gp.rhs_body.as<int>();
    rc = arnoldi_alloc(ctx, P.ab, nseg, P.maxlen, tot, k, false);
    if (rc != VIE_OK) return rc;
    rc = arnoldi_tables(ctx, P.ab, off, len);
    if (rc != VIE_OK) return rc;
  }
  VIE_HIP(P.qoff.reserve(std::max(nrhs, 1) * sizeof(int64_t)));
  VIE_HIP(P.qpoff.reserve(std::max(nrhs, 1) * sizeof(int64_t)));
  VIE_HIP(P.qlen.reserve(std::max(nrhs, 1) * sizeof(int)));
  VIE_HIP(hipMemcpyAsync(P.qoff.p, qoff.data(), nrhs * sizeof(int64_t), hipMemcpyHostToDevice,
                         ctx->stream));
  VIE_HIP(hipMemcpyAsync(P.qpoff.p, qpoff.data(), nrhs * sizeof(int64_t), hipMemcpyHostToDevice,
                         ctx->stream));
  VIE_HIP(hipMemcpyAsync(P.qlen.p, qlen.data(), nrhs * sizeof(int), hipMemcpyHostToDevice,
                         ctx->stream));
  VIE_HIP(P.R.reserve((size_t)std::max<int64_t>(tot, 1) * sizeof(c64)));
  VIE_HIP(P.seg_rhs_dev.reserve((size_t)std::max(nseg, 1) * sizeof(int)));
  VIE_HIP(P.ones.reserve((size_t)std::max(nrhs, 1) * sizeof(int)));
  if (nseg > 0)
    VIE_HIP(hipMemcpyAsync(P.seg_rhs_dev.p, P.seg_rhs.data(), nseg * sizeof(int),
                           hipMemcpyHostToDevice, ctx->stream));
  VIE_HIP(launch_fill_int(P.ones.as<int>(), nrhs, 1, ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  P.bound_rb = rb;
  P.bound_roff = roff;
  return VIE_OK;
}

// z = M^{-1} v for the bound right-hand sides (v, z device vectors at the
// bound offsets) whose device flag act_rhs[q] is set; z of the others is left
// as it is.  Device work only (no host copy, no synchronisation, no memset),
// so a caller may capture it in a graph once the block storage is sized
// (bj_prepare).
static int bj_apply(vie_ctx* ctx, BlockPrec& P, const vie_fgmres_options* fo, const void* v,
                    void* z, int vz32, const int* act_rhs) {
  const int nrhs = (int)P.bound_rb.size();
  if (P.nseg == 0) return VIE_OK;  // no block holds a voxel: the callers never get here
  vie_ctx* sub = P.sub;
  sub->stream = ctx->stream;
  sub->opt.flags = (sub->opt.flags & ~VIE_FLAG_TIMING) | (ctx->opt.flags & VIE_FLAG_TIMING);
  Group& Gp = *sub->groups[0];
  ArnoldiBufs& A = P.ab;
  const int k = fo->inner_iters;
  const int ip = fo->inner_precision == VIE_FP64 ? 0 : 1;  // block product precision
  const int nseg = P.nseg;
  const int64_t tot = P.tot;
  if (A.ls_m < k) return VIE_ESTATE;  // bj_prepare sizes the storage first
  SegSet S{A.off.as<int64_t>(), A.len.as<int>(), A.act.as<int>(), nseg, seg_blocks(P.maxlen)};
  VIE_HIP(launch_seg_act_map(nseg, P.seg_rhs_dev.as<int>(), act_rhs, A.act.as<int>(),
                             ctx->stream));
  // with FP32 block products the block basis is stored in FP32, or in
  // bfloat16 for VIE_MIXED_BF16; the work vector is FP32 either way
  A.v32 = fo->inner_precision == VIE_MIXED_BF16 ? 2 : ip;
  c64* R = P.R.as<c64>();
  double* NR = A.NR.as<double>();
  const int ldn = k + 1;
  VIE_HIP(launch_permute(nrhs, P.qoff.as<int64_t>(), P.qpoff.as<int64_t>(), P.qlen.as<int>(),
                         P.maxqlen, P.perm.as<int>(), v, vz32, R, 0, 0, act_rhs, ctx->stream));
  VIE_HIP(launch_seg_maxpy(S, nullptr, 0, 0, 0, nullptr, nullptr, 0, R, 0, A.npart.as<double>(), NR,
                           ldn, ctx->stream));
  VIE_HIP(launch_seg_normalize(S, R, 0, NR, ldn, A.V.p, A.v32, ctx->stream));
  // the block solves are approximations: with FP32 block products one
  // Gram-Schmidt pass is enough
  const double eta2 = ip ? 0.0 : 0.5;
  // packed fused products normalise the basis vector on the way in: the
  // Gram-Schmidt step leaves w and its norm partials, the next product
  // stores V_j = w / ||w|| and multiplies it
  const bool nrm_in = A.v32 == 2 && Gp.zh && xy_fused_ok(Gp.g);
  for (int j = 0; j < k; ++j) {
    // with an FP32 basis the FP32 product reads V_j and writes w in FP32
    EpiArgs e{EPI_PLAIN, nullptr, nullptr, 0, nullptr, nullptr};
    if (j > 0 && nrm_in)
      VIE_HIP(run_matvec_nrm(sub, Gp, A.w.p, A.w.p, A.at(A.V, j, tot), A.npart.as<double>(),
                             S.nblk, NR + j, ldn, A.act.as<int>()));
    else
      VIE_HIP(run_matvec(sub, Gp, ip, A.at(A.V, j, tot), A.w.p, e, A.act.as<int>(), true, A.v32));
    VIE_HIP(timed(ctx, kArnoldiKind,
                  [&] { return arnoldi_orth(ctx, A, S, tot, k, j, eta2, nrm_in); }));
  }
  // least squares of every block solve on the device, then z = V y, written
  // straight into the right-hand sides' vector order (every segment of an
  // active right-hand side is active, and the blocks partition its body)
  VIE_HIP(launch_ls_full(nseg, k, A.H1.as<c64>(), A.H2.as<c64>(), eta2 > 0 ? 1 : 0, ldn, NR, ldn,
                         A.act.as<int>(), A.ls(), A.coef.as<c64>(), ldn, A.nvs.as<int>(),
                         ctx->stream));
  VIE_HIP(launch_seg_lincomb_perm(S, A.V.p, A.v32, tot, k, A.nvs.as<int>(), A.coef.as<c64>(), ldn,
                                  P.seg_rhs_dev.as<int>(), P.qoff.as<int64_t>(),
                                  P.qpoff.as<int64_t>(), P.perm.as<int>(), z, vz32, ctx->stream));
  return VIE_OK;
}

// Size the block solves' storage for k steps and tune the block products'
// z pass (both allocate or clear memory, so they run before any capture).
static int bj_prepare(vie_ctx* ctx, BlockPrec& P, const vie_fgmres_options* fo) {
  if (P.nseg == 0) return VIE_OK;
  int rc = arnoldi_alloc(ctx, P.ab, P.nseg, P.maxlen, P.tot, fo->inner_iters, false);
  if (rc != VIE_OK) return rc;
  vie_ctx* sub = P.sub;
  sub->stream = ctx->stream;
  Group& Gs = *sub->groups[0];
  VIE_HIP(tune_z(sub, Gs, fo->inner_precision == VIE_FP64 ? 0 : 1));
  // VIE_MIXED_BF16: the block products' y and z passes in packed FP16 where
  // the grid takes them.  Spectrum scale gs = 2^-ceil(log2 max|G|) (entries
  // within 1); forward scale along each axis the power of two h_d with
  // h_d^2 N_d <= 1, so that every forward value of a unit-norm basis vector
  // stays within 1 (Cauchy-Schwarz along each transformed line).
  Gs.zh = 0;
  if (fo->inner_precision == VIE_MIXED_BF16 && h16_ok(Gs.g)) {
    const GroupGeom& g = Gs.g;
    if (!(Gs.zh_gs > 0)) {
      VIE_HIP(Gs.gmax.reserve(sizeof(unsigned)));
      VIE_HIP(hipMemsetAsync(Gs.gmax.p, 0, sizeof(unsigned), ctx->stream));
      VIE_HIP(launch_spec_absmax(Gs.spec32.p, (int64_t)6 * g.Q[0] * g.Q[1] * g.Q[2],
                                 Gs.gmax.as<unsigned>(), ctx->stream));
      unsigned bits = 0;
      VIE_HIP(hipMemcpyAsync(&bits, Gs.gmax.p, sizeof(bits), hipMemcpyDeviceToHost, ctx->stream));
      VIE_HIP(hipStreamSynchronize(ctx->stream));
      float mx = 0.f;
      memcpy(&mx, &bits, sizeof(mx));
      if (mx > 0.f && std::isfinite(mx)) {
        const float gs = exp2f(-ceilf(log2f(mx)));
        VIE_HIP(Gs.spec16.reserve((size_t)6 * g.Q[1] * g.Q[2] * (g.P[0] / 2) * 8));
        VIE_HIP(launch_spec_pairs(Gs.spec32.p, Gs.spec16.p, g, gs, ctx->stream));
        VIE_HIP(Gs.tw16y.reserve((size_t)g.P[1] * 8));
        VIE_HIP(launch_tw_h2(Gs.tw32[1].p, Gs.tw16y.p, g.P[1], ctx->stream));
        VIE_HIP(Gs.tw16z.reserve((size_t)g.P[2] * 8));
        VIE_HIP(launch_tw_h2(Gs.tw32[2].p, Gs.tw16z.p, g.P[2], ctx->stream));
        Gs.zh_gs = gs;
      }
    }
    if (Gs.zh_gs > 0) {
      float prod = Gs.zh_gs;
      for (int d = 0; d < 3; ++d) {
        int e = 0;
        while (((int64_t)1 << (2 * e)) < Gs.g.N[d]) ++e;
        Gs.hs[d] = ldexpf(1.f, -e);
        prod *= Gs.hs[d];
      }
      Gs.hout = 1.f / prod;  // a power of two: exact
      Gs.zh = 1;
    }
  }
  return VIE_OK;
}

// Pointers and sizes the captured FGMRES step chunks depend on.
static void key_bufs(std::vector<const void*>& k, std::initializer_list<const DevBuf*> bs) {
  for (const DevBuf* b : bs) {
    k.push_back(b->p);
    k.push_back((const void*)(uintptr_t)b->bytes);
  }
}
static void key_group(std::vector<const void*>& k, const Group& G) {
  key_bufs(k, {&G.chi, &G.spec64, &G.spec32, &G.tw64[0], &G.tw64[1], &G.tw64[2], &G.tw32[0],
               &G.tw32[1], &G.tw32[2], &G.vox_all, &G.chic_all, &G.line_ptr_all, &G.nb_arr,
               &G.voff_arr, &G.roff, &G.x, &G.r, &G.rh, &G.state, &G.flags, &G.bufA, &G.bufB,
               &G.rhs_body, &G.partials});
  const int ints[] = {G.g.nrhs, G.zvar[0], G.zvar[1], G.g.N[0], G.g.N[1], G.g.N[2], G.g.P[0],
                      G.g.P[1], G.g.P[2], G.zh};
  for (int v : ints) k.push_back((const void*)(intptr_t)v);
  key_bufs(k, {&G.spec16, &G.tw16y, &G.tw16z});
  for (float f : {G.hs[0], G.hs[1], G.hs[2], G.hout}) {
    uint32_t b = 0;
    memcpy(&b, &f, sizeof(b));
    k.push_back((const void*)(uintptr_t)b);
  }
}
static void key_arnoldi(std::vector<const void*>& k, const ArnoldiBufs& A) {
  key_bufs(k, {&A.V, &A.Z, &A.w, &A.H1, &A.H2, &A.NR, &A.dpart, &A.npart, &A.off, &A.len, &A.act,
               &A.nvs, &A.coef, &A.W2, &A.act2, &A.lsR, &A.lscs, &A.lssn, &A.lsg,
               &A.lsnst, &A.mc, &A.steps, &A.cycles, &A.anyf});
  k.push_back((const void*)(intptr_t)A.ls_m);
  k.push_back((const void*)(intptr_t)A.v32);
}

// Restarted FGMRES on every right-hand side of group G (bound by bind_rhs),
// from w = 0 or the learned warm start.  Arnoldi products in the context's
// precision; every cycle ends with the FP64 true residual, which alone
// decides convergence.  A right-hand side leaves a cycle early once its
// residual estimate is below tol / 2.
//
// The whole cycle runs on the device: the Givens rotations and the small
// triangular solves of the outer process and of every block solve are device
// kernels, and each right-hand side's activity is a device flag that every
// kernel reads.  The host launches the steps in chunks of kChunk (replayed
// from a captured graph unless VIE_FLAG_TIMING or VIE_FLAG_NO_GRAPH is set)
// and stops launching once the flag copied after the previous chunk says that
// no right-hand side is active (a lagged check: the GPU never waits for the
// host inside a cycle).  The host waits once per cycle, for the convergence
// flag after the FP64 residual.
static int fgmres_group(vie_ctx* ctx, Group& G, BlockPrec* P, const vie_fgmres_options* fo,
                        bool warm, std::vector<int>& steps_out, std::vector<int>& cycles_out) {
  TraceRange trace_("fgmres_group");
  const int nrhs = G.g.nrhs;
  const int m = fo->restart;
  const bool flex = P != nullptr;
  const int prec = ctx->opt.precision == VIE_MIXED ? 1 : 0;
  std::vector<int> len(nrhs);
  int maxlen = 1;
  int64_t tot = 0;
  for (int b : G.bodies) {
    const BodyRec& B = *ctx->bodies[b];
    for (int q = 0; q < B.nrhs; ++q) {
      len[B.rhs0 + q] = 3 * B.nb;
      tot = std::max<int64_t>(tot, G.roff_host[B.rhs0 + q] + 3 * (int64_t)B.nb);
    }
    maxlen = std::max(maxlen, 3 * B.nb);
  }
  if (!ctx->fgm) ctx->fgm = std::make_unique<ArnoldiBufs>();
  ArnoldiBufs& A = *ctx->fgm;
  int rc = arnoldi_alloc(ctx, A, nrhs, maxlen, tot, m, flex);
  if (rc != VIE_OK) return rc;
  rc = arnoldi_tables(ctx, A, G.roff_host, len);
  if (rc != VIE_OK) return rc;
  const SegSet S{A.off.as<int64_t>(), A.len.as<int>(), A.act.as<int>(), nrhs, seg_blocks(maxlen)};
  FinParams fp;
  fp.tol2_done = ctx->opt.tol * ctx->opt.tol;
  fp.tol2_inner = fp.tol2_done;
  fp.eta2 = 0.0;
  fp.max_iter = ctx->opt.max_iter;
  KState* st = G.state.as<KState>();
  int* flags = G.flags.as<int>();
  int* notdone = flags + nrhs;
  c64* part = G.partials.as<c64>();
  c64 *x = G.x.as<c64>(), *r = G.r.as<c64>(), *rh = G.rh.as<c64>();
  const c64* pol = G.pol.as<c64>();
  const c64* ph = G.ph.as<c64>();
  const int vb = vec_blocks_group(G);
  VIE_HIP(launch_init_zero_guess(G.g, G.bi, vb, pol, ph, x, r, rh, part, 0, nullptr, ctx->stream));
  VIE_HIP(launch_finalize(FIN_INIT, nrhs, vb, part, st, flags, fp, ctx->stream));
  if (warm) {
    std::vector<int> fb(nrhs, 0);
    rc = warm_start_init(ctx, G, fp, fb);
    if (rc != VIE_OK) return rc;
  }
  int* steps = A.steps.as<int>();
  int* cycles = A.cycles.as<int>();
  int* mc = A.mc.as<int>();
  int* anyf = A.anyf.as<int>();
  VIE_HIP(launch_fill_int(steps, nrhs, 0, ctx->stream));
  VIE_HIP(launch_fill_int(cycles, nrhs, 0, ctx->stream));
  // everything that allocates or clears memory happens before any capture
  if (flex) {
    rc = bj_prepare(ctx, *P, fo);
    if (rc != VIE_OK) return rc;
  }
  VIE_HIP(tune_z(ctx, G, prec));
  VIE_HIP(tune_z(ctx, G, 0));
  rc = ensure_hflags(ctx, std::max(nrhs, 1));
  if (rc != VIE_OK) return rc;
  const int maxit = ctx->opt.max_iter;
  // mixed precision: the basis V and the preconditioned vectors Z are stored in
  // FP32 (their products are FP32 anyway); dots, updates and x stay FP64
  A.v32 = prec;
  const DevBuf& Zb = flex ? A.Z : A.V;
  double* NR = A.NR.as<double>();
  // FP32 Arnoldi products perturb the Arnoldi relation at about 1e-7, so in the
  // mixed path one Gram-Schmidt pass is enough; the FP64 true residual at the
  // end of every cycle decides convergence either way
  const double eta2 = prec ? 0.0 : 0.5;
  const LsBufs L = A.ls();
  const double half_tol = 0.5 * ctx->opt.tol;
  const bool use_graph = !timing_on(ctx) && !(ctx->opt.flags & VIE_FLAG_NO_GRAPH);
  constexpr int kChunk = 4;

  // Arnoldi step j: z_j = M^{-1} v_j, w = A z_j, Gram-Schmidt, least squares
  auto step = [&](int j) -> int {
    void* vj = A.at(A.V, j, tot);
    void* zj = A.at(Zb, j, tot);
    if (flex) {
      const int r2 = bj_apply(ctx, *P, fo, vj, zj, A.v32, A.act.as<int>());
      if (r2 != VIE_OK) return r2;
    }
    // mixed: the FP32 product reads z_j and writes w in FP32
    EpiArgs e{EPI_PLAIN, nullptr, nullptr, 0, nullptr, nullptr};
    VIE_HIP(run_matvec(ctx, G, prec, zj, A.w.p, e, A.act.as<int>(), true, A.v32));
    VIE_HIP(timed(ctx, kArnoldiKind, [&] { return arnoldi_orth(ctx, A, S, tot, m, j, eta2); }));
    VIE_HIP(launch_ls_step(nrhs, j, A.H1.as<c64>(), A.H2.as<c64>(), eta2 > 0 ? 1 : 0, m + 1, NR,
                           m + 1, st, half_tol, A.act.as<int>(), steps, mc, L, anyf,
                           ctx->stream));
    return VIE_OK;
  };
  std::vector<const void*> key;
  if (use_graph) {
    key_group(key, G);
    key_arnoldi(key, A);
    if (flex) {
      key_group(key, *P->sub->groups[0]);
      key_arnoldi(key, P->ab);
      key_bufs(key, {&P->R, &P->perm, &P->qoff, &P->qpoff, &P->qlen, &P->seg_rhs_dev});
      const int64_t pv[] = {P->nseg, P->tot, P->maxlen, P->maxqlen, (int64_t)P->bound_rb.size(),
                            fo->inner_iters, fo->inner_precision};
      for (int64_t v : pv) key.push_back((const void*)(intptr_t)v);
    }
    const int64_t cv[] = {nrhs, m, prec, flex ? 1 : 0, tot, maxlen};
    for (int64_t v : cv) key.push_back((const void*)(intptr_t)v);
    int64_t tb = 0;
    memcpy(&tb, &half_tol, sizeof(tb));
    key.push_back((const void*)(intptr_t)tb);
    key.push_back((const void*)ctx->stream);
    if (A.chunk_key != key) {
      A.clear_graphs();
      A.chunk_key = key;
    }
  }
  // steps j0 .. j0 + jn - 1: eager, or one replay of the chunk's graph
  auto run_chunk = [&](int j0, int jn) -> int {
    if (!use_graph) {
      for (int j = j0; j < j0 + jn; ++j) {
        const int r2 = step(j);
        if (r2 != VIE_OK) return r2;
      }
      return VIE_OK;
    }
    const size_t idx = (size_t)(j0 / kChunk);
    if (A.chunk_exec.size() <= idx) A.chunk_exec.resize(idx + 1, nullptr);
    if (!A.chunk_exec[idx]) {
      hipGraph_t graph = nullptr;
      VIE_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      int r2 = VIE_OK;
      for (int j = j0; j < j0 + jn && r2 == VIE_OK; ++j) r2 = step(j);
      const hipError_t ee = hipStreamEndCapture(ctx->stream, &graph);
      if (r2 != VIE_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r2;
      }
      VIE_HIP(ee);
      hipGraphExec_t ex = nullptr;
      const hipError_t ie = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      VIE_HIP(ie);
      A.chunk_exec[idx] = ex;
    }
    VIE_HIP(hipGraphLaunch(A.chunk_exec[idx], ctx->stream));
    return VIE_OK;
  };
  for (int cycle = 0;; ++cycle) {
    // one host wait per cycle: is any right-hand side left to iterate?
    VIE_HIP(launch_any_notdone(nrhs, st, steps, maxit, anyf, ctx->stream));
    VIE_HIP(hipMemcpyAsync(ctx->hflags[0], anyf, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    VIE_HIP(hipStreamSynchronize(ctx->stream));
    if (!ctx->hflags[0][0] || cycle > maxit) break;
    VIE_HIP(launch_ls_cycle_init(nrhs, maxit, st, A.act.as<int>(), steps, mc, cycles, L,
                                 ctx->stream));
    VIE_HIP(launch_seg_maxpy(S, nullptr, 0, 0, 0, nullptr, nullptr, 0, r, 0, A.npart.as<double>(), NR,
                             m + 1, ctx->stream));
    VIE_HIP(launch_seg_normalize(S, r, 0, NR, m + 1, A.V.p, A.v32, ctx->stream));
    for (int j0 = 0, c = 0; j0 < m; j0 += kChunk, ++c) {
      rc = run_chunk(j0, std::min(kChunk, m - j0));
      if (rc != VIE_OK) return rc;
      const int slot = c & 1;
      VIE_HIP(hipMemcpyAsync(ctx->hflags[slot], anyf, sizeof(int), hipMemcpyDeviceToHost,
                             ctx->stream));
      VIE_HIP(hipEventRecord(ctx->flag_ev[slot], ctx->stream));
      if (c > 0) {  // the previous chunk's flag: stop launching once nothing is active
        VIE_HIP(hipEventSynchronize(ctx->flag_ev[slot ^ 1]));
        if (!ctx->hflags[slot ^ 1][0]) break;
        if (getenv("VIE_LOG"))
          fprintf(stderr, "vie: fgmres cycle %d: steps < %d done\n", cycle, j0);
      }
    }
    // x += Z y for every right-hand side that took steps in this cycle
    VIE_HIP(launch_ls_solve(nrhs, L, A.coef.as<c64>(), m + 1, A.nvs.as<int>(), A.act.as<int>(),
                            ctx->stream));
    VIE_HIP(launch_seg_maxpy(S, Zb.p, A.v32, tot, m, A.nvs.as<int>(), A.coef.as<c64>(), m + 1, x,
                             0, nullptr, nullptr, 0, ctx->stream));
    // true residual with the FP64 product
    EpiArgs e{EPI_RESID, rh, part, 0, pol, ph};
    VIE_HIP(run_matvec(ctx, G, 0, x, r, e, notdone));
    VIE_HIP(launch_finalize(FIN_RESTART, nrhs, e.part_blocks, part, st, flags, fp, ctx->stream));
    if (getenv("VIE_LOG")) {
      std::vector<KState> hs(nrhs);
      std::vector<int> hst(nrhs);
      VIE_HIP(hipMemcpyAsync(hs.data(), st, nrhs * sizeof(KState), hipMemcpyDeviceToHost,
                             ctx->stream));
      VIE_HIP(hipMemcpyAsync(hst.data(), steps, nrhs * sizeof(int), hipMemcpyDeviceToHost,
                             ctx->stream));
      VIE_HIP(hipStreamSynchronize(ctx->stream));
      for (int q = 0; q < nrhs; ++q)
        fprintf(stderr, "vie: fgmres rhs %d: %d steps, true rel res %.3e\n", q, hst[q],
                hs[q].bnorm2 > 0 ? sqrt(hs[q].rnorm2 / hs[q].bnorm2) : 0.0);
    }
  }
  steps_out.assign(nrhs, 0);
  cycles_out.assign(nrhs, 0);
  VIE_HIP(hipMemcpyAsync(steps_out.data(), steps, nrhs * sizeof(int), hipMemcpyDeviceToHost,
                         ctx->stream));
  VIE_HIP(hipMemcpyAsync(cycles_out.data(), cycles, nrhs * sizeof(int), hipMemcpyDeviceToHost,
                         ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  return VIE_OK;
}

// Body slot of every right-hand side of G.
static std::vector<int> rhs_slots(vie_ctx* ctx, const Group& G) {
  std::vector<int> rb(G.g.nrhs, 0);
  for (int b : G.bodies) {
    const BodyRec& B = *ctx->bodies[b];
    for (int q = 0; q < B.nrhs; ++q) rb[B.rhs0 + q] = B.slot;
  }
  return rb;
}

extern "C" int vie_solve_fgmres(vie_ctx* ctx, const vie_planewave* inc,
                                const int32_t* nrhs_per_body, const vie_fgmres_options* fo,
                                vie_stats* stats) {
  TraceRange trace_("vie_solve_fgmres");
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (!inc || !nrhs_per_body || !fo) return VIE_EINVAL;
  for (auto& Gp : ctx->groups)
    if (!valid_fgmres(fo, Gp->g)) return VIE_EINVAL;
  std::vector<int> first;
  int rc = check_channels(ctx, inc, nrhs_per_body, first);
  if (rc != VIE_OK) return rc;
  if (ctx->opt.warm_start && !ctx->cnn) return VIE_EINVAL;  // warm start needs vie_attach_cnn
  const bool blocks = fo->blocks[0] > 0;
  bool all_conv = true;
  VIE_HIP(launch_stamp(ctx->t_call.as<unsigned long long>(), ctx->stream));
  for (int gi = 0; gi < (int)ctx->groups.size(); ++gi) {
    Group& G = *ctx->groups[gi];
    rc = bind_rhs(ctx, G, inc, nrhs_per_body, first);
    if (rc != VIE_OK) return rc;
    const int nrhs = G.g.nrhs;
    if (nrhs == 0) continue;
    G.res_x0.assign(nrhs, 1.0);
    G.fallback.assign(nrhs, 0);
    G.warm_used.assign(nrhs, 0);
    G.samples_ready = false;
    BlockPrec* P = nullptr;
    if (blocks) {
      rc = bj_build(ctx, gi, fo);
      if (rc != VIE_OK) return rc;
      P = ctx->bj[gi].get();
      rc = bj_bind(ctx, G, *P, rhs_slots(ctx, G), G.roff_host, fo->inner_iters);
      if (rc != VIE_OK) return rc;
      if (P->nseg == 0) P = nullptr;  // no body voxels: nothing to precondition
    }
    std::vector<int> steps, cycles;
    rc = fgmres_group(ctx, G, P, fo, ctx->opt.warm_start != 0, steps, cycles);
    if (rc != VIE_OK) return rc;
    std::vector<KState> hs(nrhs);
    unsigned long long t0 = 0;
    VIE_HIP(hipMemcpyAsync(&t0, ctx->t_call.p, sizeof(t0), hipMemcpyDeviceToHost, ctx->stream));
    VIE_HIP(hipMemcpyAsync(hs.data(), G.state.p, nrhs * sizeof(KState), hipMemcpyDeviceToHost,
                           ctx->stream));
    VIE_HIP(hipStreamSynchronize(ctx->stream));
    for (int b : G.bodies) {
      const BodyRec& B = *ctx->bodies[b];
      for (int q = 0; q < B.nrhs; ++q) {
        const int gq = B.rhs0 + q;
        const bool conv = !hs[gq].notdone;
        all_conv &= conv;
        if (!stats) continue;
        vie_stats& o = stats[first[b] + q];
        o.iters = steps[gq];
        o.matvecs = steps[gq] + cycles[gq];
        o.cycles = cycles[gq];
        o.converged = conv;
        o.fallback = G.fallback[gq];
        o.warm = G.warm_used[gq];
        o.rel_res = hs[gq].bnorm2 > 0 ? sqrt(hs[gq].rnorm2 / hs[gq].bnorm2) : 0.0;
        o.rel_res_x0 = G.res_x0[gq];
        o.seconds = done_seconds(ctx, hs[gq], conv, t0);
      }
    }
  }
  timing_collect(ctx);
  return all_conv ? VIE_OK : VIE_ENOCONV;
}

extern "C" int vie_precond_apply(vie_ctx* ctx, const vie_fgmres_options* fo, const vie_c64* r,
                                 vie_c64* z, int32_t nvec) {
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (!fo || !r || !z || nvec < 1) return VIE_EINVAL;
  if (ctx->bodies.size() != 1) return VIE_ENOTSUP;
  BodyRec& B = *ctx->bodies[0];
  Group& G = *ctx->groups[B.group];
  if (!valid_fgmres(fo, G.g) || fo->blocks[0] < 1) return VIE_EINVAL;
  // r and z are box vectors on the body's grid (n0 voxels); the body's voxel
  // list indexes the compute window, which starts zoff layers up
  const int64_t n0 = G.n0;
  const int64_t shift = (int64_t)G.g.N[0] * G.g.N[1] * B.zoff;
  const int nb = B.nb;
  const int64_t len = 3 * (int64_t)nb;
  memset(z, 0, (size_t)nvec * 3 * n0 * sizeof(vie_c64));
  if (nb == 0) return VIE_OK;
  int rc = bj_build(ctx, B.group, fo);
  if (rc != VIE_OK) return rc;
  BlockPrec& P = *ctx->bj[B.group];
  std::vector<int64_t> roff(nvec);
  for (int q = 0; q < nvec; ++q) roff[q] = q * len;
  rc = bj_bind(ctx, G, P, std::vector<int>(nvec, B.slot), roff, fo->inner_iters);
  if (rc != VIE_OK) return rc;
  const int* vx = G.vox_host.data() + G.voff_host[B.slot];
  std::vector<c64> hv((size_t)nvec * len), hz((size_t)nvec * len);
  for (int q = 0; q < nvec; ++q)
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < nb; ++k) {
        const vie_c64& a = r[(size_t)q * 3 * n0 + (size_t)c * n0 + shift + vx[k]];
        hv[(size_t)q * len + (size_t)c * nb + k] = mk(a.re, a.im);
      }
  DevBuf dv, dz;
  VIE_HIP(dv.reserve(hv.size() * sizeof(c64)));
  VIE_HIP(dz.reserve(hv.size() * sizeof(c64)));
  VIE_HIP(hipMemcpyAsync(dv.p, hv.data(), hv.size() * sizeof(c64), hipMemcpyHostToDevice,
                         ctx->stream));
  rc = bj_prepare(ctx, P, fo);
  if (rc != VIE_OK) return rc;
  rc = bj_apply(ctx, P, fo, dv.p, dz.p, 0, P.ones.as<int>());
  if (rc != VIE_OK) return rc;
  VIE_HIP(hipMemcpyAsync(hz.data(), dz.p, hz.size() * sizeof(c64), hipMemcpyDeviceToHost,
                         ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  for (int q = 0; q < nvec; ++q)
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < nb; ++k) {
        const c64 a = hz[(size_t)q * len + (size_t)c * nb + k];
        vie_c64& o = z[(size_t)q * 3 * n0 + (size_t)c * n0 + shift + vx[k]];
        o.re = a.re;
        o.im = a.im;
      }
  return VIE_OK;
}

// --------------------------------------------------------------- products
extern "C" int vie_matvec_dev(vie_ctx* ctx, int32_t body, int32_t precision, const void* x,
                              void* y, int32_t nvec) {
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (body < 0 || body >= (int)ctx->bodies.size() || nvec < 1 || !x || !y) return VIE_EINVAL;
  if (precision != VIE_FP64 && precision != VIE_MIXED) return VIE_EINVAL;
  BodyRec& B = *ctx->bodies[body];
  Group& G = *ctx->groups[B.group];
  const int saved = G.g.nrhs;
  G.g.nrhs = nvec;
  int rc = ensure_solve_storage(ctx, G, nvec);
  if (rc != VIE_OK) {
    G.g.nrhs = saved;
    return rc;
  }
  std::vector<int> rb(nvec, B.slot);
  VIE_HIP(hipMemcpyAsync(G.rhs_body.p, rb.data(), nvec * sizeof(int), hipMemcpyHostToDevice,
                         ctx->stream));
  // Box vectors come in the bodies' grid; the product runs on the compute
  // window.  Outside the window chi = 0, so there y = x.
  const bool window = G.g.n != G.n0;
  const c64* xs = (const c64*)x;
  c64* ys = (c64*)y;
  if (window) {
    const size_t wb = (size_t)nvec * 3 * G.g.n * sizeof(c64);
    hipError_t re = G.boxX.reserve(wb);
    if (re == hipSuccess) re = G.boxY.reserve(wb);
    if (re != hipSuccess) {
      G.g.nrhs = saved;
      VIE_HIP(re);
    }
    const int64_t shift = (int64_t)G.g.N[0] * G.g.N[1] * B.zoff;
    for (int64_t r = 0; r < (int64_t)nvec * 3; ++r)  // the window of every component
      VIE_HIP(hipMemcpyAsync(G.boxX.as<c64>() + r * G.g.n, (const c64*)x + r * G.n0 + shift,
                             G.g.n * sizeof(c64), hipMemcpyDeviceToDevice, ctx->stream));
    xs = G.boxX.as<c64>();
    ys = G.boxY.as<c64>();
  }
  EpiArgs e{EPI_PLAIN, nullptr, nullptr, 0, nullptr, nullptr};
  hipError_t err = run_matvec(ctx, G, precision == VIE_MIXED ? 1 : 0, xs, ys, e, nullptr, false);
  G.g.nrhs = saved;
  VIE_HIP(err);
  if (window) {
    const int64_t shift = (int64_t)G.g.N[0] * G.g.N[1] * B.zoff;
    VIE_HIP(hipMemcpyAsync(y, x, (size_t)nvec * 3 * G.n0 * sizeof(c64), hipMemcpyDeviceToDevice,
                           ctx->stream));
    for (int64_t r = 0; r < (int64_t)nvec * 3; ++r)
      VIE_HIP(hipMemcpyAsync((c64*)y + r * G.n0 + shift, G.boxY.as<c64>() + r * G.g.n,
                             G.g.n * sizeof(c64), hipMemcpyDeviceToDevice, ctx->stream));
  }
  return VIE_OK;
}

// The product of vie_matvec_dev with every scratch buffer (FFT work arrays,
// the right-hand-side table, window copies) carved out of the static scratch
// array instead of memory the context allocates: no allocation, no host
// copy, no memset.  Layout, each part 256-byte aligned: bufA, bufB, the
// body table, then the two window copies.  The z-pass shape is the one tuned
// for this group if any, else the default.
extern "C" int vie_matvec_dev_static(vie_ctx* ctx, int32_t body, int32_t precision,
                                     const void* x, void* y, int32_t nvec) {
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (body < 0 || body >= (int)ctx->bodies.size() || nvec < 1 || !x || !y) return VIE_EINVAL;
  if (precision != VIE_FP64 && precision != VIE_MIXED) return VIE_EINVAL;
  BodyRec& B = *ctx->bodies[body];
  Group& G = *ctx->groups[B.group];
  const int prec = precision == VIE_MIXED ? 1 : 0;
  const size_t cb = prec ? sizeof(c32) : sizeof(c64);
  const bool window = G.g.n != G.n0;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t a_b = al((size_t)nvec * 3 * G.g.N[2] * G.g.N[1] * G.g.P[0] * cb);
  const size_t b_b = al((size_t)nvec * (size_t)bufB_elems(G.g) * cb);
  const size_t r_b = al((size_t)nvec * sizeof(int));
  const size_t w_b = window ? al((size_t)nvec * 3 * G.g.n * sizeof(c64)) : 0;
  const size_t need = a_b + b_b + r_b + 2 * w_b;
  if (need > (size_t)VIE_STATIC_SCRATCH_BYTES) {
    if (getenv("VIE_LOG"))
      fprintf(stderr, "vie: vie_matvec_dev_static needs %zu bytes of scratch, the limit is %zu\n",
              need, (size_t)VIE_STATIC_SCRATCH_BYTES);
    return VIE_ENOTSUP;
  }
  char* base = (char*)g_scratch_ptr[ctx->dev];
  if (!base) return VIE_ESTATE;  // the look-up at setup failed (vie_setup would have said so)
  int* rb = (int*)(base + a_b + b_b);
  c64* boxX = (c64*)(base + a_b + b_b + r_b);
  c64* boxY = (c64*)(base + a_b + b_b + r_b + w_b);
  const int saved = G.g.nrhs;
  G.g.nrhs = nvec;
  MatvecArgs m = matvec_args(G, prec, nullptr);
  m.bufA = base;
  m.bufB = base + a_b;
  m.rhs_body = rb;
  m.zvar = G.zvar[prec] >= 0 ? G.zvar[prec] : 0;
  hipError_t err = launch_fill_int(rb, nvec, B.slot, ctx->stream);
  const c64* xs = (const c64*)x;
  c64* ys = (c64*)y;
  const int64_t shift = (int64_t)G.g.N[0] * G.g.N[1] * B.zoff;
  if (window && err == hipSuccess) {
    // the window of every component: nvec * 3 rows of n from rows of n0
    err = hipMemcpy2DAsync(boxX, G.g.n * sizeof(c64), (const c64*)x + shift, G.n0 * sizeof(c64),
                           G.g.n * sizeof(c64), (size_t)nvec * 3, hipMemcpyDeviceToDevice,
                           ctx->stream);
    xs = boxX;
    ys = boxY;
  }
  EpiArgs e{EPI_PLAIN, nullptr, nullptr, 0, nullptr, nullptr};
  if (err == hipSuccess) err = launch_matvec(m, prec, xs, ys, e, ctx->stream, nullptr, nullptr);
  G.g.nrhs = saved;
  VIE_HIP(err);
  if (window) {
    VIE_HIP(hipMemcpyAsync(y, x, (size_t)nvec * 3 * G.n0 * sizeof(c64), hipMemcpyDeviceToDevice,
                           ctx->stream));
    VIE_HIP(hipMemcpy2DAsync((c64*)y + shift, G.n0 * sizeof(c64), boxY, G.g.n * sizeof(c64),
                             G.g.n * sizeof(c64), (size_t)nvec * 3, hipMemcpyDeviceToDevice,
                             ctx->stream));
  }
  return VIE_OK;
}

extern "C" int vie_matvec(vie_ctx* ctx, int32_t body, int32_t precision, const vie_c64* x,
                          vie_c64* y, int32_t nvec) {
  TraceRange trace_("vie_matvec");
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (body < 0 || body >= (int)ctx->bodies.size() || nvec < 1 || !x || !y) return VIE_EINVAL;
  Group& G = *ctx->groups[ctx->bodies[body]->group];
  const size_t bytes = (size_t)nvec * 3 * G.n0 * sizeof(c64);
  DevBuf dx, dy;
  VIE_HIP(dx.reserve(bytes));
  VIE_HIP(dy.reserve(bytes));
  VIE_HIP(hipMemcpyAsync(dx.p, x, bytes, hipMemcpyHostToDevice, ctx->stream));
  int rc = vie_matvec_dev(ctx, body, precision, dx.p, dy.p, nvec);
  if (rc != VIE_OK) return rc;
  VIE_HIP(hipMemcpyAsync(y, dy.p, bytes, hipMemcpyDeviceToHost, ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  timing_collect(ctx);
  return VIE_OK;
}

extern "C" int vie_get_current(vie_ctx* ctx, int32_t body, int32_t rhs, vie_c64* w) {
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (body < 0 || body >= (int)ctx->bodies.size() || !w) return VIE_EINVAL;
  BodyRec& B = *ctx->bodies[body];
  if (rhs < 0 || rhs >= B.nrhs) return VIE_EINVAL;
  Group& G = *ctx->groups[B.group];
  const int64_t n0 = G.n0;
  const int64_t shift = (int64_t)G.g.N[0] * G.g.N[1] * B.zoff;  // window -> body grid
  std::vector<c64> c((size_t)3 * B.nb);
  if (B.nb > 0) {
    VIE_HIP(hipMemcpyAsync(c.data(), G.x.as<c64>() + G.roff_host[B.rhs0 + rhs],
                           c.size() * sizeof(c64), hipMemcpyDeviceToHost, ctx->stream));
    VIE_HIP(hipStreamSynchronize(ctx->stream));
  }
  memset(w, 0, (size_t)3 * n0 * sizeof(vie_c64));
  const int* vx = G.vox_host.data() + G.voff_host[B.slot];
  for (int comp = 0; comp < 3; ++comp)
    for (int k = 0; k < B.nb; ++k) {
      w[comp * n0 + shift + vx[k]].re = c[(size_t)comp * B.nb + k].re;
      w[comp * n0 + shift + vx[k]].im = c[(size_t)comp * B.nb + k].im;
    }
  return VIE_OK;
}

// -------------------------------------------------------------- far field
// Far field of every right-hand side of body B at ndir directions given as
// (r-hat, e1, e2) triples (9 doubles each, e1 and e2 orthonormal and
// perpendicular to r-hat): F[(rhs * ndir + d) * 2 + {0,1}] = (e1.F, e2.F).
static int far_project(vie_ctx* ctx, BodyRec& B, const std::vector<double>& dirs, int ndir,
                       vie_c64* F) {
  Group& G = *ctx->groups[B.group];
  const size_t outn = (size_t)B.nrhs * ndir * 2;
  if (B.nb == 0) {
    memset(F, 0, outn * sizeof(vie_c64));
    return VIE_OK;
  }
  if (G.far.size() < G.bodies.size()) G.far.resize(G.bodies.size());
  if (!G.far[B.slot]) {
    std::unique_ptr<Group::Far> fr(new Group::Far);
    far_blocks_build(G.vox_host.data() + G.voff_host[B.slot], B.nb, G.g.N, fr->fb);
    VIE_HIP(fr->vi.reserve(fr->fb.vi.size() * sizeof(int)));
    VIE_HIP(fr->org.reserve(fr->fb.org.size() * sizeof(int)));
    VIE_HIP(hipMemcpyAsync(fr->vi.p, fr->fb.vi.data(), fr->fb.vi.size() * sizeof(int),
                           hipMemcpyHostToDevice, ctx->stream));
    VIE_HIP(hipMemcpyAsync(fr->org.p, fr->fb.org.data(), fr->fb.org.size() * sizeof(int),
                           hipMemcpyHostToDevice, ctx->stream));
    G.far[B.slot] = std::move(fr);
  }
  const Group::Far& fr = *G.far[B.slot];
  const int ks = far_split_total(fr.fb, ndir);
  VIE_HIP(G.dirs.reserve(dirs.size() * sizeof(double)));
  VIE_HIP(G.part.reserve((size_t)ks * ndir * 3 * sizeof(c64)));
  VIE_HIP(G.wd.reserve(far_pack_elems(fr.fb.ntiles) * sizeof(c64)));
  VIE_HIP(G.F.reserve(outn * sizeof(c64)));
  VIE_HIP(hipMemcpyAsync(G.dirs.p, dirs.data(), dirs.size() * sizeof(double),
                         hipMemcpyHostToDevice, ctx->stream));
  VIE_HIP(timed(ctx, 12, [&] {
    return launch_farfield_mfma(G.x.as<c64>(), G.roff_host.data() + B.rhs0, B.nrhs, B.nb, fr.fb,
                                fr.vi.as<int>(), fr.org.as<int>(), G.dirs.as<double>(), ndir,
                                ctx->opt.k0, G.h, B.origin, G.wd.as<c64>(), G.part.as<c64>(),
                                G.F.as<c64>(), ctx->stream);
  }));
  VIE_HIP(hipMemcpyAsync(F, G.F.p, outn * sizeof(c64), hipMemcpyDeviceToHost, ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  timing_collect(ctx);
  return VIE_OK;
}

// r-hat, theta-hat, phi-hat of the direction (t, p) into D[0..8]
static void sph_frame(double t, double p, double* D) {
  const double st = sin(t), ct = cos(t), sp = sin(p), cp = cos(p);
  D[0] = st * cp; D[1] = st * sp; D[2] = ct;
  D[3] = ct * cp; D[4] = ct * sp; D[5] = -st;
  D[6] = -sp;     D[7] = cp;      D[8] = 0.0;
}

extern "C" int vie_farfield(vie_ctx* ctx, int32_t body, const double* theta, const double* phi,
                            int32_t ndir, vie_c64* F) {
  TraceRange trace_("vie_farfield");
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (body < 0 || body >= (int)ctx->bodies.size() || ndir < 1 || !theta || !phi || !F)
    return VIE_EINVAL;
  BodyRec& B = *ctx->bodies[body];
  if (B.nrhs < 1) return VIE_ESTATE;
  std::vector<double> dirs((size_t)ndir * 9);
  for (int d = 0; d < ndir; ++d) {
    if (!isfinite(theta[d]) || !isfinite(phi[d])) return VIE_EINVAL;
    sph_frame(theta[d], phi[d], &dirs[(size_t)d * 9]);
  }
  return far_project(ctx, B, dirs, ndir, F);
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on P_n from
// the cosine initial guess, P_n and P_n' by the three-term recurrence.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // P_0, P_1
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = n == 0 ? 1.0 : (n == 1 ? z : p1);
      const double pm = n == 1 ? 1.0 : p0;  // P_{n-1}
      dp = n * (z * pn - pm) / (z * z - 1.0);
      const double dz = pn / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

extern "C" int vie_transfer_na(vie_ctx* ctx, int32_t body, const vie_na_detector* det,
                               int32_t ndet, int32_t n_rad, int32_t n_az, vie_c64* T) {
  TraceRange trace_("vie_transfer_na");
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (body < 0 || body >= (int)ctx->bodies.size() || ndet < 1 || !det || !T || n_rad < 1 ||
      n_az < 1 || n_rad > 256 || n_az > 1024 || (int64_t)ndet * n_rad * n_az > (1 << 22))
    return VIE_EINVAL;
  BodyRec& B = *ctx->bodies[body];
  if (B.nrhs < 1) return VIE_ESTATE;
  std::vector<double> gx, gw;
  gauss_legendre(n_rad, gx, gw);
  // quadrature directions of every detector: (r-hat, theta-hat, phi-hat) and
  // the weight times (p . theta-hat, p . phi-hat)
  std::vector<double> dirs;
  std::vector<vie_c64> cw;  // per direction: weight * p.theta-hat, weight * p.phi-hat
  std::vector<int> first(ndet + 1, 0);
  for (int a = 0; a < ndet; ++a) {
    const vie_na_detector& D = det[a];
    if (!isfinite(D.theta0) || !isfinite(D.phi0) || !(D.alpha >= 0.0) || D.alpha > M_PI)
      return VIE_EINVAL;
    for (int c = 0; c < 3; ++c)
      if (!isfinite(D.pol[c].re) || !isfinite(D.pol[c].im)) return VIE_EINVAL;
    double ax[9];
    sph_frame(D.theta0, D.phi0, ax);  // local frame: u = r0, e1 = theta0-hat, e2 = phi0-hat
    auto add = [&](double ca, double beta, double wt) {
      const double sa = sqrt(fmax(0.0, 1.0 - ca * ca)), cb = cos(beta), sb = sin(beta);
      double r[3];
      for (int k = 0; k < 3; ++k) r[k] = ca * ax[k] + sa * (cb * ax[3 + k] + sb * ax[6 + k]);
      const double t = acos(fmax(-1.0, fmin(1.0, r[2]))), p = atan2(r[1], r[0]);
      double F9[9];
      sph_frame(t, p, F9);
      // sph_frame rebuilt r-hat from (t, p); keep the exact node direction
      F9[0] = r[0]; F9[1] = r[1]; F9[2] = r[2];
      dirs.insert(dirs.end(), F9, F9 + 9);
      vie_c64 pt{0, 0}, pp{0, 0};
      for (int k = 0; k < 3; ++k) {
        pt.re += D.pol[k].re * F9[3 + k]; pt.im += D.pol[k].im * F9[3 + k];
        pp.re += D.pol[k].re * F9[6 + k]; pp.im += D.pol[k].im * F9[6 + k];
      }
      cw.push_back({wt * pt.re, wt * pt.im});
      cw.push_back({wt * pp.re, wt * pp.im});
    };
    if (D.alpha == 0.0) {
      add(1.0, 0.0, 1.0);  // point detector on the axis
    } else {
      const double c0 = cos(D.alpha), omega = 2.0 * M_PI * (1.0 - c0);
      for (int i = 0; i < n_rad; ++i) {
        const double ca = 0.5 * (1.0 - c0) * gx[i] + 0.5 * (1.0 + c0);  // [-1,1] -> [cos alpha, 1]
        const double wr = 0.5 * (1.0 - c0) * gw[i];
        for (int j = 0; j < n_az; ++j)
          add(ca, 2.0 * M_PI * (j + 0.5) / n_az, wr * (2.0 * M_PI / n_az) / omega);
      }
    }
    first[a + 1] = (int)(dirs.size() / 9);
  }
  const int nd = first[ndet];
  std::vector<vie_c64> F((size_t)B.nrhs * nd * 2);
  const int rc = far_project(ctx, B, dirs, nd, F.data());
  if (rc != VIE_OK) return rc;
  for (int q = 0; q < B.nrhs; ++q)
    for (int a = 0; a < ndet; ++a) {
      double re = 0.0, im = 0.0;
      for (int d = first[a]; d < first[a + 1]; ++d)
        for (int k = 0; k < 2; ++k) {
          const vie_c64 f = F[((size_t)q * nd + d) * 2 + k], c = cw[(size_t)d * 2 + k];
          re += c.re * f.re - c.im * f.im;
          im += c.re * f.im + c.im * f.re;
        }
      T[(size_t)q * ndet + a] = {re, im};
    }
  return VIE_OK;
}

// ------------------------------------------------------- two-photon (host)
extern "C" int hom_g2(const vie_c64 T[4], const double* omega, double sigma, const double* dtau,
                      int32_t ndelay, int32_t norm, double* g2, double* Nc_raw, double* Nc_norm) {
  if (!T) return VIE_EINVAL;
  if (norm != VIE_NORM_R1 && norm != VIE_NORM_R2) return VIE_EINVAL;
  if (ndelay < 0 || (ndelay > 0 && !dtau)) return VIE_EINVAL;
  if ((Nc_raw || Nc_norm) && ndelay > 0 && !(sigma > 0)) return VIE_EINVAL;
  for (int i = 0; i < 4; ++i)
    if (!isfinite(T[i].re) || !isfinite(T[i].im)) return VIE_EINVAL;
  const double w1 = omega ? omega[0] : 1.0, w2 = omega ? omega[1] : 1.0;
  if (!(w1 > 0) || !(w2 > 0) || !isfinite(w1) || !isfinite(w2)) return VIE_EINVAL;
  // the channel weights enter as sqrt(w_j) on every coefficient of channel j
  // (the field operators of eqs. 8-9)
  const double s1 = sqrt(w1), s2 = sqrt(w2);
  const c64 a1 = s1 * mk(T[0].re, T[0].im), a2 = s2 * mk(T[1].re, T[1].im);
  const c64 b1 = s1 * mk(T[2].re, T[2].im), b2 = s2 * mk(T[3].re, T[3].im);
  auto ab2 = [](c64 z) { return z.re * z.re + z.im * z.im; };
  const c64 Ad = a1 * b2, Ae = a2 * b1;  // direct and exchange path amplitudes
  const c64 sum = Ad + Ae;
  const double G1a = ab2(a1) + ab2(a2), G1b = ab2(b1) + ab2(b2);  // marginal intensities
  if (g2) {
    const double den = G1a * G1b;
    *g2 = den > 0 ? ab2(sum) / den : NAN;
  }
  if (ndelay > 0 && (Nc_raw || Nc_norm)) {
    const double sp = sigma * sqrt(M_PI);
    const double d2 = ab2(Ad), e2 = ab2(Ae);
    const double cross = 2.0 * (Ad.re * Ae.re + Ad.im * Ae.im);  // 2 Re(Ad conj(Ae))
    const double D = norm == VIE_NORM_R1 ? sp * (d2 + e2) : sp * G1a * G1b;
    for (int k = 0; k < ndelay; ++k) {
      const double c = exp(-(dtau[k] * dtau[k]) / (sigma * sigma));
      const double raw = sp * (d2 + e2 + cross * c);
      if (Nc_raw) Nc_raw[k] = raw;
      if (Nc_norm) Nc_norm[k] = D > 0 ? raw / D : NAN;
    }
  }
  return VIE_OK;
}

// The grid a body is computed on: its compute window, the circulant lengths
// and the window's z offset.
extern "C" int vie_grid(vie_ctx* ctx, int32_t body, int32_t* grid, int32_t* fft,
                        int32_t* offset) {
  if (!ctx) return VIE_EINVAL;
  if (body < 0 || body >= (int)ctx->bodies.size()) return VIE_EINVAL;
  const BodyRec& B = *ctx->bodies[body];
  const Group& G = *ctx->groups[B.group];
  for (int a = 0; a < 3; ++a) {
    if (grid) grid[a] = G.g.N[a];
    if (fft) fft[a] = G.g.P[a];
    if (offset) offset[a] = a == 2 ? B.zoff : 0;
  }
  return VIE_OK;
}

extern "C" int vie_self_term(int32_t kind, double k0, double h, vie_c64* s) {
  if (!s || !(k0 > 0) || !(h > 0) || !isfinite(k0) || !isfinite(h)) return VIE_EINVAL;
  double re, im;
  if (kind == 0)
    self_term_sphere(k0, h, &re, &im);
  else if (kind == 1)
    self_term_cube(k0, h, &re, &im);
  else
    return VIE_EINVAL;
  s->re = re;
  s->im = im;
  return VIE_OK;
}

// Classical fourth-order correlation (eq. 27) of the coherent superposition
// of the two channels' responses: |T_a1 + T_a2|^2 |T_b1 + T_b2|^2.
extern "C" int hom_classical_p2(const vie_c64 T[4], double* p2) {
  if (!T || !p2) return VIE_EINVAL;
  for (int i = 0; i < 4; ++i)
    if (!isfinite(T[i].re) || !isfinite(T[i].im)) return VIE_EINVAL;
  const double ar = T[0].re + T[1].re, ai = T[0].im + T[1].im;
  const double br = T[2].re + T[3].re, bi = T[2].im + T[3].im;
  *p2 = (ar * ar + ai * ai) * (br * br + bi * bi);
  return VIE_OK;
}

// ------------------------------------------------------- network (C ABI)
extern "C" int64_t vie_cnn_num_params(void) { return cnn_offsets().total; }

extern "C" int vie_cnn_create(uint64_t seed, vie_cnn** out) {
  if (!out) return VIE_EINVAL;
  *out = nullptr;
  vie_cnn* net = new (std::nothrow) vie_cnn();
  if (!net) return VIE_ENOMEM;
  if (cnn_alloc(net->c) != hipSuccess) {
    cnn_free(net->c);
    delete net;
    return VIE_ENOMEM;
  }
  // He-normal weights (last layer x0.1, unused output channels zero), zero biases
  const CnnLayerOffsets o = cnn_offsets();
  std::vector<float> p((size_t)o.total, 0.f);
  uint64_t st = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  auto next = [&]() {  // splitmix64
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto unif = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
  for (int l = 0; l < kCnnLayers; ++l) {
    const int ci = kCnnCh[l], co = kCnnCh[l + 1];
    const double sd = sqrt(2.0 / (27.0 * ci)) * (l + 1 == kCnnLayers ? 0.1 : 1.0);
    for (int t = 0; t < 27; ++t)
      for (int a = 0; a < co; ++a)
        for (int b = 0; b < ci; ++b) {
          const double g = sqrt(-2.0 * log(unif())) * cos(6.283185307179586 * unif());
          const bool dead = (l + 1 == kCnnLayers && a >= kCnnOut) || (l == 0 && b >= kCnnFeat);
          p[o.w[l] + ((size_t)t * co + a) * ci + b] = dead ? 0.f : (float)(sd * g);
        }
  }
  if (hipMemcpy(net->c.p, p.data(), p.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      cnn_refresh_bf16(net->c, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    cnn_free(net->c);
    delete net;
    return VIE_EDEVICE;
  }
  *out = net;
  return VIE_OK;
}

extern "C" void vie_cnn_destroy(vie_cnn* net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  cnn_free(net->c);
  delete net;
}

extern "C" int vie_cnn_params(vie_cnn* net, float* host, int64_t n, int32_t set) {
  if (!net || !host || n != cnn_offsets().total) return VIE_EINVAL;
  vie_ctx* ctx = nullptr;
  if (set) {
    for (int64_t i = 0; i < n; ++i)
      if (!isfinite(host[i])) return VIE_EINVAL;
    VIE_HIP(hipMemcpy(net->c.p, host, n * 4, hipMemcpyHostToDevice));
    VIE_HIP(hipMemset(net->c.m, 0, n * 4));
    VIE_HIP(hipMemset(net->c.v, 0, n * 4));
    net->c.step = 0;
    VIE_HIP(cnn_refresh_bf16(net->c, nullptr));
    VIE_HIP(hipDeviceSynchronize());
  } else {
    VIE_HIP(hipDeviceSynchronize());
    VIE_HIP(hipMemcpy(host, net->c.p, n * 4, hipMemcpyDeviceToHost));
  }
  return VIE_OK;
}

extern "C" int vie_cnn_adam_state(vie_cnn* net, float* m, float* v, int64_t n, int64_t* step,
                                  int32_t set) {
  if (!net || !m || !v || !step || n != cnn_offsets().total) return VIE_EINVAL;
  vie_ctx* ctx = nullptr;
  if (set) {
    if (*step < 0) return VIE_EINVAL;
    for (int64_t i = 0; i < n; ++i)
      if (!isfinite(m[i]) || !isfinite(v[i]) || v[i] < 0) return VIE_EINVAL;
    VIE_HIP(hipDeviceSynchronize());
    VIE_HIP(hipMemcpy(net->c.m, m, n * 4, hipMemcpyHostToDevice));
    VIE_HIP(hipMemcpy(net->c.v, v, n * 4, hipMemcpyHostToDevice));
    net->c.step = *step;
  } else {
    VIE_HIP(hipDeviceSynchronize());
    VIE_HIP(hipMemcpy(m, net->c.m, n * 4, hipMemcpyDeviceToHost));
    VIE_HIP(hipMemcpy(v, net->c.v, n * 4, hipMemcpyDeviceToHost));
    *step = net->c.step;
  }
  return VIE_OK;
}

extern "C" int vie_attach_cnn(vie_ctx* ctx, vie_cnn* net) {
  if (!ctx) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  ctx->cnn = net;
  return VIE_OK;
}

static bool valid_dims(const int32_t* d) {
  return d && d[0] > 0 && d[1] > 0 && d[2] > 0 && d[0] <= 512 && d[1] <= 512 && d[2] <= 512;
}

extern "C" int vie_cnn_sample_dev(vie_ctx* ctx, int32_t body, int32_t rhs, void* feat,
                                  void* target, int32_t* dims) {
  if (!ctx || !dims) return VIE_EINVAL;
  if (ctx->poisoned) return VIE_ESTATE;
  if (body < 0 || body >= (int)ctx->bodies.size()) return VIE_EINVAL;
  BodyRec& B = *ctx->bodies[body];
  if (rhs < 0 || rhs >= B.nrhs) return VIE_EINVAL;
  Group& G = *ctx->groups[B.group];
  for (int a = 0; a < 3; ++a) dims[a] = G.box_d[3 * B.slot + a];
  if (!feat && !target) return VIE_OK;
  const int q = B.rhs0 + rhs;
  std::vector<KState> hs(G.g.nrhs);
  VIE_HIP(hipMemcpyAsync(hs.data(), G.state.p, hs.size() * sizeof(KState), hipMemcpyDeviceToHost,
                         ctx->stream));
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  if (!G.samples_ready) {
    // r = b (solution x kept), v = A_32 b for every right-hand side
    const int vb = vec_blocks_group(G);
    VIE_HIP(launch_init_zero_guess(G.g, G.bi, vb, G.pol.as<c64>(), G.ph.as<c64>(), G.x.as<c64>(),
                                   G.r.as<c64>(), G.rh.as<c64>(), G.partials.as<c64>(), 1,
                                   nullptr, ctx->stream));
    int rc = krylov_inputs(ctx, G);
    if (rc != VIE_OK) return rc;
    G.samples_ready = true;
  }
  const double bn2 = hs[q].bnorm2;
  if (feat) {
    int rc = build_features(ctx, G, q, B.slot, feat);
    if (rc != VIE_OK) return rc;
  }
  if (target) {
    const int nb = B.nb;
    const double s = nb > 0 && bn2 > 0 ? sqrt(bn2 / nb) : 0.0;
    VIE_HIP(launch_cnn_target((float*)target, dims, &G.box_lo[3 * B.slot], G.g.N,
                              G.vox_all.as<int>() + G.voff_host[B.slot], nb,
                              G.x.as<c64>() + G.roff_host[q], s, ctx->stream));
  }
  VIE_HIP(hipStreamSynchronize(ctx->stream));
  return VIE_OK;
}

extern "C" int vie_cnn_infer_dev(vie_cnn* net, const int32_t* dims, const void* feat, void* out,
                                 void* stream) {
  if (!net || !valid_dims(dims) || !feat || !out) return VIE_EINVAL;
  vie_ctx* ctx = nullptr;
  const int d[3] = {dims[0], dims[1], dims[2]};
  VIE_HIP(cnn_forward(net->c, d, (const bf16raw*)feat, (float*)out, (hipStream_t)stream));
  return VIE_OK;
}

extern "C" int vie_cnn_grad_dev(vie_cnn* net, const int32_t* dims, const void* feat,
                                const void* target, float* grad_host, float* loss,
                                void* stream) {
  if (!net || !valid_dims(dims) || !feat || !target) return VIE_EINVAL;
  vie_ctx* ctx = nullptr;
  const int d[3] = {dims[0], dims[1], dims[2]};
  hipStream_t s = (hipStream_t)stream;
  VIE_HIP(cnn_forward(net->c, d, (const bf16raw*)feat, nullptr, s));
  float l = 0.f;
  VIE_HIP(cnn_backward(net->c, d, (const float*)target, &l, s));
  if (loss) *loss = l;
  if (grad_host) {
    VIE_HIP(hipMemcpyAsync(grad_host, net->c.g, net->c.off.total * 4, hipMemcpyDeviceToHost, s));
    VIE_HIP(hipStreamSynchronize(s));
  }
  return VIE_OK;
}

extern "C" int vie_cnn_train_step_dev(vie_cnn* net, const int32_t* dims, const void* feat,
                                      const void* target, float lr, float* loss, void* stream) {
  if (!net || !valid_dims(dims) || !feat || !target || !(lr > 0)) return VIE_EINVAL;
  vie_ctx* ctx = nullptr;
  const int d[3] = {dims[0], dims[1], dims[2]};
  hipStream_t s = (hipStream_t)stream;
  VIE_HIP(cnn_forward(net->c, d, (const bf16raw*)feat, nullptr, s));
  VIE_HIP(cnn_backward(net->c, d, (const float*)target, loss, s));
  VIE_HIP(cnn_adam(net->c, lr, s));
  return VIE_OK;
}

// ------------------------------------------------------------------ misc
extern "C" int vie_kernel_times(vie_ctx* ctx, const char** names, double* ms, int64_t* cnt,
                                int32_t* nkinds, int32_t reset) {
  if (!ctx || !nkinds) return VIE_EINVAL;
  timing_collect(ctx);
  for (auto& P : ctx->bj) {  // block products of the sub-contexts
    if (!P || !P->sub) continue;
    timing_collect(P->sub);
    for (int k = 0; k < 17; ++k) {
      const int src = k < 10 ? k : kH16Kind0 + k - 10;
      const int dst = k < 10 ? kBlockKind0 + k : kBlockH16Kind0 + k - 10;
      ctx->kind_ms[dst] += P->sub->kind_ms[src];
      ctx->kind_cnt[dst] += P->sub->kind_cnt[src];
      P->sub->kind_ms[src] = 0;
      P->sub->kind_cnt[src] = 0;
    }
  }
  const int n = std::min<int>(*nkinds, kNumKinds);
  for (int k = 0; k < n; ++k) {
    if (names) names[k] = kKindNames[k];
    if (ms) ms[k] = ctx->kind_ms[k];
    if (cnt) cnt[k] = ctx->kind_cnt[k];
  }
  *nkinds = kNumKinds;
  if (reset) {
    for (int k = 0; k < kNumKinds; ++k) {
      ctx->kind_ms[k] = 0;
      ctx->kind_cnt[k] = 0;
    }
  }
  return VIE_OK;
}

extern "C" const char* vie_strerror(int code) {
  switch (code) {
    case VIE_OK: return "ok";
    case VIE_EINVAL: return "invalid argument";
    case VIE_ENOMEM: return "out of memory";
    case VIE_EDEVICE: return "HIP device error (context poisoned)";
    case VIE_ENOCONV: return "not converged within max_iter";
    case VIE_ENOTSUP: return "unsupported request";
    case VIE_ESTATE: return "context poisoned or not prepared";
    default: return "unknown error";
  }
}
