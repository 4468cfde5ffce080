// Far-field amplitude (eq. 25 with the radiation-zone Green's function):
//   F(r) = k0^2 h^3 / (4 pi) (I - r r) sum_n w_n exp(-i k0 r . r_n),
// reported as (F_theta, F_phi) = (theta-hat . F, phi-hat . F).
//
// The sum over voxels is a dense complex contraction [directions x voxels] x
// [voxels x 3R] run on FP64 MFMA (v_mfma_f64_16x16x4f64).  The phase matrix is
// never stored: the body voxels are grouped into aligned blocks of 16 voxels
// (shape bx x by x bz, chosen per body to minimise padding), and for a voxel
// at block origin o_b plus offset u the phase factors as
//   exp(-i k0 r.(o + h(o_b + u))) = S(r, b) A(r, u),
// S(r, b) = exp(-i k0 r.(o + h o_b)),   A(r, u) = exp(-i k0 h r.u).
// A is the same for every block, so it stays in registers as the MFMA's left
// operand for the whole kernel; each block contributes
//   G(r, b, qc) = sum_u A(r, u) W(b, u, qc)   (16x16x16 complex tiles on MFMA)
// and is scaled by S(r, b) (one sincos per direction and block) and summed.
// The accumulation over blocks is split across workgroups (K-split) and
// reduced in fixed order by a second kernel that projects onto theta-hat /
// phi-hat and applies the constant.
#include <algorithm>
#include <vector>

#include "kernels.h"

namespace vie {

typedef double d4 __attribute__((ext_vector_type(4)));

static constexpr int FF_RB = 1;          // right-hand sides per pass
static constexpr int FF_QC = 3 * FF_RB;  // complex columns per block (rhs x component)
static constexpr int FF_BS = 16;         // voxels per block (MFMA K = 4 per step, 4 steps)
static constexpr int FF_TB = 16;         // blocks per tile (MFMA N)
static constexpr int FF_WAVES = 4;       // waves per workgroup, 16 directions each
static constexpr int FF_DIRS = 16 * FF_WAVES;
static constexpr int FF_TILE = FF_QC * FF_BS * FF_TB;  // c64 per packed tile

// ------------------------------------------------------------ host: blocks
namespace {
const int kShapes[][3] = {{16, 1, 1}, {8, 2, 1}, {4, 4, 1}, {4, 2, 2}, {2, 4, 2},
                          {2, 2, 4}, {1, 4, 4}, {2, 8, 1}, {1, 16, 1}, {1, 1, 16}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

struct VoxIJK {
  int i, j, z;
};
}  // namespace

void far_blocks_build(const int* vox, int nb, const int N[3], FarBlocks& fb) {
  std::vector<VoxIJK> p(nb);
  for (int k = 0; k < nb; ++k) {
    const int lin = vox[k];
    p[k] = {lin % N[0], (lin / N[0]) % N[1], lin / (N[0] * N[1])};
  }
  // blocks per band of H z layers for every shape with bz dividing H
  // (aligned blocks of such shapes never cross a band boundary)
  auto count_bands = [&](int H, std::vector<std::vector<int64_t>>& cnt) {
    const int nbands = (N[2] + H - 1) / H;
    cnt.assign(kNumShapes, std::vector<int64_t>(nbands, -1));
    std::vector<uint8_t> mark;
    for (int s = 0; s < kNumShapes; ++s) {
      const int bx = kShapes[s][0], by = kShapes[s][1], bz = kShapes[s][2];
      if (H % bz) continue;
      const int gx = (N[0] + bx - 1) / bx, gy = (N[1] + by - 1) / by, gz = (N[2] + bz - 1) / bz;
      mark.assign((size_t)gx * gy * gz, 0);
      std::fill(cnt[s].begin(), cnt[s].end(), 0);
      for (const VoxIJK& v : p) {
        const size_t key = ((size_t)(v.z / bz) * gy + v.j / by) * gx + v.i / bx;
        if (!mark[key]) {
          mark[key] = 1;
          ++cnt[s][v.z / H];
        }
      }
    }
    return nbands;
  };
  // pick the band height (4 or 16 layers) and per-band shape with the fewest blocks
  int bestH = 16;
  std::vector<int> best_choice;
  int64_t best_total = -1;
  for (int H : {4, 16}) {
    std::vector<std::vector<int64_t>> cnt;
    const int nbands = count_bands(H, cnt);
    std::vector<int> choice(nbands, 0);
    int64_t total = 0;
    for (int band = 0; band < nbands; ++band) {
      int64_t bc = -1;
      for (int s = 0; s < kNumShapes; ++s)
        if (cnt[s][band] >= 0 && (bc < 0 || cnt[s][band] < bc)) {
          bc = cnt[s][band];
          choice[band] = s;
        }
      total += bc;
    }
    if (best_total < 0 || total < best_total) {
      best_total = total;
      bestH = H;
      best_choice = choice;
    }
  }
  // one group per shape in use; blocks numbered in (z, y, x) block order
  fb.groups.clear();
  fb.org.clear();
  fb.vi.clear();
  fb.nblk = 0;
  int tiles = 0;
  for (int s = 0; s < kNumShapes; ++s) {
    bool used = false;
    for (int c : best_choice) used |= (c == s);
    if (!used) continue;
    const int bx = kShapes[s][0], by = kShapes[s][1], bz = kShapes[s][2];
    const int gx = (N[0] + bx - 1) / bx, gy = (N[1] + by - 1) / by, gz = (N[2] + bz - 1) / bz;
    std::vector<int> id((size_t)gx * gy * gz, -1);
    for (const VoxIJK& v : p)
      if (best_choice[v.z / bestH] == s) id[((size_t)(v.z / bz) * gy + v.j / by) * gx + v.i / bx] = 0;
    const size_t base = fb.org.size() / 4;
    int nblk = 0;
    for (int zb = 0; zb < gz; ++zb)
      for (int yb = 0; yb < gy; ++yb)
        for (int xb = 0; xb < gx; ++xb) {
          int& e = id[((size_t)zb * gy + yb) * gx + xb];
          if (e < 0) continue;
          e = nblk++;
          fb.org.insert(fb.org.end(), {xb * bx, yb * by, zb * bz, 0});
        }
    if (nblk == 0) continue;  // a shape chosen only for empty bands
    const int padded = (nblk + FF_TB - 1) / FF_TB * FF_TB;
    fb.org.resize((base + padded) * 4, 0);
    fb.vi.resize((base + padded) * FF_BS, -1);
    for (int k = 0; k < nb; ++k) {
      const VoxIJK& v = p[k];
      if (best_choice[v.z / bestH] != s) continue;
      const int b = id[((size_t)(v.z / bz) * gy + v.j / by) * gx + v.i / bx];
      const int u = v.i % bx + bx * (v.j % by + by * (v.z % bz));
      fb.vi[(base + b) * FF_BS + u] = k;
    }
    FarGroup gr;
    gr.shape[0] = bx;
    gr.shape[1] = by;
    gr.shape[2] = bz;
    gr.tile0 = tiles;
    gr.ntiles = padded / FF_TB;
    fb.groups.push_back(gr);
    tiles += gr.ntiles;
    fb.nblk += nblk;
  }
  fb.ntiles = tiles;
}

// ------------------------------------------------------------ kernels
struct RoffArg {
  int64_t r[FF_RB];
};

// Wd[tile][qc][u][s] = w of right-hand side q, component c at offset u of
// block tile*16 + s (zero where the block has no body voxel).
__global__ void k_ff_pack(const c64* __restrict__ w, RoffArg ro, int nq, int nb,
                          const int* __restrict__ blk_vi, int ntiles, c64* __restrict__ Wd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ntiles * FF_TILE) return;
  const int s = (int)(e % FF_TB);
  const int u = (int)((e / FF_TB) % FF_BS);
  const int qc = (int)((e / (FF_TB * FF_BS)) % FF_QC);
  const int64_t tile = e / FF_TILE;
  const int q = qc / 3, c = qc % 3;
  const int vi = blk_vi[(tile * FF_TB + s) * FF_BS + u];
  c64 v = mk(0.0, 0.0);
  if (vi >= 0 && q < nq) v = w[ro.r[q] + (int64_t)c * nb + vi];
  Wd[e] = v;
}

struct FfGeom {
  double k0, h, o[3];
  int bx, by;
};

// sin and cos of x for |x| < 1e9: Cody-Waite reduction by pi/2 with a two-part
// constant (FMA), then Taylor polynomials on |r| <= pi/4 through r^17 (sin)
// and r^16 (cos); absolute error about 2e-16.  Branch-free, so it schedules
// between the matrix instructions.
__device__ __forceinline__ void ff_sincos(double x, double& sn, double& cs) {
  const double n = rint(x * 0.63661977236758134308);
  double r = fma(-n, 1.5707963267948966192, x);
  r = fma(-n, 6.123233995736766036e-17, r);
  const int q = (int)n;
  const double r2 = r * r;
  double ps = 2.8114572543455207632e-15;    // 1/17!
  ps = fma(ps, r2, -7.6471637318198164759e-13);  // -1/15!
  ps = fma(ps, r2, 1.6059043836821614599e-10);   // 1/13!
  ps = fma(ps, r2, -2.5052108385441718775e-08);  // -1/11!
  ps = fma(ps, r2, 2.7557319223985890653e-06);   // 1/9!
  ps = fma(ps, r2, -1.9841269841269841270e-04);  // -1/7!
  ps = fma(ps, r2, 8.3333333333333333333e-03);   // 1/5!
  ps = fma(ps, r2, -1.6666666666666666667e-01);  // -1/3!
  const double s0 = fma(r * r2, ps, r);
  double pc = 4.7794773323873852974e-14;    // 1/16!
  pc = fma(pc, r2, -1.1470745597729724714e-11);  // -1/14!
  pc = fma(pc, r2, 2.0876756987868098979e-09);   // 1/12!
  pc = fma(pc, r2, -2.7557319223985890653e-07);  // -1/10!
  pc = fma(pc, r2, 2.4801587301587301587e-05);   // 1/8!
  pc = fma(pc, r2, -1.3888888888888888889e-03);  // -1/6!
  pc = fma(pc, r2, 4.1666666666666666667e-02);   // 1/4!
  pc = fma(pc, r2, -0.5);
  const double c0 = fma(r2, pc, 1.0);
  const bool swap = q & 1;
  const double s1 = swap ? c0 : s0, c1 = swap ? s0 : c0;
  sn = (q & 2) ? -s1 : s1;
  cs = ((q + 1) & 2) ? -c1 : c1;
}

// exp(i x) from a 256-entry table of exp(2 pi i k / 256) in LDS: x = k pi/128
// + e with |e| <= pi/256 (two-part FMA reduction), then Taylor polynomials of
// cos e through e^6 and sin e through e^7 (truncation below 1e-19) and one
// complex product with the table entry.
constexpr int FF_NT = 256;
__device__ __forceinline__ c64 ff_expi(double x, const c64* sT) {
  const double kf = rint(x * 40.743665431525205957);  // 128 / pi
  double e = fma(-kf, 2.4543692606170259375e-02, x);  // fl(pi) / 128
  e = fma(-kf, 9.5675531183386971e-19, e);            // (pi - fl(pi)) / 128
  const c64 t = sT[(int)kf & (FF_NT - 1)];
  const double e2 = e * e;
  double pc = fma(e2, -1.3888888888888888889e-03, 4.1666666666666666667e-02);
  pc = fma(e2, pc, -0.5);
  const double c = fma(e2, pc, 1.0);
  double ps = fma(e2, -1.9841269841269841270e-04, 8.3333333333333333333e-03);
  ps = fma(e2, ps, -1.6666666666666666667e-01);
  const double sn = fma(e * e2, ps, e);
  return mk(t.re * c - t.im * sn, fma(t.re, sn, t.im * c));
}

// packed tile t -> registers (FF_TILE / 256 c64 and one block origin per thread)
constexpr int FF_PER = FF_TILE / (FF_DIRS * 4);
struct FfPre {
  c64 v[FF_PER];
  int4 o;
};

__device__ __forceinline__ FfPre ff_fetch(const c64* __restrict__ Wd,
                                          const int4* __restrict__ org, int t) {
  FfPre p;
  const c64* src = Wd + (int64_t)t * FF_TILE;
#pragma unroll
  for (int k = 0; k < FF_PER; ++k) p.v[k] = src[k * FF_DIRS * 4 + threadIdx.x];
  p.o = threadIdx.x < FF_TB ? org[(int64_t)t * FF_TB + threadIdx.x] : make_int4(0, 0, 0, 0);
  return p;
}

__device__ __forceinline__ void ff_store(c64* sW, int4* sOrg, const FfPre& p) {
#pragma unroll
  for (int k = 0; k < FF_PER; ++k) sW[k * FF_DIRS * 4 + threadIdx.x] = p.v[k];
  if (threadIdx.x < FF_TB) sOrg[threadIdx.x] = p.o;
}

struct FfRows {
  double p0[4], cx[4], cy[4], cz[4];
};

// G(r, b, qc) = sum_u A(r, u) W(b, u, qc) for one staged tile (complex as
// four real products), and the block scale S(r, b) of this lane's column.
__device__ __forceinline__ void ff_tile(const c64* sW, const int4* sOrg, const c64* sT,
                                        const double (&aR)[4],
                                        const double (&aI)[4], const double (&aIn)[4],
                                        const FfRows& rw, int lane, d4 (&gR)[FF_QC],
                                        d4 (&gI)[FF_QC], c64 (&S)[4]) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    c64 b[FF_QC];
#pragma unroll
    for (int qc = 0; qc < FF_QC; ++qc)
      b[qc] = sW[(qc * FF_BS + 4 * ks + (lane >> 4)) * FF_TB + (lane & 15)];
    if (ks == 0) {
#pragma unroll
      for (int qc = 0; qc < FF_QC; ++qc) {
        gR[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(aR[ks], b[qc].re, d4{0.0, 0.0, 0.0, 0.0},
                                                      0, 0, 0);
        gI[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(aR[ks], b[qc].im, d4{0.0, 0.0, 0.0, 0.0},
                                                      0, 0, 0);
      }
    } else {
#pragma unroll
      for (int qc = 0; qc < FF_QC; ++qc) {
        gR[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(aR[ks], b[qc].re, gR[qc], 0, 0, 0);
        gI[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(aR[ks], b[qc].im, gI[qc], 0, 0, 0);
      }
    }
#pragma unroll
    for (int qc = 0; qc < FF_QC; ++qc) {
      gR[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(aIn[ks], b[qc].im, gR[qc], 0, 0, 0);
      gI[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(aI[ks], b[qc].re, gI[qc], 0, 0, 0);
    }
  }
  const int4 ob = sOrg[lane & 15];
  const double ox = ob.x, oy = ob.y, oz = ob.z;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double ang = fma(rw.cz[r], oz, fma(rw.cy[r], oy, fma(rw.cx[r], ox, rw.p0[r])));
    S[r] = ff_expi(ang, sT);
  }
}

__device__ __forceinline__ void ff_accum(const d4 (&gR)[FF_QC], const d4 (&gI)[FF_QC],
                                         const c64 (&S)[4], c64 (&acc)[4][FF_QC]) {
#pragma unroll
  for (int qc = 0; qc < FF_QC; ++qc)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r][qc] = cfma(S[r], mk(gR[qc][r], gI[qc][r]), acc[r][qc]);
}

// One workgroup: 64 directions (16 per wave) against the blocks of tiles
// [t0, t1).  Tiles are double-buffered in LDS (one barrier per tile) with a
// register prefetch; two waves per SIMD so that one wave's scale-and-
// accumulate and phase work runs while the other's matrix products execute.
__global__ __launch_bounds__(FF_DIRS * 4) __attribute__((amdgpu_waves_per_eu(2))) void k_ff_mfma(
    const c64* __restrict__ Wd, const int4* __restrict__ org, int ntiles, int tiles_per_split,
    const double* __restrict__ dirs, int nd, FfGeom fg, int nq, c64* __restrict__ part) {
  __shared__ c64 sW[2][FF_TILE];
  __shared__ int4 sOrg[2][FF_TB];
  __shared__ c64 sT[FF_NT];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < FF_NT; k += FF_DIRS * 4) {
    double sn, cs;
    ff_sincos(k * (2.0 * M_PI / FF_NT), sn, cs);
    sT[k] = mk(cs, sn);
  }  // visible after the first barrier of the tile loop
  const int dbase = blockIdx.x * FF_DIRS + wave * 16;
  const int t0 = blockIdx.y * tiles_per_split;
  const int t1 = min(ntiles, t0 + tiles_per_split);

  // left operand A(r, u): direction dbase + lane%16, offsets u = 4 ks + lane/16
  double aR[4], aI[4], aIn[4];
  {
    const int d = dbase + (lane & 15);
    double rx = 0, ry = 0, rz = 0;
    if (d < nd) {
      rx = dirs[d * 9 + 0];
      ry = dirs[d * 9 + 1];
      rz = dirs[d * 9 + 2];
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int u = 4 * ks + (lane >> 4);
      const int du = u % fg.bx, dv = (u / fg.bx) % fg.by, dw = u / (fg.bx * fg.by);
      const double ang = -fg.k0 * fg.h * (rx * du + ry * dv + rz * dw);
      double sn, cs;
      ff_sincos(ang, sn, cs);
      aR[ks] = cs;
      aI[ks] = sn;
      aIn[ks] = -sn;
    }
  }
  // output rows of this lane (FP64 16x16x4 result layout: row lane/16 + 4 r,
  // column lane % 16): directions dbase + lane/16 + 4 r
  FfRows rw;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int d = dbase + (lane >> 4) + 4 * r;
    double rx = 0, ry = 0, rz = 0;
    if (d < nd) {
      rx = dirs[d * 9 + 0];
      ry = dirs[d * 9 + 1];
      rz = dirs[d * 9 + 2];
    }
    rw.p0[r] = -fg.k0 * (rx * fg.o[0] + ry * fg.o[1] + rz * fg.o[2]);
    rw.cx[r] = -fg.k0 * fg.h * rx;
    rw.cy[r] = -fg.k0 * fg.h * ry;
    rw.cz[r] = -fg.k0 * fg.h * rz;
  }
  c64 acc[4][FF_QC];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int qc = 0; qc < FF_QC; ++qc) acc[r][qc] = mk(0.0, 0.0);

  d4 gR[FF_QC], gI[FF_QC];
  c64 S[4];
  FfPre pre;
  if (t0 < t1) pre = ff_fetch(Wd, org, t0);
  for (int t = t0; t < t1; ++t) {
    const int cb = (t - t0) & 1;
    ff_store(sW[cb], sOrg[cb], pre);
    if (t + 1 < t1) pre = ff_fetch(Wd, org, t + 1);
    __syncthreads();
    ff_tile(sW[cb], sOrg[cb], sT, aR, aI, aIn, rw, lane, gR, gI, S);
    ff_accum(gR, gI, S, acc);
  }
  // sum over the 16 column blocks (lanes sharing lane / 16), fixed pattern
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int qc = 0; qc < FF_QC; ++qc) {
      double re = acc[r][qc].re, im = acc[r][qc].im;
#pragma unroll
      for (int m = 8; m >= 1; m >>= 1) {
        re += __shfl_xor(re, m, 64);
        im += __shfl_xor(im, m, 64);
      }
      acc[r][qc] = mk(re, im);
    }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int d = dbase + (lane >> 4) + 4 * r;
      if (d >= nd) continue;
#pragma unroll
      for (int qc = 0; qc < FF_QC; ++qc) {
        const int q = qc / 3, c = qc % 3;
        if (q < nq) part[(((int64_t)blockIdx.y * nq + q) * nd + d) * 3 + c] = acc[r][qc];
      }
    }
  }
}

__global__ void k_farfield_project(const c64* __restrict__ part, int ksplit, int nr, int nd,
                                   const double* __restrict__ dirs, double scale,
                                   c64* __restrict__ F) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nr * nd) return;
  const int q = e / nd, d = e % nd;
  c64 v[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  for (int k = 0; k < ksplit; ++k)
    for (int c = 0; c < 3; ++c) v[c] = v[c] + part[(((int64_t)k * nr + q) * nd + d) * 3 + c];
  const double* D = dirs + d * 9;
  c64 ft = mk(0.0, 0.0), fp = mk(0.0, 0.0);
  for (int c = 0; c < 3; ++c) {
    ft = ft + D[3 + c] * v[c];
    fp = fp + D[6 + c] * v[c];
  }
  F[(int64_t)e * 2 + 0] = scale * ft;
  F[(int64_t)e * 2 + 1] = scale * fp;
}

static int far_split(int ntiles, int nd) {
  if (ntiles <= 0) return 0;
  const int dblocks = (nd + FF_DIRS - 1) / FF_DIRS;
  const int want = std::max(1, 1024 / dblocks);
  const int ks = std::min(ntiles, want);
  const int tps = (ntiles + ks - 1) / ks;
  return (ntiles + tps - 1) / tps;
}

int far_split_total(const FarBlocks& fb, int nd) {
  int ks = 0;
  for (const FarGroup& gr : fb.groups) ks += far_split(gr.ntiles, nd);
  return ks;
}

size_t far_pack_elems(int ntiles) { return (size_t)ntiles * FF_TILE; }

hipError_t launch_farfield_mfma(const c64* w, const int64_t* roff_host, int nr, int nb,
                                const FarBlocks& fb, const int* blk_vi, const int* blk_org,
                                const double* dirs, int nd, double k0, double h,
                                const double* origin, c64* Wd, c64* part, c64* F,
                                hipStream_t s) {
  const int ntiles = fb.ntiles;
  const int kst = far_split_total(fb, nd);
  FfGeom fg;
  fg.k0 = k0;
  fg.h = h;
  fg.o[0] = origin[0];
  fg.o[1] = origin[1];
  fg.o[2] = origin[2];
  const double scale = k0 * k0 * h * h * h / (4.0 * M_PI);
  for (int q0 = 0; q0 < nr; q0 += FF_RB) {
    const int nq = std::min(FF_RB, nr - q0);
    RoffArg ro;
    for (int q = 0; q < FF_RB; ++q) ro.r[q] = q < nq ? roff_host[q0 + q] : 0;
    const int64_t tot = (int64_t)ntiles * FF_TILE;
    k_ff_pack<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(w, ro, nq, nb, blk_vi, ntiles, Wd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one launch per block shape; each writes its own range of K-split partials
    int ks0 = 0;
    for (const FarGroup& gr : fb.groups) {
      const int ks = far_split(gr.ntiles, nd);
      if (ks == 0) continue;
      const int tps = (gr.ntiles + ks - 1) / ks;
      fg.bx = gr.shape[0];
      fg.by = gr.shape[1];
      dim3 grid((nd + FF_DIRS - 1) / FF_DIRS, ks);
      k_ff_mfma<<<grid, FF_DIRS * 4, 0, s>>>(
          Wd + (int64_t)gr.tile0 * FF_TILE, (const int4*)blk_org + (int64_t)gr.tile0 * FF_TB,
          gr.ntiles, tps, dirs, nd, fg, nq, part + (int64_t)ks0 * nq * nd * 3);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      ks0 += ks;
    }
    k_farfield_project<<<(nq * nd + 255) / 256, 256, 0, s>>>(part, kst, nq, nd, dirs, scale,
                                                              F + (int64_t)q0 * nd * 2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vie
