// Learned warm start: 3x3x3 convolutions as implicit GEMMs on bf16 MFMA
// (gfx950's v_mfma_f32_16x16x32_bf16, fp32 accumulation; the 16-deep
// v_mfma_f32_16x16x16_bf16 where a reduction step has only 16 channels), with
// training kernels.
//
// Convolution (forward and backward-data): a workgroup of 4 waves computes
// an 8x8x4 voxel tile (256 GEMM rows) x Cout, K = 27 taps x Cin.  The halo
// tile (10x10x6 voxels, channels-last, padded channel stride) and the whole
// weight tensor sit in LDS; blocks are persistent over tiles so the weights
// are loaded once per block.  Wave w owns tile z-plane w: four 16-row MFMA
// tiles (two y-rows of 8 x each) per output-channel tile.
// Weight gradient: rows = Cout, columns = (tap, Cin), reduction over the
// tile voxels; activations and gradients are staged channels-first in LDS so
// that four consecutive voxels form one operand quad.  Per-block partials are
// summed in fixed order by a second kernel (deterministic).
#include <math.h>
#include <string.h>

#include "cnn.h"

namespace vie {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// One 16x16 output tile += A (16 x K) B (K x 16) over K = 32 (or 16): lane l
// holds row / column l % 16 and the K slice 8 (l / 16) .. + 7 (4 (l / 16) .. +
// 3) of its operands, and receives D[4 (l / 16) + i][l % 16], i = 0..3.  Only
// the pairing of A and B slices matters for the sum, so any fixed K order
// that both operands share gives the same product.
__device__ __forceinline__ v4f mfma32(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16raw f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (bf16raw)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16raw h) { return __uint_as_float(((uint32_t)h) << 16); }

CnnLayerOffsets cnn_offsets() {
  CnnLayerOffsets o;
  int64_t at = 0;
  for (int l = 0; l < kCnnLayers; ++l) {
    o.w[l] = at;
    at += 27 * (int64_t)kCnnCh[l] * kCnnCh[l + 1];
    o.b[l] = at;
    at += kCnnCh[l + 1];
  }
  o.total = at;
  return o;
}

constexpr int TX = 8, TY = 8, TZ = 4;  // weight-gradient tile (256 voxels)
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int HV = HX * HY * HZ;
// Convolution tile: 8 x 8 x FZ voxels, one z-plane per wave of an
// 8-wave workgroup (two waves per SIMD).
constexpr int FZ = 8, FNT = 64 * FZ;
constexpr int HVF = HX * HY * (FZ + 2);

struct ConvDims {
  int d0, d1, d2, tx, ty, tz, ntiles;
};

// Tiles of tx x ty x tz voxels (tz = TZ for the weight gradient, FZ for the
// convolutions) covering the box.
static ConvDims conv_dims(const int d[3], int tdz) {
  ConvDims c;
  c.d0 = d[0];
  c.d1 = d[1];
  c.d2 = d[2];
  c.tx = (d[0] + TX - 1) / TX;
  c.ty = (d[1] + TY - 1) / TY;
  c.tz = (d[2] + tdz - 1) / tdz;
  c.ntiles = c.tx * c.ty * c.tz;
  return c;
}

// MODE 0: + bias, ReLU -> bf16; MODE 1: + bias -> fp32; MODE 2: * (ref > 0) -> bf16
// Persistent workgroups: the weights are staged once; every tile's halo is
// fetched into registers while the previous tile's MFMAs run, then stored to
// LDS between two barriers.
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(FNT) void k_conv3d(const bf16raw* __restrict__ in,
                                                const bf16raw* __restrict__ w,
                                                const float* __restrict__ bias,
                                                bf16raw* __restrict__ outb,
                                                float* __restrict__ outf,
                                                const bf16raw* __restrict__ ref, ConvDims cd) {
  // 32-deep MFMA steps when the channels allow; padded channel stride keeps
  // every operand slice 16-byte aligned (8-byte for the 16-deep form)
  constexpr bool X32 = CIN % 32 == 0;
  constexpr int KS = X32 ? 32 : 16;
  constexpr int CP = X32 ? CIN + 8 : CIN + 4;
  constexpr int NCT = COUT / 16;
  constexpr int NQ = HVF * (CIN / 4);  // 8-byte halo items
  constexpr int PF = (NQ + FNT - 1) / FNT;
  __shared__ __align__(16) bf16raw s_in[HVF * CP];
  __shared__ __align__(16) bf16raw s_w[27 * COUT * CP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kq = lane >> 4;
  for (int i = tid; i < 27 * COUT * (CIN / 4); i += FNT) {
    const int c4 = i % (CIN / 4), row = i / (CIN / 4);
    *(uint2*)&s_w[row * CP + 4 * c4] = *(const uint2*)&w[(size_t)row * CIN + 4 * c4];
  }
  uint2 pre[PF];
  auto fetch = [&](int tile) {
    const int tx = tile % cd.tx, ty = (tile / cd.tx) % cd.ty, tz = tile / (cd.tx * cd.ty);
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * FZ;
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int i = tid + p * FNT;
      const int c4 = i % (CIN / 4), v = i / (CIN / 4);
      const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
      const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
      pre[p] = make_uint2(0u, 0u);
      if (i < NQ && gx >= 0 && gx < cd.d0 && gy >= 0 && gy < cd.d1 && gz >= 0 && gz < cd.d2)
        pre[p] = *(const uint2*)&in[((size_t)(gz * cd.d1 + gy) * cd.d0 + gx) * CIN + 4 * c4];
    }
  };
  if ((int)blockIdx.x < cd.ntiles) fetch(blockIdx.x);
  for (int tile = blockIdx.x; tile < cd.ntiles; tile += gridDim.x) {
    const int tx = tile % cd.tx, ty = (tile / cd.tx) % cd.ty, tz = tile / (cd.tx * cd.ty);
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * FZ;
    __syncthreads();  // the previous tile's operand reads are done
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int i = tid + p * FNT;
      if (i < NQ) {
        const int c4 = i % (CIN / 4), v = i / (CIN / 4);
        *(uint2*)&s_in[v * CP + 4 * c4] = pre[p];
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < cd.ntiles) fetch(tile + gridDim.x);
    v4f acc[4][NCT];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[rt][ct] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
    for (int tap = 0; tap < 27; ++tap) {
      const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
#pragma unroll
      for (int kc = 0; kc < CIN / KS; ++kc) {
        const int ko = KS * kc + (KS / 4) * kq;  // this lane's K slice
        if constexpr (X32) {
          v8bf a[4], b[NCT];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            const int ly = 2 * rt + (r >> 3), lx = r & 7;
            const int hv = ((wave + 1 + dz) * HY + (ly + 1 + dy)) * HX + (lx + 1 + dx);
            a[rt] = *(const v8bf*)&s_in[hv * CP + ko];
          }
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct)
            b[ct] = *(const v8bf*)&s_w[(tap * COUT + ct * 16 + r) * CP + ko];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) acc[rt][ct] = mfma32(a[rt], b[ct], acc[rt][ct]);
        } else {
          v4s a[4], b[NCT];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            const int ly = 2 * rt + (r >> 3), lx = r & 7;
            const int hv = ((wave + 1 + dz) * HY + (ly + 1 + dy)) * HX + (lx + 1 + dx);
            a[rt] = *(const v4s*)&s_in[hv * CP + ko];
          }
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct)
            b[ct] = *(const v4s*)&s_w[(tap * COUT + ct * 16 + r) * CP + ko];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) acc[rt][ct] = mfma16(a[rt], b[ct], acc[rt][ct]);
        }
      }
    }
    // lane holds D[row = 4 kq + i][col = r]
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 4 * kq + i;
          const int gx = x0 + (row & 7), gy = y0 + 2 * rt + (row >> 3), gz = z0 + wave;
          if (gx < cd.d0 && gy < cd.d1 && gz < cd.d2) {
            const size_t vox = (size_t)(gz * cd.d1 + gy) * cd.d0 + gx;
            const int co = ct * 16 + r;
            float val = acc[rt][ct][i];
            if (MODE == 0) {
              val += bias[co];
              outb[vox * COUT + co] = f2bf(val > 0.f ? val : 0.f);
            } else if (MODE == 1) {
              outf[vox * COUT + co] = val + bias[co];
            } else {
              outb[vox * COUT + co] = f2bf(bf2f(ref[vox * COUT + co]) > 0.f ? val : 0.f);
            }
          }
        }
  }
}

// dW[tap][co][ci] = sum_m in[m + tap][ci] g[m][co];  db[co] = sum_m g[m][co]
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv3d_wgrad(const bf16raw* __restrict__ in,
                                                      const bf16raw* __restrict__ g,
                                                      float* __restrict__ part, ConvDims cd) {
  constexpr int NCOL = 27 * CIN / 16;
  constexpr int NRT = COUT / 16;
  constexpr int CPW = (NCOL + 3) / 4;
  constexpr int HVP = HV + 4;
  constexpr int MP = 256 + 8;  // 16-byte aligned gradient rows
  constexpr int NW = 27 * COUT * CIN;
  __shared__ __align__(16) bf16raw s_inT[CIN * HVP];
  __shared__ __align__(16) bf16raw s_gT[COUT * MP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kq = lane >> 4;
  v4f acc[CPW][NRT];
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) acc[j][rt] = v4f{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int tile = blockIdx.x; tile < cd.ntiles; tile += gridDim.x) {
    const int tx = tile % cd.tx, ty = (tile / cd.tx) % cd.ty, tz = tile / (cd.tx * cd.ty);
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    __syncthreads();
    for (int i = tid; i < HV * (CIN / 4); i += 256) {
      const int c4 = i % (CIN / 4), v = i / (CIN / 4);
      const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
      const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
      uint2 val = make_uint2(0u, 0u);
      if (gx >= 0 && gx < cd.d0 && gy >= 0 && gy < cd.d1 && gz >= 0 && gz < cd.d2)
        val = *(const uint2*)&in[((size_t)(gz * cd.d1 + gy) * cd.d0 + gx) * CIN + 4 * c4];
      s_inT[(4 * c4 + 0) * HVP + v] = (bf16raw)(val.x & 0xFFFFu);
      s_inT[(4 * c4 + 1) * HVP + v] = (bf16raw)(val.x >> 16);
      s_inT[(4 * c4 + 2) * HVP + v] = (bf16raw)(val.y & 0xFFFFu);
      s_inT[(4 * c4 + 3) * HVP + v] = (bf16raw)(val.y >> 16);
    }
    for (int i = tid; i < 256 * (COUT / 4); i += 256) {
      const int c4 = i % (COUT / 4), m = i / (COUT / 4);
      const int gx = x0 + (m & 7), gy = y0 + ((m >> 3) & 7), gz = z0 + (m >> 6);
      uint2 val = make_uint2(0u, 0u);
      if (gx < cd.d0 && gy < cd.d1 && gz < cd.d2)
        val = *(const uint2*)&g[((size_t)(gz * cd.d1 + gy) * cd.d0 + gx) * COUT + 4 * c4];
      s_gT[(4 * c4 + 0) * MP + m] = (bf16raw)(val.x & 0xFFFFu);
      s_gT[(4 * c4 + 1) * MP + m] = (bf16raw)(val.x >> 16);
      s_gT[(4 * c4 + 2) * MP + m] = (bf16raw)(val.y & 0xFFFFu);
      s_gT[(4 * c4 + 3) * MP + m] = (bf16raw)(val.y >> 16);
    }
    __syncthreads();
    if (tid < COUT) {
      for (int m = 0; m < 256; ++m) bsum += bf2f(s_gT[tid * MP + m]);
    }
    for (int ks = 0; ks < 8; ++ks) {
      const int m0 = 32 * ks + 8 * kq;  // this lane's 8 voxels m0..m0+7: one x-row
      const int lz = m0 >> 6, ly = (m0 >> 3) & 7;
      v8bf a[NRT];
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt) a[rt] = *(const v8bf*)&s_gT[(rt * 16 + r) * MP + m0];
#pragma unroll
      for (int j = 0; j < CPW; ++j) {
        const int c = wave + 4 * j;
        if (c < NCOL) {
          const int col = 16 * c + r;
          const int tap = col / CIN, ci = col % CIN;
          const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
          const int hv = ((lz + 1 + dz) * HY + (ly + 1 + dy)) * HX + (1 + dx);
          const bf16raw* p = &s_inT[ci * HVP + hv];
          v8bf b;
#pragma unroll
          for (int e = 0; e < 8; ++e) b[e] = __builtin_bit_cast(__bf16, p[e]);
#pragma unroll
          for (int rt = 0; rt < NRT; ++rt) acc[j][rt] = mfma32(a[rt], b, acc[j][rt]);
        }
      }
    }
  }
  float* pb = part + (size_t)blockIdx.x * (NW + COUT);
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = wave + 4 * j;
    if (c < NCOL) {
      const int col = 16 * c + r;
      const int tap = col / CIN, ci = col % CIN;
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int co = rt * 16 + 4 * kq + i;
          pb[((size_t)tap * COUT + co) * CIN + ci] = acc[j][rt][i];
        }
    }
  }
  if (tid < COUT) pb[NW + tid] = bsum;
}

__global__ void k_reduce_parts(const float* __restrict__ part, int nblk, int n,
                               float* __restrict__ out) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * n + j];
    out[j] = s;
  }
}

// masked relative L2 loss over outputs 0..5; mask = feature channel 0 > 0
__global__ __launch_bounds__(256) void k_loss_partial(const float* __restrict__ out,
                                                      const float* __restrict__ tgt,
                                                      const bf16raw* __restrict__ feat,
                                                      size_t nvox, float* __restrict__ part) {
  __shared__ float sn[256], sd[256];
  float num = 0.f, den = 0.f;
  for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < nvox; v += (size_t)gridDim.x * 256) {
    if (bf2f(feat[v * kCnnIn]) > 0.f) {
#pragma unroll
      for (int c = 0; c < kCnnOut; ++c) {
        const float t = tgt[v * kCnnOut + c], d = out[v * 16 + c] - t;
        num += d * d;
        den += t * t;
      }
    }
  }
  sn[threadIdx.x] = num;
  sd[threadIdx.x] = den;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sn[threadIdx.x] += sn[threadIdx.x + o];
      sd[threadIdx.x] += sd[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * 2] = sn[0];
    part[blockIdx.x * 2 + 1] = sd[0];
  }
}

__global__ void k_loss_final(const float* __restrict__ part, int nblk, float* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float n = 0.f, d = 0.f;
    for (int b = 0; b < nblk; ++b) {
      n += part[2 * b];
      d += part[2 * b + 1];
    }
    loss[0] = n;
    loss[1] = d;
  }
}

__global__ __launch_bounds__(256) void k_loss_grad(const float* __restrict__ out,
                                                   const float* __restrict__ tgt,
                                                   const bf16raw* __restrict__ feat,
                                                   const float* __restrict__ loss, size_t nvox,
                                                   bf16raw* __restrict__ g) {
  const float inv = loss[1] > 0.f ? 2.f / loss[1] : 0.f;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nvox * 16;
       e += (size_t)gridDim.x * 256) {
    const size_t v = e / 16;
    const int c = (int)(e % 16);
    float val = 0.f;
    if (c < kCnnOut && bf2f(feat[v * kCnnIn]) > 0.f) val = inv * (out[e] - tgt[v * kCnnOut + c]);
    g[e] = f2bf(val);
  }
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  }
}

// bf16 weight copies: forward [27][Cout][Cin]; backward-data [27][Cin][Cout]
// with tap t' = 26 - t (the adjoint of a same-padded convolution).
__global__ void k_refresh_bf16(const float* __restrict__ p, bf16raw* __restrict__ wf,
                               bf16raw* __restrict__ wb, CnnLayerOffsets off) {
  for (int l = 0; l < kCnnLayers; ++l) {
    const int ci_n = kCnnCh[l], co_n = kCnnCh[l + 1];
    const int64_t n = 27 * (int64_t)ci_n * co_n;
    const float* W = p + off.w[l];
    // bf16 weights are packed without the biases: layer offset in bf16 arrays
    int64_t wo = 0;
    for (int q = 0; q < l; ++q) wo += 27 * (int64_t)kCnnCh[q] * kCnnCh[q + 1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
      const int tap = (int)(i / ((int64_t)co_n * ci_n));
      const int co = (int)((i / ci_n) % co_n), ci = (int)(i % ci_n);
      const bf16raw h = f2bf(W[i]);
      wf[wo + i] = h;
      wb[wo + ((int64_t)(26 - tap) * ci_n + ci) * co_n + co] = h;
    }
  }
}

// ------------------------------------------------- features / target / gather
__device__ __forceinline__ size_t box_index(int lin, const int N[3], const int lo[3],
                                            const int d[3]) {
  const int i = lin % N[0], j = (lin / N[0]) % N[1], l = lin / (N[0] * N[1]);
  return ((size_t)(l - lo[2]) * d[1] + (j - lo[1])) * d[0] + (i - lo[0]);
}

struct Box {
  int d[3], lo[3], N[3];
};

struct KrylovIn {
  const c64* v[kCnnKrylov];
  double inv[kCnnKrylov];
};

__global__ void k_cnn_features(bf16raw* __restrict__ feat, Box bx, const int* __restrict__ vox,
                               const double* __restrict__ chic, int nb, KrylovIn kin) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += gridDim.x * blockDim.x) {
    const size_t v = box_index(vox[k], bx.N, bx.lo, bx.d);
    bf16raw* f = feat + v * kCnnIn;
    f[0] = f2bf((float)(chic[k] * 0.25));
#pragma unroll
    for (int q = 0; q < kCnnKrylov; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const c64 bv = kin.v[q][(size_t)c * nb + k];
        f[1 + 6 * q + 2 * c] = f2bf((float)(bv.re * kin.inv[q]));
        f[2 + 6 * q + 2 * c] = f2bf((float)(bv.im * kin.inv[q]));
      }
  }
}

__global__ void k_cnn_target(float* __restrict__ tgt, Box bx, const int* __restrict__ vox, int nb,
                             const c64* __restrict__ w, double inv_s) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += gridDim.x * blockDim.x) {
    const size_t v = box_index(vox[k], bx.N, bx.lo, bx.d);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const c64 wv = w[(size_t)c * nb + k];
      tgt[v * kCnnOut + 2 * c] = (float)(wv.re * inv_s);
      tgt[v * kCnnOut + 2 * c + 1] = (float)(wv.im * inv_s);
    }
  }
}

__global__ void k_cnn_gather(c64* __restrict__ x, const float* __restrict__ out, Box bx,
                             const int* __restrict__ vox, int nb, double s) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += gridDim.x * blockDim.x) {
    const size_t v = box_index(vox[k], bx.N, bx.lo, bx.d);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      x[(size_t)c * nb + k] = mk(s * out[v * 16 + 2 * c], s * out[v * 16 + 2 * c + 1]);
  }
}

static Box mkbox(const int d[3], const int lo[3], const int N[3]) {
  Box b;
  for (int a = 0; a < 3; ++a) {
    b.d[a] = d[a];
    b.lo[a] = lo[a];
    b.N[a] = N[a];
  }
  return b;
}

static int grid_for(int64_t n, int per = 256) {
  int64_t b = (n + per - 1) / per;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_cnn_features(bf16raw* feat, const int d[3], const int lo[3], const int N[3],
                               const int* vox, const double* chic, int nb,
                               const c64* const vec[kCnnKrylov], const double inv[kCnnKrylov],
                               hipStream_t st) {
  const size_t nv = (size_t)d[0] * d[1] * d[2];
  hipError_t e = hipMemsetAsync(feat, 0, nv * kCnnIn * sizeof(bf16raw), st);
  if (e != hipSuccess || nb == 0) return e;
  KrylovIn kin;
  for (int q = 0; q < kCnnKrylov; ++q) {
    kin.v[q] = vec[q];
    kin.inv[q] = inv[q];
  }
  k_cnn_features<<<grid_for(nb), 256, 0, st>>>(feat, mkbox(d, lo, N), vox, chic, nb, kin);
  return hipGetLastError();
}

hipError_t launch_cnn_target(float* tgt, const int d[3], const int lo[3], const int N[3],
                             const int* vox, int nb, const c64* w, double s, hipStream_t st) {
  const size_t nv = (size_t)d[0] * d[1] * d[2];
  hipError_t e = hipMemsetAsync(tgt, 0, nv * kCnnOut * sizeof(float), st);
  if (e != hipSuccess || nb == 0) return e;
  k_cnn_target<<<grid_for(nb), 256, 0, st>>>(tgt, mkbox(d, lo, N), vox, nb, w,
                                             s > 0 ? 1.0 / s : 0.0);
  return hipGetLastError();
}

hipError_t launch_cnn_gather(c64* x, const float* out, const int d[3], const int lo[3],
                             const int N[3], const int* vox, int nb, double s, hipStream_t st) {
  if (nb == 0) return hipSuccess;
  k_cnn_gather<<<grid_for(nb), 256, 0, st>>>(x, out, mkbox(d, lo, N), vox, nb, s);
  return hipGetLastError();
}

// ------------------------------------------------------------------ host
static int64_t bf16_weights_total() {
  int64_t n = 0;
  for (int l = 0; l < kCnnLayers; ++l) n += 27 * (int64_t)kCnnCh[l] * kCnnCh[l + 1];
  return n;
}
static int64_t bf16_weight_offset(int l) {
  int64_t n = 0;
  for (int q = 0; q < l; ++q) n += 27 * (int64_t)kCnnCh[q] * kCnnCh[q + 1];
  return n;
}

hipError_t cnn_alloc(Cnn& c) {
  c.off = cnn_offsets();
  const size_t np = (size_t)c.off.total;
  hipError_t e;
  if ((e = hipMalloc(&c.p, np * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&c.m, np * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&c.v, np * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&c.g, np * 4)) != hipSuccess) return e;
  if ((e = hipMemset(c.m, 0, np * 4)) != hipSuccess) return e;
  if ((e = hipMemset(c.v, 0, np * 4)) != hipSuccess) return e;
  const size_t nw = (size_t)bf16_weights_total();
  if ((e = hipMalloc(&c.wf, nw * 2)) != hipSuccess) return e;
  if ((e = hipMalloc(&c.wb, nw * 2)) != hipSuccess) return e;
  if ((e = hipMalloc(&c.loss, 4 * 4096 * 2)) != hipSuccess) return e;
  if ((e = hipHostMalloc(&c.hostloss, 2 * sizeof(float))) != hipSuccess) return e;
  return hipSuccess;
}

void cnn_free(Cnn& c) {
  void* ps[] = {c.p, c.m, c.v, c.g, c.wf, c.wb, c.out, c.wpart, c.loss, c.gbuf[0], c.gbuf[1],
                c.act[1], c.act[2], c.act[3]};
  for (void* q : ps)
    if (q) (void)hipFree(q);
  if (c.hostloss) (void)hipHostFree(c.hostloss);
  c = Cnn();
}

// persistent grids: convolutions one 149 KB-LDS workgroup per CU, weight
// gradients two 4-wave workgroups per CU (per-block partials: kMaxConvBlocks)
static constexpr int kConvBlocks = 256;
static constexpr int kMaxConvBlocks = 512;

hipError_t cnn_ensure_ws(Cnn& c, size_t vox) {
  if (vox <= c.ws_vox) return hipSuccess;
  void* old[] = {c.out, c.gbuf[0], c.gbuf[1], c.act[1], c.act[2], c.act[3], c.wpart};
  for (void* q : old)
    if (q) (void)hipFree(q);
  c.out = nullptr;
  c.gbuf[0] = c.gbuf[1] = c.act[1] = c.act[2] = c.act[3] = nullptr;
  c.wpart = nullptr;
  c.ws_vox = 0;
  hipError_t e;
  if ((e = hipMalloc(&c.out, vox * 16 * 4)) != hipSuccess) return e;
  for (int k = 0; k < 2; ++k)
    if ((e = hipMalloc(&c.gbuf[k], vox * 32 * 2)) != hipSuccess) return e;
  for (int l = 1; l < kCnnLayers; ++l)
    if ((e = hipMalloc(&c.act[l], vox * kCnnCh[l] * 2)) != hipSuccess) return e;
  const size_t maxlayer = 27 * 32 * 32 + 32;
  if ((e = hipMalloc(&c.wpart, (size_t)kMaxConvBlocks * maxlayer * 4)) != hipSuccess) return e;
  c.ws_vox = vox;
  return hipSuccess;
}

hipError_t cnn_refresh_bf16(Cnn& c, hipStream_t s) {
  k_refresh_bf16<<<256, 256, 0, s>>>(c.p, c.wf, c.wb, c.off);
  return hipGetLastError();
}

template <int CIN, int COUT, int MODE>
static void conv(const ConvDims& cd, const bf16raw* in, const bf16raw* w, const float* bias,
                 bf16raw* ob, float* of, const bf16raw* ref, hipStream_t s) {
  const int grid = cd.ntiles < kConvBlocks ? cd.ntiles : kConvBlocks;
  k_conv3d<CIN, COUT, MODE><<<grid, FNT, 0, s>>>(in, w, bias, ob, of, ref, cd);
}

template <int CIN, int COUT>
static void wgrad(const ConvDims& cd, const bf16raw* in, const bf16raw* g, float* part,
                  float* out, hipStream_t s) {
  const int grid = cd.ntiles < kMaxConvBlocks ? cd.ntiles : kMaxConvBlocks;
  k_conv3d_wgrad<CIN, COUT><<<grid, 256, 0, s>>>(in, g, part, cd);
  const int n = 27 * CIN * COUT + COUT;
  k_reduce_parts<<<(n + 255) / 256, 256, 0, s>>>(part, grid, n, out);
}

hipError_t cnn_forward(Cnn& c, const int d[3], const bf16raw* feat, float* out, hipStream_t s) {
  const ConvDims cd = conv_dims(d, FZ);
  hipError_t e = cnn_ensure_ws(c, (size_t)d[0] * d[1] * d[2]);
  if (e != hipSuccess) return e;
  c.act[0] = const_cast<bf16raw*>(feat);
  conv<32, 32, 0>(cd, feat, c.wf + bf16_weight_offset(0), c.p + c.off.b[0], c.act[1], nullptr,
                  nullptr, s);
  conv<32, 32, 0>(cd, c.act[1], c.wf + bf16_weight_offset(1), c.p + c.off.b[1], c.act[2],
                  nullptr, nullptr, s);
  conv<32, 32, 0>(cd, c.act[2], c.wf + bf16_weight_offset(2), c.p + c.off.b[2], c.act[3],
                  nullptr, nullptr, s);
  conv<32, 16, 1>(cd, c.act[3], c.wf + bf16_weight_offset(3), c.p + c.off.b[3], nullptr,
                  out ? out : c.out, nullptr, s);
  return hipGetLastError();
}

hipError_t cnn_backward(Cnn& c, const int d[3], const float* target, float* loss_host,
                        hipStream_t s) {
  const ConvDims cd = conv_dims(d, FZ), cw = conv_dims(d, TZ);
  const size_t nv = (size_t)d[0] * d[1] * d[2];
  const int lb = grid_for((int64_t)nv, 256) < 1024 ? grid_for((int64_t)nv, 256) : 1024;
  k_loss_partial<<<lb, 256, 0, s>>>(c.out, target, c.act[0], nv, c.loss + 2);
  k_loss_final<<<1, 64, 0, s>>>(c.loss + 2, lb, c.loss);
  k_loss_grad<<<grid_for((int64_t)nv * 16), 256, 0, s>>>(c.out, target, c.act[0], c.loss, nv,
                                                         c.gbuf[0]);
  // layer 4 (32 -> 16): weight gradient, then data gradient masked by ReLU'
  wgrad<32, 16>(cw, c.act[3], c.gbuf[0], c.wpart, c.g + c.off.w[3], s);
  conv<16, 32, 2>(cd, c.gbuf[0], c.wb + bf16_weight_offset(3), nullptr, c.gbuf[1], nullptr,
                  c.act[3], s);
  wgrad<32, 32>(cw, c.act[2], c.gbuf[1], c.wpart, c.g + c.off.w[2], s);
  conv<32, 32, 2>(cd, c.gbuf[1], c.wb + bf16_weight_offset(2), nullptr, c.gbuf[0], nullptr,
                  c.act[2], s);
  wgrad<32, 32>(cw, c.act[1], c.gbuf[0], c.wpart, c.g + c.off.w[1], s);
  conv<32, 32, 2>(cd, c.gbuf[0], c.wb + bf16_weight_offset(1), nullptr, c.gbuf[1], nullptr,
                  c.act[1], s);
  wgrad<32, 32>(cw, c.act[0], c.gbuf[1], c.wpart, c.g + c.off.w[0], s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (loss_host) {
    if ((e = hipMemcpyAsync(c.hostloss, c.loss, 2 * sizeof(float), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *loss_host = c.hostloss[1] > 0 ? c.hostloss[0] / c.hostloss[1] : 0.f;
  }
  return hipSuccess;
}

hipError_t cnn_adam(Cnn& c, float lr, hipStream_t s) {
  c.step += 1;
  const float c1 = 1.f - powf(0.9f, (float)c.step), c2 = 1.f - powf(0.999f, (float)c.step);
  k_adam<<<grid_for(c.off.total), 256, 0, s>>>(c.p, c.m, c.v, c.g, c.off.total, lr, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return cnn_refresh_bf16(c, s);
}

}  // namespace vie
