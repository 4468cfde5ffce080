// Far-field amplitude (eq. 25 with the radiation-zone Green's function):
//   F(r) = k0^2 h^3 / (4 pi) (I - r r) sum_n w_n exp(-i k0 r . r_n),
// reported as (F_theta, F_phi) = (theta-hat . F, phi-hat . F).
//
// Contraction over the body voxels n, split across workgroups (K-split) and
// reduced in fixed order by a second kernel that also projects onto
// theta-hat / phi-hat and applies the constant.
#include "kernels.h"

namespace vie {

static constexpr int FF_D = 64;   // directions per workgroup
static constexpr int FF_S = 4;    // voxel sub-lanes per direction
static constexpr int FF_NR = 4;   // right-hand sides per pass
static constexpr int FF_CH = 64;  // voxels staged in LDS per step

struct RoffArg {
  int64_t r[FF_NR];
};

__global__ __launch_bounds__(FF_D* FF_S) void k_farfield_sum(
    const c64* __restrict__ w, RoffArg ro, int nr, const int* __restrict__ vox, int nb,
    int chunk, const double* __restrict__ dirs, int nd, double k0, double h, double o0, double o1,
    double o2, int N1, int N2, c64* __restrict__ part) {
  __shared__ int sidx[FF_CH][3];
  __shared__ c64 sw[FF_CH][FF_NR][3];
  const int dl = threadIdx.x % FF_D, sl = threadIdx.x / FF_D;
  const int d = blockIdx.x * FF_D + dl;
  const int ks = blockIdx.y;
  const int v0 = ks * chunk, v1 = min(nb, v0 + chunk);
  double rx = 0, ry = 0, rz = 0;
  if (d < nd) {
    rx = dirs[d * 9 + 0];
    ry = dirs[d * 9 + 1];
    rz = dirs[d * 9 + 2];
  }
  const double ph0 = -k0 * (rx * o0 + ry * o1 + rz * o2);
  const double ax = -k0 * h * rx, ay = -k0 * h * ry, az = -k0 * h * rz;
  c64 acc[FF_NR][3];
#pragma unroll
  for (int q = 0; q < FF_NR; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[q][c] = mk(0.0, 0.0);
  for (int base = v0; base < v1; base += FF_CH) {
    __syncthreads();
    for (int k = threadIdx.x; k < FF_CH; k += blockDim.x) {
      const int vi = base + k;
      if (vi < v1) {
        const int lin = vox[vi];
        sidx[k][0] = lin % N1;
        sidx[k][1] = (lin / N1) % N2;
        sidx[k][2] = lin / (N1 * N2);
        for (int q = 0; q < FF_NR; ++q)
          for (int c = 0; c < 3; ++c)
            sw[k][q][c] = (q < nr) ? w[ro.r[q] + (int64_t)c * nb + vi] : mk(0.0, 0.0);
      } else {
        sidx[k][0] = sidx[k][1] = sidx[k][2] = 0;
        for (int q = 0; q < FF_NR; ++q)
          for (int c = 0; c < 3; ++c) sw[k][q][c] = mk(0.0, 0.0);
      }
    }
    __syncthreads();
    for (int k = sl; k < FF_CH; k += FF_S) {
      const double ang = ph0 + ax * sidx[k][0] + ay * sidx[k][1] + az * sidx[k][2];
      double sn, cs;
      sincos(ang, &sn, &cs);
      const c64 e = mk(cs, sn);
#pragma unroll
      for (int q = 0; q < FF_NR; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[q][c] = cfma(e, sw[k][q][c], acc[q][c]);
    }
  }
  // reduce the FF_S sub-lanes through LDS (reuse sw)
  __syncthreads();
  c64* red = &sw[0][0][0];  // FF_CH*FF_NR*3 = 768 >= FF_D*FF_S? use two rounds per q
  for (int q = 0; q < FF_NR; ++q) {
    for (int c = 0; c < 3; ++c) {
      red[threadIdx.x] = acc[q][c];
      __syncthreads();
      if (sl == 0 && d < nd && q < nr) {
        c64 s = red[dl];
        for (int u = 1; u < FF_S; ++u) s = s + red[u * FF_D + dl];
        part[(((int64_t)ks * nr + q) * nd + d) * 3 + c] = s;
      }
      __syncthreads();
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

hipError_t launch_farfield_ks(const GroupGeom& g, const c64* w, const int64_t* roff_host,
                              int nr, const int* vox, int nb, const double* dirs, int nd,
                              double k0, double h, const double* origin, c64* part, int chunk,
                              c64* F, hipStream_t s) {
  const int ks = (nb + chunk - 1) / chunk;
  for (int q0 = 0; q0 < nr; q0 += FF_NR) {
    const int nq = nr - q0 < FF_NR ? nr - q0 : FF_NR;
    RoffArg ro;
    for (int q = 0; q < FF_NR; ++q) ro.r[q] = q < nq ? roff_host[q0 + q] : 0;
    dim3 grid((nd + FF_D - 1) / FF_D, ks);
    k_farfield_sum<<<grid, FF_D * FF_S, 0, s>>>(w, ro, nq, vox, nb, chunk, dirs, nd, k0, h,
                                                origin[0], origin[1], origin[2], g.N[0], g.N[1],
                                                part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double scale = k0 * k0 * h * h * h / (4.0 * M_PI);
    k_farfield_project<<<(nq * nd + 255) / 256, 256, 0, s>>>(part, ks, nq, nd, dirs, scale,
                                                              F + (int64_t)q0 * nd * 2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vie
