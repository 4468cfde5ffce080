// Spectrum of the discrete Green operator (setup, FP64).
//
// The off-diagonal blocks k0^2 h^3 G(r_m - r_n) depend only on the integer
// displacement d = (m - n), so the product is a 3-D discrete convolution
// (Sec. II-C: uniform voxelisation gives a convolution structure that the
// FFT accelerates).  Embedding it in a circulant of length P >= 2N - 1 per
// axis: sample d in [-(N-1), N-1] at index d mod P, zero elsewhere; the
// diagonal (d = 0) holds the self term s on xx, yy, zz.  The dyadic Green's
// function is (I + grad grad / k0^2) e^{i k0 R} / (4 pi R), differentiated in
// closed form.  Each component is even or odd along each axis, so its DFT
// has the same parity and only the octant [0, P/2]^3 is stored.
#include "kernels.h"

namespace vie {

__global__ void k_green_sample(c64* __restrict__ work, GroupGeom g, int ab, double h, double k0,
                               double self_re, double self_im) {
  const int64_t M = (int64_t)g.P[0] * g.P[1] * g.P[2];
  static const int A_[6] = {0, 0, 0, 1, 1, 2};
  static const int B_[6] = {0, 1, 2, 1, 2, 2};
  const int ca = A_[ab], cb = B_[ab];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M;
       e += (int64_t)gridDim.x * blockDim.x) {
    int idx[3];
    idx[0] = (int)(e % g.P[0]);
    idx[1] = (int)((e / g.P[0]) % g.P[1]);
    idx[2] = (int)(e / ((int64_t)g.P[0] * g.P[1]));
    int d[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
      if (idx[a] <= g.N[a] - 1)
        d[a] = idx[a];
      else if (idx[a] >= g.P[a] - (g.N[a] - 1))
        d[a] = idx[a] - g.P[a];
      else
        ok = false;
    }
    c64 val = mk(0.0, 0.0);
    if (ok) {
      if (d[0] == 0 && d[1] == 0 && d[2] == 0) {
        if (ca == cb) val = mk(self_re, self_im);
      } else {
        const double R[3] = {h * d[0], h * d[1], h * d[2]};
        const double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
        const double kr = k0 * r;
        double sn, cs;
        sincos(kr, &sn, &cs);
        const double inv = 1.0 / (4.0 * M_PI * r);
        const c64 gg = mk(cs * inv, sn * inv);  // e^{ikr} / (4 pi r)
        const double ikr = 1.0 / kr, ikr2 = ikr * ikr;
        const c64 A = mk(1.0 - ikr2, ikr);              // 1 + i/(kr) - 1/(kr)^2
        const c64 B = mk(3.0 * ikr2 - 1.0, -3.0 * ikr);  // 3/(kr)^2 - 3i/(kr) - 1
        const double uu = (R[ca] / r) * (R[cb] / r);
        c64 t = mk(B.re * uu, B.im * uu);
        if (ca == cb) t = t + A;
        val = (k0 * k0 * h * h * h) * (gg * t);
      }
    }
    work[e] = val;
  }
}

// spec[y][z][x][ab] over the octant: the six components of a frequency are
// one contiguous record (the z pass reads it with wide loads), scaled by 1/M.
__global__ void k_octant(const c64* __restrict__ work, c64* __restrict__ s64,
                         c32* __restrict__ s32, GroupGeom g, int ab) {
  const int64_t oct = (int64_t)g.Q[0] * g.Q[1] * g.Q[2];
  const double inv = 1.0 / ((double)g.P[0] * g.P[1] * g.P[2]);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < oct;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(e % g.Q[0]);
    const int y = (int)((e / g.Q[0]) % g.Q[1]);
    const int z = (int)(e / ((int64_t)g.Q[0] * g.Q[1]));
    const c64 v = work[((int64_t)z * g.P[1] + y) * g.P[0] + x];
    const c64 w = mk(v.re * inv, v.im * inv);
    const int64_t o = (((int64_t)y * g.Q[2] + z) * g.Q[0] + x) * 6 + ab;
    s64[o] = w;
    if (s32) s32[o] = mk((float)w.re, (float)w.im);
  }
}

static double self_term_re(double k0, double h) {
  const double a = h * cbrt(3.0 / (4.0 * M_PI));
  const double x = k0 * a;
  return -1.0 / 3.0 + (2.0 / 3.0) * (cos(x) + x * sin(x) - 1.0);
}
static double self_term_im(double k0, double h) { return k0 * k0 * k0 * h * h * h / (6.0 * M_PI); }

hipError_t launch_green_sample(c64* work, const GroupGeom& g, int ab, double h, double k0,
                               hipStream_t s) {
  k_green_sample<<<2048, 256, 0, s>>>(work, g, ab, h, k0, self_term_re(k0, h),
                                      self_term_im(k0, h));
  return hipGetLastError();
}

hipError_t launch_octant(const c64* work, c64* s64, c32* s32, const GroupGeom& g, int ab,
                         hipStream_t s) {
  k_octant<<<1024, 256, 0, s>>>(work, s64, s32, g, ab);
  return hipGetLastError();
}

}  // namespace vie
