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
#include <math.h>

#include <vector>

#include "green.h"

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

// Exact-cube self term: s = -1/3 + (2 k0^2 / 3) I with I the integral of
// e^{i k0 r} / (4 pi r) over the voxel (a cube of edge h about the collocation
// point).  The -1/3 is the cube's static principal value (depolarisation
// I/3, by cubic symmetry); the remainder of the dyadic kernel is integrable
// with trace 2 g.  In spherical coordinates the radial integral is
// elementary, int_0^R r e^{ikr} dr = (e^{ikR}(1 - ikR) - 1) / k^2, and the
// solid angle is covered through the six (equal) faces: on the face x = h/2,
// dOmega = (h/2) dy dz / R^3.  Gauss-Legendre on a quarter face (the
// integrand is smooth there, R >= h/2).
static void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double t = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double dt = p1 / dp;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - t);  // on [0, 1]
    w[i] = 1.0 / ((1.0 - t * t) * dp * dp);
  }
}

void cube_green_integral(double k0, double h, double* re, double* im) {
  const double c = 0.5 * h;
  std::vector<double> x, w;
  gauss_legendre01(40, x, w);
  double sr = 0.0, si = 0.0;
  for (size_t i = 0; i < x.size(); ++i)
    for (size_t j = 0; j < x.size(); ++j) {
      const double y = c * x[i], z = c * x[j];
      const double R = sqrt(c * c + y * y + z * z);
      const double t = k0 * R;
      // e^{it}(1 - it) - 1 = (t sin t - 2 sin^2(t/2)) + i (sin t - t cos t),
      // the imaginary part by its series where the difference would cancel
      const double sh = sin(0.5 * t);
      const double fr = t * sin(t) - 2.0 * sh * sh;
      double fi;
      if (t < 0.1) {
        const double t2 = t * t;
        fi = t * t2 * (1.0 / 3 - t2 * (1.0 / 30 - t2 * (1.0 / 840 - t2 * (1.0 / 45360 - t2 / 3991680))));
      } else {
        fi = sin(t) - t * cos(t);
      }
      const double wt = w[i] * w[j] * c * c * c / (R * R * R);  // quarter-face area c^2 times dOmega factor
      sr += wt * fr;
      si += wt * fi;
    }
  // six faces x four quarters, 1 / (4 pi), radial integral / k0^2
  const double f = 24.0 / (4.0 * M_PI) / (k0 * k0);
  *re = f * sr;
  *im = f * si;
}

void self_term_cube(double k0, double h, double* re, double* im) {
  double ir, ii;
  cube_green_integral(k0, h, &ir, &ii);
  *re = -1.0 / 3.0 + (2.0 * k0 * k0 / 3.0) * ir;
  *im = (2.0 * k0 * k0 / 3.0) * ii;
}

void self_term_sphere(double k0, double h, double* re, double* im) {
  *re = self_term_re(k0, h);
  *im = self_term_im(k0, h);
}

hipError_t launch_green_sample_self(c64* work, const GroupGeom& g, int ab, double h, double k0,
                                    double s_re, double s_im, hipStream_t s) {
  k_green_sample<<<2048, 256, 0, s>>>(work, g, ab, h, k0, s_re, s_im);
  return hipGetLastError();
}

hipError_t launch_octant(const c64* work, c64* s64, c32* s32, const GroupGeom& g, int ab,
                         hipStream_t s) {
  k_octant<<<1024, 256, 0, s>>>(work, s64, s32, g, ab);
  return hipGetLastError();
}

}  // namespace vie
