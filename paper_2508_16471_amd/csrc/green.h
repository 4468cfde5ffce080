// Self-term variants of the Green spectrum setup.
#pragma once

#include "kernels.h"

namespace vie {

// Default self term (equal-volume sphere, radiation-reaction imaginary part).
void self_term_sphere(double k0, double h, double* re, double* im);

// Self term with the exact cube cell: -1/3 + (2 k0^2 / 3) times the integral of
// e^{i k0 r} / (4 pi r) over the voxel (edge h) about its centre.
void self_term_cube(double k0, double h, double* re, double* im);

// The integral of e^{i k0 r} / (4 pi r) over the cube of edge h about its
// centre (the cell's own potential coefficient of the rooftop operator).
void cube_green_integral(double k0, double h, double* re, double* im);

// launch_green_sample with a given self term s (diagonal samples xx, yy, zz).
hipError_t launch_green_sample_self(c64* work, const GroupGeom& g, int ab, double h, double k0,
                                    double s_re, double s_im, hipStream_t s);

}  // namespace vie
