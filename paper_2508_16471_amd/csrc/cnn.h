// Learned warm start: a 4-layer 3x3x3 convolutional network evaluated on a
// body's bounding box (channels-last bf16 activations, fp32 accumulation on
// bf16 MFMA), with its training kernels (backward data / weight, loss, Adam).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "common.h"

namespace vie {

using bf16raw = uint16_t;

// Architecture: 32 -> 32 -> 32 -> 32 -> 16 channels, ReLU between layers.
// Input features (25 used): chi/4 and the Krylov vectors b, A b, A^2 b, A^3 b
// (FP32 products), each divided by its rms over the body (re, im of x, y, z);
// outputs 0..5 = w/s (re,im x 3) with s = rms of |b| over the body.
constexpr int kCnnLayers = 4;
constexpr int kCnnCh[kCnnLayers + 1] = {32, 32, 32, 32, 16};
constexpr int kCnnKrylov = 4;
constexpr int kCnnFeat = 1 + 6 * kCnnKrylov;
constexpr int kCnnIn = 32;  // feature channels (padded)
constexpr int kCnnOut = 6;

struct CnnLayerOffsets {
  int64_t w[kCnnLayers], b[kCnnLayers], total;
};
CnnLayerOffsets cnn_offsets();  // parameter layout: per layer W[27][Cout][Cin] then b[Cout]

struct Cnn {
  CnnLayerOffsets off;
  float* p = nullptr;      // fp32 master parameters
  float* m = nullptr;      // Adam moments
  float* v = nullptr;
  float* g = nullptr;      // gradients
  bf16raw* wf = nullptr;   // bf16 weights, forward layout [27][Cout][Cin]
  bf16raw* wb = nullptr;   // bf16 weights, backward-data layout [27][Cin][Cout] (flipped taps)
  int64_t step = 0;
  // workspace (grown on demand)
  size_t ws_vox = 0;
  bf16raw* act[kCnnLayers] = {nullptr};  // layer inputs (act[0] = features)
  bf16raw* gbuf[2] = {nullptr, nullptr}; // activation gradients (ping-pong)
  float* out = nullptr;                  // network output [vox][16] fp32
  float* wpart = nullptr;                // weight-gradient partials
  float* loss = nullptr;                 // [2] numerator, denominator
  float* hostloss = nullptr;
};

hipError_t cnn_alloc(Cnn& c);
void cnn_free(Cnn& c);
hipError_t cnn_ensure_ws(Cnn& c, size_t vox);
hipError_t cnn_refresh_bf16(Cnn& c, hipStream_t s);          // after parameters change
// forward on feat [d2][d1][d0][16] bf16; keeps layer inputs in c.act; out fp32 [vox][16]
hipError_t cnn_forward(Cnn& c, const int d[3], const bf16raw* feat, float* out, hipStream_t s);
// loss (masked relative L2 over outputs 0..5, mask = feature channel 0 > 0) and
// backward; gradients accumulate into c.g (zeroed first).  loss_host may be null.
hipError_t cnn_backward(Cnn& c, const int d[3], const float* target, float* loss_host,
                        hipStream_t s);
hipError_t cnn_adam(Cnn& c, float lr, hipStream_t s);

// features of one right-hand side on its body's box: Krylov vectors vec[k]
// body-compressed (component-major, nb voxels) with scales inv[k] (1/rms);
// box origin lo[3] and dims d[3].
hipError_t launch_cnn_features(bf16raw* feat, const int d[3], const int lo[3], const int N[3],
                               const int* vox, const double* chic, int nb,
                               const c64* const vec[kCnnKrylov], const double inv[kCnnKrylov],
                               hipStream_t st);
hipError_t launch_cnn_target(float* tgt, const int d[3], const int lo[3], const int N[3],
                             const int* vox, int nb, const c64* w, double s, hipStream_t st);
hipError_t launch_cnn_gather(c64* x, const float* out, const int d[3], const int lo[3],
                             const int N[3], const int* vox, int nb, double s, hipStream_t st);

}  // namespace vie
