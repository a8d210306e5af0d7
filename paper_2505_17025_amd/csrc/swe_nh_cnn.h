// swe_nh_cnn.h -- host interface of the warm-start network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "swe_nh_common.h"

namespace swenh {

// byte offsets of the network's buffers inside a workspace
struct CnnLayout {
  size_t wpk[6];    // BF16 packed weights (forward)
  size_t wpk_t[6];  // BF16 packed weights (input gradient: transposed, flipped taps)
  size_t act[5];    // BF16 NHWC activations of layers 0..4
  size_t out;       // FP32 output [n][h][w]
  size_t dy_a, dy_b, dy16;  // BF16 NHWC gradients
  size_t part, part_b;      // weight-gradient partial sums
  size_t mse_part, mse_w;
  int nblk_w;
  size_t bytes;
};

int64_t cnn_param_count();
CnnLayout cnn_layout(int n, int h, int w);
CnnLayout cnn_layout_infer(int n, int h, int w);
void cnn_pack_weights(const float* params, char* ws, const CnnLayout& L, bool with_transposed,
                      hipStream_t s);
// box (device, nullable): [x0, y0, x1, y1) of the image, the pixel tiles to
// compute (tiles outside it keep their old values)
void cnn_forward(const float* params, const uint16_t* x, int n, int h, int w, char* ws,
                 const CnnLayout& L, float* out, hipStream_t s, const int* box = nullptr);
void cnn_backward(const float* params, const uint16_t* x, const float* dout, int n, int h, int w,
                  char* ws, const CnnLayout& L, float* grad, hipStream_t s);
// network input of the grid (org null) or of its w x h window at org = (i0, j0)
// (device), in the window's NHWC layout
void cnn_features(const Chan* ch, const double* ds, int nx, int ny, double dx, double dy,
                  const double* scale, const double* t, const double* dt, const double* ht,
                  const double* mt, const double* nt, const uint8_t* mask, uint16_t* out,
                  hipStream_t s, const int* org = nullptr, int w = 0, int h = 0);

}  // namespace swenh
