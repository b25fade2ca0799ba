// Internal launchers of the learned-guess network kernels (net.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace smgn {
// Upper bound on the weight-gradient partial sums (floats): the pixel chunk
// of smgn::wgrad grows until the per-chunk partials fit (8 MiB).
constexpr size_t kWgradMaxPartials = (size_t)2 << 20;
// pixel chunk and partial-sum floats of smgn::wgrad for a layer
int wgrad_chunk(int npix, int cout, int cin);
size_t wgrad_partials(int npix, int cout, int cin);
// 3x3 convolution with fused forms (see k_conv3 in net.hip): the input
// (optionally the decoder's concatenation, channels 0..31 upsampled from
// `lo`), the output and the optional pooled copy / 1x1 output layer.
struct ConvIn {
  const unsigned short* in;  // ics elements per pixel (the skip half at channel 32 when lo is set)
  const unsigned short* lo;  // or null
  int ics, cin;
  const unsigned short* W;
  const float* bias;
};
struct ConvOut {
  unsigned short* out;  // or null
  int ocs, cout;
  const unsigned short* mask;
  int mcs;
  bool relu;
  unsigned short* pooled;  // or null
  int pcs;
  const unsigned short* w1;  // or null
  const float* b1;
  float* y1;
};
hipError_t conv3x(const ConvIn& in, const ConvOut& out, int N, int H, int Wd, hipStream_t st);
// 3x3 convolution (MFMA): see k_conv3 in net.hip for the layout.
hipError_t conv3(const unsigned short* in, int ics, int cin, const unsigned short* W, const float* bias,
                 unsigned short* out, int ocs, int cout, const unsigned short* mask, int mcs, bool relu, int N, int H,
                 int Wd, hipStream_t st);
// weight and bias gradients of a 3x3 convolution (dW overwritten, db accumulated)
hipError_t wgrad(const unsigned short* g, int gcs, int cout, const unsigned short* x, int xcs, int cin, float* part,
                 size_t part_floats, float* dW, float* db, int N, int H, int Wd, hipStream_t st);
hipError_t flip_weights(const unsigned short* W, int cout, int cin, unsigned short* Wd, hipStream_t st);
hipError_t pool(const unsigned short* in, int ics, unsigned short* out, int ocs, int C, int N, int H, int Wd,
                hipStream_t st);
hipError_t up(const unsigned short* in, int ics, unsigned short* out, int ocs, int C, int N, int H, int Wd,
              hipStream_t st);
hipError_t up_back(const unsigned short* gin, int gcs, const unsigned short* mask, int mcs, unsigned short* gout, int ocs,
                   int C, int N, int H, int Wd, hipStream_t st);
hipError_t pool_back(const unsigned short* gpool, int pcs, const unsigned short* skip, int scs, const unsigned short* e,
                     int ecs, unsigned short* gout, int ocs, int C, int N, int H, int Wd, hipStream_t st);
hipError_t to_bf16(const float* in, unsigned short* out, size_t n, hipStream_t st);
hipError_t out_layer(const unsigned short* d, int dcs, int C, const unsigned short* w, const float* b, float* y, int npix,
                     hipStream_t st);
hipError_t out_layer_back(const float* gy, const unsigned short* d, int dcs, const unsigned short* w, unsigned short* gd,
                          int gcs, int npix, float* dw, float* db, hipStream_t st);
hipError_t mse(const float* y, const float* t, float* gy, int n, float* loss, hipStream_t st);
hipError_t adam(float* p, const float* g, float* m, float* v, unsigned short* pb, int n, float lr, float b1, float b2,
                float eps, int step, hipStream_t st);
hipError_t params_bf16(const float* p, unsigned short* pb, int n, hipStream_t st);
hipError_t fill_f32(float* p, size_t n, float v, hipStream_t st);
}  // namespace smgn
