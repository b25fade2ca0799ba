// Host description of the learned-guess network: parameter layout, state
// buffers and the workspace of one batch shape (net.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "smg.h"

namespace smg {

constexpr int kNetMaxLevels = 6;

struct NetLayer {
  int kind;         // 3: 3x3 convolution, 1: 1x1 output layer
  int cin, cout;
  size_t w_off, b_off;  // offsets into the parameter vector
};

// Byte offsets of one batch shape's arrays in the caller's work buffer.
struct NetWork {
  int n, H, W;
  size_t x32, xb, y, gy, tgt;
  size_t h[kNetMaxLevels], a[kNetMaxLevels], cat[kNetMaxLevels], ad[kNetMaxLevels], d[kNetMaxLevels];
  size_t ebot;
  size_t g32a[kNetMaxLevels], g32b[kNetMaxLevels], g64[kNetMaxLevels];
  size_t part, part_floats;
  size_t bytes;
};

struct NetDef {
  int levels, ch, in_ch;
  std::vector<NetLayer> layers;
  size_t n_params = 0;
  // bound state: FP32 parameters, gradients, Adam moments; BF16 copy
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
  unsigned short *pb = nullptr, *wflip = nullptr;

  NetDef(int levels, int ch, int in_ch);
  size_t state_bytes() const;
  void bind(char* state);
  NetWork work_layout(int n, int H, int W) const;
  // forward: x32 (FP32 NHWC) -> y (train: keep every activation the
  // backward pass reads; otherwise the concatenations are read in place and
  // the top decoder output is not stored); backward: gy -> g (overwritten)
  smg_status forward(char* work, const NetWork& w, hipStream_t st, bool train) const;
  smg_status backward(char* work, const NetWork& w, hipStream_t st) const;
};

}  // namespace smg

struct smg_net {
  smg::NetDef def;
  char* state = nullptr;
  int step = 0;
  smg_net(int l, int c, int i) : def(l, c, i) {}
};
